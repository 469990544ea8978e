"""Requests captured as HIP graphs (frsd_graph_create / frsd_graph_launch):
replays with catalogues of different sizes and contents in the captured
buffers, with the program's own eager work and synchronisations between
them, each checked against the eager path on the same data (1e-5 of the
largest value for FP32 plans, 1e-10 for FP64) and against the FP64 oracle
(the parity tolerance)."""

import sys

import numpy as np
import pytest

from oracle import estimator as est
from test_gpu_parity import _bk_case, _cfg, _check_bk, _check_pk

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _fill(buf, cat, torch):
    n = len(cat["w"])
    for key in ("pos", "w", "nbar"):
        buf[key][:n].copy_(torch.as_tensor(np.ascontiguousarray(cat[key]), dtype=buf[key].dtype))


@pytest.mark.parametrize("precision", [32, 64])
def test_graph_replays_match_eager_requests(gpu_lib, precision):
    import torch
    F = gpu_lib
    dev = torch.device("cuda:0")
    _log(f"case: graph capture of a 48^3 request, precision={precision}")
    gal, ran, alpha, prm = _bk_case(161, N=48, nbk=5, n_gal=3000, n_ran=15000)
    gal_b, ran_b, _, _ = _bk_case(162, N=48, nbk=5, n_gal=2000, n_ran=9000)
    alpha_b = 2000 / 9000
    cap = len(gal["w"]) + len(ran["w"])
    cfg = _cfg(F, prm, precision, cap)
    plan = F.Plan(cfg, device=dev, stream=torch.cuda.Stream(dev))
    eager = F.Plan(cfg, device=dev, stream=torch.cuda.Stream(dev))
    gbuf = {k: torch.zeros((len(gal["w"]), 3) if k == "pos" else len(gal["w"]), dtype=torch.float64, device=dev)
            for k in ("pos", "w", "nbar")}
    rbuf = {k: torch.zeros((len(ran["w"]), 3) if k == "pos" else len(ran["w"]), dtype=torch.float64, device=dev)
            for k in ("pos", "w", "nbar")}
    _fill(gbuf, gal, torch)
    _fill(rbuf, ran, torch)
    torch.cuda.synchronize()
    graph = plan.capture(gbuf, rbuf, alpha)
    close = 1e-5 if precision == 32 else 1e-10

    def replay(cat_g, cat_r, a):
        _fill(gbuf, cat_g, torch)
        _fill(rbuf, cat_r, torch)
        torch.cuda.synchronize()
        graph.launch(len(cat_g["w"]), len(cat_r["w"]), a)
        torch.cuda.synchronize()
        out = {k: v.cpu().numpy().copy() for k, v in plan.pk_buf.items()}
        out.update({"bk_" + k: v.cpu().numpy().copy() for k, v in plan.bk_buf.items()})
        return out

    def eager_run(cat_g, cat_r, a):
        return eager.run(F.device_catalog(cat_g, dev), F.device_catalog(cat_r, dev), a)

    results = []
    for rep, (g, r, a) in enumerate(((gal, ran, alpha), (gal_b, ran_b, alpha_b), (gal, ran, alpha),
                                     (gal_b, ran_b, alpha_b))):
        _log(f"  replay {rep}: {len(g['w'])} + {len(r['w'])} objects")
        got = replay(g, r, a)
        ref = eager_run(g, r, a)          # eager work and a synchronisation between replays
        np.testing.assert_array_equal(got["n_modes"], ref["n_modes"])
        np.testing.assert_array_equal(got["bk_nt"], ref["bk_nt"])
        np.testing.assert_allclose(got["scalars"], ref["scalars"], rtol=1e-12)
        for key in ("p0", "p2", "p4", "p4b", "s00", "bk_t0", "bk_t2", "bk_t4", "bk_sn0", "bk_sn2", "bk_sn4"):
            scale = np.max(np.abs(ref[key]))
            assert np.max(np.abs(got[key] - ref[key])) <= close * scale, (rep, key)
        if rep < 2:
            fields = est.multipole_fields(g, r, a, prm, with_w=True)
            _check_pk(got, est.pk_multipoles(g, r, a, prm, fields=fields), prm, precision)
            _check_bk(got, est.bk_multipoles(g, r, a, prm, fields=fields), prm, precision, plan)
        results.append(got)
    # the replays of one catalogue agree with each other, and the two differ
    assert np.max(np.abs(results[0]["p0"] - results[2]["p0"])) <= close * np.max(np.abs(results[0]["p0"]))
    assert np.max(np.abs(results[0]["p0"] - results[1]["p0"])) > 1e-3 * np.max(np.abs(results[0]["p0"]))
    with pytest.raises(F.FrsdError) as ei:
        graph.launch(len(gal["w"]) + 1, len(ran["w"]), alpha)
    assert ei.value.code == F.FRSD_ENOMEM
    del graph


@pytest.mark.parametrize("precision", [32, 64])
def test_batch_graph_replays_match_eager_batches(gpu_lib, precision):
    """A batch of three 48^3 requests captured as one graph
    (frsd_graph_create_batch), replayed with other sizes, contents and alpha
    per request (frsd_graph_launch_batch), with eager batches and
    synchronisations between the replays: each replay against the eager
    batch on the same data and against the oracle."""
    import torch
    F = gpu_lib
    dev = torch.device("cuda:0")
    _log(f"case: graph capture of a batch of three 48^3 requests, precision={precision}")
    sets = []
    for k in range(3):
        g, r, a, prm = _bk_case(170 + k, N=48, nbk=1, n_gal=2500 + 400 * k, n_ran=12000 + 1500 * k)
        g2, r2, _, _ = _bk_case(180 + k, N=48, nbk=1, n_gal=1600 + 300 * k, n_ran=8000 + 900 * k)
        sets.append(((g, r, a), (g2, r2, len(g2["w"]) / len(r2["w"]))))
    prm.bk_nbins = 0
    cap = max(len(s[0][0]["w"]) + len(s[0][1]["w"]) for s in sets)
    cfg = _cfg(F, prm, precision, cap)
    stream = torch.cuda.Stream(dev)
    plans = [F.Plan(cfg, device=dev, stream=stream) for _ in sets]
    eager = [F.Plan(cfg, device=dev, stream=stream) for _ in sets]

    def buffers(c):
        return {k: torch.zeros((len(c["w"]), 3) if k == "pos" else len(c["w"]), dtype=torch.float64, device=dev)
                for k in ("pos", "w", "nbar")}

    gbufs = [buffers(s[0][0]) for s in sets]
    rbufs = [buffers(s[0][1]) for s in sets]
    for k, s in enumerate(sets):
        _fill(gbufs[k], s[0][0], torch)
        _fill(rbufs[k], s[0][1], torch)
    torch.cuda.synchronize()
    graph = F.capture_batch(plans, gbufs, rbufs, [s[0][2] for s in sets])
    close = 1e-5 if precision == 32 else 1e-10
    for rep, which in enumerate((0, 1, 0, 1)):
        reqs = [s[which] for s in sets]
        _log(f"  replay {rep}: " + ", ".join(f"{len(g['w'])} + {len(r['w'])}" for g, r, _ in reqs))
        for k, (g, r, _) in enumerate(reqs):
            _fill(gbufs[k], g, torch)
            _fill(rbufs[k], r, torch)
        torch.cuda.synchronize()
        graph.launch([len(g["w"]) for g, _, _ in reqs], [len(r["w"]) for _, r, _ in reqs], [a for _, _, a in reqs])
        torch.cuda.synchronize()
        got = [{k: v.cpu().numpy().copy() for k, v in p.pk_buf.items()} for p in plans]
        ref = F.run_batch(eager, [F.device_catalog(g, dev) for g, _, _ in reqs],
                          [F.device_catalog(r, dev) for _, r, _ in reqs], [a for _, _, a in reqs])
        for k, (g, r, a) in enumerate(reqs):
            np.testing.assert_array_equal(got[k]["n_modes"], ref[k]["n_modes"])
            np.testing.assert_allclose(got[k]["scalars"], ref[k]["scalars"], rtol=1e-12)
            for key in ("p0", "p2", "p4", "p4b", "s00"):
                scale = np.max(np.abs(ref[k][key]))
                assert np.max(np.abs(got[k][key] - ref[k][key])) <= close * scale, (rep, k, key)
            if rep < 2:
                _check_pk(got[k], est.pk_multipoles(g, r, a, prm), prm, precision)
    with pytest.raises(F.FrsdError):
        F.frsd_graph_launch(graph.handle, 10, 10, 0.1, stream.cuda_stream)  # a batch graph needs the batch call
