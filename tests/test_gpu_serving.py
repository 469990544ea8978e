"""Serving: requests in flight together on separate plans and streams give
the same results as each request alone (the stated tolerance: 2e-4 per bin
for FP32 plans against the FP64 oracle), and a workspace is reused across
requests without carrying anything over."""

import sys

import numpy as np
import pytest

from oracle import estimator as est
from test_gpu_parity import _bk_case, _cfg, _check_bk, _check_pk

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_results_same_alone_and_in_the_mix(gpu_lib):
    import torch
    _log("case: three FP32 48^3 requests alone, then in flight together on three streams")
    dev = torch.device("cuda:0")
    cases = [_bk_case(61 + i) for i in range(3)]
    n_max = max(len(g["w"]) + len(r["w"]) for g, r, _, _ in cases)
    prm = cases[0][3]
    cfg = _cfg(gpu_lib, prm, 32, n_max)
    cats = [(gpu_lib.device_catalog(g, dev), gpu_lib.device_catalog(r, dev), a) for g, r, a, _ in cases]
    torch.cuda.synchronize()

    alone_plan = gpu_lib.Plan(cfg, device=dev)
    alone = [alone_plan.run(g, r, a) for g, r, a in cats]

    plans = [gpu_lib.Plan(cfg, device=dev, stream=torch.cuda.Stream(dev)) for _ in cats]
    torch.cuda.synchronize()
    for plan, (g, r, a) in zip(plans, cats):  # enqueue all three before any result is read
        plan.mesh_assign(g, r, a)
        plan.pk()
        plan.bk()
    torch.cuda.synchronize()
    for i, plan in enumerate(plans):
        assert plan.status() == 0
        mix = {k: v.cpu().numpy() for k, v in plan.pk_buf.items()}
        mix.update({"bk_" + k: v.cpu().numpy() for k, v in plan.bk_buf.items()})
        gal, ran, alpha, prm_i = cases[i]
        fields = est.multipole_fields(gal, ran, alpha, prm_i, with_w=True)
        _check_pk(mix, est.pk_multipoles(gal, ran, alpha, prm_i, fields=fields), prm_i, 32)
        _check_bk(mix, est.bk_multipoles(gal, ran, alpha, prm_i, fields=fields), prm_i, 32, plan)
        np.testing.assert_array_equal(mix["n_modes"], alone[i]["n_modes"])
        np.testing.assert_array_equal(mix["bk_nt"], alone[i]["bk_nt"])
        for key in ("p0", "p2", "p4", "p4b", "bk_t0", "bk_t2", "bk_t4"):
            scale = np.max(np.abs(alone[i][key]))
            assert np.max(np.abs(mix[key] - alone[i][key])) <= 1e-5 * scale, (i, key)


def test_mixed_sizes_in_flight(gpu_lib):
    """Requests of different mesh sizes and bin sets in flight together: a
    48^3 (gather assignment), a 64^3 (x-sweep assignment) and a 96^3 FP32
    plan, each on its own stream, enqueued before any result is read; each
    result equals the same request run alone (1e-5 of the largest value) and
    the FP64 oracle (2e-4 per bin)."""
    import torch
    _log("case: 48^3, 64^3 and 96^3 FP32 requests in flight together")
    dev = torch.device("cuda:0")
    cases = [_bk_case(111, N=48, nbk=5), _bk_case(112, N=64, nbk=6, n_gal=4000, n_ran=20000),
             _bk_case(113, N=96, nbk=8, n_gal=8000, n_ran=40000)]
    cases[2][3].pk_nbins = 20
    cfgs = [_cfg(gpu_lib, prm, 32, len(g["w"]) + len(r["w"])) for g, r, _, prm in cases]
    cats = [(gpu_lib.device_catalog(g, dev), gpu_lib.device_catalog(r, dev), a) for g, r, a, _ in cases]
    torch.cuda.synchronize()
    alone = [gpu_lib.Plan(cfg, device=dev).run(g, r, a) for cfg, (g, r, a) in zip(cfgs, cats)]
    plans = [gpu_lib.Plan(cfg, device=dev, stream=torch.cuda.Stream(dev)) for cfg in cfgs]
    torch.cuda.synchronize()
    for plan, (g, r, a) in zip(plans, cats):
        plan.mesh_assign(g, r, a)
        plan.pk()
        plan.bk()
    torch.cuda.synchronize()
    for i, plan in enumerate(plans):
        assert plan.status() == 0
        mix = {k: v.cpu().numpy() for k, v in plan.pk_buf.items()}
        mix.update({"bk_" + k: v.cpu().numpy() for k, v in plan.bk_buf.items()})
        gal, ran, alpha, prm = cases[i]
        fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
        _check_pk(mix, est.pk_multipoles(gal, ran, alpha, prm, fields=fields), prm, 32)
        _check_bk(mix, est.bk_multipoles(gal, ran, alpha, prm, fields=fields), prm, 32, plan)
        np.testing.assert_array_equal(mix["n_modes"], alone[i]["n_modes"])
        np.testing.assert_array_equal(mix["bk_nt"], alone[i]["bk_nt"])
        for key in ("p0", "p2", "p4", "p4b", "bk_t0", "bk_t2", "bk_t4"):
            scale = np.max(np.abs(alone[i][key]))
            assert np.max(np.abs(mix[key] - alone[i][key])) <= 1e-5 * scale, (i, key)


@pytest.mark.parametrize("precision,cached", [(32, False), (64, True)])
def test_batch_server_results_same_alone_and_in_the_mix(gpu_lib, precision, cached):
    """The continuous-batching server (paper_1506_02729_amd/serve.py): ten
    48^3 requests submitted together to two groups of four plans, so that
    batches of up to four form while others run, each result equal to the
    same request alone (within 1e-5 of the largest value for FP32, 1e-11 for
    FP64) and two of them to the oracle; with cached randoms every request
    shares one random catalogue."""
    import torch
    from paper_1506_02729_amd.serve import BatchServer
    dev = torch.device("cuda:0")
    _log(f"case: batch server, 10 requests, precision={precision} cached={cached}")
    cases = [_bk_case(190 + i, nbk=1, n_gal=1500 + 200 * i, n_ran=9000 + 500 * i) for i in range(10)]
    prm = cases[0][3]
    prm.bk_nbins = 0
    ran0 = cases[0][1]
    if cached:
        cases = [(g, ran0, len(g["w"]) / len(ran0["w"]), p) for g, _, _, p in cases]
    cap = max(len(g["w"]) + len(r["w"]) for g, r, _, _ in cases)
    cfg = _cfg(gpu_lib, prm, precision, cap)
    cfg.random_cache = cached
    r0 = gpu_lib.device_catalog(ran0, dev)
    server = BatchServer(cfg, groups=2, group_size=4, device=dev, randoms=r0 if cached else None)
    cats = [(gpu_lib.device_catalog(g, dev), None if cached else gpu_lib.device_catalog(r, dev), a)
            for g, r, a, _ in cases]
    torch.cuda.synchronize()
    reqs = [server.submit(g, a, r) for g, r, a in cats]
    done = server.drain()
    assert sorted(r.rid for r in done) == [r.rid for r in reqs]
    assert max(server.batch_sizes) > 1 and sum(server.batch_sizes) == len(reqs)
    assert server.rejected() == 0
    alone = gpu_lib.Plan(cfg, device=dev)
    if cached:
        alone.random_cache(r0)
    close = 1e-5 if precision == 32 else 1e-11
    for k, (req, (g, r, a)) in enumerate(zip(reqs, cats)):
        ref = alone.run_cached(g, a, bispectrum=False) if cached else alone.run(g, r, a, bispectrum=False)
        np.testing.assert_array_equal(req.result["n_modes"], ref["n_modes"])
        np.testing.assert_allclose(req.result["scalars"], ref["scalars"], rtol=1e-12)
        for key in ("p0", "p2", "p4", "p4b", "s00"):
            scale = np.max(np.abs(ref[key]))
            assert np.max(np.abs(req.result[key] - ref[key])) <= close * scale, (k, key)
        if k in (0, 7):
            gh, rh, ah, _ = cases[k]
            _check_pk(req.result, est.pk_multipoles(gh, rh, ah, prm), prm, precision)
