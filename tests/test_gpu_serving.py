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
