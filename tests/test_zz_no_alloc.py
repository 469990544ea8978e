"""The entry point that allocates nothing (frsd_run_static), through the C ABI,
against the existing entry points (frsd_plan_init, frsd_mesh_assign,
frsd_pk_multipoles, frsd_bk_multipoles on a caller workspace) and the FP64
oracle: two calls in a row on one device's static scratch, the second with
a smaller catalogue (and then a smaller plan), so stale scratch contents
from the first call would show.  Tolerance of the parity tests: counts and
N^T exact, 2e-4 per bin against the oracle (FP32 plans), and 1e-5 of the
largest value against the workspace path."""

import sys

import numpy as np
import pytest

from oracle import estimator as est
from test_gpu_parity import _bk_case, _cfg, _check_bk, _check_pk

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _outputs(F, torch, plan):
    """Fresh output arrays and their C structs for one static call."""
    dev = plan.device
    f64 = dict(dtype=torch.float64, device=dev)
    nb = plan.cfg.pk_nbins
    pk = {"n_modes": torch.full((nb,), -1, dtype=torch.int64, device=dev)}
    for key in ("k_eff", "p0", "p2", "p4", "s00", "s20", "s40", "p4b", "s22"):
        pk[key] = torch.full((nb,), np.nan, **f64)
    pk["scalars"] = torch.full((4,), np.nan, **f64)
    bk = {key: torch.full((plan.ntri,), np.nan, **f64)
          for key in ("nt", "t0", "t2", "t4", "b0", "b2", "b4", "sn0", "sn2", "sn4")}
    po, bo = F.frsd_pk_out(), F.frsd_bk_out()
    for name in F.PK_ARRAYS:
        setattr(po, name, pk[name].data_ptr())
    for name in F.BK_ARRAYS:
        setattr(bo, name, bk[name].data_ptr() if name in bk else None)
    return pk, bk, po, bo


def _static_run(F, torch, plan, g, r, alpha):
    pk, bk, po, bo = _outputs(F, torch, plan)
    F.frsd_run_static(plan.handle, F._c_catalog(g), F._c_catalog(r), alpha, po, bo, plan.stream.cuda_stream)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in pk.items()}
    out.update({"bk_" + k: v.cpu().numpy() for k, v in bk.items()})
    return out


def _compare(out, ref_ws, gal, ran, alpha, prm, plan):
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
    _check_pk(out, est.pk_multipoles(gal, ran, alpha, prm, fields=fields), prm, 32)
    _check_bk(out, est.bk_multipoles(gal, ran, alpha, prm, fields=fields), prm, 32, plan)
    np.testing.assert_array_equal(out["n_modes"], ref_ws["n_modes"])
    np.testing.assert_array_equal(out["bk_nt"], ref_ws["bk_nt"])
    for key in ("p0", "p2", "p4", "p4b", "s00", "bk_t0", "bk_t2", "bk_t4", "bk_sn0", "bk_sn2"):
        scale = np.max(np.abs(ref_ws[key]))
        assert np.max(np.abs(out[key] - ref_ws[key])) <= 1e-5 * scale, key


def test_static_entry_point_matches_workspace_path(gpu_lib):
    import torch
    F = gpu_lib
    dev = torch.device("cuda:0")
    _log("case: frsd_run_static, 48^3 FP32 plan, 3000 + 15000 then 1200 + 6000 objects")
    gal, ran, alpha, prm = _bk_case(121, N=48, nbk=5)
    plan = F.Plan(_cfg(F, prm, 32, len(gal["w"]) + len(ran["w"])), device=dev)
    assert plan.ws_bytes <= 128 << 20
    small = (_bk_case(122, N=48, nbk=5, n_gal=1200, n_ran=6000))
    for g_h, r_h, a in ((gal, ran, alpha), (small[0], small[1], small[2])):
        g, r = F.device_catalog(g_h, dev), F.device_catalog(r_h, dev)
        ref_ws = plan.run(g, r, a)                   # existing entry points, caller workspace
        out = _static_run(F, torch, plan, g, r, a)   # static scratch
        _compare(out, ref_ws, g_h, r_h, a, prm, plan)

    _log("case: frsd_run_static on a smaller plan (32^3, 3 bins) after the 48^3 one")
    g32, r32, a32, prm32 = _bk_case(123, N=32, nbk=3, n_gal=1000, n_ran=5000)
    prm32.pk_nbins = 8
    plan32 = F.Plan(_cfg(F, prm32, 32, len(g32["w"]) + len(r32["w"])), device=dev)
    g, r = F.device_catalog(g32, dev), F.device_catalog(r32, dev)
    ref_ws = plan32.run(g, r, a32)
    out = _static_run(F, torch, plan32, g, r, a32)
    _compare(out, ref_ws, g32, r32, a32, prm32, plan32)


def test_static_entry_point_rejects_large_plans(gpu_lib):
    import torch
    F = gpu_lib
    _log("case: frsd_run_static with a plan larger than the scratch")
    gal, ran, alpha, prm = _bk_case(124, N=96, nbk=8)
    h = F.frsd_plan_create(_cfg(F, prm, 32, 60000).to_c())
    assert F.frsd_plan_workspace_bytes(h) > 128 << 20
    dev = torch.device("cuda:0")
    g, r = F.device_catalog(gal, dev), F.device_catalog(ran, dev)
    po, bo = F.frsd_pk_out(), F.frsd_bk_out()
    with pytest.raises(F.FrsdError) as ei:
        F.frsd_run_static(h, F._c_catalog(g), F._c_catalog(r), alpha, po, bo, None)
    assert ei.value.code == F.FRSD_ENOMEM
    assert "static scratch" in str(ei.value)
    F.frsd_plan_destroy(h)
