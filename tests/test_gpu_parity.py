"""GPU parity: the HIP path against the FP64 oracle on identical seeded inputs.

Bins counts and the triangle list must match exactly; floating point must
agree within 1e-10 (FP64 plans) or 2e-4 (FP32 plans) relative per bin, the
relative error being taken against max(|ref|, c_b) with the conditioning
scale c_b = (2 ell + 1) sum_b |A_ell| |A_0| / (N_b I22) for P_ell (and the
analogous sum of |F_ell F_0 F_0| for B_ell), because P_2, P_4 and B_ell can
cross zero.
"""

import math
import sys

import numpy as np
import pytest

from oracle import estimator as est
from paper_1506_02729_amd import synth

pytestmark = pytest.mark.gpu

TOL = {64: 1e-10, 32: 2e-4}
_ORACLE_CACHE = {}   # oracle results shared by the precisions of one case


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cfg(F, prm: est.Params, precision, max_objects, m_grid=None):
    return F.Config(n_grid=prm.n_grid, box=prm.box, observer=prm.observer, order=prm.order,
                    interlace=prm.interlace, compensate=prm.compensate, ell_max=prm.ell_max,
                    precision=precision, pk_kmin=prm.pk_kmin, pk_dk=prm.pk_dk, pk_nbins=prm.pk_nbins,
                    bk_kmin=prm.bk_kmin, bk_dk=prm.bk_dk, bk_nbins=prm.bk_nbins,
                    bk_grid=prm.m_grid if m_grid is None else m_grid, max_objects=max_objects)


def _run_gpu(F, prm, precision, gal, ran, alpha, in_dtype=None, m_grid=None):
    import torch
    dev = torch.device("cuda:0")
    n = len(gal["w"]) + (len(ran["w"]) if ran is not None else 0)
    plan = F.Plan(_cfg(F, prm, precision, max(n, 1), m_grid), device=dev)
    dt = in_dtype or torch.float64
    g = F.device_catalog(gal, dev, dt)
    r = F.device_catalog(ran, dev, dt) if ran is not None else None
    out = plan.run(g, r, alpha)
    return out, plan


def _rel(gpu, ref, floor):
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), floor)


def _check_pk(out, ref, prm, precision):
    tol = TOL[precision]
    np.testing.assert_array_equal(out["n_modes"], ref["n_modes"])
    nb = ref["n_modes"].astype(float)
    assert np.max(_rel(out["k_eff"], ref["k_eff"], 0)) < 1e-12
    I22 = ref["I22"]
    np.testing.assert_allclose(out["scalars"], [ref["I22"], ref["N0"], ref["I33"], ref["W3"]], rtol=1e-12)
    floor0 = ref["S00"] / (nb * I22)
    e0 = _rel(out["p0"], ref["P0"], floor0)
    assert np.max(e0) < tol, ("P0", e0)
    for ell in (2, 4):
        if ell > prm.ell_max:
            continue
        floor = (2 * ell + 1) * ref[f"C{ell}0"] / (nb * I22)
        e = _rel(out[f"p{ell}"], ref[f"P{ell}"], floor)
        assert np.max(e) < tol, (f"P{ell}", e)
    e = _rel(out["s00"], ref["S00"], 0)
    assert np.max(e) < tol
    if prm.ell_max >= 2:
        # split hexadecapole: floor from the magnitudes of its three terms
        floor4b = (17.5 * ref["S22"] + 5.0 * ref["C20"] + 3.5 * ref["S00"]) / (nb * I22)
        e = _rel(out["p4b"], ref["P4b"], floor4b)
        assert np.max(e) < tol, ("P4b", e)
        assert np.max(_rel(out["s22"], ref["S22"], 0)) < tol
    else:
        assert np.all(np.isnan(out["p4b"]))


def _check_bk(out, ref, prm, precision, plan):
    tol = TOL[precision]
    np.testing.assert_array_equal(plan.triangles, ref["triangles"])
    np.testing.assert_array_equal(out["bk_nt"], ref["NT"])
    ok = ref["NT"] > 0
    for ell in (0, 2, 4):
        if ell > prm.ell_max:
            continue
        e = _rel(out[f"bk_t{ell}"][ok], ref[f"T{ell}"][ok], ref[f"C{ell}"][ok])
        assert np.max(e) < tol, (f"T{ell}", np.max(e))
        floor = (2 * ell + 1) * ref[f"C{ell}"][ok] / (ref["NT"][ok] * ref["I33"])
        e = _rel(out[f"bk_b{ell}"][ok], ref[f"B{ell}"][ok], floor)
        assert np.max(e) < tol, (f"B{ell}", np.max(e))
    assert np.all(np.isnan(out["bk_b0"][~ok]))
    e = _rel(out["bk_sn0"], ref["SN0"], np.abs(ref["SN0"]))
    assert np.max(e) < tol
    for ell in (2, 4):
        if ell <= prm.ell_max:
            e = _rel(out[f"bk_sn{ell}"], ref[f"SN{ell}"], np.max(np.abs(ref[f"SN{ell}"])))
            assert np.max(e) < tol


# ---------------------------------------------------------------------------

def _tiny_config():
    gal, ran, alpha, obs = synth.tiny_survey(seed=1000)
    kf = 2 * math.pi / 500.0
    prm = est.Params(n_grid=64, box=500.0, observer=obs, order=2, interlace=False, compensate=True,
                     ell_max=4, pk_kmin=0.0, pk_dk=2 * kf, pk_nbins=16)
    return gal, ran, alpha, prm


@pytest.mark.parametrize("precision", [64, 32])
def test_pk_tiny_survey_cic(gpu_lib, precision):
    """64^3 CIC, no interlacing, compensated, 16 bins of 2 k_f up to Nyquist."""
    _log(f"case: pk tiny survey 64^3 CIC precision={precision}")
    gal, ran, alpha, prm = _tiny_config()
    ref = est.pk_multipoles(gal, ran, alpha, prm)
    out, _ = _run_gpu(gpu_lib, prm, precision, gal, ran, alpha)
    _check_pk(out, ref, prm, precision)


def _bk_case(seed, N=48, order=3, interlace=True, ell_max=4, nbk=5, n_gal=3000, n_ran=15000):
    rng = np.random.Generator(np.random.PCG64(seed))
    box = 600.0
    gal = synth.uniform_box(n_gal, box, rng, nbar=n_gal / box**3, w=0.6)
    ran = synth.uniform_box(n_ran, box, rng, nbar=n_gal / box**3, w=0.6)
    gal["w"] = 0.4 + 0.4 * rng.random(n_gal)
    ran["w"] = 0.4 + 0.4 * rng.random(n_ran)
    ran["nbar"] = ran["nbar"] * (0.5 + rng.random(n_ran))
    kf = 2 * math.pi / box
    prm = est.Params(n_grid=N, box=box, observer=(-200.0, 310.0, -150.0), order=order, interlace=interlace,
                     compensate=True, ell_max=ell_max, pk_kmin=0.5 * kf, pk_dk=1.7 * kf, pk_nbins=13,
                     bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=nbk)
    return gal, ran, n_gal / n_ran, prm


@pytest.mark.parametrize("precision,order,interlace", [(64, 3, True), (32, 3, True), (64, 1, False),
                                                       (32, 2, True), (64, 4, True), (32, 4, True),
                                                       (32, 4, False)])
def test_pk_bk_interlaced(gpu_lib, precision, order, interlace):
    _log(f"case: pk+bk 48^3 order={order} interlace={interlace} precision={precision}")
    gal, ran, alpha, prm = _bk_case(7 + order, order=order, interlace=interlace)
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
    refp = est.pk_multipoles(gal, ran, alpha, prm, fields=fields)
    refb = est.bk_multipoles(gal, ran, alpha, prm, fields=fields)
    out, plan = _run_gpu(gpu_lib, prm, precision, gal, ran, alpha)
    _check_pk(out, refp, prm, precision)
    _check_bk(out, refb, prm, precision, plan)


@pytest.mark.parametrize("precision", [64, 32])
def test_pruned_fft_passes_192(gpu_lib, precision):
    """N = 192 with k_max = 40.5 k_f: the forward FFT passes keep only
    frequencies |n_d| <= 40 in column blocks that do not divide N."""
    _log(f"case: pk+bk 192^3 pruned FFT precision={precision}")
    if "pruned192" not in _ORACLE_CACHE:
        gal, ran, alpha, prm = _bk_case(23, N=192, n_gal=30000, n_ran=150000)
        kf = prm.kf
        prm.pk_kmin, prm.pk_dk, prm.pk_nbins = 0.5 * kf, 2.0 * kf, 20
        prm.bk_nbins = 6
        fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
        refp = est.pk_multipoles(gal, ran, alpha, prm, fields=fields)
        refb = est.bk_multipoles(gal, ran, alpha, prm, fields=fields)
        _ORACLE_CACHE["pruned192"] = (gal, ran, alpha, prm, refp, refb)
    gal, ran, alpha, prm, refp, refb = _ORACLE_CACHE["pruned192"]
    out, plan = _run_gpu(gpu_lib, prm, precision, gal, ran, alpha)
    _check_pk(out, refp, prm, precision)
    _check_bk(out, refb, prm, precision, plan)


@pytest.mark.parametrize("precision,m_gpu", [(64, 50), (32, 50), (64, 56), (32, 56), (64, 343), (32, 343),
                                             (64, 360), (32, 360)])
def test_radix5_triangle_grids(gpu_lib, precision, m_gpu):
    """The triangle search on 5- and 7-smooth real-space grids: M = 50 and
    56 (run-time schedules 5, 5, 2 and 7, 8), M = 343 and 360 (compiled
    schedules 7, 7, 7 and 3, 3, 5, 8).  Any M > 3 n_c gives the exact
    closed-triangle sums, so the oracle keeps its own grid (M = 54 here) and
    the results must agree."""
    _log(f"case: pk+bk 48^3 bk_grid={m_gpu} precision={precision}")
    if "radix5" not in _ORACLE_CACHE:
        gal, ran, alpha, prm = _bk_case(29)
        fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
        refp = est.pk_multipoles(gal, ran, alpha, prm, fields=fields)
        refb = est.bk_multipoles(gal, ran, alpha, prm, fields=fields)
        _ORACLE_CACHE["radix5"] = (gal, ran, alpha, prm, refp, refb)
    gal, ran, alpha, prm, refp, refb = _ORACLE_CACHE["radix5"]
    assert est.bk_grid(prm) == 54
    out, plan = _run_gpu(gpu_lib, prm, precision, gal, ran, alpha, m_grid=m_gpu)
    _check_pk(out, refp, prm, precision)
    _check_bk(out, refb, prm, precision, plan)


@pytest.mark.parametrize("precision,order,interlace", [(64, 3, True), (32, 3, True), (64, 2, False),
                                                       (32, 4, True)])
def test_sparse_survey_region(gpu_lib, precision, order, interlace):
    """Objects confined to a region that wraps the periodic x boundary and
    covers a band of y, plus one isolated pair of objects: most node columns
    and x slabs are empty, and the occupancy masks (from the cell counts,
    dilated by the kernel reach across the boundary) must leave the result
    equal to the dense oracle one."""
    _log(f"case: sparse survey region order={order} interlace={interlace} precision={precision}")
    rng = np.random.Generator(np.random.PCG64(31 + order))
    box, N = 600.0, 48

    def region(n, w):
        u = rng.random((n, 3))
        u[:, 0] = (0.25 * u[:, 0] - 0.1) % 1.0    # x in [0.9, 1) and [0, 0.15)
        u[:, 1] = 0.3 + 0.2 * u[:, 1]             # y in [0.3, 0.5)
        u[:2] = [[0.55, 0.8, 0.2], [0.56, 0.81, 0.9]]
        pos = np.minimum(u * box, np.nextafter(box, 0.0))
        return {"pos": pos, "w": w + 0.4 * rng.random(n), "nbar": np.full(n, 3e-5) * (0.5 + rng.random(n))}

    gal, ran = region(3000, 0.4), region(15000, 0.4)
    kf = 2 * math.pi / box
    prm = est.Params(n_grid=N, box=box, observer=(-200.0, 310.0, -150.0), order=order, interlace=interlace,
                     compensate=True, ell_max=4, pk_kmin=0.5 * kf, pk_dk=1.7 * kf, pk_nbins=13,
                     bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=5)
    alpha = 3000 / 15000
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
    refp = est.pk_multipoles(gal, ran, alpha, prm, fields=fields)
    refb = est.bk_multipoles(gal, ran, alpha, prm, fields=fields)
    out, plan = _run_gpu(gpu_lib, prm, precision, gal, ran, alpha)
    _check_pk(out, refp, prm, precision)
    _check_bk(out, refb, prm, precision, plan)


@pytest.mark.parametrize("precision,order,interlace", [(32, 1, True), (32, 2, True), (32, 3, True), (32, 1, False),
                                                       (32, 3, False), (32, 4, True), (32, 4, False),
                                                       (64, 1, True), (64, 2, True), (64, 3, True), (64, 2, False)])
def test_fp32_assignment_orders_64(gpu_lib, precision, order, interlace):
    """Plans on N = 64 (a multiple of 64: the x-sweep assignment for orders
    1-3, FP32 and FP64 instantiations, with the half-cell trimming of the
    TSC main and CIC twin windows; the gather for PCS) for every order with
    and without interlacing, against the FP64 oracle."""
    _log(f"case: pk+bk 64^3 precision={precision} order={order} interlace={interlace}")
    gal, ran, alpha, prm = _bk_case(41 + order, N=64, order=order, interlace=interlace, n_gal=4000, n_ran=20000)
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
    refp = est.pk_multipoles(gal, ran, alpha, prm, fields=fields)
    refb = est.bk_multipoles(gal, ran, alpha, prm, fields=fields)
    out, plan = _run_gpu(gpu_lib, prm, precision, gal, ran, alpha)
    _check_pk(out, refp, prm, precision)
    _check_bk(out, refb, prm, precision, plan)


def test_ell_max_two_and_float32_inputs(gpu_lib):
    _log("case: ell_max=2, float32 catalogue into FP64 plan")
    gal, ran, alpha, prm = _bk_case(3, ell_max=2, nbk=4)
    # the oracle sees exactly the float32-rounded positions
    for c in (gal, ran):
        for k in ("pos", "w", "nbar"):
            c[k] = c[k].astype(np.float32).astype(np.float64)
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
    refp = est.pk_multipoles(gal, ran, alpha, prm, fields=fields)
    refb = est.bk_multipoles(gal, ran, alpha, prm, fields=fields)
    import torch
    out, plan = _run_gpu(gpu_lib, prm, 64, gal, ran, alpha, in_dtype=torch.float32)
    _check_pk(out, refp, prm, 64)
    _check_bk(out, refb, prm, 64, plan)
    assert np.all(np.isnan(out["p4"]))


def test_empty_randoms_and_repeat_calls(gpu_lib):
    """No randoms: I22 = I33 = 0, normalised outputs are NaN/inf, raw sums
    stay valid; a second call on the same plan gives the same result."""
    _log("case: empty randoms, repeated calls")
    gal, ran, alpha, prm = _bk_case(11, nbk=3)
    fields = est.multipole_fields(gal, None, 0.0, prm, with_w=True)
    refp = est.pk_multipoles(gal, None, 0.0, prm, fields=fields)
    out, plan = _run_gpu(gpu_lib, prm, 64, gal, None, 0.0)
    np.testing.assert_array_equal(out["n_modes"], refp["n_modes"])
    assert np.max(_rel(out["s00"], refp["S00"], 0)) < 1e-10
    assert out["scalars"][0] == 0.0
    import torch
    g = gpu_lib.device_catalog(gal, torch.device("cuda:0"), torch.float64)
    again = plan.run(g, None, 0.0)
    np.testing.assert_allclose(again["s20"], out["s20"], rtol=1e-12)


def test_no_caching_by_input_identity(gpu_lib):
    """Served requests recompute everything: the same device buffers refilled
    with another catalogue of the same size give that catalogue's spectra
    (each checked against the oracle), and the first catalogue again gives
    its own spectra, on one plan and workspace."""
    _log("case: no caching by buffer identity (FP32, 48^3, pk + bk)")
    import torch
    dev = torch.device("cuda:0")
    gal_a, ran_a, alpha, prm = _bk_case(51)
    gal_b, ran_b, _, _ = _bk_case(52)
    plan = gpu_lib.Plan(_cfg(gpu_lib, prm, 32, len(gal_a["w"]) + len(ran_a["w"])), device=dev)
    g = gpu_lib.device_catalog(gal_a, dev, torch.float64)
    r = gpu_lib.device_catalog(ran_a, dev, torch.float64)

    def refill(dst, src):
        for key in ("pos", "w", "nbar"):
            dst[key].copy_(torch.as_tensor(np.ascontiguousarray(src[key]), dtype=torch.float64))

    results = []
    for gal, ran in ((gal_a, ran_a), (gal_b, ran_b), (gal_a, ran_a)):
        refill(g, gal)
        refill(r, ran)
        out = plan.run(g, r, alpha)
        fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
        _check_pk(out, est.pk_multipoles(gal, ran, alpha, prm, fields=fields), prm, 32)
        _check_bk(out, est.bk_multipoles(gal, ran, alpha, prm, fields=fields), prm, 32, plan)
        results.append(out)
    assert np.max(np.abs(results[0]["p0"] - results[1]["p0"])) > 1e-3 * np.max(np.abs(results[0]["p0"]))


def test_out_of_box_objects_are_rejected(gpu_lib):
    _log("case: out-of-box rejection")
    gal, ran, alpha, prm = _bk_case(13, nbk=0)
    gal["pos"][:5] = -1.0
    gal["pos"][5:7] = prm.box + 10.0
    import torch
    dev = torch.device("cuda:0")
    plan = gpu_lib.Plan(_cfg(gpu_lib, prm, 64, len(gal["w"]) + len(ran["w"])), device=dev)
    g = gpu_lib.device_catalog(gal, dev)
    r = gpu_lib.device_catalog(ran, dev)
    with pytest.raises(gpu_lib.FrsdError) as ei:
        plan.run(g, r, alpha)
    assert ei.value.code == gpu_lib.FRSD_EDOM
    assert plan.status() == 7
    # the rejected objects contribute nothing: same as dropping them
    keep = {k: v[7:] for k, v in gal.items()}
    ref = est.pk_multipoles(keep, ran, alpha, prm)
    got = {k: v.cpu().numpy() for k, v in plan.pk_buf.items()}
    assert np.max(_rel(got["s00"], ref["S00"], 0)) < 1e-10


def test_capacity_and_order_errors(gpu_lib):
    _log("case: error codes")
    gal, ran, alpha, prm = _bk_case(17, nbk=2)
    import torch
    dev = torch.device("cuda:0")
    plan = gpu_lib.Plan(_cfg(gpu_lib, prm, 32, 100), device=dev)
    g = gpu_lib.device_catalog(gal, dev, torch.float32)
    r = gpu_lib.device_catalog(ran, dev, torch.float32)
    with pytest.raises(gpu_lib.FrsdError) as ei:
        plan.mesh_assign(g, r, alpha)
    assert ei.value.code == gpu_lib.FRSD_ENOMEM
    with pytest.raises(gpu_lib.FrsdError) as ei:
        plan.bk()
    assert ei.value.code == gpu_lib.FRSD_ESTATE
