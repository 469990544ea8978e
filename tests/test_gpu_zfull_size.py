"""Full-size parity: the 512^3 lognormal-mock workload, in the launch
configuration the benchmark times, against stored FP64 oracle results.

``tests/golden/h512_golden.json`` is written by
``tests/golden/make_h512_golden.py``, which runs only the oracle: P_0,2,4 in
all 60 bins and B_0,2,4 with N^T on the triangles whose three bins lie in a
fixed sample of bins.  The GPU draws the same seeded mock; the stored
catalogue digest proves it is bit-identical before any number is compared.
Tolerances and conditioning floors are those of the small-case parity tests:
1e-10 (FP64 plans) and 2e-4 (FP32 plans) relative per bin against
max(|ref|, c_b).
"""

import json
import os
import sys

import numpy as np
import pytest

from paper_1506_02729_amd import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "h512_golden.json")
TOL = {64: 1e-10, 32: 2e-4}


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(gpu, ref, floor):
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), floor)


@pytest.fixture(scope="module")
def h512():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    import bench
    wl = bench.workload(False)
    _log("case: H512 mock generation (seed 2000)")
    gal, ran, alpha, obs, _ = synth.lognormal_mock(n_mesh=wl["n_mesh"], box=wl["box"], n_gal=wl["n_gal"],
                                                   n_ran=wl["n_ran"], seed=2000)
    digest = synth.catalog_digest(gal, ran, alpha, obs)
    # same seed, same generator, same NumPy: a different digest is an error
    assert digest == gold["catalog_sha256"], (
        f"this host drew a different mock ({digest[:16]} vs stored {gold['catalog_sha256'][:16]})")
    from paper_1506_02729_amd import fastrsd as F
    dev = torch.device("cuda:0")
    yield dict(gold=gold, wl=wl, F=F, bench=bench, alpha=alpha, obs=obs, n_obj=len(gal["w"]) + len(ran["w"]),
               g=F.device_catalog(gal, dev), r=F.device_catalog(ran, dev))
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [64, 32])
def test_h512_against_oracle(h512, precision):
    import torch
    _log(f"case: H512 full-size parity precision={precision}")
    F, gold = h512["F"], h512["gold"]
    tol = TOL[precision]
    cfg = h512["bench"].make_config(F, h512["wl"], precision, h512["obs"], h512["n_obj"])
    plan = F.Plan(cfg, device=torch.device("cuda:0"))
    from paper_1506_02729_amd import autotune
    _log(f"  launch parameters of the benchmark: {autotune.apply(plan)}")  # as bench.py times them
    out = plan.run(h512["g"], h512["r"], h512["alpha"])
    assert plan.status() == 0

    pk, sc = gold["pk"], gold["scalars"]
    nb = np.asarray(pk["n_modes"])
    np.testing.assert_array_equal(out["n_modes"], nb)
    assert np.max(_rel(out["k_eff"], np.asarray(pk["k_eff"]), 0)) < 1e-12
    np.testing.assert_allclose(out["scalars"], [sc["I22"], sc["N0"], sc["I33"], sc["W3"]], rtol=1e-12)
    I22 = sc["I22"]
    floors = {0: np.asarray(pk["S00"]) / (nb * I22)}
    for ell in (2, 4):
        floors[ell] = (2 * ell + 1) * np.asarray(pk[f"C{ell}0"]) / (nb * I22)
    for ell in (0, 2, 4):
        e = _rel(out[f"p{ell}"], np.asarray(pk[f"P{ell}"]), floors[ell])
        _log(f"  P{ell}: max rel err {e.max():.3e}")
        assert e.max() < tol, (f"P{ell}", e)

    bk = gold["bk"]
    idx = np.asarray(bk["index"])
    np.testing.assert_array_equal(plan.triangles[idx], np.asarray(bk["triangles"]))
    nt = np.asarray(bk["NT"])
    np.testing.assert_array_equal(out["bk_nt"][idx], nt)
    ok = nt > 0
    for ell in (0, 2, 4):
        C = np.asarray(bk[f"C{ell}"])[ok]
        e = _rel(out[f"bk_t{ell}"][idx][ok], np.asarray(bk[f"T{ell}"])[ok], C)
        _log(f"  T{ell}: max rel err {e.max():.3e} over {ok.sum()} triangles")
        assert e.max() < tol, (f"T{ell}", e)
        floor = (2 * ell + 1) * C / (nt[ok] * sc["I33"])
        e = _rel(out[f"bk_b{ell}"][idx][ok], np.asarray(bk[f"B{ell}"])[ok], floor)
        assert e.max() < tol, (f"B{ell}", e)
    assert np.all(np.isnan(out["bk_b0"][idx][~ok]))
    sn0 = np.asarray(bk["SN0"])
    assert np.max(_rel(out["bk_sn0"][idx], sn0, np.abs(sn0))) < tol
    for ell in (2, 4):
        sn = np.asarray(bk[f"SN{ell}"])
        assert np.max(_rel(out[f"bk_sn{ell}"][idx], sn, np.max(np.abs(sn)))) < tol
    del plan
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# 1024^3: streamed moment meshes against the stored FP64 oracle results
# (tests/golden/cfg5_golden.json, written by make_cfg5_golden.py: P_0, P_2
# and the split hexadecapole P_4b in 100 bins of 0.005 h/Mpc).

GOLDEN_1024 = os.path.join(HERE, "golden", "cfg5_golden.json")


@pytest.fixture(scope="module")
def mesh1024():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    with open(GOLDEN_1024) as fh:
        gold = json.load(fh)
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_cfg5_golden as m5
    _log("case: 1024^3 mock generation (seed 5000, r_smooth 3)")
    gal, ran, alpha, obs, _ = m5.mock()
    digest = synth.catalog_digest(gal, ran, alpha, obs)
    assert digest == gold["catalog_sha256"], (
        f"this host drew a different mock ({digest[:16]} vs stored {gold['catalog_sha256'][:16]})")
    from paper_1506_02729_amd import fastrsd as F
    dev = torch.device("cuda:0")
    n_obj = len(gal["w"]) + len(ran["w"])
    g, r = F.device_catalog(gal, dev), F.device_catalog(ran, dev)
    del gal, ran
    yield dict(gold=gold, F=F, m5=m5, alpha=alpha, obs=obs, n_obj=n_obj, g=g, r=r)
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", [64, 32])
def test_1024_streamed_against_oracle(mesh1024, precision):
    """Streamed plan (two complex slots resident) at N = 1024, P_0, P_2, P_4b
    per bin against the oracle, floors as in the small-case tests; P_4 (22
    moments) is not in the stored results and is checked as finite."""
    import torch
    _log(f"case: 1024^3 streamed parity precision={precision}")
    F, gold, m5 = mesh1024["F"], mesh1024["gold"], mesh1024["m5"]
    tol = TOL[precision]
    cfg = F.Config(n_grid=m5.N, box=m5.BOX, observer=mesh1024["obs"], order=3, interlace=True, compensate=True,
                   ell_max=4, precision=precision, pk_kmin=0.0, pk_dk=m5.PK_DK, pk_nbins=m5.PK_NBINS,
                   max_objects=mesh1024["n_obj"], stream_moments=True)
    plan = F.Plan(cfg, device=torch.device("cuda:0"))
    out = plan.run(mesh1024["g"], mesh1024["r"], mesh1024["alpha"], bispectrum=False)
    pk, sc = gold["pk"], gold["scalars"]
    nb = np.asarray(pk["n_modes"])
    np.testing.assert_array_equal(out["n_modes"], nb)
    np.testing.assert_allclose(out["scalars"], [sc["I22"], sc["N0"], sc["I33"], sc["W3"]], rtol=1e-12)
    I22 = sc["I22"]
    floors = {"P0": np.asarray(pk["S00"]) / (nb * I22), "P2": 5 * np.asarray(pk["C20"]) / (nb * I22),
              "P4b": (17.5 * np.asarray(pk["S22"]) + 5 * np.asarray(pk["C20"]) + 3.5 * np.asarray(pk["S00"]))
              / (nb * I22)}
    for key, name in (("P0", "p0"), ("P2", "p2"), ("P4b", "p4b")):
        e = _rel(out[name], np.asarray(pk[key]), floors[key])
        _log(f"  {key}: max rel err {e.max():.3e}")
        assert e.max() < tol, (key, e)
    assert np.all(np.isfinite(out["p4"]))
    del plan
    torch.cuda.empty_cache()
