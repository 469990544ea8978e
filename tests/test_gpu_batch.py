"""GPU parity of request batches (frsd_pk_batch): several requests on plans
of one shape share one forward-FFT launch per pass and one binning launch.
Each request of a batch is checked against the oracle (tolerances of
``test_gpu_parity``: 1e-10 FP64, 2e-4 FP32 per bin) and against the same
request run alone through frsd_mesh_assign + frsd_pk_multipoles (within
1e-5 of the largest value for FP32, whose node sums depend on the order of
objects within a cell, and 1e-11 for FP64).  The plans are left as after
that sequence: the bispectrum and the status follow per plan.
"""

import sys

import numpy as np
import pytest

from oracle import estimator as est
from test_gpu_parity import _bk_case, _cfg, _check_bk, _check_pk

pytestmark = pytest.mark.gpu

CLOSE = {32: 1e-5, 64: 1e-11}
KEYS = ("p0", "p2", "p4", "p4b", "s00", "s20", "s40", "k_eff")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests(n, N, interlace=True, ell_max=4, nbk=0, seed=900):
    """n catalogues of different sizes on one configuration (the first's)."""
    reqs = []
    prm = None
    for r in range(n):
        gal, ran, alpha, p = _bk_case(seed + r, N=N, interlace=interlace, ell_max=ell_max, nbk=max(nbk, 1),
                                      n_gal=1500 + 700 * r, n_ran=9000 + 1100 * (r % 4))
        if prm is None:
            prm = p
            if nbk == 0:
                prm.bk_nbins = 0
            if N < 48:
                prm.pk_nbins = 9  # top edge 15.8 k_f, below the Nyquist frequency of N = 32
        reqs.append((gal, ran, alpha))
    return reqs, prm


def _same(a, b, close, keys=KEYS):
    for key in keys:
        if np.all(np.isnan(b[key])):
            assert np.all(np.isnan(a[key])), key
            continue
        scale = np.nanmax(np.abs(b[key]))
        assert np.nanmax(np.abs(a[key] - b[key])) <= close * scale, key
    np.testing.assert_array_equal(a["n_modes"], b["n_modes"])
    np.testing.assert_allclose(a["scalars"], b["scalars"], rtol=1e-12)


@pytest.mark.parametrize("precision,N,interlace,ell_max,nbk,n_req", [
    (32, 64, True, 4, 5, 3),    # compiled FFT length, x-sweep (16-node runs), bispectrum after the batch
    (64, 64, True, 4, 5, 3),
    (32, 128, True, 4, 0, 4),   # x-sweep with 32-node runs (4 x 256 workgroups)
    (32, 48, False, 2, 0, 3),   # slots pairing two planes, P_ell only
    (64, 80, True, 4, 0, 3),    # run-time FFT length (pencil kernels)
    (32, 80, False, 4, 0, 3),
])
def test_batch_matches_alone_and_oracle(gpu_lib, precision, N, interlace, ell_max, nbk, n_req):
    import torch
    dev = torch.device("cuda:0")
    _log(f"case: batch of {n_req} N={N} interlace={interlace} ell_max={ell_max} nbk={nbk} precision={precision}")
    reqs, prm = _requests(n_req, N, interlace, ell_max, nbk)
    cap = max(len(g["w"]) + len(r["w"]) for g, r, _ in reqs)
    cfg = _cfg(gpu_lib, prm, precision, cap)
    plans = [gpu_lib.Plan(cfg, device=dev) for _ in reqs]
    gals = [gpu_lib.device_catalog(g, dev) for g, _, _ in reqs]
    rans = [gpu_lib.device_catalog(r, dev) for _, r, _ in reqs]
    outs = gpu_lib.run_batch(plans, gals, rans, [a for _, _, a in reqs])
    alone = gpu_lib.Plan(cfg, device=dev)
    for k, (g, r, a) in enumerate(reqs):
        fields = est.multipole_fields(g, r, a, prm, with_w=True)
        refp = est.pk_multipoles(g, r, a, prm, fields=fields)
        _check_pk(outs[k], refp, prm, precision)
        _same(outs[k], alone.run(gals[k], rans[k], a, bispectrum=False), CLOSE[precision])
        if nbk:
            # the batch's binning wrote each request's low-k fields into its own workspace
            refb = est.bk_multipoles(g, r, a, prm, fields=fields)
            bk = {"bk_" + key: v.cpu().numpy().copy() for key, v in plans[k].bk().items()}
            _check_bk(bk, refb, prm, precision, plans[k])
        assert plans[k].status() == 0
    if nbk:
        # a batch after the bispectrum calls (which took the mesh regions), the requests in reverse order
        again = gpu_lib.run_batch(plans, gals[::-1], rans[::-1], [a for _, _, a in reqs][::-1])
        for k in range(n_req):
            _same(again[k], outs[n_req - 1 - k], CLOSE[precision])


@pytest.mark.parametrize("precision", [32, 64])
def test_batch_against_random_caches(gpu_lib, precision):
    """rans = None: every plan holds the randoms' spectra (frsd_random_cache)
    and each request's galaxies, with its own alpha, are combined with them."""
    import torch
    dev = torch.device("cuda:0")
    _log(f"case: batch of 4 against random caches N=64 precision={precision}")
    reqs, prm = _requests(4, 64, seed=940)
    ran = reqs[0][1]
    alphas = [len(g["w"]) / len(ran["w"]) for g, _, _ in reqs]
    cap = max(max(len(g["w"]) for g, _, _ in reqs), len(ran["w"]))
    cfg = _cfg(gpu_lib, prm, precision, cap)
    cfg.random_cache = True
    rd = gpu_lib.device_catalog(ran, dev)
    plans = [gpu_lib.Plan(cfg, device=dev) for _ in reqs]
    for p in plans:
        p.random_cache(rd)
    gals = [gpu_lib.device_catalog(g, dev) for g, _, _ in reqs]
    outs = gpu_lib.run_batch(plans, gals, None, alphas)
    alone = gpu_lib.Plan(cfg, device=dev)
    alone.random_cache(rd)
    for k, (g, _, _) in enumerate(reqs):
        refp = est.pk_multipoles(g, ran, alphas[k], prm)
        _check_pk(outs[k], refp, prm, precision)
        _same(outs[k], alone.run_cached(gals[k], alphas[k], bispectrum=False), CLOSE[precision])


def test_largest_batch(gpu_lib):
    """FRSD_MAX_BATCH requests at N = 32 (FP64), one of them without galaxies;
    then a second, smaller batch on the same plans; then a plain
    frsd_pk_multipoles call on one plan repeats its batched result."""
    import torch
    dev = torch.device("cuda:0")
    n = gpu_lib.FRSD_MAX_BATCH
    _log(f"case: batch of {n} N=32 FP64, then a batch of 5")
    reqs, prm = _requests(n, 32, seed=960)
    empty = {"pos": np.zeros((0, 3)), "w": np.zeros(0), "nbar": np.zeros(0)}
    reqs[5] = (empty, reqs[5][1], reqs[5][2])
    cap = max(len(g["w"]) + len(r["w"]) for g, r, _ in reqs)
    cfg = _cfg(gpu_lib, prm, 64, cap)
    plans = [gpu_lib.Plan(cfg, device=dev) for _ in range(n)]
    gals = [gpu_lib.device_catalog(g, dev) for g, _, _ in reqs]
    rans = [gpu_lib.device_catalog(r, dev) for _, r, _ in reqs]
    outs = gpu_lib.run_batch(plans, gals, rans, [a for _, _, a in reqs])
    refs = [est.pk_multipoles(g, r, a, prm) for g, r, a in reqs]
    for k in range(n):
        if k == 5:
            np.testing.assert_array_equal(outs[k]["n_modes"], refs[k]["n_modes"])
            assert np.max(np.abs(outs[k]["s00"] - refs[k]["S00"]) / np.abs(refs[k]["S00"])) < 1e-10
        _check_pk(outs[k], refs[k], prm, 64)
    # a smaller batch on plans 3, 1, 4, 0, 2 (new order, other requests)
    order = [3, 1, 4, 0, 2]
    sub = [reqs[k + 8] for k in range(5)]
    outs2 = gpu_lib.run_batch([plans[k] for k in order], [gals[k + 8] for k in range(5)],
                              [rans[k + 8] for k in range(5)], [a for _, _, a in sub])
    for j in range(5):
        _check_pk(outs2[j], refs[j + 8], prm, 64)
    # plan 3 holds request 8's meshes: P_ell again from them
    again = {k: v.cpu().numpy().copy() for k, v in plans[3].pk().items()}
    _same(again, outs2[0], CLOSE[64])


def test_batch_catalogue_dtypes(gpu_lib):
    """FP32 catalogues in a batch (the ingest reads them as they are), a
    batch mixing FP32 and FP64 catalogues (ingested one request at a time),
    and page-locked host catalogues, on FP64 plans; the oracle gets the same
    FP32-rounded catalogues."""
    import torch
    dev = torch.device("cuda:0")
    _log("case: batch catalogue dtypes N=48 FP64")
    reqs, prm = _requests(3, 48, seed=980)

    def rounded(c):
        return {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in c.items()}

    cap = max(len(g["w"]) + len(r["w"]) for g, r, _ in reqs)
    cfg = _cfg(gpu_lib, prm, 64, cap)
    plans = [gpu_lib.Plan(cfg, device=dev) for _ in reqs]
    for dts in ((torch.float32,) * 3, (torch.float32, torch.float64, torch.float32)):
        gals = [gpu_lib.device_catalog(g, dev, dt) for (g, _, _), dt in zip(reqs, dts)]
        rans = [gpu_lib.device_catalog(r, dev, dt) for (_, r, _), dt in zip(reqs, dts)]
        outs = gpu_lib.run_batch(plans, gals, rans, [a for _, _, a in reqs])
        for k, ((g, r, a), dt) in enumerate(zip(reqs, dts)):
            if dt == torch.float32:
                g, r = rounded(g), rounded(r)
            _check_pk(outs[k], est.pk_multipoles(g, r, a, prm), prm, 64)
    # catalogues in page-locked host memory, read in place by the ingest kernels
    gals = [gpu_lib.pinned_catalog(g) for g, _, _ in reqs]
    rans = [gpu_lib.pinned_catalog(r) for _, r, _ in reqs]
    outs = gpu_lib.run_batch(plans, gals, rans, [a for _, _, a in reqs])
    for k, (g, r, a) in enumerate(reqs):
        _check_pk(outs[k], est.pk_multipoles(g, r, a, prm), prm, 64)
