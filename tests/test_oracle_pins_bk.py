"""Pins of the oracle's normalisations, bispectrum prefactors and shot-noise
terms against what the paper and the mathematics fix (CPU only).

* closed forms of the scalar sums I22, I33, N_0 and the w^3 sum (Sec. III.A
  eqs. I22def, N0true; Sec. III.B eq. Noise0; I33 read as alpha sum_r
  nbar^2 w^3);
* P_0, P_2, P_4 of a Poisson-sampled deterministic field against the exact
  expectation (normalisation I22, shot noise N_0, prefactors 2 ell + 1;
  Sec. III.A eqs. P0_impl-P4_impl);
* B_ell prefactors and T_220 placement in the plane-parallel limit against
  direct triangle enumeration (Sec. III.B eqs. BispMono, BispQuad; Sec. II.C
  eq. Bhexa2);
* a random-phase Gaussian field gives triangle sums consistent with zero;
* the thin-shell shot noise (eq. SNbisp2thin) against the exact eq. SNbisp2
  in lattice configurations where the thin-shell form is exact.
"""

import math

import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import brute, estimator as est
from paper_1506_02729_amd import synth

FAR = 1e12   # observer distance in box units for the plane-parallel limit


def _uniform(seed, ng, nr, box, nbar, w):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.uniform_box(ng, box, rng, nbar, w), synth.uniform_box(nr, box, rng, nbar, w)


# --------------------------------------------------------------------------
# scalar sums
# --------------------------------------------------------------------------

def test_scalar_sums_closed_forms():
    """Constant nbar and w: I22 = alpha N_r nbar w^2 = nbar^2 w^2 V,
    I33 = alpha N_r nbar^2 w^3 = nbar^3 w^3 V, N_0 = (N_g + alpha^2 N_r) w^2,
    W3 = (N_g - alpha^3 N_r) w^3; I22 and I33 do not depend on the galaxies
    and scale as w_r^2 nbar and w_r^3 nbar^2."""
    box, ng, nr, nbar, w = 500.0, 3000, 12000, 3000 / 500.0**3, 0.6
    gal, ran = _uniform(17, ng, nr, box, nbar, w)
    alpha = ng / nr
    sc = est.scalars(gal, ran, alpha)
    V = box**3
    assert sc["I22"] == pytest.approx(alpha * nr * nbar * w**2, rel=1e-13)
    assert sc["I22"] == pytest.approx(nbar**2 * w**2 * V, rel=1e-13)
    assert sc["I33"] == pytest.approx(alpha * nr * nbar**2 * w**3, rel=1e-13)
    assert sc["I33"] == pytest.approx(nbar**3 * w**3 * V, rel=1e-13)
    assert sc["N0"] == pytest.approx((ng + alpha**2 * nr) * w**2, rel=1e-13)
    assert sc["W3"] == pytest.approx((ng - alpha**3 * nr) * w**3, rel=1e-13)
    # galaxies do not enter I22, I33; randoms' weights and densities do
    gal2 = dict(gal, w=gal["w"] * 1.7, nbar=gal["nbar"] * 3.0)
    sc2 = est.scalars(gal2, ran, alpha)
    assert sc2["I22"] == sc["I22"] and sc2["I33"] == sc["I33"]
    ran2 = dict(ran, w=ran["w"] * 2.0, nbar=ran["nbar"] * 3.0)
    sc3 = est.scalars(gal, ran2, alpha)
    assert sc3["I22"] == pytest.approx(sc["I22"] * 4.0 * 3.0, rel=1e-13)
    assert sc3["I33"] == pytest.approx(sc["I33"] * 8.0 * 9.0, rel=1e-13)
    assert sc3["N0"] == pytest.approx(ng * w**2 + alpha**2 * nr * 4 * w**2, rel=1e-13)
    assert sc3["W3"] == pytest.approx(ng * w**3 - alpha**3 * nr * 8 * w**3, rel=1e-13)


# --------------------------------------------------------------------------
# P_ell normalisation: Poisson sampling of a deterministic field
# --------------------------------------------------------------------------

def _full_modes(N):
    f = np.fft.fftfreq(N, d=1.0 / N).astype(np.int64)
    nx, ny, nz = np.meshgrid(f, f, f, indexing="ij")
    return nx, ny, nz


def test_pk_normalisation_of_poisson_sampled_field():
    """Galaxies Poisson-sampled on the nodes of a fixed field lambda(x)
    (mean 40 per node, Kaiser-shaped fluctuations of rms 0.3), uniform random
    nodes, NGP without compensation and a distant observer along z.  Then
    F(n) = S(n) + noise with S = DFT of lambda and noise variance
    V = sum lambda + alpha^2 N_r, and F_l = L_l(nhat_z) F_0, so the exact
    expectations are
        E[P_0] = sum_b |S|^2 / (N_b I22),
        E[P_l] = (2l+1) sum_b L_l(mu) (|S|^2 + V) / (N_b I22),
    with I22 = alpha N_r nbar.  Every bin must agree within 5 sigma (the
    mode-by-mode variance 2|S|^2 V + V^2), which fixes N_0, I22 and the
    factors 1, 5, 9 (a wrong factor or normalisation is many sigma off)."""
    N, box, f = 32, 500.0, 0.7
    rng = np.random.Generator(np.random.PCG64(4040))
    cat, amp2 = synth.kaiser_nodes(N, box, f, rng)
    delta = cat["w"].reshape(N, N, N)
    delta *= 0.3 / delta.std()
    lam = 40.0 * np.clip(1.0 + delta, 0.0, None)
    counts = rng.poisson(lam)
    h = box / N
    idx = np.arange(N)
    gx, gy, gz = np.meshgrid(idx, idx, idx, indexing="ij")
    nodes = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1) * h
    gpos = np.repeat(nodes, counts.ravel(), axis=0)
    nbar = lam.sum() / box**3
    gal = {"pos": gpos, "w": np.ones(len(gpos)), "nbar": np.full(len(gpos), nbar)}
    n_r = 4 * int(lam.sum())
    rpos = nodes[rng.integers(0, N**3, n_r)]
    ran = {"pos": rpos, "w": np.ones(n_r), "nbar": np.full(n_r, nbar)}
    alpha = lam.sum() / n_r
    kf = 2 * math.pi / box
    nbins = 7
    prm = est.Params(n_grid=N, box=box, observer=(box / 2, box / 2, -FAR * box), order=1, interlace=False,
                     compensate=False, ell_max=4, pk_kmin=0.0, pk_dk=2 * kf, pk_nbins=nbins)
    res = est.pk_multipoles(gal, ran, alpha, prm)

    S = np.fft.fftn(lam)
    V = lam.sum() + alpha**2 * n_r
    I22 = alpha * n_r * nbar
    nx, ny, nz = _full_modes(N)
    m2 = nx * nx + ny * ny + nz * nz
    mu = nz / np.sqrt(np.maximum(m2, 1))
    b = np.floor(np.sqrt(m2) / 2.0).astype(int)          # edges 2 b k_f
    b = np.where((m2 > 0) & (b < nbins), b, -1)
    S2 = np.abs(S) ** 2
    var = 2 * S2 * V + V * V
    zs = []
    for ell in (0, 2, 4):
        L = eval_legendre(ell, mu)
        for k in range(nbins):
            sel = b == k
            nb = sel.sum()
            if ell == 0:
                pred = np.sum(S2[sel]) / (nb * I22)
            else:
                pred = (2 * ell + 1) * np.sum(L[sel] * (S2[sel] + V)) / (nb * I22)
            # n and -n carry the same |F|^2: the sum over the full shell has twice
            # the variance of a sum over independent modes
            sig = (2 * ell + 1) * math.sqrt(2.0 * np.sum((L[sel] ** 2) * var[sel])) / (nb * I22)
            zs.append((res[f"P{ell}"][k] - pred) / sig)
    zs = np.array(zs)
    assert np.all(np.abs(zs) < 5.0), zs
    assert np.mean(zs**2) < 4.0, zs
    assert np.all(res["n_modes"] == np.bincount(b[b >= 0], minlength=nbins))


# --------------------------------------------------------------------------
# B_ell prefactors, the zero-area hexadecapole, Gaussian fields
# --------------------------------------------------------------------------

def _pp_case(seed=23, N=32, nb=3, bk_kmin=1.5, bk_dk=3.0):
    box = 500.0
    kf = 2 * math.pi / box
    gal, ran = _uniform(seed, 500, 2500, box, 500 / box**3, 0.7)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    gal["w"] = 0.5 + rng.random(len(gal["w"]))
    ran["w"] = 0.5 + rng.random(len(ran["w"]))
    prm = est.Params(n_grid=N, box=box, observer=(box / 2, box / 2, -FAR * box), order=2, interlace=False,
                     compensate=True, ell_max=4, bk_kmin=bk_kmin * kf, bk_dk=bk_dk * kf, bk_nbins=nb)
    return gal, ran, 0.2, prm


def _value(field, N):
    return lambda n: est.gather_full(field, N, n[:, 0], n[:, 1], n[:, 2])


def _legendre_z(ell):
    return lambda n: eval_legendre(ell, n[:, 2] / np.sqrt(np.sum(n * n, axis=1))) + 0j


def test_bispectrum_prefactors_plane_parallel():
    """Distant observer: F_l(q) = L_l(qhat_z) F_0(q), so
    B_l^raw = (2l+1) sum_T L_l(qhat1_z) F_0 F_0 F_0 / (N^T I33) and
    B4za = [35/2 sum_T L_2(qhat1_z) L_2(qhat2_z) - 5 sum_T L_2(qhat1_z)
    - 7/2 sum_T 1] F_0 F_0 F_0 / (N^T I33), by direct triangle enumeration
    with the monopole field alone."""
    gal, ran, alpha, prm = _pp_case()
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
    res = est.bk_multipoles(gal, ran, alpha, prm, fields=fields, zero_area=True)
    tri = res["triangles"]
    e2 = est.squared_edges(prm.bk_kmin, prm.bk_dk, prm.bk_nbins, prm.kf)
    F0 = _value(fields[0], prm.n_grid)
    L2, L4 = _legendre_z(2), _legendre_z(4)
    L2F0 = lambda n: L2(n) * F0(n)  # noqa: E731
    cnt, (s000, s2, s4, s22) = brute.triangle_enumeration_many(
        [(F0, F0, F0), (L2F0, F0, F0), (lambda n: L4(n) * F0(n), F0, F0), (L2F0, L2F0, F0)], e2, tri)
    np.testing.assert_array_equal(cnt, res["NT"])
    I33 = est.scalars(gal, ran, alpha)["I33"]
    ok = cnt > 0
    for ell, s in ((0, s000), (2, s2), (4, s4)):
        pred = (2 * ell + 1) * s.real / (cnt * I33)
        scale = (2 * ell + 1) * res[f"C{ell}"] / (cnt * I33)
        assert np.max(np.abs(res[f"B{ell}"][ok] - pred[ok]) / scale[ok]) < 1e-8, ell
    pred = (17.5 * s22.real - 5.0 * s2.real - 3.5 * s000.real) / (cnt * I33)
    scale = (17.5 * res["C220"] + 5.0 * res["C2"] + 3.5 * res["C0"]) / (cnt * I33)
    assert np.max(np.abs(res["B4za"][ok] - pred[ok]) / scale[ok]) < 1e-8
    # B4za is not B4 for general triangles (it is a true multipole only for zero area)
    assert np.max(np.abs(res["B4za"][ok] - res["B4"][ok]) / scale[ok]) > 1e-3


def test_zero_area_hexadecapole_equals_b4_for_collinear_triangles():
    """Bins [2.7, 3.0) and [1.2, 1.5) k_f: the only closed lattice triangles
    of (b1, b2, b3) = (5, 0, 0) are q2 = q3, q1 = -2 q2 (|q2|^2 = 2), all of
    zero area, where delta_2(qhat_1, q2) = delta_2(q2) (Sec. II.C); in the
    plane-parallel limit the split of L_2^2 is then exact and
    B4za = B4 triangle by triangle."""
    gal, ran, alpha, prm = _pp_case(seed=29, bk_kmin=1.2, bk_dk=0.3, nb=6)
    tri = np.array([[5, 0, 0]])
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
    res = est.bk_multipoles(gal, ran, alpha, prm, triangles=tri, fields=fields, zero_area=True)
    assert res["NT"][0] == 12
    scale = 9 * res["C4"][0] / (res["NT"][0] * res["I33"])
    assert abs(res["B4za"][0] - res["B4"][0]) < 1e-8 * scale


def test_gaussian_field_triangle_sums_consistent_with_zero():
    """One object per node carrying a random-phase Kaiser field (no Poisson
    noise): the phases of F(q1) F(q2) F(q3) are uniform, so E[B_l] = 0 and
    every T_l is consistent with zero within its Gaussian spread
    sqrt(s sum_T |L_l F F F|^2) (s = 6, 2, 1 for equilateral, isosceles,
    scalene bin triples); their mean over triangles too."""
    N, box = 32, 500.0
    rng = np.random.Generator(np.random.PCG64(777))
    cat, _ = synth.kaiser_nodes(N, box, 0.7, rng)
    kf = 2 * math.pi / box
    prm = est.Params(n_grid=N, box=box, observer=(box / 2, box / 2, -FAR * box), order=1, interlace=False,
                     compensate=False, ell_max=4, bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=3)
    fields = est.multipole_fields(cat, None, 0.0, prm)
    tri = est.triangle_list(prm)
    ts = est.bk_triangle_sums(fields, prm, tri)
    e2 = est.squared_edges(prm.bk_kmin, prm.bk_dk, prm.bk_nbins, prm.kf)
    F0 = _value(fields[0], N)
    eq = (tri[:, 0] == tri[:, 1]) & (tri[:, 1] == tri[:, 2])
    iso = (tri[:, 0] == tri[:, 1]) | (tri[:, 1] == tri[:, 2])
    s = np.where(eq, 6.0, np.where(iso, 2.0, 1.0))
    ok = ts["NT"] > 0
    P = lambda n: np.abs(F0(n)) ** 2 + 0j  # noqa: E731
    Lz = {ell: _legendre_z(ell) for ell in (0, 2, 4)}
    _, vs = brute.triangle_enumeration_many(
        [(lambda n, e=ell: np.abs(Lz[e](n)) ** 2 * P(n), P, P) for ell in (0, 2, 4)], e2, tri)
    for ell, v in zip((0, 2, 4), vs):
        z = ts[f"T{ell}"][ok] / np.sqrt(s[ok] * v.real[ok])
        assert np.all(np.abs(z) < 5.0), (ell, z)
        assert abs(z.mean()) < 3.0 / math.sqrt(ok.sum()) + 0.3, (ell, z.mean())
    # the same statistic is far from zero when the triangle phases are aligned:
    # |F| itself (all phases zero) gives z of many sigma
    mag = {0: np.abs(fields[0]) + 0j}
    ta = est.bk_triangle_sums(mag, prm, tri)
    assert np.min(ta["T0"][ok] / np.sqrt(s[ok] * vs[0].real[ok])) > 5.0


# --------------------------------------------------------------------------
# shot noise (Sec. III.B eqs. Noise0, SNbisp2, SNbisp2thin)
# --------------------------------------------------------------------------

def test_shell_sums_of_w2_multipoles_plane_parallel():
    """Distant observer: F_l = L_l(khat_z) F_0 and F^w_l = L_l(khat_z) F^w_0
    per mode, so S_lw = sum_b Re F_l (F^w_0)^* and Q_lw = sum_b Re F_0
    (F^w_l)^* both equal sum_b L_l(khat_z) Re F_0 (F^w_0)^*."""
    gal, ran, alpha, prm = _pp_case(seed=31, N=32, nb=4)
    prm.pk_kmin, prm.pk_dk, prm.pk_nbins = 0.0, 2 * prm.kf, 8
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w_ell=True)
    for kmin, dk, nb in ((prm.pk_kmin, prm.pk_dk, prm.pk_nbins), (prm.bk_kmin, prm.bk_dk, prm.bk_nbins)):
        sh = est.shell_sums(fields, prm, kmin, dk, nb)
        nx, ny, nz = _full_modes(prm.n_grid)
        m2 = nx * nx + ny * ny + nz * nz
        e2 = est.squared_edges(kmin, dk, nb, prm.kf)
        b = np.searchsorted(e2, m2, side="right") - 1
        b = np.where((m2 > 0) & (b >= 0) & (b < nb), b, -1)
        sel = b >= 0
        n = np.stack([nx[sel], ny[sel], nz[sel]], axis=1)
        g = (_value(fields[0], prm.n_grid)(n) * np.conj(_value(fields["w"], prm.n_grid)(n))).real
        for ell in (2, 4):
            ref = np.bincount(b[sel], weights=_legendre_z(ell)(n).real * g, minlength=nb)
            scale = np.bincount(b[sel], weights=np.abs(g), minlength=nb)
            assert np.max(np.abs(sh[f"S{ell}w"] - ref) / scale) < 1e-9
            assert np.max(np.abs(sh[f"Q{ell}w"] - ref) / scale) < 1e-9


def _exact_shot_noise(fields, prm, tri, I33, ell, mixed):
    """Eq. SNbisp2 by triangle enumeration; ``mixed(n1, n_i)`` gives
    F^w_l(qhat_1, -q_i) for the sides i = 2, 3."""
    N = prm.n_grid
    e2 = est.squared_edges(prm.bk_kmin, prm.bk_dk, prm.bk_nbins, prm.kf)
    Fl, F0, Fw = (_value(fields[k], N) for k in (ell, 0, "w"))
    one = lambda n: np.ones(len(n), dtype=complex)  # noqa: E731
    cnt, a = brute.triangle_enumeration_slots(lambda n: Fl(n) * np.conj(Fw(n)), one, one, e2, tri)
    total = a.real.copy()
    # sides 2 and 3 need q1 and q_i together: enumerate them by hand
    nc = int(math.ceil(math.sqrt(e2[-1])) - 1)
    r = np.arange(-nc, nc + 1)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    m2 = np.sum(g * g, axis=1)
    bb = np.searchsorted(e2, m2, side="right") - 1
    bb = np.where((m2 > 0) & (bb >= 0) & (bb < len(e2) - 1), bb, -1)
    for t, (b1, b2, b3) in enumerate(tri):
        n1, n2 = g[bb == b1], g[bb == b2]
        n3 = -(n1[:, None, :] + n2[None, :, :])
        m3 = np.sum(n3 * n3, axis=-1)
        ok = (m3 >= e2[b3]) & (m3 < e2[b3 + 1]) & (m3 > 0)
        i1, i2 = np.nonzero(ok)
        q1, q2, q3 = n1[i1], n2[i2], n3[i1, i2]
        total[t] += np.sum(F0(q2) * mixed(q1, q2)).real + np.sum(F0(q3) * mixed(q1, q3)).real
    return (2 * ell + 1) * total / (cnt * I33), cnt


def test_thin_shell_shot_noise_exact_for_collinear_triangles():
    """Any observer: when every closed triangle of a bin triple has
    q2 = q3 = -q1/2 (bins [2.7, 3.0) and [1.2, 1.5) k_f, one triangle per
    mode of b1 and of b2), qhat_1 = -qhat_i, so F^w_l(qhat_1, -q_i) is the
    ordinary F^w_l(-q_i) and L_l(qhat_1 . qhat_i) = 1 at the bin centres
    (cosine clamped to -1): eq. SNbisp2thin is eq. SNbisp2 exactly, for every
    ell."""
    box = 500.0
    kf = 2 * math.pi / box
    gal, ran = _uniform(37, 500, 2500, box, 500 / box**3, 0.7)
    alpha = 0.2
    prm = est.Params(n_grid=32, box=box, observer=(-300.0, 150.0, 700.0), order=3, interlace=True,
                     compensate=True, ell_max=4, bk_kmin=1.2 * kf, bk_dk=0.3 * kf, bk_nbins=6)
    tri = np.array([[5, 0, 0]])
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w_ell=True)
    res = est.bk_multipoles(gal, ran, alpha, prm, triangles=tri, fields=fields)
    c12, c13 = est.triangle_cosines(prm, tri)
    assert c12[0] == -1.0 and c13[0] == -1.0
    for ell in (2, 4):
        Fwl = _value(fields[f"w{ell}"], prm.n_grid)
        ex, cnt = _exact_shot_noise(fields, prm, tri, res["I33"], ell, lambda q1, qi: np.conj(Fwl(qi)))
        assert cnt[0] == 12
        assert abs(res[f"SN{ell}"][0] - ex[0]) <= 1e-9 * abs(ex[0])
        # the q_2, q_3 terms carry weight here: the q1 term alone is off
        assert abs(res[f"SN{ell}_q1"][0] - ex[0]) > 1e-3 * abs(ex[0])


def test_thin_shell_shot_noise_exact_for_right_angle_triangles_plane_parallel():
    """Bins centred on 1 and sqrt(2) k_f (width (sqrt 2 - 1)/2 k_f): the
    closed triangles of (b1, b2, b3) = (2, 0, 0) are q2, q3 two perpendicular
    unit vectors and q1 = -(q2 + q3), so qhat_1 . qhat_i = -1/sqrt 2 exactly
    at the bin centres; each q2 sits in four triangles whose q1 are related
    by the four-fold rotation about q2, over which the average of
    L_2(qhat_1 . zhat) is L_2(qhat_1 . qhat_2) L_2(qhat_2 . zhat) exactly.
    With a distant observer F^w_2(qhat_1, q) = L_2(qhat_1 . zhat) F^w_0(q),
    so eq. SNbisp2thin equals eq. SNbisp2 for ell = 2, with the factor
    L_2(-1/sqrt 2) = 1/4."""
    box = 500.0
    kf = 2 * math.pi / box
    dk = (math.sqrt(2) - 1) / 2
    gal, ran = _uniform(41, 500, 2500, box, 500 / box**3, 0.7)
    alpha = 0.2
    prm = est.Params(n_grid=32, box=box, observer=(box / 2, box / 2, -FAR * box), order=2, interlace=False,
                     compensate=True, ell_max=4, bk_kmin=(1 - dk / 2) * kf, bk_dk=dk * kf, bk_nbins=3)
    tri = np.array([[2, 0, 0]])
    np.testing.assert_allclose(est.bin_centres(prm), [1.0, 1.0 + dk, math.sqrt(2)], rtol=1e-14)
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w_ell=True)
    res = est.bk_multipoles(gal, ran, alpha, prm, triangles=tri, fields=fields)
    c12, c13 = est.triangle_cosines(prm, tri)
    np.testing.assert_allclose([c12[0], c13[0]], [-1 / math.sqrt(2)] * 2, rtol=1e-14)
    Fw0 = _value(fields["w"], prm.n_grid)
    L2 = _legendre_z(2)
    ex, cnt = _exact_shot_noise(fields, prm, tri, res["I33"], 2, lambda q1, qi: L2(q1) * np.conj(Fw0(qi)))
    assert cnt[0] == 24
    assert abs(res["SN2"][0] - ex[0]) <= 1e-8 * abs(ex[0])
    assert abs(res["SN2_q1"][0] - ex[0]) > 1e-3 * abs(ex[0])


def test_triangle_cosines_from_vectors():
    """Law of cosines at the bin centres against explicit lattice vectors
    whose lengths are the centres (1, sqrt 2, sqrt 3 k_f)."""
    box = 500.0
    kf = 2 * math.pi / box
    d = (math.sqrt(2) - 1)
    prm = est.Params(n_grid=32, box=box, observer=(0, 0, 0), bk_kmin=(1 - d / 2) * kf, bk_dk=d * kf, bk_nbins=2)
    c = est.bin_centres(prm)
    np.testing.assert_allclose(c, [1.0, math.sqrt(2)], rtol=1e-14)
    q2, q3 = np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    q1 = -(q2 + q3)
    c12, c13 = est.triangle_cosines(prm, [[1, 0, 0]])
    np.testing.assert_allclose(c12, q1 @ q2 / (np.linalg.norm(q1) * np.linalg.norm(q2)), rtol=1e-14)
    np.testing.assert_allclose(c13, q1 @ q3 / (np.linalg.norm(q1) * np.linalg.norm(q3)), rtol=1e-14)
