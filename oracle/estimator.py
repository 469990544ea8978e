"""FP64 NumPy oracle of the power-spectrum and bispectrum multipole estimators.

Test infrastructure only (see the package docstring).  The paper's notation
is kept: F_0, Q^{ab}, A_ell (= F_ell, the overdensity multipoles), I22, N_0,
N^T, I33.  Conventions (the paper leaves them open; the readings are listed
with the design notes of the repository):

* Forward transforms use exp(-i k.x).  Every reported number is the real
  part of a shell or triangle sum that is symmetric under n -> -n, so the
  sign of the exponent does not change any output (Sec. III.A eq. F0 uses
  exp(+ik.x), Sec. II.B eq. deltaell uses exp(-ik.x)).
* Integer wave-vectors n follow numpy.fft.fftfreq; k = k_f n, k_f = 2 pi / L.
* Objects carry signs: +1 for galaxies, -alpha for randoms (eq. F0).
* Line of sight is per object, x_hat_j = (x_j - o)/|x_j - o| (eq. Qab).
* Mass assignment uses the B-spline kernels of order p (1 NGP, 2 CIC, 3 TSC,
  4 PCS) with nodes at integer grid coordinates, periodic wrap; the
  interlaced twin grid has nodes at half-integer coordinates
  (Sec. III.A, the paragraph after eq. Nelltrue).
* Bins: b covers [kmin + b dk, kmin + (b+1) dk); membership is decided on
  the integer |n|^2 against squared edges in k_f units, snapped to the
  nearest integer when within 1e-9 relative.  DC is never binned.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from itertools import product

import os

import numpy as np
import scipy.fft as sfft

_WORKERS = max(1, min(16, os.cpu_count() or 1))

# ---------------------------------------------------------------------------
# Moment tensors (Sec. II.B eqs. delta2b and delta4b)
# ---------------------------------------------------------------------------

#: index tuples of the moment meshes: the monopole, the 6 independent
#: components of Q_ij and the 15 of Q_ijkl (x=0, y=1, z=2)
MOMENTS_2 = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0)]
MOMENTS_4 = [
    (0, 0, 0, 0), (1, 1, 1, 1), (2, 2, 2, 2),
    (0, 0, 0, 1), (0, 0, 0, 2), (1, 1, 1, 0), (1, 1, 1, 2), (2, 2, 2, 0), (2, 2, 2, 1),
    (0, 0, 1, 1), (1, 1, 2, 2), (2, 2, 0, 0),
    (0, 0, 1, 2), (1, 1, 0, 2), (2, 2, 0, 1),
]
MOMENTS = [()] + MOMENTS_2 + MOMENTS_4


def multiplicity(idx: tuple) -> int:
    """Number of distinct orderings of a symmetric-tensor index tuple.

    This is the weight each independent component carries when the full
    contraction k_i k_j Q_ij (or k_i k_j k_k k_l Q_ijkl) is written over the
    independent components only: 1,1,1,2,2,2 for rank 2 and 1 (x3), 4 (x6),
    6 (x3), 12 (x3) for rank 4 (Sec. II.B eqs. delta2b, delta4b).
    """
    counts = [idx.count(a) for a in range(3)]
    m = math.factorial(len(idx))
    for c in counts:
        m //= math.factorial(c)
    return m


def moments_for(ell_max: int):
    """Moment index tuples needed for multipoles up to ell_max."""
    if ell_max == 0:
        return MOMENTS[:1]
    if ell_max == 2:
        return MOMENTS[:7]
    if ell_max == 4:
        return list(MOMENTS)
    raise ValueError("ell_max must be 0, 2 or 4")


def monomial(v: np.ndarray, idx: tuple) -> np.ndarray:
    """Product v_{i1} v_{i2} ... over the index tuple, row-wise (v: n x 3)."""
    out = np.ones(v.shape[0], dtype=np.float64)
    for a in idx:
        out = out * v[:, a]
    return out


def los_unit(pos: np.ndarray, observer) -> np.ndarray:
    """Per-object line of sight x_hat_j = (x_j - o)/|x_j - o| (Sec. III.A eq. Qab)."""
    r = np.asarray(pos, dtype=np.float64) - np.asarray(observer, dtype=np.float64)[None, :]
    return r / np.linalg.norm(r, axis=1)[:, None]


def legendre(ell: int, mu):
    """Legendre polynomials L_0, L_2, L_4 written out."""
    mu = np.asarray(mu, dtype=np.float64)
    if ell == 0:
        return np.ones_like(mu)
    if ell == 2:
        return 0.5 * (3.0 * mu**2 - 1.0)
    if ell == 4:
        return (35.0 * mu**4 - 30.0 * mu**2 + 3.0) / 8.0
    raise ValueError(ell)


# ---------------------------------------------------------------------------
# Mass assignment (Sec. III.A eq. mapFFT and the paragraph after it)
# ---------------------------------------------------------------------------

def bspline(p: int, d):
    """Hockney-Eastwood assignment kernel of order p at distance d (grid units)."""
    d = np.asarray(d, dtype=np.float64)
    a = np.abs(d)
    if p == 1:
        # half-open cell so that every point has exactly one node, floor(u + 1/2)
        return np.where((d >= -0.5) & (d < 0.5), 1.0, 0.0)
    if p == 2:
        return np.where(a < 1.0, 1.0 - a, 0.0)
    if p == 3:
        return np.where(a < 0.5, 0.75 - a * a,
                        np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))
    if p == 4:
        return np.where(a < 1.0, (4.0 - 6.0 * a * a + 3.0 * a**3) / 6.0,
                        np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))
    raise ValueError("order must be 1..4")


def first_node(u: np.ndarray, p: int) -> np.ndarray:
    """Lowest grid node reached by an object at grid coordinate u.

    Odd orders centre on the nearest node floor(u + 1/2); even orders on the
    cell floor(u).  The kernel support then covers nodes first..first+p-1.
    """
    if p % 2 == 1:
        return np.floor(u + 0.5).astype(np.int64) - (p - 1) // 2
    return np.floor(u).astype(np.int64) - (p // 2 - 1)


def assign_mesh(u: np.ndarray, weight: np.ndarray, n_grid: int, p: int) -> np.ndarray:
    """Real mesh m[i] = sum_j weight_j prod_d W_p(u_jd - i_d), periodic.

    u: (n, 3) grid coordinates (position / cell size), weight: (n,).
    """
    N = n_grid
    mesh = np.zeros(N**3, dtype=np.float64)
    if u.shape[0] == 0:
        return mesh.reshape(N, N, N)
    i0 = [first_node(u[:, d], p) for d in range(3)]
    wt = [[bspline(p, u[:, d] - (i0[d] + a)) for a in range(p)] for d in range(3)]
    for a, b, c in product(range(p), repeat=3):
        idx = (((i0[0] + a) % N) * N + ((i0[1] + b) % N)) * N + ((i0[2] + c) % N)
        mesh += np.bincount(idx, weights=weight * wt[0][a] * wt[1][b] * wt[2][c],
                            minlength=N**3)
    return mesh.reshape(N, N, N)


# ---------------------------------------------------------------------------
# Parameters, bins
# ---------------------------------------------------------------------------

@dataclass
class Params:
    n_grid: int
    box: float
    observer: tuple
    order: int = 3
    interlace: bool = True
    compensate: bool = True
    ell_max: int = 4
    pk_kmin: float = 0.0
    pk_dk: float = 0.0
    pk_nbins: int = 0
    bk_kmin: float = 0.0
    bk_dk: float = 0.0
    bk_nbins: int = 0
    m_grid: int = 0          # real-space grid of the triangle search; 0 = smallest valid
    assign: object = field(default=None, repr=False)  # optional faster assign_mesh

    @property
    def kf(self) -> float:
        return 2.0 * math.pi / self.box


def squared_edges(kmin: float, dk: float, nbins: int, kf: float) -> np.ndarray:
    """Squared bin edges in k_f units, snapped to integers within 1e-9 relative."""
    e = (kmin + dk * np.arange(nbins + 1, dtype=np.float64)) / kf
    e2 = e * e
    r = np.rint(e2)
    snap = np.abs(e2 - r) <= 1e-9 * np.maximum(r, 1.0)
    return np.where(snap, r, e2)


def bin_of(m2: np.ndarray, e2: np.ndarray) -> np.ndarray:
    """Bin index of integer |n|^2 values (-1 when outside every bin or DC)."""
    nb = len(e2) - 1
    b = np.searchsorted(e2, m2, side="right") - 1
    ok = (b >= 0) & (b < nb) & (m2 > 0)
    return np.where(ok, b, -1)


def smooth_size(n: int) -> int:
    """Smallest 2^a 3^b that is >= n."""
    best = None
    a = 1
    while a < 4 * n:
        b = a
        while b < 4 * n:
            if b >= n and (best is None or b < best):
                best = b
            b *= 3
        a *= 2
    return best


def bk_grid(prm: Params) -> int:
    """Real-space grid M of the triangle search.

    A triangle n1 + n2 + n3 = 0 is detected by the grid sum modulo M; with
    every component |n_d| <= n_c, spurious closures n1+n2+n3 = M e (e != 0)
    are impossible when M > 3 n_c (Sec. III.B eqs. Factorize, F_k).
    """
    e2 = squared_edges(prm.bk_kmin, prm.bk_dk, prm.bk_nbins, prm.kf)
    if e2[-1] > (prm.n_grid // 2) ** 2 * (1 + 1e-12):
        raise ValueError("bispectrum k_max beyond Nyquist")
    etop = math.sqrt(e2[-1])
    nc = int(math.ceil(etop) - 1)
    need = smooth_size(3 * nc + 1)
    if prm.m_grid:
        if prm.m_grid < 3 * nc + 1:
            raise ValueError("m_grid too small for exact triangle closure")
        return prm.m_grid
    return need


# ---------------------------------------------------------------------------
# Fourier-space multipole fields (Sec. II.B, Sec. III.A)
# ---------------------------------------------------------------------------

def signed_freq(N: int) -> np.ndarray:
    return np.fft.fftfreq(N, d=1.0 / N).astype(np.int64)


def half_grid(N: int):
    """Integer wave-vector components on the numpy rfftn half grid."""
    f = signed_freq(N)
    fz = np.arange(N // 2 + 1, dtype=np.int64)
    nx, ny, nz = np.meshgrid(f, f, fz, indexing="ij")
    return nx, ny, nz


def combined_catalog(gal, ran, alpha):
    """Positions and signed weights of the galaxy-minus-random field (eq. F0)."""
    pg, wg = gal["pos"], gal["w"]
    if ran is not None and len(ran["w"]) > 0:
        pos = np.concatenate([pg, ran["pos"]])
        w = np.concatenate([wg, -alpha * ran["w"]])
        w2 = np.concatenate([wg**2, alpha**2 * ran["w"] ** 2])
    else:
        pos, w, w2 = pg, wg, wg**2
    return np.asarray(pos, np.float64), np.asarray(w, np.float64), np.asarray(w2, np.float64)


def fourier_of_weights(u, weight, prm: Params, nx, ny, nz, u_twin=None):
    """Compensated, interlaced Fourier transform of one weighted point set.

    Returns sum_j weight_j exp(-i k.x_j) as estimated on the grid: the
    interlaced pair 1/2 [X + exp(-i pi (nx+ny+nz)/N) Y] (Y from the twin grid
    whose nodes sit at half-integer coordinates), divided by the kernel
    window prod_d sinc(pi n_d / N)^p when compensation is on.
    """
    N, p = prm.n_grid, prm.order
    assign = prm.assign or assign_mesh
    X = sfft.rfftn(assign(u, weight, N, p), workers=_WORKERS)
    if prm.interlace:
        ut = u - 0.5 if u_twin is None else u_twin
        Y = sfft.rfftn(assign(ut, weight, N, p), workers=_WORKERS)
        X = 0.5 * (X + np.exp(-1j * np.pi * (nx + ny + nz) / N) * Y)
    if prm.compensate:
        win = np.ones(X.shape)
        for n in (nx, ny, nz):
            win = win * np.sinc(n / N) ** p      # np.sinc(t) = sin(pi t)/(pi t)
        X = X / win
    return X


def multipole_fields(gal, ran, alpha, prm: Params, with_w: bool = False,
                     sign: int = -1, with_w_ell: bool = False):
    """A_0, A_2, A_4 (and A_0^w, A_2^w, A_4^w) on the rfftn half grid.

    A_0 = F_0 (eq. F0); A_2 = 3/2 khat_a khat_b Q^{ab} - 1/2 A_0 (eq. F2 with
    Q^{ab} of eq. Qab); A_4 = 35/8 khat^4 Q^{abcd} - 5/2 A_2 - 7/8 A_0
    (eq. delta4 in the survey form).  A_0^w is the w^2-weighted monopole
    F_0^w with weights w^2 for galaxies and alpha^2 w^2 for randoms
    (the definition after eq. SNbisp2).  With ``with_w_ell`` also
    F^w_2(q) = F^w_2(qhat, q) and F^w_4 (the same definition with
    L_ell(qhat . xhat_j), i.e. the same combination as A_2 and A_4 of the
    w^2-weighted moment meshes), keys "w2" and "w4".  ``sign=+1`` conjugates
    every field, i.e. uses exp(+ik.x) as written in eq. F0.
    """
    N = prm.n_grid
    pos, w, w2 = combined_catalog(gal, ran, alpha)
    u = pos / (prm.box / N)
    ut = u - 0.5                      # coordinates on the interlaced twin grid
    xhat = los_unit(pos, prm.observer)
    nx, ny, nz = half_grid(N)
    kk = np.sqrt((nx * nx + ny * ny + nz * nz).astype(np.float64))
    kk[0, 0, 0] = 1.0
    khat = (nx / kk, ny / kk, nz / kk)

    def khat_mono(idx):
        out = np.ones(nx.shape)
        for a in idx:
            out = out * khat[a]
        return out

    fields = {}
    A0 = fourier_of_weights(u, w, prm, nx, ny, nz, ut)
    fields[0] = A0
    if prm.ell_max >= 2:
        s = np.zeros_like(A0)
        for idx in MOMENTS_2:
            s += multiplicity(idx) * khat_mono(idx) * fourier_of_weights(
                u, w * monomial(xhat, idx), prm, nx, ny, nz, ut)
        A2 = 1.5 * s - 0.5 * A0
        fields[2] = A2
    if prm.ell_max >= 4:
        s = np.zeros_like(A0)
        for idx in MOMENTS_4:
            s += multiplicity(idx) * khat_mono(idx) * fourier_of_weights(
                u, w * monomial(xhat, idx), prm, nx, ny, nz, ut)
        fields[4] = 35.0 / 8.0 * s - 2.5 * fields[2] - 7.0 / 8.0 * A0
    if with_w or with_w_ell:
        fields["w"] = fourier_of_weights(u, w2, prm, nx, ny, nz, ut)
    if with_w_ell and prm.ell_max >= 2:
        s = np.zeros_like(A0)
        for idx in MOMENTS_2:
            s += multiplicity(idx) * khat_mono(idx) * fourier_of_weights(
                u, w2 * monomial(xhat, idx), prm, nx, ny, nz, ut)
        fields["w2"] = 1.5 * s - 0.5 * fields["w"]
        if prm.ell_max >= 4:
            s = np.zeros_like(A0)
            for idx in MOMENTS_4:
                s += multiplicity(idx) * khat_mono(idx) * fourier_of_weights(
                    u, w2 * monomial(xhat, idx), prm, nx, ny, nz, ut)
            fields["w4"] = 35.0 / 8.0 * s - 2.5 * fields["w2"] - 7.0 / 8.0 * fields["w"]
    if sign > 0:
        fields = {k: np.conj(v) for k, v in fields.items()}
    return fields


# ---------------------------------------------------------------------------
# Normalisation and shot noise (Sec. III.A eqs. I22def, N0true; Sec. III.B)
# ---------------------------------------------------------------------------

def scalars(gal, ran, alpha):
    """I22, N_0, I33 and the w^3 shot-noise sum.

    I22 = alpha sum_r nbar w^2 (eq. I22def); N_0 = (sum_g + alpha^2 sum_r) w^2
    (eq. N0true, true galaxy shot noise); I33 = alpha sum_r nbar^2 w^3 (not
    defined in the paper; the reading is the cubic analogue of I22);
    W3 = (sum_g - alpha^3 sum_r) w^3 (eq. Noise0).
    """
    wg = np.asarray(gal["w"], np.float64)
    if ran is not None and len(ran["w"]) > 0:
        wr = np.asarray(ran["w"], np.float64)
        nr = np.asarray(ran["nbar"], np.float64)
    else:
        wr = np.zeros(0)
        nr = np.zeros(0)
    return {
        "I22": alpha * np.sum(nr * wr**2),
        "N0": np.sum(wg**2) + alpha**2 * np.sum(wr**2),
        "I33": alpha * np.sum(nr**2 * wr**3),
        "W3": np.sum(wg**3) - alpha**3 * np.sum(wr**3),
    }


# ---------------------------------------------------------------------------
# Power spectrum multipoles (Sec. III.A eqs. P0_impl, P2_impl, P4_impl)
# ---------------------------------------------------------------------------

def half_weights(N: int, nz: np.ndarray) -> np.ndarray:
    """Multiplicity of each half-grid mode in the full grid (n and -n)."""
    return np.where((nz > 0) & (nz < N // 2), 2.0, 1.0)


def shell_sums(fields, prm: Params, kmin, dk, nbins):
    """Full-grid shell sums over |k| bins (eq. shell).

    N_b = number of modes, k_eff = mean |k|, S_l0 = sum Re[A_l A_0^*],
    S_22 = sum |A_2|^2 (the autocorrelation of the quadrupole field, used by
    the split hexadecapole of Sec. II.B eq. P4fast), S_0w = sum Re[A_0 A_0w^*],
    S_lw = sum Re[A_l A_0w^*], and with the w^2-weighted multipoles
    Q_lw = sum Re[A_0 (A_l^w)^*] (the q_2, q_3 terms of eq. SNbisp2thin).
    """
    N = prm.n_grid
    nx, ny, nz = half_grid(N)
    m2 = nx * nx + ny * ny + nz * nz
    e2 = squared_edges(kmin, dk, nbins, prm.kf)
    if e2[-1] > (N // 2) ** 2 * (1 + 1e-12):
        raise ValueError("k_max beyond Nyquist")
    b = bin_of(m2, e2).ravel()
    hw = half_weights(N, nz).ravel()
    sel = b >= 0
    bb = b[sel]
    wsel = hw[sel]
    out = {"n_modes": np.bincount(bb, weights=wsel, minlength=nbins).astype(np.int64)}
    kmag = prm.kf * np.sqrt(m2.astype(np.float64)).ravel()[sel]
    out["k_eff"] = np.bincount(bb, weights=wsel * kmag, minlength=nbins) / np.maximum(out["n_modes"], 1)
    A0 = fields[0].ravel()[sel]
    for ell in (0, 2, 4):
        if ell in fields:
            prod_ = fields[ell].ravel()[sel] * np.conj(A0)
            out[f"S{ell}0"] = np.bincount(bb, weights=wsel * prod_.real, minlength=nbins)
            out[f"C{ell}0"] = np.bincount(bb, weights=wsel * np.abs(prod_), minlength=nbins)
    if 2 in fields:
        out["S22"] = np.bincount(bb, weights=wsel * np.abs(fields[2].ravel()[sel]) ** 2, minlength=nbins)
    if "w" in fields:
        Aw = np.conj(fields["w"].ravel()[sel])
        for ell in (0, 2, 4):
            if ell in fields:
                out[f"S{ell}w"] = np.bincount(bb, weights=wsel * (fields[ell].ravel()[sel] * Aw).real,
                                              minlength=nbins)
    for ell in (2, 4):
        if f"w{ell}" in fields:
            out[f"Q{ell}w"] = np.bincount(bb, weights=wsel * (A0 * np.conj(fields[f"w{ell}"].ravel()[sel])).real,
                                          minlength=nbins)
    return out


def pk_multipoles(gal, ran, alpha, prm: Params, fields=None):
    """P_0, P_2, P_4 of the survey estimator (Sec. III.A eqs. P0_impl-P4_impl),
    and the split hexadecapole P_4b (Sec. II.B eqs. factorizeL4, split, P4fast).

    P_4b: L_4 = 35/18 L_2^2 - 5/9 L_2 - 7/18 with L_2^2 split over the two
    objects of a pair turns 9 F_4 F_0^* into 35/2 |F_2|^2 - 5 F_2 F_0^* -
    7/2 |F_0|^2, so P_4b = (35/2 S_22 - 5 S_20 - 7/2 S_00) / (N_b I22) with the
    raw S_00: the self pairs (an object with itself, where the split is exact)
    then carry the same zero-mean term as in P_4, and no N_0 is subtracted.
    Needs only the monopole and quadrupole fields (7 FFTs).
    """
    if fields is None:
        fields = multipole_fields(gal, ran, alpha, prm)
    sc = scalars(gal, ran, alpha)
    res = shell_sums(fields, prm, prm.pk_kmin, prm.pk_dk, prm.pk_nbins)
    nb = res["n_modes"].astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        res["P0"] = (res["S00"] / nb - sc["N0"]) / sc["I22"]
        if "S20" in res:
            res["P2"] = 5.0 * res["S20"] / (nb * sc["I22"])
        if "S40" in res:
            res["P4"] = 9.0 * res["S40"] / (nb * sc["I22"])
        if "S22" in res:
            res["P4b"] = (17.5 * res["S22"] - 5.0 * res["S20"] - 3.5 * res["S00"]) / (nb * sc["I22"])
    res.update(sc)
    return res


# ---------------------------------------------------------------------------
# Bispectrum multipoles (Sec. III.B eqs. BispMono-SNbisp2thin, Factorize, F_k)
# ---------------------------------------------------------------------------

def triangle_list(prm: Params) -> np.ndarray:
    """Triangles b1 >= b2 >= b3 whose shells can close.

    With the multipole taken on the largest side (Sec. II.C eq. YBisp), the
    list keeps every bin triple with lo(b1) < hi(b2) + hi(b3) in k_f units,
    a superset of the triples with closed lattice triangles since
    |n1| = |n2 + n3| <= |n2| + |n3|.  Lexicographic order in (b1, b2, b3).
    """
    e = np.sqrt(squared_edges(prm.bk_kmin, prm.bk_dk, prm.bk_nbins, prm.kf))
    tri = []
    for b1 in range(prm.bk_nbins):
        for b2 in range(b1 + 1):
            for b3 in range(b2 + 1):
                if e[b1] < e[b2 + 1] + e[b3 + 1]:
                    tri.append((b1, b2, b3))
    return np.array(tri, dtype=np.int64).reshape(-1, 3)


def lowk_modes(prm: Params):
    """All integer n (full signed range) inside the bispectrum bins, with bin index."""
    e2 = squared_edges(prm.bk_kmin, prm.bk_dk, prm.bk_nbins, prm.kf)
    nc = int(math.ceil(math.sqrt(e2[-1])) - 1)
    r = np.arange(-nc, nc + 1, dtype=np.int64)
    nx, ny, nz = np.meshgrid(r, r, r, indexing="ij")
    m2 = nx * nx + ny * ny + nz * nz
    b = bin_of(m2, e2)
    sel = b >= 0
    return nx[sel], ny[sel], nz[sel], b[sel]


def gather_full(field_half: np.ndarray, N: int, nx, ny, nz) -> np.ndarray:
    """Values at arbitrary signed n from a half-grid array, via A(-n) = A(n)^*."""
    neg = nz < 0
    sx = np.where(neg, -nx, nx) % N
    sy = np.where(neg, -ny, ny) % N
    sz = np.where(neg, -nz, nz)
    v = field_half[sx, sy, sz]
    return np.where(neg, np.conj(v), v)


def shell_field(values, nx, ny, nz, M: int) -> np.ndarray:
    """F_k(x) = sum_{n in shell} F(n) exp(+2 pi i n.x / M) on an M^3 grid (eq. F_k).

    Returns the real part; the imaginary part is asserted to vanish to
    round-off (the shell spectrum is Hermitian).
    """
    spec = np.zeros((M, M, M), dtype=np.complex128)
    spec[nx % M, ny % M, nz % M] = values
    f = sfft.ifftn(spec, workers=_WORKERS) * (M**3)
    scale = np.sum(np.abs(values)) + 1e-300
    assert np.max(np.abs(f.imag)) <= 1e-10 * scale, "shell field not real"
    return f.real


def bk_triangle_sums(fields, prm: Params, triangles=None, indicators_only=False, t220=False):
    """T_ell(b1,b2,b3) = M^-3 sum_x F_{ell,b1}(x) F_{0,b2}(x) F_{0,b3}(x) and N^T.

    The grid sum over real space equals the sum over closed triangles
    q1 + q2 + q3 = 0 with q_i in shell b_i (eq. Factorize), exact when
    M > 3 n_c.  N^T is the same sum with unit fields (eq. NT, exact
    discrete count), rounded to the nearest integer.  With ``t220`` also
    T_220 = M^-3 sum_x F_{2,b1} F_{2,b2} F_{0,b3}, the triangle sum of the
    zero-area hexadecapole (Sec. II.C eq. Bhexa2: delta_2 on q1 and q2).
    """
    M = bk_grid(prm)
    N = prm.n_grid
    if triangles is None:
        triangles = triangle_list(prm)
    nx, ny, nz, b = lowk_modes(prm)
    needed = sorted(set(np.asarray(triangles).ravel().tolist()))
    cache = {}

    def get(kind, bin_):
        key = (kind, bin_)
        if key not in cache:
            s = b == bin_
            if kind == "I":
                vals = np.ones(int(s.sum()), dtype=np.complex128)
            else:
                vals = gather_full(fields[kind], N, nx[s], ny[s], nz[s])
            cache[key] = shell_field(vals, nx[s], ny[s], nz[s], M)
        return cache[key]

    out = {"NT": np.zeros(len(triangles))}
    ells = [] if indicators_only else [e for e in (0, 2, 4) if e in fields]
    t220 = t220 and 2 in ells
    for ell in ells:
        out[f"T{ell}"] = np.zeros(len(triangles))
        out[f"C{ell}"] = np.zeros(len(triangles))
    if t220:
        out["T220"] = np.zeros(len(triangles))
        out["C220"] = np.zeros(len(triangles))
    for t, (b1, b2, b3) in enumerate(np.asarray(triangles)):
        out["NT"][t] = np.rint(np.sum(get("I", b1) * get("I", b2) * get("I", b3)) / M**3)
        if ells:
            pair = get(0, b2) * get(0, b3)
            for ell in ells:
                f1 = get(ell, b1)
                out[f"T{ell}"][t] = np.sum(f1 * pair) / M**3
                out[f"C{ell}"][t] = np.sum(np.abs(f1 * pair)) / M**3
        if t220:
            prod = get(2, b1) * get(2, b2) * get(0, b3)
            out["T220"][t] = np.sum(prod) / M**3
            out["C220"][t] = np.sum(np.abs(prod)) / M**3
        # drop fields no longer needed by later triangles in lexicographic order
        if len(cache) > 64:
            cache.clear()
    out["M"] = M
    return out


def bin_centres(prm: Params) -> np.ndarray:
    """Centres of the bispectrum bins in k_f units (mid-points of the edges)."""
    e = np.sqrt(squared_edges(prm.bk_kmin, prm.bk_dk, prm.bk_nbins, prm.kf))
    return 0.5 * (e[:-1] + e[1:])


def triangle_cosines(prm: Params, triangles) -> tuple:
    """cos(q1, q2) and cos(q1, q3) of a closed triangle with sides at the bin
    centres (law of cosines: q3^2 = q1^2 + q2^2 + 2 q1.q2), clamped to
    [-1, 1] for bin triples that do not close at their centres."""
    c = bin_centres(prm)
    t = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    k1, k2, k3 = c[t[:, 0]], c[t[:, 1]], c[t[:, 2]]
    c12 = np.clip((k3 * k3 - k1 * k1 - k2 * k2) / (2.0 * k1 * k2), -1.0, 1.0)
    c13 = np.clip((k2 * k2 - k1 * k1 - k3 * k3) / (2.0 * k1 * k3), -1.0, 1.0)
    return c12, c13


def bk_multipoles(gal, ran, alpha, prm: Params, triangles=None, fields=None, zero_area=False, tsums=None):
    """B_0, B_2, B_4 of the survey estimator with thin-shell shot noise.

    B_ell^raw = (2 ell + 1) T_ell / (N^T I33) (eqs. BispMono, BispQuad).
    Shot noise in the thin-shell form (eq. SNbisp2thin):
      N^(0) = sum_i S_0w(b_i)/(N_{b_i} I33) - 2 W3 / I33,
      N^(l) = (2l+1)/I33 [S_lw(b1)/N_{b1} + sum_{i=2,3} L_l(qhat_1 . qhat_i) Q_lw(b_i)/N_{b_i}]
    with S_lw = sum Re F_l F_0w^*, Q_lw = sum Re F_0 (F^w_l)^* and the cosines
    at the bin centres (``triangle_cosines``).  "SN{l}_q1" is the first term
    alone; "SN{l}" needs the w^2-weighted multipoles (fields "w2", "w4",
    ``multipole_fields(with_w_ell=True)``) and is the q1 term otherwise.
    With ``zero_area`` also the zero-area hexadecapole of Sec. II.C
    eq. Bhexa2 in the survey normalisation,
      B4za = [35/2 T_220 - 5 T_2 - 7/2 T_0] / (N^T I33)
    (no shot noise subtracted).  Triangles with N^T = 0 give NaN.  ``tsums``
    takes triangle sums already computed for these triangles (e.g. by
    ``bk_triangle_sums_streamed``).
    """
    if triangles is None:
        triangles = triangle_list(prm)
    triangles = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    if fields is None:
        fields = multipole_fields(gal, ran, alpha, prm, with_w=True)
    sc = scalars(gal, ran, alpha)
    ts = tsums if tsums is not None else bk_triangle_sums(fields, prm, triangles, t220=zero_area)
    sh = shell_sums(fields, prm, prm.bk_kmin, prm.bk_dk, prm.bk_nbins)
    nt = ts["NT"]
    res = {"triangles": triangles, "NT": nt, "M": ts["M"], "bins": sh}
    with np.errstate(divide="ignore", invalid="ignore"):
        for ell in (0, 2, 4):
            if f"T{ell}" not in ts:
                continue
            res[f"T{ell}"] = ts[f"T{ell}"]
            res[f"C{ell}"] = ts[f"C{ell}"]
            res[f"B{ell}"] = np.where(nt > 0, (2 * ell + 1) * ts[f"T{ell}"] / (nt * sc["I33"]), np.nan)
        if "T220" in ts:
            res["T220"] = ts["T220"]
            res["C220"] = ts["C220"]
            res["B4za"] = np.where(nt > 0, (17.5 * ts["T220"] - 5.0 * ts["T2"] - 3.5 * ts["T0"]) / (nt * sc["I33"]),
                                   np.nan)
        nb = sh["n_modes"].astype(np.float64)
        if "S0w" in sh:
            per_bin = sh["S0w"] / nb
            b1, b2, b3 = triangles.T
            res["SN0"] = (per_bin[b1] + per_bin[b2] + per_bin[b3]) / sc["I33"] - 2.0 * sc["W3"] / sc["I33"]
            c12, c13 = triangle_cosines(prm, triangles)
            for ell in (2, 4):
                if f"S{ell}w" in sh:
                    q1 = (2 * ell + 1) * (sh[f"S{ell}w"] / nb)[b1] / sc["I33"]
                    res[f"SN{ell}_q1"] = q1
                    res[f"SN{ell}"] = q1
                    if f"Q{ell}w" in sh:
                        per = sh[f"Q{ell}w"] / nb
                        res[f"SN{ell}"] = q1 + (2 * ell + 1) * (legendre(ell, c12) * per[b2]
                                                                + legendre(ell, c13) * per[b3]) / sc["I33"]
    res.update(sc)
    return res


def bk_triangle_sums_streamed(fields, prm: Params, triangles, scratch_path: str, chunk: int = 1 << 17,
                              t220: bool = False):
    """The sums of ``bk_triangle_sums`` for grids whose shell fields do not all
    fit in memory (the same definition, Sec. III.B eqs. Factorize, F_k, NT).

    Every shell field needed (the unit indicator and F_0, F_2, F_4 of each
    bin, eq. F_k) is computed once by ``shell_field`` and written to a
    memory-mapped file at ``scratch_path``.  The grid sum over x is then taken
    over chunks of cells: for each chunk the (pair x cell) array of products
    F_{0,b2}(x) F_{0,b3}(x) times the (cell x field) array of F_{l,b1}(x)
    gives the chunk's contribution to every sum_x F_{0,b2} F_{0,b3} F_{l,b1}
    at once (a matrix product as a step), accumulated in float64; the
    absolute values give the conditioning sums C_l, the indicators N^T, and
    with ``t220`` the pair F_{2,b2} F_{0,b3} against F_{2,b1} gives T_220.
    """
    M = bk_grid(prm)
    N = prm.n_grid
    triangles = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    nb = prm.bk_nbins
    nx, ny, nz, b = lowk_modes(prm)
    ells = [e for e in (0, 2, 4) if e in fields]
    kinds = ["I"] + ells
    t220 = t220 and 2 in ells
    ncell = M**3
    store = np.lib.format.open_memmap(scratch_path, mode="w+", dtype=np.float64, shape=(len(kinds) * nb, ncell))
    for ki, kind in enumerate(kinds):
        for bin_ in range(nb):
            sel = b == bin_
            if kind == "I":
                vals = np.ones(int(sel.sum()), dtype=np.complex128)
            else:
                vals = gather_full(fields[kind], N, nx[sel], ny[sel], nz[sel])
            store[ki * nb + bin_] = shell_field(vals, nx[sel], ny[sel], nz[sel], M).ravel()
    store.flush()
    pairs = sorted({(int(t[1]), int(t[2])) for t in triangles})
    pidx = {p: i for i, p in enumerate(pairs)}
    p2 = np.array([p[0] for p in pairs])
    p3 = np.array([p[1] for p in pairs])
    row = {k: ki * nb for ki, k in enumerate(kinds)}
    nd = len(ells) * nb
    acc_nt = np.zeros((len(pairs), nb))
    acc_t = np.zeros((len(pairs), nd))
    acc_c = np.zeros((len(pairs), nd))
    acc_220 = np.zeros((len(pairs), nb))
    acc_c220 = np.zeros((len(pairs), nb))
    for c0 in range(0, ncell, chunk):
        blk = np.array(store[:, c0:c0 + chunk])
        ind = blk[row["I"]:row["I"] + nb]
        acc_nt += (ind[p2] * ind[p3]) @ ind.T
        f0 = blk[row[0]:row[0] + nb]
        data = np.concatenate([blk[row[e]:row[e] + nb] for e in ells])
        pr = f0[p2] * f0[p3]
        acc_t += pr @ data.T
        acc_c += np.abs(pr) @ np.abs(data).T
        if t220:
            f2 = blk[row[2]:row[2] + nb]
            pr2 = f2[p2] * f0[p3]
            acc_220 += pr2 @ f2.T
            acc_c220 += np.abs(pr2) @ np.abs(f2).T
    del store
    os.remove(scratch_path)
    pi = np.array([pidx[(int(t[1]), int(t[2]))] for t in triangles])
    b1 = triangles[:, 0]
    out = {"NT": np.rint(acc_nt[pi, b1] / M**3), "M": M}
    for li, ell in enumerate(ells):
        out[f"T{ell}"] = acc_t[pi, li * nb + b1] / M**3
        out[f"C{ell}"] = acc_c[pi, li * nb + b1] / M**3
    if t220:
        out["T220"] = acc_220[pi, b1] / M**3
        out["C220"] = acc_c220[pi, b1] / M**3
    return out
