"""Brute-force twins that pin the oracle (test infrastructure only).

Each routine computes a quantity of the estimator by a route that shares no
step with ``oracle.estimator`` beyond the definition itself:

* ``kernel_dft_multipoles`` -- per-mode direct sum over objects of
  s_j w_j L_ell(khat . xhat_j) K_j(n), where K_j(n) is the discrete Fourier
  transform of object j's assignment kernel on the grid.  This is what the
  22-FFT decomposition (Sec. II.B eqs. delta2b, delta4b; Sec. III.A
  eq. mapFFT) must reproduce to round-off.  The B-spline kernels are
  evaluated here from the truncated-power formula, not the piecewise form.
* ``literal_multipoles`` -- sum_j s_j w_j exp(-i k.x_j) L_ell(khat . xhat_j),
  the continuous-position form of eqs. F0/F2; equal to the above when every
  object sits on a grid node and p <= 2 without interlacing.
* ``triangle_enumeration`` -- closed triangles n1 + n2 + n3 = 0 enumerated
  directly (the delta function of eqs. BispMono, NT), no FFT.
* ``shell_mode_counts`` -- lattice-point counts per shell by counting, for
  each (nx, ny), the admissible nz with integer square roots.
"""

from __future__ import annotations

import math

import numpy as np


def _truncated_power_bspline(p: int, x):
    """Centred cardinal B-spline of order p (degree p-1) at x.

    W_p(x) = 1/(p-1)! sum_{k=0}^{p} (-1)^k C(p,k) (x + p/2 - k)_+^{p-1}.
    For p = 1 the half-open box [-1/2, 1/2) is used.
    """
    x = np.asarray(x, dtype=np.float64)
    if p == 1:
        return ((x >= -0.5) & (x < 0.5)).astype(np.float64)
    acc = np.zeros_like(x)
    for k in range(p + 1):
        t = x + p / 2.0 - k
        acc += (-1) ** k * math.comb(p, k) * np.where(t > 0, t, 0.0) ** (p - 1)
    return acc / math.factorial(p - 1)


def _legendre(ell, mu):
    # Bonnet recursion, independent of the closed forms in the estimator
    p0 = np.ones_like(mu)
    if ell == 0:
        return p0
    p1 = mu
    for n in range(1, ell):
        p0, p1 = p1, ((2 * n + 1) * mu * p1 - n * p0) / (n + 1)
    return p1


def _kernel_dft_1d(u, n, N, p):
    """sum_i W_p(u - i) exp(-2 pi i n i / N) for each object (1D)."""
    base = np.floor(u).astype(np.int64)
    acc = np.zeros(u.shape, dtype=np.complex128)
    for off in range(-3, 4):
        i = base + off
        # NGP: the node owning u is floor(u + 1/2), i.e. u - i in [-1/2, 1/2)
        acc += _truncated_power_bspline(p, u - i) * np.exp(-2j * np.pi * n * i / N)
    return acc


def _catalog(gal, ran, alpha):
    if ran is not None and len(ran["w"]) > 0:
        pos = np.concatenate([gal["pos"], ran["pos"]])
        w = np.concatenate([gal["w"], -alpha * np.asarray(ran["w"])])
    else:
        pos, w = gal["pos"], gal["w"]
    return np.asarray(pos, np.float64), np.asarray(w, np.float64)


def kernel_dft_multipoles(gal, ran, alpha, n_grid, box, observer, order,
                          interlace, compensate, modes, ells=(0, 2, 4)):
    """Per-mode F_ell(n) by a direct sum over objects (no mesh, no FFT).

    modes: (m, 3) integer wave-vectors.  Returns {ell: (m,) complex}.
    """
    pos, w = _catalog(gal, ran, alpha)
    N = n_grid
    u = pos / (box / N)
    r = pos - np.asarray(observer, np.float64)
    xh = r / np.sqrt(np.sum(r * r, axis=1))[:, None]
    out = {ell: np.zeros(len(modes), dtype=np.complex128) for ell in ells}
    for t, n in enumerate(np.asarray(modes, dtype=np.int64)):
        K = np.ones(len(w), dtype=np.complex128)
        for d in range(3):
            K = K * _kernel_dft_1d(u[:, d], n[d], N, order)
        if interlace:
            K2 = np.ones(len(w), dtype=np.complex128)
            for d in range(3):
                K2 = K2 * _kernel_dft_1d(u[:, d] - 0.5, n[d], N, order)
            K = 0.5 * (K + np.exp(-1j * np.pi * n.sum() / N) * K2)
        if compensate:
            win = 1.0
            for d in range(3):
                a = math.pi * n[d] / N
                win *= (math.sin(a) / a if a != 0 else 1.0) ** order
            K = K / win
        nn = math.sqrt(float(n @ n))
        mu = (xh @ n) / nn if nn > 0 else np.zeros(len(w))
        for ell in ells:
            out[ell][t] = np.sum(w * _legendre(ell, mu) * K)
    return out


def literal_multipoles(gal, ran, alpha, box, observer, modes, ells=(0, 2, 4)):
    """sum_j s_j w_j exp(-i k.x_j) L_ell(khat . xhat_j) at the given modes."""
    pos, w = _catalog(gal, ran, alpha)
    r = pos - np.asarray(observer, np.float64)
    xh = r / np.sqrt(np.sum(r * r, axis=1))[:, None]
    kf = 2 * math.pi / box
    out = {ell: np.zeros(len(modes), dtype=np.complex128) for ell in ells}
    for t, n in enumerate(np.asarray(modes, dtype=np.int64)):
        k = kf * n.astype(np.float64)
        ph = np.exp(-1j * (pos @ k))
        nn = math.sqrt(float(n @ n))
        mu = (xh @ n) / nn if nn > 0 else np.zeros(len(w))
        for ell in ells:
            out[ell][t] = np.sum(w * _legendre(ell, mu) * ph)
    return out


def shell_mode_counts(e2_edges):
    """Number of integer vectors with e2[b] <= |n|^2 < e2[b+1], n != 0."""
    e2 = [float(v) for v in e2_edges]
    nb = len(e2) - 1
    top = e2[-1]
    R = int(math.isqrt(int(math.ceil(top)))) + 1

    def count_below(x2y2, bound):
        # number of integer nz with x2y2 + nz^2 < bound
        lim = bound - x2y2
        if lim <= 0:
            return 0
        # largest nz >= 0 with nz^2 < lim
        z = math.isqrt(int(math.floor(lim)))
        while z * z >= lim:
            z -= 1
        while (z + 1) * (z + 1) < lim:
            z += 1
        return 2 * z + 1

    counts = [0] * nb
    for x in range(-R, R + 1):
        for y in range(-R, R + 1):
            s = x * x + y * y
            below = [count_below(s, e) for e in e2]
            for b in range(nb):
                counts[b] += below[b + 1] - below[b]
    # remove DC if it fell in the first bin
    if e2[0] <= 0 < e2[1]:
        counts[0] -= 1
    return counts


def triangle_enumeration(value_fn, e2_edges, triangles, ells=(0, 2, 4)):
    """Direct sums over closed lattice triangles.

    value_fn(ell, nvec[k, 3]) -> complex values of F_ell at signed modes.
    For each (b1, b2, b3): count = #{(n1, n2): n1 in b1, n2 in b2,
    -(n1+n2) in b3} and T_ell = sum F_ell(n1) F_0(n2) F_0(n3).
    """
    e2 = np.asarray(e2_edges, dtype=np.float64)
    nc = int(math.ceil(math.sqrt(e2[-1])) - 1)
    r = np.arange(-nc, nc + 1)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    m2 = np.sum(g * g, axis=1)
    b = np.searchsorted(e2, m2, side="right") - 1
    b = np.where((m2 > 0) & (b >= 0) & (b < len(e2) - 1), b, -1)
    shells = {i: g[b == i] for i in range(len(e2) - 1)}
    cnt = np.zeros(len(triangles))
    sums = {ell: np.zeros(len(triangles), dtype=np.complex128) for ell in ells}
    for t, (b1, b2, b3) in enumerate(triangles):
        n1 = shells[b1]
        n2 = shells[b2]
        n3 = -(n1[:, None, :] + n2[None, :, :])
        m3 = np.sum(n3 * n3, axis=-1)
        ok = (m3 >= e2[b3]) & (m3 < e2[b3 + 1]) & (m3 > 0)
        cnt[t] = ok.sum()
        if cnt[t] == 0:
            continue
        i1, i2 = np.nonzero(ok)
        v2 = value_fn(0, n2[i2])
        v3 = value_fn(0, n3[i1, i2])
        for ell in ells:
            sums[ell][t] = np.sum(value_fn(ell, n1[i1]) * v2 * v3)
    return cnt, sums


def triangle_enumeration_slots(f1, f2, f3, e2_edges, triangles):
    """Direct sums over closed lattice triangles with a function per side.

    For each (b1, b2, b3): sum of f1(n1) f2(n2) f3(n3) over n1 in b1, n2 in
    b2 and n3 = -(n1 + n2) in b3 (the delta function of eq. NT), and the
    count of such triangles.  f_i(nvec[k, 3]) -> complex values.
    """
    cnt, sums = triangle_enumeration_many([(f1, f2, f3)], e2_edges, triangles)
    return cnt, sums[0]


def triangle_enumeration_many(products, e2_edges, triangles):
    """``triangle_enumeration_slots`` for several products (f1, f2, f3) over
    one enumeration of the closed triangles; returns the count and a list of
    sums, one per product."""
    e2 = np.asarray(e2_edges, dtype=np.float64)
    nc = int(math.ceil(math.sqrt(e2[-1])) - 1)
    r = np.arange(-nc, nc + 1)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    m2 = np.sum(g * g, axis=1)
    b = np.searchsorted(e2, m2, side="right") - 1
    b = np.where((m2 > 0) & (b >= 0) & (b < len(e2) - 1), b, -1)
    shells = {i: g[b == i] for i in range(len(e2) - 1)}
    cnt = np.zeros(len(triangles))
    sums = [np.zeros(len(triangles), dtype=np.complex128) for _ in products]
    for t, (b1, b2, b3) in enumerate(triangles):
        n1 = shells[b1]
        n2 = shells[b2]
        n3 = -(n1[:, None, :] + n2[None, :, :])
        m3 = np.sum(n3 * n3, axis=-1)
        ok = (m3 >= e2[b3]) & (m3 < e2[b3 + 1]) & (m3 > 0)
        cnt[t] = ok.sum()
        if cnt[t] == 0:
            continue
        i1, i2 = np.nonzero(ok)
        q1, q2, q3 = n1[i1], n2[i2], n3[i1, i2]
        for k, (f1, f2, f3) in enumerate(products):
            sums[k][t] = np.sum(f1(q1) * f2(q2) * f3(q3))
    return cnt, sums
