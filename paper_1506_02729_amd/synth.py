"""Seeded synthetic catalogs shaped like the paper's workloads.

This module generates inputs only: it holds none of the estimator's
arithmetic (no mass assignment, no multipole combination, no binning).  The
oracle-side tests and the GPU path both draw their inputs from here.

Catalog dictionaries hold ``pos`` (n x 3 float64, box frame [0, L)^3, Mpc/h),
``w`` (FKP weights) and ``nbar`` (mean density at each object).

Generators (seed = 1000 * workload + stream, NumPy ``Generator(PCG64)``):

* ``uniform_box``     -- uniform points in a cube (tiny cases, shot noise).
* ``tiny_survey``     -- 2e4 galaxies + 1e5 randoms in a 500 Mpc/h cube,
  observer at (-300, -300, -300), FKP weights with P_FKP = 1e4.
* ``lognormal_mock``  -- a BOSS-like survey: lognormal density on a mesh,
  linear radial redshift-space displacement s = x - f xhat (u . xhat)
  (Sec. I eq. RSDmap), cut to a radial shell over a spherical cap.
* ``kaiser_nodes``    -- one object per grid node carrying a fixed-amplitude
  Kaiser field (1 + f mu^2) sqrt(P) exp(i phi), mu measured along +z.
"""

from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

_WORKERS = max(1, min(16, os.cpu_count() or 1))


def rng_for(workload: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * workload + stream))


def uniform_box(n: int, box: float, rng: np.random.Generator, nbar: float | None = None,
                w: float | None = None) -> dict:
    pos = rng.random((n, 3)) * box
    pos = np.minimum(pos, np.nextafter(box, 0.0))
    nb = n / box**3 if nbar is None else nbar
    ww = 1.0 if w is None else w
    return {"pos": pos, "w": np.full(n, ww), "nbar": np.full(n, nb)}


def tiny_survey(n_gal: int = 20_000, n_ran: int = 100_000, box: float = 500.0,
                observer=(-300.0, -300.0, -300.0), p_fkp: float = 1.0e4, seed: int = 1000):
    """Uniform galaxies and randoms in a cube with constant nbar and FKP weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nbar = n_gal / box**3
    w = 1.0 / (1.0 + nbar * p_fkp)
    gal = uniform_box(n_gal, box, rng, nbar, w)
    ran = uniform_box(n_ran, box, rng, nbar, w)
    return gal, ran, n_gal / n_ran, tuple(float(v) for v in observer)


def power_law_bump(k, amp=None, k_pivot=0.02, slope=2.3, p_at_01=1.2e4):
    """P(k) = A k / (1 + (k/k_pivot)^slope), A fixed by P(0.1) (Mpc/h)^3."""
    if amp is None:
        amp = p_at_01 * (1.0 + (0.1 / k_pivot) ** slope) / 0.1
    k = np.asarray(k, dtype=np.float64)
    return amp * k / (1.0 + (k / k_pivot) ** slope)


def _kgrid(N, box):
    kf = 2.0 * math.pi / box
    f = np.fft.fftfreq(N, d=1.0 / N) * kf
    fz = np.arange(N // 2 + 1) * kf
    return f, fz


def _in_survey(pos, observer, r_min, r_max, cos_max, axis):
    r = pos - observer[None, :]
    rr = np.sqrt(np.sum(r * r, axis=1))
    c = (r @ axis) / np.maximum(rr, 1e-300)
    return (rr >= r_min) & (rr < r_max) & (c >= cos_max)


def survey_volume(r_min, r_max, cap_deg):
    omega = 2.0 * math.pi * (1.0 - math.cos(math.radians(cap_deg)))
    return omega * (r_max**3 - r_min**3) / 3.0


def lognormal_mock(n_mesh: int = 512, box: float = 3500.0, n_gal: float = 8.0e5,
                   n_ran: int = 40_000_000, f: float = 0.7, seed: int = 2000,
                   r_min: float = 1150.0, r_max: float = 1750.0, cap_deg: float = 60.0,
                   observer=(-400.0, 1750.0, 1750.0), p_fkp: float = 1.0e4,
                   ran_seed: int | None = None, make_randoms: bool = True, r_smooth: float = 0.0):
    """Lognormal redshift-space mock in a shell x cap survey.

    G is Gaussian on an n_mesh^3 grid with power P(k) (``power_law_bump``);
    delta = exp(G - sigma^2/2) - 1 with sigma^2 = V^-1 sum_{n != 0} P(k_n).
    The linear displacement u(k) = -i k G(k)/k^2 (so that div u = G) moves
    each galaxy along its line of sight, s = x - f xhat (u . xhat).  Galaxies
    are Poisson-sampled per cell with mean nbar h^3 (1 + delta), placed
    uniformly inside the cell, displaced, and kept if s lies in the survey.
    Randoms are uniform in r^3 and in solid angle over the cap.
    Constant nbar = n_gal / V_survey and w = 1 / (1 + nbar P_FKP).
    With make_randoms=False the random catalogue is returned empty (alpha is
    still N_g / n_ran, for a random catalogue drawn separately).
    r_smooth > 0 (Mpc/h) multiplies P(k) by exp(-k^2 r_smooth^2), which keeps
    sigma^2 finite on fine meshes: the power law alone gives sigma^2 = 2.1,
    6.9 and 22.5 at N = 256, 512, 1024 in the 3500 Mpc/h box, and at 22.5
    single cells hold millions of galaxies; r_smooth = 3 gives 2.6 at 1024.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    N, L = n_mesh, box
    h = L / N
    obs = np.asarray(observer, dtype=np.float64)
    axis = np.array([1.0, 0.0, 0.0])
    cos_max = math.cos(math.radians(cap_deg))
    vol = survey_volume(r_min, r_max, cap_deg)
    nbar = n_gal / vol
    w = 1.0 / (1.0 + nbar * p_fkp)

    kx, kz = _kgrid(N, L)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    pk = power_law_bump(np.sqrt(k2))
    if r_smooth > 0.0:
        pk *= np.exp(-k2 * r_smooth**2)
    pk[0, 0, 0] = 0.0
    # sigma^2 over the full grid: half-grid modes 0 < nz < N/2 count twice
    mult = np.full(N // 2 + 1, 2.0)
    mult[0] = 1.0
    mult[-1] = 1.0
    sigma2 = float(np.sum(pk * mult[None, None, :]) / L**3)

    white = rng.standard_normal((N, N, N))
    gk = sfft.rfftn(white, workers=_WORKERS)
    del white
    gk *= np.sqrt(pk / h**3)
    del pk
    delta = sfft.irfftn(gk, s=(N, N, N), axes=(0, 1, 2), workers=_WORKERS)
    np.exp(delta - 0.5 * sigma2, out=delta)           # 1 + delta
    lam = (nbar * h**3) * delta.ravel()
    del delta
    counts = rng.poisson(lam)
    del lam
    cells = np.repeat(np.arange(N**3, dtype=np.int64), counts)
    del counts
    ix = cells // (N * N)
    iy = (cells // N) % N
    iz = cells % N
    pos = (np.stack([ix, iy, iz], axis=1) + rng.random((len(cells), 3))) * h
    r = pos - obs[None, :]
    xhat = r / np.sqrt(np.sum(r * r, axis=1))[:, None]
    ux = np.zeros(len(cells))
    k2[0, 0, 0] = 1.0
    for d, kd in enumerate((kx[:, None, None], kx[None, :, None], kz[None, None, :])):
        comp = sfft.irfftn(-1j * kd * gk / k2, s=(N, N, N), axes=(0, 1, 2), workers=_WORKERS).ravel()
        ux += comp[cells] * xhat[:, d]
        del comp
    del gk, k2
    s = pos - f * xhat * ux[:, None]
    keep = _in_survey(s, obs, r_min, r_max, cos_max, axis)
    keep &= np.all((s >= 0.0) & (s < L), axis=1)
    gpos = s[keep]
    ng = len(gpos)
    gal = {"pos": gpos, "w": np.full(ng, w), "nbar": np.full(ng, nbar)}

    if make_randoms:
        rr = np.random.Generator(np.random.PCG64(seed + 500 if ran_seed is None else ran_seed))
        ran = {"pos": _cap_randoms(rr, int(n_ran), obs, r_min, r_max, cos_max),
               "w": np.full(int(n_ran), w), "nbar": np.full(int(n_ran), nbar)}
    else:
        ran = {"pos": np.zeros((0, 3)), "w": np.zeros(0), "nbar": np.zeros(0)}
    alpha = ng / float(n_ran)
    meta = {"nbar": nbar, "w": w, "sigma2": sigma2, "volume": vol, "n_gal": ng}
    return gal, ran, alpha, tuple(obs.tolist()), meta


def _cap_randoms(rng, n, obs, r_min, r_max, cos_max):
    out = np.empty((n, 3))
    chunk = 4_000_000
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        u = rng.random((m, 3))
        r = (r_min**3 + u[:, 0] * (r_max**3 - r_min**3)) ** (1.0 / 3.0)
        c = cos_max + u[:, 1] * (1.0 - cos_max)
        sn = np.sqrt(np.maximum(0.0, 1.0 - c * c))
        phi = 2.0 * math.pi * u[:, 2]
        out[s:s + m, 0] = obs[0] + r * c
        out[s:s + m, 1] = obs[1] + r * sn * np.cos(phi)
        out[s:s + m, 2] = obs[2] + r * sn * np.sin(phi)
    return out


def kaiser_nodes(N: int, box: float, f: float, rng: np.random.Generator, pk=None):
    """One object per grid node carrying a fixed-amplitude Kaiser field.

    The field's Fourier amplitude at mode n is (1 + f mu^2) sqrt(P(k)) with a
    uniformly random phase (Hermitian), mu = n_z/|n|.  Objects sit exactly on
    nodes i*h with weight delta_s(x_i).  Returns (catalog, amplitude2) where
    amplitude2 is the half-grid array of (1 + f mu^2)^2 P(k).
    """
    f_ = np.fft.fftfreq(N, d=1.0 / N)
    fz = np.arange(N // 2 + 1)
    nx, ny, nz = np.meshgrid(f_, f_, fz, indexing="ij")
    n2 = nx**2 + ny**2 + nz**2
    nn = np.sqrt(np.where(n2 > 0, n2, 1.0))
    mu = nz / nn
    kf = 2.0 * math.pi / box
    p = np.ones_like(nn) if pk is None else pk(kf * nn)
    amp = (1.0 + f * mu**2) * np.sqrt(p)
    amp[0, 0, 0] = 0.0
    # unit-modulus phases from the transform of real white noise are Hermitian
    # by construction, so the field below has exactly the amplitude amp
    wn = np.fft.rfftn(rng.standard_normal((N, N, N)))
    phase = wn / np.maximum(np.abs(wn), 1e-300)
    spec = amp * phase
    field = np.fft.irfftn(spec, s=(N, N, N), axes=(0, 1, 2))
    amp2 = amp**2
    idx = np.arange(N)
    gx, gy, gz = np.meshgrid(idx, idx, idx, indexing="ij")
    pos = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1) * (box / N)
    cat = {"pos": pos, "w": field.ravel().copy(), "nbar": np.ones(N**3)}
    return cat, amp2


def catalog_digest(gal: dict, ran: dict, alpha: float, observer) -> str:
    """SHA-256 of a catalogue pair (float64 bytes of every array, alpha and the
    observer), to tell whether two hosts drew bit-identical mocks."""
    import hashlib
    h = hashlib.sha256()
    for cat in (gal, ran):
        for key in ("pos", "w", "nbar"):
            h.update(np.ascontiguousarray(cat[key], dtype=np.float64).tobytes())
    h.update(np.asarray([alpha, *observer], dtype=np.float64).tobytes())
    return h.hexdigest()


def lognormal_pool(n_mocks: int, seed0: int = 2000, **kw):
    """Pool of mocks sharing one random catalogue (that of mock 0, seed0 +
    500), as a covariance run does: galaxy catalogues from seeds seed0 + 10 i.
    Returns a list of (gal, alpha) and the shared (ran, observer)."""
    gal0, ran, alpha0, obs, _ = lognormal_mock(seed=seed0, **kw)
    out = [(gal0, alpha0)]
    for i in range(1, n_mocks):
        g, _, a, _, _ = lognormal_mock(seed=seed0 + 10 * i, ran_seed=seed0 + 500, make_randoms=False, **kw)
        out.append((g, a))
    return out, ran, obs
