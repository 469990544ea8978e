"""FP64 CPU oracle for the FFT multipole estimators of Scoccimarro,
"Fast Estimators for Redshift-Space Clustering" (arXiv:1506.02729).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything here.  Only
the test-suite, the smoke check in ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is a plain, slow, obviously correct NumPy implementation, in
float64, of what the estimator computes:

* ``estimator``  -- gridding of moment weights, FFTs, multipole combination,
  shell binning, P_ell, the FFT triangle search, N^T and B_ell
  (Sec. III.A eqs. F0-Nelltrue and mapFFT, Sec. III.B eqs. BispMono-F_k).
* ``brute``      -- brute-force twins used to pin the estimator: per-mode
  direct sums over objects, direct triangle enumeration, lattice-point
  counts.

Parity unpinned: the l > 0 thin-shell shot-noise q1 term (SN2, SN4) has no
pin beyond its formula, and I33 (not defined in the paper; read as
alpha sum_r nbar^2 w^3) is pinned only through its definition.

It shares no code with the GPU path.  Every function cites the passage of
the paper it follows.
"""

from . import estimator, brute  # noqa: F401
from .estimator import Params, pk_multipoles, bk_multipoles  # noqa: F401
