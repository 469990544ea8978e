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
  direct sums over objects, direct triangle enumeration (with any function
  per side), lattice-point counts.

Every function is pinned by a test in ``tests/test_oracle_pins.py`` or
``tests/test_oracle_pins_bk.py`` against something other than itself: brute
force over objects or lattice triangles, closed forms (I22, I33, N_0, W3 for
constant nbar and w), exact expectations (P_ell of a Poisson-sampled fixed
field), the plane-parallel limit (B_ell prefactors, the w^2-weighted shell
sums), and lattice configurations in which the thin-shell shot noise equals
its exact triangle sum.

It shares no code with the GPU path.  Every function cites the passage of
the paper it follows.
"""

from . import estimator, brute  # noqa: F401
from .estimator import Params, pk_multipoles, bk_multipoles  # noqa: F401
