"""Write the FP64 oracle's results for the 256^3 bispectrum workload.

Runs only the oracle (``oracle/``) on the seeded lognormal mock of
``paper_1506_02729_amd.synth.lognormal_mock`` at N = 256 (2e5 galaxies, 1e7
randoms, box 3500 Mpc/h, seed 3000): interlaced TSC, P_0,2,4 in 45 bins of
0.005 h/Mpc (to 0.225 < k_Nyquist), and for ALL 5416 triangles of 37 bins of
3 k_f (centres m 3 k_f, m = 1..37, top edge 112.5 k_f = 0.202 h/Mpc):
N^T, T_0,2,4 with their conditioning sums, B_0,2,4, the thin-shell shot noise
(complete for every ell, from the w^2-weighted multipoles F^w_2, F^w_4, and
the q1 term alone), and the zero-area hexadecapole T_220 / B4za.  The
triangle sums are taken on the M = 343 grid by
``estimator.bk_triangle_sums_streamed`` (any M > 3 n_c = 336 gives the exact
closed-triangle sums).  The result goes to ``cfg3_golden.json`` beside this
script with the SHA-256 of the catalogue.

Usage:  python tests/golden/make_cfg3_golden.py [scratch.npy]
        (about an hour on 8 cores; ~50 GB of scratch disk for the shell fields)
"""

from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import assign_c  # noqa: E402
from oracle import estimator as est  # noqa: E402
from paper_1506_02729_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "cfg3_golden.json")
SEED = 3000
N, BOX, N_GAL, N_RAN = 256, 3500.0, 2.0e5, 10_000_000
PK_DK, PK_NBINS = 0.005, 45
BK_NBINS = 37
M_ORACLE = 343


def params(observer):
    kf = 2 * math.pi / BOX
    return est.Params(n_grid=N, box=BOX, observer=observer, order=3, interlace=True, compensate=True, ell_max=4,
                      pk_kmin=0.0, pk_dk=PK_DK, pk_nbins=PK_NBINS, bk_kmin=1.5 * kf, bk_dk=3 * kf,
                      bk_nbins=BK_NBINS, m_grid=M_ORACLE, assign=assign_c.assign_mesh)


def mock():
    return synth.lognormal_mock(n_mesh=N, box=BOX, n_gal=N_GAL, n_ran=N_RAN, seed=SEED)


def main():
    scratch = sys.argv[1] if len(sys.argv) > 1 else os.path.join("/tmp", "cfg3_shells.npy")
    t0 = time.time()
    gal, ran, alpha, observer, _ = mock()
    digest = synth.catalog_digest(gal, ran, alpha, observer)
    print(f"mock: {len(gal['w'])} galaxies, {len(ran['w'])} randoms, sha256 {digest[:16]}", flush=True)
    prm = params(observer)
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True, with_w_ell=True)
    print(f"fields {time.time() - t0:.0f} s", flush=True)
    pk = est.pk_multipoles(gal, ran, alpha, prm, fields=fields)
    tri = est.triangle_list(prm)
    ts = est.bk_triangle_sums_streamed(fields, prm, tri, scratch, t220=True)
    print(f"triangle sums of {len(tri)} triangles {time.time() - t0:.0f} s", flush=True)
    bk = est.bk_multipoles(gal, ran, alpha, prm, triangles=tri, fields=fields, zero_area=True, tsums=ts)

    def lst(a):
        return [float(v) for v in np.asarray(a, dtype=np.float64)]

    out = {
        "about": "FP64 oracle results for the 256^3 lognormal mock (seed 3000), written by make_cfg3_golden.py",
        "catalog_sha256": digest,
        "n_gal": int(len(gal["w"])), "n_ran": int(len(ran["w"])), "alpha": float(alpha),
        "observer": [float(v) for v in observer], "M_oracle": M_ORACLE,
        "scalars": {k: float(pk[k]) for k in ("I22", "N0", "I33", "W3")},
        "pk": {"n_modes": [int(v) for v in pk["n_modes"]], "k_eff": lst(pk["k_eff"]),
               **{f"P{ell}": lst(pk[f"P{ell}"]) for ell in (0, 2, 4)}, "P4b": lst(pk["P4b"]),
               **{f"S{ell}0": lst(pk[f"S{ell}0"]) for ell in (0, 2, 4)}, "S22": lst(pk["S22"]),
               **{f"C{ell}0": lst(pk[f"C{ell}0"]) for ell in (0, 2, 4)}},
        "bk": {"triangles": [[int(b) for b in t] for t in tri],
               "NT": lst(bk["NT"]),
               **{f"T{ell}": lst(bk[f"T{ell}"]) for ell in (0, 2, 4)},
               **{f"C{ell}": lst(bk[f"C{ell}"]) for ell in (0, 2, 4)},
               **{f"B{ell}": lst(bk[f"B{ell}"]) for ell in (0, 2, 4)},
               **{f"SN{ell}": lst(bk[f"SN{ell}"]) for ell in (0, 2, 4)},
               **{f"SN{ell}_q1": lst(bk[f"SN{ell}_q1"]) for ell in (2, 4)},
               "T220": lst(bk["T220"]), "C220": lst(bk["C220"]), "B4za": lst(bk["B4za"])},
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
