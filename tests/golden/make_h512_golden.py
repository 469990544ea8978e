"""Write the FP64 oracle's results for the 512^3 lognormal-mock workload.

Runs only the oracle (``oracle/``) on the seeded mock of
``paper_1506_02729_amd.synth.lognormal_mock`` (8e5 galaxies, 4e7 randoms,
box 3500 Mpc/h, seed 2000): interlaced TSC on N = 512, P_0,2,4 in 60 bins of
0.005 h/Mpc, and B_0,2,4 with N^T on a sample of the 5416 triangles of 37
bins of 3 k_f (every triangle whose three bins lie in SAMPLE_BINS).  The
result goes to ``h512_golden.json`` beside this script together with the
SHA-256 of the catalogue, so a GPU test can check that it drew the same mock.

Usage:  python tests/golden/make_h512_golden.py      (about 20 minutes, ~25 GB)
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

OUT = os.path.join(HERE, "h512_golden.json")
SEED = 2000
N, BOX, N_GAL, N_RAN = 512, 3500.0, 8.0e5, 40_000_000
PK_DK, PK_NBINS = 0.005, 60
BK_NBINS = 37
SAMPLE_BINS = (0, 1, 8, 17, 18, 26, 36)


def params(observer):
    kf = 2 * math.pi / BOX
    return est.Params(n_grid=N, box=BOX, observer=observer, order=3, interlace=True, compensate=True, ell_max=4,
                      pk_kmin=0.0, pk_dk=PK_DK, pk_nbins=PK_NBINS, bk_kmin=1.5 * kf, bk_dk=3 * kf,
                      bk_nbins=BK_NBINS, assign=assign_c.assign_mesh)


def main():
    t0 = time.time()
    gal, ran, alpha, observer, _ = synth.lognormal_mock(n_mesh=N, box=BOX, n_gal=N_GAL, n_ran=N_RAN, seed=SEED)
    digest = synth.catalog_digest(gal, ran, alpha, observer)
    print(f"mock: {len(gal['w'])} galaxies, {len(ran['w'])} randoms, sha256 {digest[:16]}", flush=True)
    prm = params(observer)
    fields = est.multipole_fields(gal, ran, alpha, prm, with_w=True)
    print(f"fields {time.time() - t0:.0f} s", flush=True)
    pk = est.pk_multipoles(gal, ran, alpha, prm, fields=fields)
    tri_all = est.triangle_list(prm)
    keep = np.all(np.isin(tri_all, SAMPLE_BINS), axis=1)
    index = np.nonzero(keep)[0]
    bk = est.bk_multipoles(gal, ran, alpha, prm, triangles=tri_all[index], fields=fields)
    print(f"bispectrum sample of {len(index)} triangles {time.time() - t0:.0f} s", flush=True)

    def lst(a):
        return [float(v) for v in np.asarray(a, dtype=np.float64)]

    out = {
        "about": "FP64 oracle results for the 512^3 lognormal mock (seed 2000), written by make_h512_golden.py",
        "catalog_sha256": digest,
        "n_gal": int(len(gal["w"])), "n_ran": int(len(ran["w"])), "alpha": float(alpha),
        "observer": [float(v) for v in observer],
        "scalars": {k: float(pk[k]) for k in ("I22", "N0", "I33", "W3")},
        "pk": {"n_modes": [int(v) for v in pk["n_modes"]], "k_eff": lst(pk["k_eff"]),
               **{f"P{ell}": lst(pk[f"P{ell}"]) for ell in (0, 2, 4)},
               **{f"S{ell}0": lst(pk[f"S{ell}0"]) for ell in (0, 2, 4)},
               **{f"C{ell}0": lst(pk[f"C{ell}0"]) for ell in (0, 2, 4)}},
        "bk": {"index": [int(v) for v in index], "triangles": [[int(b) for b in t] for t in tri_all[index]],
               "NT": lst(bk["NT"]),
               **{f"T{ell}": lst(bk[f"T{ell}"]) for ell in (0, 2, 4)},
               **{f"C{ell}": lst(bk[f"C{ell}"]) for ell in (0, 2, 4)},
               **{f"B{ell}": lst(bk[f"B{ell}"]) for ell in (0, 2, 4)},
               **{f"SN{ell}": lst(bk[f"SN{ell}"]) for ell in (0, 2, 4)}},
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
