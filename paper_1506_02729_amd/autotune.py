"""Autotuner of a plan's launch parameters, cached as JSON per plan shape.

The tunable parameters are those of ``frsd_tuning`` (include/fastrsd.h):
the workgroup count of the matrix-core contraction, of the persistent
forward z pass and of the binning kernel, the number of shell-field pairs
per inverse-FFT launch, and the x run of the x-sweep assignment's
workgroup tiles.  None changes a result beyond rounding order.
The radix schedules of the FFT lengths are fixed at compile time (one
schedule per length), so the tuner chooses launch tiles only.

Search: coordinate descent.  For each parameter in turn, every candidate is
timed over a few requests (per-kernel HIP-event durations from
``frsd_profile``, summed over the kernels that parameter drives), the
fastest is kept, and the next parameter is tuned with it in place.  The
result is stored under a key of the plan shape (precision, N, order,
interlacing, ell_max, M, bins) in a JSON file; ``apply`` sets a plan's
tuning from that file when its shape is there.
"""

from __future__ import annotations

import json
import os

from . import fastrsd as F

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

CANDIDATES = {
    "tri_wg": (512, 768, 1024, 1536, 2048),
    "row_grid": (1024, 2048, 4096, 8192),
    "bin_blocks": (1024, 2048, 4096),
    "pair_batch": (2, 4, 8, 16),
    "sweep_x": (16, 32, 64),
}
AFFECTS = {
    "tri_wg": ("triple", "tri_reduce"),
    "row_grid": ("fft_z",),
    "bin_blocks": ("bin", "bin_reduce"),
    "pair_batch": ("shell_z", "shell_y", "shell_x"),
    "sweep_x": ("grid", "grid_twin"),
}


def shape_key(cfg: F.Config, bk_grid: int) -> str:
    return (f"p{cfg.precision}_N{cfg.n_grid}_o{cfg.order}_i{int(cfg.interlace)}_l{cfg.ell_max}"
            f"_bl{cfg.bk_ell_max}_M{bk_grid}_pk{cfg.pk_nbins}_bk{cfg.bk_nbins}")


def load(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def apply(plan: F.Plan, path: str = DEFAULT_CACHE) -> dict | None:
    """Set plan's tuning from the cache if its shape is there; returns it."""
    entry = load(path).get(shape_key(plan.cfg, plan.bk_grid))
    if not entry:
        return None
    F.frsd_plan_set_tuning(plan.handle, entry["tuning"])
    return entry["tuning"]


def _time(plan: F.Plan, run_request, kernels, reps: int, sync) -> float:
    run_request(plan)             # first request with these parameters, untimed
    sync()
    F.frsd_profile(True)
    F.frsd_profile_report()
    for _ in range(reps):
        run_request(plan)
    sync()
    rep = F.frsd_profile_report()
    F.frsd_profile(False)
    return sum(rep[k][1] for k in kernels if k in rep) / reps


def tune(plan: F.Plan, run_request, sync, reps: int = 3, path: str | None = DEFAULT_CACHE, log=print) -> dict:
    """Coordinate descent over CANDIDATES on `plan`; run_request(plan)
    enqueues one request, sync() waits for the device.  Writes the result
    into the JSON cache at `path` (None: no file) and returns it."""
    best = F.frsd_plan_get_tuning(plan.handle)
    timings = {}
    for name, cands in CANDIDATES.items():
        if name in ("tri_wg", "pair_batch") and plan.ntri == 0:
            continue
        res = {}
        for v in cands:
            trial = dict(best, **{name: v})
            F.frsd_plan_set_tuning(plan.handle, trial)
            res[v] = _time(plan, run_request, AFFECTS[name], reps, sync)
        pick = min(res, key=res.get)
        best[name] = pick
        timings[name] = {str(k): round(v, 4) for k, v in res.items()}
        log(f"autotune {name}: " + ", ".join(f"{k}: {v:.3f} ms" for k, v in res.items()) + f" -> {pick}")
    F.frsd_plan_set_tuning(plan.handle, best)
    entry = {"tuning": best, "ms_per_request": timings, "reps": reps}
    if path:
        cache = load(path)
        cache[shape_key(plan.cfg, plan.bk_grid)] = entry
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return entry
