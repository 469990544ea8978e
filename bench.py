"""Throughput of the FFT multipole estimators on one MI355X.

One step = one request: a synthetic BOSS-like mock through the whole hot path:
ingest + sort, interlaced TSC assignment of the 22 moment meshes and the
w^2 mesh, their forward FFTs, multipole combination and binning into
P_0, P_2, P_4 (60 bins to k = 0.3 h/Mpc), shell-filtered inverse FFTs on the
M = 343 grid and the triple-product sums of B_0, B_2, B_4 over all 5416
triangles of 37 bins of width 3 k_f up to k = 0.2 h/Mpc.  The served FP32
measurement is a closed loop of --steps requests cycling a pool of --mocks
distinct mocks (galaxy catalogues of distinct seeds sharing one random
catalogue, as in a covariance run); catalogues are resident in HBM before
the timed region and nothing is cached between requests.  --streams
requests are in flight at once, each on its own plan (workspace) and HIP
stream, so the kernels of consecutive requests overlap; the value is
requests over the wall time of the whole loop.  The plain FP64 leg runs one
mock at a time.

Prints one JSON line (see the "metric" key).  --gpus N > 1 is refused: the
build targets one GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mocks/s for P_0,2,4+B_0,2,4 at 512^3 (served FP32 vs plain FP64), HBM %, p99 ms"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30                 # calibration copy: reads and writes 1 GiB
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {"grid": "grid.hip", "grid_twin": "grid.hip", "fft_z": "fft.hip", "fft_y": "fft.hip",
                  "fft_x": "fft.hip", "triple": "triple_mfma.hip", "bin": "pk.hip", "shell_x": "bk.hip",
                  "shell_y": "bk.hip", "shell_z": "bk.hip"}
FP32_VEC_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


def workload(quick: bool):
    box = 3500.0
    kf = 2 * math.pi / box
    if quick:
        return dict(name="Q256: lognormal mock 2.0e5 galaxies + 1.0e7 randoms, N=256 TSC interlaced, "
                         "P_ell 45 bins to k=0.225, B_ell 37 bins of 3k_f (5416 triangles), M=343",
                    n_mesh=256, n_gal=2.0e5, n_ran=10_000_000, pk_dk=0.005, pk_nbins=45,
                    bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=37, box=box)
    return dict(name="H512: lognormal mock 8.0e5 galaxies + 4.0e7 randoms in a 3500 Mpc/h box, N=512 TSC "
                     "interlaced, 23 moment meshes, P_ell l=0,2,4 in 60 bins of 0.005 to k=0.3, B_ell l=0,2,4 "
                     "over 5416 triangles of 37 bins of 3k_f to k=0.202, M=343",
                n_mesh=512, n_gal=8.0e5, n_ran=40_000_000, pk_dk=0.005, pk_nbins=60,
                bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=37, box=box)


def make_config(F, wl, precision, observer, max_objects):
    return F.Config(n_grid=wl["n_mesh"], box=wl["box"], observer=observer, order=3, interlace=True,
                    compensate=True, ell_max=4, precision=precision, pk_kmin=0.0, pk_dk=wl["pk_dk"],
                    pk_nbins=wl["pk_nbins"], bk_kmin=wl["bk_kmin"], bk_dk=wl["bk_dk"],
                    bk_nbins=wl["bk_nbins"], max_objects=max_objects)


def algorithmic_cost(name, plan_cfg, n_obj, n_slot, M, n_out, tbytes):
    """Algorithmic bytes (HBM-bound kernels) or flops of one launch."""
    N = plan_cfg.n_grid
    cplx = 2 * tbytes
    mesh = n_slot * N**3 * cplx
    if name in ("grid", "grid_twin"):  # one grid's planes (half the mesh) written once, every record read once
        return "hbm", mesh // 2 + n_obj * 4 * tbytes
    if name.startswith("fft_"):  # read + write every mesh once per pass
        return "hbm", 2 * mesh
    if name == "shell_x":       # write two real M^3 fields per pair of 8 per launch
        return "hbm", 16 * M**3 * tbytes
    if name == "triple":        # 3 flops per listed output (triangle x multipole) per cell, on the matrix cores
        return "mfma", 3.0 * n_out * M**3
    return None, None


def source_hash(kernel):
    import hashlib
    src = KERNEL_SOURCES.get(kernel)
    if src is None:
        return None
    h = hashlib.sha256()
    for f in (src, "device.h", "frsd_internal.h"):
        with open(os.path.join(ROOT, "paper_1506_02729_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, if the kernel
    source is unchanged since the counters were taken; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            tab = json.load(fh)
    except (OSError, ValueError):
        return None
    e = tab.get(kernel)
    if not e or e.get("source_hash") != source_hash(kernel):
        return None
    return e.get("bytes_per_launch")


def run_steps(F, torch, plans, mocks, steps, timed: bool):
    """Serve `steps` requests cycling the pool; request i goes to plan i % len(plans)
    (one stream and workspace per plan, so consecutive requests overlap)."""
    if not isinstance(plans, (list, tuple)):
        plans = [plans]
    lat = []
    for i in range(steps):
        g, r, a = mocks[i % len(mocks)]
        plan = plans[i % len(plans)]
        if timed:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(plan.stream)
        plan.mesh_assign(g, r, a)
        plan.pk()
        plan.bk()
        if timed:
            e1.record(plan.stream)
            lat.append((e0, e1))
    return lat


def cpu_baseline(wl, gal, ran, alpha, observer, M):
    """FP64 oracle timed on a bounded sample of the same workload, scaled to one mock."""
    from oracle import estimator as est
    N = wl["n_mesh"]
    n_obj = len(gal["w"]) + len(ran["w"])
    t = {}
    sample = 1_000_000
    pos = ran["pos"][:sample]
    u = pos / (wl["box"] / N)
    w = -alpha * ran["w"][:sample]
    t0 = time.perf_counter()
    est.assign_mesh(u, w, N, 3)
    t["grid_1moment_1e6obj"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    mesh = np.random.default_rng(0).standard_normal((N, N, N))
    t1 = time.perf_counter()
    np.fft.rfftn(mesh)
    t["rfftn"] = time.perf_counter() - t1
    del mesh
    prm = est.Params(n_grid=N, box=wl["box"], observer=observer, pk_kmin=0.0, pk_dk=wl["pk_dk"],
                     pk_nbins=wl["pk_nbins"])
    fields = {0: np.ones((N, N, N // 2 + 1), complex), 2: np.ones((N, N, N // 2 + 1), complex),
              4: np.ones((N, N, N // 2 + 1), complex)}
    t0 = time.perf_counter()
    est.shell_sums(fields, prm, 0.0, wl["pk_dk"], wl["pk_nbins"])
    t["bin"] = time.perf_counter() - t0
    del fields
    bprm = est.Params(n_grid=N, box=wl["box"], observer=observer, bk_kmin=wl["bk_kmin"], bk_dk=wl["bk_dk"],
                      bk_nbins=wl["bk_nbins"])
    nx, ny, nz, b = est.lowk_modes(bprm)
    sel = b == wl["bk_nbins"] // 2
    t0 = time.perf_counter()
    f = est.shell_field(np.ones(int(sel.sum()), complex), nx[sel], ny[sel], nz[sel], M)
    t["shell_ifft"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(3):
        float(np.sum(f * f * f))
    t["triangle_sum"] = (time.perf_counter() - t0) / 3
    del f
    n_tri, n_ell, n_mom, n_fields = 5416, 3, 23, 111
    per_mock = (t["grid_1moment_1e6obj"] * (n_obj / sample) * n_mom * 2 + t["rfftn"] * n_mom * 2 + t["bin"]
                + t["shell_ifft"] * n_fields + t["triangle_sum"] * n_tri * n_ell)
    return {"value": 1.0 / per_mock, "unit": "mocks/s", "cores": 1, "kind": "oracle",
            "seconds_per_mock": per_mock,
            "sample": ("FP64 NumPy oracle stages timed once each on this host and scaled to one mock: TSC "
                       "assignment of 1e6 randoms for one moment plane (x %.0f objects x 46 planes), one "
                       "512^3 rfftn (x 46), the 60-bin shell sums of 3 multipoles, one %d^3 shell inverse "
                       "FFT (x 111), one %d^3 triple-product sum (x 5416 triangles x 3 multipoles)"
                       % (n_obj / sample, M, M)),
            "stage_seconds": {k: round(v, 4) for k, v in t.items()}}


def oracle_check(F, torch, plan, mock0, gold_path):
    """FP32 result of pool mock 0 against the stored FP64 oracle results for
    that mock (written by tests/golden/make_h512_golden.py), if the catalogue
    digest matches; max relative error per multipole with the conditioning
    floors of the parity tests."""
    from paper_1506_02729_amd import synth
    try:
        with open(gold_path) as fh:
            gold = json.load(fh)
    except OSError:
        return None
    g_host, ran_host, alpha, obs, g_dev, r_dev = mock0
    if synth.catalog_digest(g_host, ran_host, alpha, obs) != gold["catalog_sha256"]:
        return {"skipped": "catalogue digest differs from the stored oracle run"}
    out = plan.run(g_dev, r_dev, alpha)
    pk, sc, bk = gold["pk"], gold["scalars"], gold["bk"]
    nb = np.asarray(pk["n_modes"], dtype=float)
    res = {"bins": len(nb), "triangles": len(bk["index"])}
    floors = {0: np.asarray(pk["S00"]) / (nb * sc["I22"])}
    for ell in (2, 4):
        floors[ell] = (2 * ell + 1) * np.asarray(pk[f"C{ell}0"]) / (nb * sc["I22"])
    for ell in (0, 2, 4):
        ref = np.asarray(pk[f"P{ell}"])
        res[f"P{ell}_max_rel"] = float(np.max(np.abs(out[f"p{ell}"] - ref) / np.maximum(np.abs(ref), floors[ell])))
    idx = np.asarray(bk["index"])
    nt = np.asarray(bk["NT"])
    ok = nt > 0
    res["NT_exact"] = bool(np.array_equal(out["bk_nt"][idx], nt))
    for ell in (0, 2, 4):
        ref = np.asarray(bk[f"T{ell}"])[ok]
        C = np.asarray(bk[f"C{ell}"])[ok]
        res[f"T{ell}_max_rel"] = float(np.max(np.abs(out[f"bk_t{ell}"][idx][ok] - ref) / np.maximum(np.abs(ref), C)))
    return res


def open_loop(args, F, torch, synth, dev, log):
    """Open-loop serving of requests of mixed mesh sizes: Poisson arrivals
    (exponential gaps of mean --mean-gap s), N uniform in {256, 384, 512},
    N_g uniform in [3e5, the pool size] and N_r = 50 N_g taken as prefixes of
    shuffled pool catalogues resident in HBM, P_ell to min(0.3, k_Ny) in bins
    of 0.005 and B_ell on 18 bins of 3 k_f (k <= 0.1).  Admission by HBM
    footprint: every mesh size starts with one plan (workspace + stream); a
    queued request takes a free plan of its size, or a new one when the
    workspaces (exact sizes from the plan) stay within --hbm-budget-gb, or
    waits.  Latency runs from arrival to the P_ell and B_ell arrays on the
    host."""
    from collections import deque
    box = 3500.0
    kf = 2 * math.pi / box
    rng = np.random.Generator(np.random.PCG64(4000))
    t0 = time.perf_counter()
    pool, ran, observer = synth.lognormal_pool(4, seed0=4100, n_mesh=512, box=box, n_gal=8.0e5, n_ran=40_000_000)

    def shuffled(c, seed):
        perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(c["w"]))
        return {k: v[perm] for k, v in c.items()}

    gals = [F.device_catalog(shuffled(g, 4200 + i), dev) for i, (g, _) in enumerate(pool)]
    rand = F.device_catalog(shuffled(ran, 4300), dev)
    ng_max = min(len(g["w"]) for g, _ in pool)
    nr_all = len(ran["w"])
    log(f"open loop: pool of {len(gals)} mocks, {ng_max}+ galaxies, {nr_all} randoms in {time.perf_counter() - t0:.1f} s")
    sizes = (256, 384, 512)
    plans, nbins, cfgs, ws_bytes = {}, {}, {}, {}
    budget = args.hbm_budget_gb * 1e9
    for N in sizes:
        kny = math.pi * N / box
        nbins[N] = min(60, int(math.floor(kny / 0.005 - 1e-9)))  # bins of 0.005 to min(0.3, k_Ny)
        cfg = F.Config(n_grid=N, box=box, observer=observer, order=3, interlace=True, compensate=True, ell_max=4,
                       precision=32, pk_kmin=0.0, pk_dk=0.005, pk_nbins=nbins[N], bk_kmin=1.5 * kf, bk_dk=3 * kf,
                       bk_nbins=18, max_objects=ng_max + nr_all)
        cfgs[N] = cfg
        h = F.frsd_plan_create(cfg.to_c())
        ws_bytes[N] = F.frsd_plan_workspace_bytes(h)
        F.frsd_plan_destroy(h)
        plans[N] = [F.Plan(cfg, device=dev, stream=torch.cuda.Stream(dev))]
    used = sum(ws_bytes[N] for N in sizes)
    if used > budget:
        raise SystemExit(f"--hbm-budget-gb {args.hbm_budget_gb} is below one workspace per size ({used / 1e9:.1f} GB)")
    n = args.open_loop
    arrive = np.cumsum(rng.exponential(args.mean_gap, n))
    n_of = rng.choice(np.array(sizes), n)
    ng_of = rng.integers(300_000, ng_max + 1, n)
    mock_of = rng.integers(0, len(gals), n)

    def submit(pl, k):
        ng = int(ng_of[k])
        nr = min(50 * ng, nr_all)
        g = {key: v[:ng] for key, v in gals[mock_of[k]].items()}
        r = {key: v[:nr] for key, v in rand.items()}
        pl.mesh_assign(g, r, ng / nr)
        pl.pk()
        pl.bk()

    for N in sizes:  # one untimed request per plan: code objects loaded, tables resident
        for pl in plans[N]:
            submit(pl, 0)
    torch.cuda.synchronize()
    free = {id(pl): True for N in sizes for pl in plans[N]}
    queue, inflight, lat, sizes_done = deque(), [], [], []
    i = 0
    t0 = time.perf_counter()
    while i < n or queue or inflight:
        now = time.perf_counter() - t0
        while i < n and arrive[i] <= now:
            queue.append(i)
            i += 1
        for rec in list(inflight):
            pl, ev, k = rec
            if ev.query():
                host = [pl.pk_buf[key].cpu() for key in ("p0", "p2", "p4")]
                host += [pl.bk_buf[key].cpu() for key in ("b0", "b2", "b4")]
                lat.append(time.perf_counter() - t0 - arrive[k])
                sizes_done.append(int(n_of[k]))
                inflight.remove(rec)
                free[id(pl)] = True
        for k in list(queue):  # admit every queued request that has (or may allocate) a plan of its size
            N = int(n_of[k])
            pl = next((p for p in plans[N] if free[id(p)]), None)
            if pl is None and used + ws_bytes[N] <= budget:
                pl = F.Plan(cfgs[N], device=dev, stream=torch.cuda.Stream(dev))
                plans[N].append(pl)
                used += ws_bytes[N]
                free[id(pl)] = True
            if pl is None:
                continue
            queue.remove(k)
            free[id(pl)] = False
            submit(pl, k)
            ev = torch.cuda.Event()
            ev.record(pl.stream)
            inflight.append((pl, ev, k))
        time.sleep(0.0002)
    elapsed = time.perf_counter() - t0
    for N in sizes:
        for pl in plans[N]:
            assert pl.status() == 0
    lat_ms = 1e3 * np.asarray(lat)
    sz = np.asarray(sizes_done)
    per_size = {str(N): {"requests": int((sz == N).sum()), "p50_ms": float(np.percentile(lat_ms[sz == N], 50)),
                         "p99_ms": float(np.percentile(lat_ms[sz == N], 99))} for N in sizes if (sz == N).any()}
    out = {"metric": "open-loop request latency p99 (arrival to host result), mixed N in {256, 384, 512}",
           "value": float(np.percentile(lat_ms, 99)), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "requests": n, "p50_ms": float(np.percentile(lat_ms, 50)), "mocks_per_s": n / elapsed,
           "mean_gap_s": args.mean_gap, "hbm_budget_gb": args.hbm_budget_gb,
           "plans_per_size": {str(N): len(plans[N]) for N in sizes}, "workspace_gb": used / 1e9, "per_size": per_size,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "open loop: lognormal pool (4 mocks, 8e5 galaxies, 4e7 randoms, 3500 Mpc/h box), "
                                  "prefixes N_g in [3e5, pool], N_r = 50 N_g, P_ell l=0,2,4 to min(0.3, k_Ny), "
                                  "B_ell l=0,2,4 on 18 bins of 3 k_f",
                      "pk_bins": {str(N): nbins[N] for N in sizes}}}
    print(json.dumps(out), flush=True)



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64, help="requests served in the timed closed loop")
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--mocks", type=int, default=16, help="distinct mocks in the pool, cycled")
    ap.add_argument("--streams", type=int, default=3,
                    help="requests in flight: one plan (workspace) and HIP stream each, default priority")
    ap.add_argument("--kernel-steps", type=int, default=8,
                    help="requests served one at a time after the timed loop, for per-kernel timings and the roofline")
    ap.add_argument("--quick", action="store_true", help="256^3 workload for development runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--open-loop", type=int, default=0,
                    help="instead of the closed loop: this many open-loop requests of mixed mesh sizes")
    ap.add_argument("--mean-gap", type=float, default=0.5, help="open loop: mean inter-arrival time (s)")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0,
                    help="open loop: device memory for plan workspaces (admission by footprint)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB elementwise copy first (counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1506_02729_amd import fastrsd as F
    from paper_1506_02729_amd import synth

    dev = torch.device("cuda:0")
    wl = workload(args.quick)
    if args.calibrate_copy:
        a = torch.ones(COPY_BYTES // 4, device=dev, dtype=torch.float32)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if args.open_loop > 0:
        open_loop(args, F, torch, synth, dev, log)
        return

    # pool of distinct mocks sharing one random catalogue (a covariance run)
    t0 = time.perf_counter()
    pool, ran, observer = synth.lognormal_pool(args.mocks, seed0=2000, n_mesh=wl["n_mesh"], box=wl["box"],
                                               n_gal=wl["n_gal"], n_ran=wl["n_ran"])
    log(f"pool of {len(pool)} mocks ({min(len(g['w']) for g, _ in pool)}-{max(len(g['w']) for g, _ in pool)} "
        f"galaxies, {len(ran['w'])} shared randoms) in {time.perf_counter() - t0:.1f} s")
    max_obj = max(len(g["w"]) for g, _ in pool) + len(ran["w"])
    r_dev = F.device_catalog(ran, dev)
    dev_mocks = [(F.device_catalog(g, dev), r_dev, a) for g, a in pool]

    # ---- served FP32: closed loop over the pool ---------------------------
    cfg = make_config(F, wl, 32, observer, max_obj)
    t0 = time.perf_counter()
    nstream = max(1, args.streams)
    plans = [F.Plan(cfg, device=dev, stream=torch.cuda.Stream(dev) if nstream > 1 else None)
             for _ in range(nstream)]
    plan = plans[0]
    torch.cuda.synchronize()
    log(f"fp32 plan init (tables + N^T) {time.perf_counter() - t0:.2f} s, {nstream} workspace(s) of "
        f"{plan.ws_bytes / 1e9:.1f} GB")
    run_steps(F, torch, plans, dev_mocks, max(args.warmup, nstream), False)
    torch.cuda.synchronize()
    log("warmup done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = run_steps(F, torch, plans, dev_mocks, args.steps, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat_ms = np.array([a.elapsed_time(b) for a, b in lat])
    for pl_ in plans:
        rej = pl_.status()
        assert rej == 0, f"{rej} objects rejected"
    last = (args.steps - 1) % len(dev_mocks)
    last_plan = plans[(args.steps - 1) % nstream]
    p32 = {k: v.cpu().numpy().copy() for k, v in last_plan.pk_buf.items()}
    b32 = {k: v.cpu().numpy().copy() for k, v in last_plan.bk_buf.items()}
    # per-kernel durations with one request in flight (overlapping requests
    # would fold the other request's kernels into each duration)
    F.frsd_profile(True)
    F.frsd_profile_report()
    run_steps(F, torch, plans[:1], dev_mocks, max(1, args.kernel_steps), False)
    torch.cuda.synchronize()
    kern = F.frsd_profile_report()
    F.frsd_profile(False)
    log(f"fp32: {args.steps} requests in {elapsed:.3f} s")
    gold = None if args.quick else oracle_check(
        F, torch, plan, (pool[0][0], ran, pool[0][1], observer, dev_mocks[0][0], r_dev),
        os.path.join(ROOT, "tests", "golden", "h512_golden.json"))

    n_slot = 23
    tbytes = 4
    M = plan.bk_grid
    assert f"M={M}" in wl["name"], (M, wl["name"])
    n_out = plan.ntri * 3
    ks = max(1, args.kernel_steps)
    n_obj_kern = float(np.mean([len(pool[i % len(pool)][0]["w"]) for i in range(ks)])) + len(ran["w"])
    kernels = {k: {"launches": n, "total_ms": round(ms, 3), "avg_ms": round(ms / n, 4)} for k, (n, ms) in kern.items()}
    dom = max(kern, key=lambda k: kern[k][1])
    n_launch, tot_ms = kern[dom]
    avg_s = tot_ms / n_launch / 1e3
    bound, cost = algorithmic_cost(dom, cfg, n_obj_kern, n_slot, M, n_out, tbytes)
    if cost is None:
        bound = None
    if bound == "hbm":
        roof = {"kernel": dom, "bound": "hbm", "achieved": cost / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif bound == "mfma":
        roof = {"kernel": dom, "bound": "mfma", "achieved": cost / avg_s / 1e12, "peak": BF16_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        roof = {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None}
    if roof["achieved"] is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["avg_launch_ms"] = avg_s * 1e3
    roof["traffic"] = measured_traffic(dom)
    del plan, last_plan, plans
    torch.cuda.empty_cache()

    # ---- plain FP64: one mock at a time ------------------------------------
    fp64 = None
    if not args.no_fp64 and args.fp64_steps > 0:
        cfg64 = make_config(F, wl, 64, observer, max_obj)
        plan64 = F.Plan(cfg64, device=dev)
        run_steps(F, torch, plan64, dev_mocks[last:last + 1], 1, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.fp64_steps):
            run_steps(F, torch, plan64, dev_mocks[last:last + 1], 1, False)
            torch.cuda.synchronize()
        e64 = time.perf_counter() - t0
        p64 = {k: v.cpu().numpy().copy() for k, v in plan64.pk_buf.items()}
        b64 = {k: v.cpu().numpy().copy() for k, v in plan64.bk_buf.items()}
        # FP32 and FP64 on the same (last served) mock; P_ell errors relative to
        # max(|P_ell|, (2 ell + 1) x the raw monopole power S00 / (N_b I22))
        cmp = {}
        nb = p64["n_modes"]
        raw0 = p64["s00"] / (nb * p64["scalars"][0])
        for ell in (0, 2, 4):
            ref = p64[f"p{ell}"]
            floor = (2 * ell + 1) * raw0
            cmp[f"P{ell}_max_rel"] = float(np.max(np.abs(p32[f"p{ell}"] - ref) / np.maximum(np.abs(ref), floor)))
        ok = b64["nt"] > 0
        for ell in (0, 2, 4):
            ref = b64[f"t{ell}"][ok]
            cmp[f"T{ell}_max_rel_vs_max"] = float(np.max(np.abs(b32[f"t{ell}"][ok] - ref)) / np.max(np.abs(ref)))
        fp64 = {"value": args.fp64_steps / e64, "unit": "mocks/s", "steps": args.fp64_steps,
                "ms_per_step": 1e3 * e64 / args.fp64_steps, "fp32_vs_fp64": cmp}
        del plan64
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, pool[0][0], ran, pool[0][1], observer, M)

    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "mocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "requests": args.steps, "mocks_in_pool": len(pool),
                   "in_flight": nstream, "kernel_timing": f"{max(1, args.kernel_steps)} requests, one in flight",
                   "precision": "fp32 served (closed loop), fp64 plain (one mock at a time)"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "roofline": roof,
        "kernels": kernels,
        "fp32_vs_oracle": gold,
        "fp64_plain": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
