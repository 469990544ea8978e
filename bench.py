"""Throughput of the FFT multipole estimators on one MI355X.

One step = one request: a synthetic BOSS-like mock through the whole hot path:
ingest + sort, interlaced TSC assignment of the 15 independent moment meshes
(the 22 of the paper less those fixed by the trace relations) and the w^2
mesh, their forward FFTs, multipole combination and binning into
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
mock at a time.  Per-kernel durations come from a separate pass with one
request in flight (HIP events on the launch stream), with each kernel's
algorithmic HBM bytes (and, when the committed counter summary matches the
kernel source, its counter bytes) against the 8 TB/s peak; the triple
product is priced in bf16 MFMA flops against 2.5 PF/s.

The "serving" object is the served covariance run (Poisson arrivals of
uneven mocks on 256^3, 384^3 and 512^3 meshes, admission by HBM footprint,
p50/p99 latency, the plain FP64 path one request at a time beside it),
"small_mesh_batches" the covariance mocks of --batch-study on 64^3 and 128^3
meshes (one at a time, three streams, and request batches of frsd_pk_batch),
and "cpu_baseline" the FP64 oracle on this host's cores.

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
N_SLOT_H512 = 16  # complex slots of an interlaced l_max = 4 plan with the w^2 plane (15 moments + F_0^w)
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
                     "interlaced, 16 moment meshes, P_ell l=0,2,4 in 60 bins of 0.005 to k=0.3, B_ell l=0,2,4 "
                     "over 5416 triangles of 37 bins of 3k_f to k=0.202, M=343",
                n_mesh=512, n_gal=8.0e5, n_ran=40_000_000, pk_dk=0.005, pk_nbins=60,
                bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=37, box=box)


def make_config(F, wl, precision, observer, max_objects):
    return F.Config(n_grid=wl["n_mesh"], box=wl["box"], observer=observer, order=3, interlace=True,
                    compensate=True, ell_max=4, precision=precision, pk_kmin=0.0, pk_dk=wl["pk_dk"],
                    pk_nbins=wl["pk_nbins"], bk_kmin=wl["bk_kmin"], bk_dk=wl["bk_dk"],
                    bk_nbins=wl["bk_nbins"], max_objects=max_objects)


def _squared_edges(kmin, dk, nb, kf):
    """Squared bin edges in k_f units, snapped to integers within 1e-9 relative (the plan's rule)."""
    e = (kmin + dk * np.arange(nb + 1, dtype=np.float64)) / kf
    e2 = e * e
    r = np.rint(e2)
    return np.where(np.abs(e2 - r) <= 1e-9 * np.maximum(r, 1.0), r, e2)


def _below(e2top):
    """Largest integer strictly below sqrt(e2top)."""
    c = int(math.floor(math.sqrt(e2top)))
    while c > 0 and c * c >= e2top:
        c -= 1
    while (c + 1) * (c + 1) < e2top:
        c += 1
    return c


def plan_geometry(cfg, M):
    """Kept frequency range, binning sphere and bispectrum bins of a plan
    (the same rules the library applies when it builds the plan)."""
    kf = 2 * math.pi / cfg.box
    pk_e2 = _squared_edges(cfg.pk_kmin, cfg.pk_dk, cfg.pk_nbins, kf)
    g = {"N": cfg.n_grid, "M": M, "nc_p": _below(pk_e2[-1]), "pk_len": int(math.ceil(pk_e2[-1]))}
    g["nmax"], g["m2max"] = g["nc_p"], g["pk_len"] - 1
    if cfg.bk_nbins:
        bk_e2 = _squared_edges(cfg.bk_kmin, cfg.bk_dk, cfg.bk_nbins, kf)
        g["nc_b"] = _below(bk_e2[-1])
        g["nmax"] = max(g["nmax"], g["nc_b"])
        g["m2max"] = max(g["m2max"], int(math.ceil(bk_e2[-1])) - 1)
        m = np.arange(1, int(math.ceil(bk_e2[-1])))
        b = np.searchsorted(bk_e2, m, side="right") - 1
        g["bk_hi"] = [int(m[b == i].max()) if np.any(b == i) else -1 for i in range(cfg.bk_nbins)]
    return g


def live_masks(positions, N, box, lo=-2, hi=1):
    """Node columns (x, y) within reach of an object (cell columns holding an
    object, dilated by the TSC window cells [lo, hi], periodic) and x slabs
    holding such a column."""
    occ = np.zeros((N, N), dtype=bool)
    h = box / N
    for pos in positions:
        for s0 in range(0, len(pos), 4_000_000):
            c = np.clip(np.floor(pos[s0:s0 + 4_000_000, :2] / h).astype(np.int64), 0, N - 1)
            occ[c[:, 0], c[:, 1]] = True
    col = np.zeros_like(occ)
    for dx in range(lo, hi + 1):
        for dy in range(lo, hi + 1):
            col |= np.roll(np.roll(occ, -dx, axis=0), -dy, axis=1)
    return col, col.any(axis=1)


def _count_disc(nmax, m2max):
    r = np.arange(-nmax, nmax + 1)
    a2 = (r * r)[:, None] + (r * r)[None, :]
    return int(np.sum(a2 <= m2max))


def _count_sphere(nmax, m2max):
    r = np.arange(-nmax, nmax + 1)
    r2 = r * r
    a2 = r2[:, None, None] + r2[None, :, None] + r2[None, None, :]
    return int(np.sum(a2 <= m2max))


def algorithmic_traffic(geom, col, xm, n_obj, n_slot, n_field, tb, n_batch_pairs=8):
    """Algorithmic HBM bytes per launch of the memory-bound kernels: every
    element a pass must read or write counted once (live survey columns and
    slabs only, kept frequencies only), for an FP32 plan (tb = 4).  Shell
    passes: the launch average over the request's batches of n_batch_pairs field pairs."""
    N, M, nmax, m2max = geom["N"], geom["M"], geom["nmax"], geom["m2max"]
    c = 2 * tb
    live_cols = int(col.sum())
    live_rows = col.sum(axis=1)
    nkz = 2 * nmax + 1
    n_disc, n_sph = _count_disc(nmax, m2max), _count_sphere(nmax, m2max)
    out = {}
    out["grid"] = out["grid_twin"] = live_cols * N * tb * n_slot + n_obj * 4 * tb
    out["fft_z"] = n_slot * (live_cols * N * 2 * tb + live_cols * nkz * c)
    out["fft_y"] = n_slot * (int(live_rows[xm].sum()) * nkz * c + int(xm.sum()) * n_disc * c)
    out["fft_x"] = n_slot * (n_disc * int(xm.sum()) * c + n_sph * c)
    out["bin"] = n_slot * n_sph * c
    nc = geom.get("nc_b")
    if nc is not None:
        nb = len(geom["bk_hi"])
        r = np.arange(-nc, nc + 1)
        a2 = (r * r)[:, None] + (r * r)[None, :]
        npair = (n_field + 1) // 2
        z = y = x = 0
        for p in range(npair):
            hp = max(geom["bk_hi"][f % nb] for f in (2 * p, 2 * p + 1) if f < n_field)
            cols = int(np.sum(a2 <= hp))
            nix = int(np.sum(r * r <= hp))
            z += cols * M * c
            y += cols * M * c + nix * M * M * c
            x += nix * M * M * c + min(2, n_field - 2 * p) * M**3 * tb
        nl = (npair + n_batch_pairs - 1) // n_batch_pairs
        out["shell_z"], out["shell_y"], out["shell_x"] = z // nl, y // nl, x // nl
        out["triple"] = n_field * M**3 * tb
    return out


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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(wl, gal, ran, alpha, observer, M):
    """The FP64 oracle on this host's cores: the small 64^3 power-spectrum case
    end to end, and the H512 stages timed on a bounded sample and scaled to
    one mock.  The oracle's FFTs run with scipy workers on all cores (at most
    16), its assignment loop (plain C, OpenMP) on OMP_NUM_THREADS threads;
    the shell sums and triangle sums are single-threaded NumPy."""
    from oracle import assign_c
    from oracle import estimator as est
    from paper_1506_02729_amd import synth
    import scipy.fft as sfft
    assign_c.build()
    nproc = os.cpu_count() or 1
    fft_threads = est._WORKERS
    omp_threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
    N = wl["n_mesh"]
    n_obj = len(gal["w"]) + len(ran["w"])
    t = {}
    # the small power-spectrum case, end to end (64^3 CIC, 2e4 + 1e5 objects)
    g1, r1, a1, o1 = synth.tiny_survey(seed=1000)
    kf1 = 2 * math.pi / 500.0
    prm1 = est.Params(n_grid=64, box=500.0, observer=o1, order=2, interlace=False, compensate=True, ell_max=4,
                      pk_kmin=0.0, pk_dk=2 * kf1, pk_nbins=16, assign=assign_c.assign_mesh)
    t0 = time.perf_counter()
    est.pk_multipoles(g1, r1, a1, prm1)
    t["small_pk_64_end_to_end"] = time.perf_counter() - t0
    # H512 stages
    sample = 4_000_000
    u = ran["pos"][:sample] / (wl["box"] / N)
    w = -alpha * ran["w"][:sample]
    assign_c.assign_mesh(u, w, N, 3)
    t0 = time.perf_counter()
    assign_c.assign_mesh(u, w, N, 3)
    t["assign_1plane_4e6obj"] = time.perf_counter() - t0
    mesh = np.random.default_rng(0).standard_normal((N, N, N))
    t0 = time.perf_counter()
    sfft.rfftn(mesh, workers=fft_threads)
    t["rfftn_512"] = time.perf_counter() - t0
    del mesh
    prm = est.Params(n_grid=N, box=wl["box"], observer=observer, pk_kmin=0.0, pk_dk=wl["pk_dk"],
                     pk_nbins=wl["pk_nbins"])
    fields = {0: np.ones((N, N, N // 2 + 1), complex), 2: np.ones((N, N, N // 2 + 1), complex),
              4: np.ones((N, N, N // 2 + 1), complex)}
    t0 = time.perf_counter()
    est.shell_sums(fields, prm, 0.0, wl["pk_dk"], wl["pk_nbins"])
    t["bin_60"] = time.perf_counter() - t0
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
        pair = f * f
        float(np.sum(f * pair))
    t["triangle_sum"] = (time.perf_counter() - t0) / 3
    del f
    n_tri, n_ell, n_mom, n_fields = 5416, 3, 23, 111
    per_mock = (t["assign_1plane_4e6obj"] * (n_obj / sample) * n_mom * 2 + t["rfftn_512"] * n_mom * 2 + t["bin_60"]
                + t["shell_ifft"] * n_fields + t["triangle_sum"] * n_tri * n_ell)
    return {"value": 1.0 / per_mock, "unit": "mocks/s", "cores": max(fft_threads, omp_threads), "kind": "oracle",
            "seconds_per_mock": per_mock, "nproc": nproc, "cpu_model": _cpu_model(),
            "threads": {"fft": fft_threads, "assign": omp_threads, "bin": 1, "triangle_sum": 1},
            "sample": ("FP64 oracle on this host: H512 stages timed once each and scaled to one mock -- TSC "
                       "assignment of 4e6 randoms for one moment plane (x %.1f for all objects, x 46 planes), one "
                       "512^3 rfftn (x 46), the 60-bin shell sums of 3 multipoles, one %d^3 shell inverse FFT "
                       "(x 111), one %d^3 triangle sum (x 5416 triangles x 3 multipoles); plus the 64^3 CIC "
                       "P_ell case of 2e4 + 1e5 objects end to end" % (n_obj / sample, M, M)),
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


def served_with_random_cache(args, F, torch, wl, dev_mocks, r_dev, observer, max_obj, nstream, ref, log):
    """The closed loop again with the pool's shared random catalogue cached per
    plan (frsd_random_cache once, untimed; then frsd_mesh_assign_cached on
    each mock's galaxies), the covariance-run use of a fixed survey mask.
    Reported beside the headline value, which caches nothing."""
    dev = dev_mocks[0][0]["pos"].device
    cfg = make_config(F, wl, 32, observer, max_obj)
    cfg.random_cache = True
    plans = [F.Plan(cfg, device=dev, stream=torch.cuda.Stream(dev)) for _ in range(nstream)]
    if not args.no_tuning:
        from paper_1506_02729_amd import autotune
        for pl in plans:
            autotune.apply(pl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl in plans:
        pl.random_cache(r_dev)
    torch.cuda.synchronize()
    t_cache = time.perf_counter() - t0

    def loop(steps):
        for i in range(steps):
            g, _, a = dev_mocks[i % len(dev_mocks)]
            pl = plans[i % len(plans)]
            pl.mesh_assign_cached(g, a)
            pl.pk()
            pl.bk()

    loop(max(args.warmup, nstream))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for pl in plans:
        assert pl.status() == 0
    last, p32, b32 = ref
    pl = plans[0]
    g, _, a = dev_mocks[last]
    pl.mesh_assign_cached(g, a)
    pk, bk = pl.pk(), pl.bk()
    torch.cuda.synchronize()
    diff = {}
    for key in ("p0", "p2", "p4"):
        v = pk[key].cpu().numpy()
        diff[key] = float(np.max(np.abs(v - p32[key])) / np.max(np.abs(p32[key])))
    for key in ("t0", "t2", "t4"):
        v = bk[key].cpu().numpy()
        ok = b32["nt"] > 0
        diff[key] = float(np.max(np.abs(v[ok] - b32[key][ok])) / np.max(np.abs(b32[key][ok])))
    log(f"fp32 with the random cache: {args.steps} requests in {elapsed:.3f} s (cache {t_cache:.2f} s)")
    out = {"value": args.steps / elapsed, "unit": "mocks/s", "ms_per_step": 1e3 * elapsed / args.steps,
           "in_flight": nstream, "cache_build_s_all_plans": t_cache, "workspace_gb": plans[0].ws_bytes / 1e9,
           "max_rel_diff_vs_uncached": diff}
    del plans, pl
    return out


def large_mesh(args, F, torch, synth, dev, log):
    """The large-mesh precision sweep: one 1024^3 mesh in the 3500 Mpc/h box,
    a lognormal mock of 4e6 galaxies and 2e8 randoms (seed 5000, P(k) smoothed
    at 3 Mpc/h), interlaced TSC, P_0,2,4 and P_4b in 100 bins of 0.005 to
    k = 0.5, on streamed plans, FP32 and FP64: with two complex slots of
    moment meshes resident (the smallest workspace) and with as many slots as
    the free HBM holds, in as few equal groups as that allows.  Reports each
    run's time and workspace, the FP32 error per bin against FP64, and both
    against the stored FP64 oracle results (P_0, P_2, P_4b) when the catalogue
    digest matches."""
    N, box = 1024, 3500.0
    t0 = time.perf_counter()
    gal, ran, alpha, observer, _ = synth.lognormal_mock(n_mesh=N, box=box, n_gal=4.0e6, n_ran=200_000_000, seed=5000,
                                                        r_smooth=3.0)
    digest = synth.catalog_digest(gal, ran, alpha, observer)
    log(f"large mesh: mock of {len(gal['w'])} + {len(ran['w'])} objects in {time.perf_counter() - t0:.0f} s")
    t0 = time.perf_counter()
    g, r = F.device_catalog(gal, dev), F.device_catalog(ran, dev)
    torch.cuda.synchronize()
    log(f"large mesh: catalogues on the device in {time.perf_counter() - t0:.1f} s")
    n_obj = len(gal["w"]) + len(ran["w"])
    del ran
    res, outs = {}, {}
    n_mom = 15
    for prec in (32, 64):
        cfg = F.Config(n_grid=N, box=box, observer=observer, order=3, interlace=True, compensate=True, ell_max=4,
                       precision=prec, pk_kmin=0.0, pk_dk=0.005, pk_nbins=100, max_objects=n_obj,
                       stream_moments=True)
        torch.cuda.empty_cache()
        free = torch.cuda.mem_get_info(dev)[0] - (8 << 30)  # headroom for torch and the outputs
        fit = max(s for s in range(1, n_mom + 1)
                  if s == 1 or F.workspace_bytes(F.Config(**{**cfg.__dict__, "stream_slots": s})) <= free)
        groups = -(-n_mom // fit)
        for slots in sorted({2, -(-n_mom // groups)}):
            cfg.stream_slots = slots
            t0 = time.perf_counter()
            plan = F.Plan(cfg, device=dev)
            torch.cuda.synchronize()
            log(f"large mesh fp{prec} x{slots}: plan of {plan.ws_bytes / 1e9:.1f} GB initialised in "
                f"{time.perf_counter() - t0:.1f} s")
            for rep in range(2):
                t1 = time.perf_counter()
                plan.mesh_assign(g, r, alpha)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                plan.pk()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1
                log(f"large mesh fp{prec} x{slots} run {rep}: assignment + transforms {t2 - t1:.2f} s, total {dt:.2f} s")
            assert plan.status() == 0
            o = {k: v.cpu().numpy().copy() for k, v in plan.pk_buf.items()}
            if prec in outs:  # the groupings agree to rounding
                for key in ("p0", "p2", "p4", "p4b"):
                    d = np.max(np.abs(o[key] - outs[prec][key])) / np.max(np.abs(outs[prec][key]))
                    assert d < (1e-5 if prec == 32 else 1e-11), (prec, slots, key, d)
            outs[prec] = o
            res[f"fp{prec}_slots{slots}"] = {"seconds": dt, "groups": -(-n_mom // slots),
                                             "workspace_gb": plan.ws_bytes / 1e9}
            del plan
            torch.cuda.empty_cache()
    p32, p64 = outs[32], outs[64]
    nb = p64["n_modes"].astype(float)
    raw0 = p64["s00"] / (nb * p64["scalars"][0])
    cmp = {}
    for ell in (0, 2, 4):
        ref = p64[f"p{ell}"]
        e = np.abs(p32[f"p{ell}"] - ref) / np.maximum(np.abs(ref), (2 * ell + 1) * raw0)
        cmp[f"P{ell}"] = {"max_rel": float(e.max()), "median_rel": float(np.median(e))}
    e = np.abs(p32["p4b"] - p64["p4b"]) / np.maximum(np.abs(p64["p4b"]), 9 * raw0)
    cmp["P4b"] = {"max_rel": float(e.max()), "median_rel": float(np.median(e))}
    res["fp32_vs_fp64_per_bin"] = cmp
    gold_path = os.path.join(ROOT, "tests", "golden", "cfg5_golden.json")
    try:
        with open(gold_path) as fh:
            gold = json.load(fh)
    except OSError:
        gold = None
    if gold and gold["catalog_sha256"] == digest:
        pk, sc = gold["pk"], gold["scalars"]
        gnb = np.asarray(pk["n_modes"], dtype=float)
        vs = {"n_modes_exact": bool(np.array_equal(p64["n_modes"], np.asarray(pk["n_modes"])))}
        floors = {0: np.asarray(pk["S00"]) / (gnb * sc["I22"]), 2: 5 * np.asarray(pk["C20"]) / (gnb * sc["I22"])}
        floor4b = (17.5 * np.asarray(pk["S22"]) + 5 * np.asarray(pk["C20"]) + 3.5 * np.asarray(pk["S00"])) / (gnb * sc["I22"])
        for prec, o in ((32, p32), (64, p64)):
            for ell in (0, 2):
                e = np.abs(o[f"p{ell}"] - np.asarray(pk[f"P{ell}"])) / np.maximum(np.abs(np.asarray(pk[f"P{ell}"])), floors[ell])
                vs[f"fp{prec}_P{ell}_max_rel"] = float(e.max())
            e = np.abs(o["p4b"] - np.asarray(pk["P4b"])) / np.maximum(np.abs(np.asarray(pk["P4b"])), floor4b)
            vs[f"fp{prec}_P4b_max_rel"] = float(e.max())
        res["vs_oracle"] = vs
    else:
        res["vs_oracle"] = None if gold is None else {"skipped": "catalogue digest differs from the stored oracle run"}
    return {"metric": "large-mesh precision sweep: P_0,2,4 at 1024^3, streamed moments, FP32 vs FP64 vs oracle",
            "config": {"workload": "lognormal mock 4e6 galaxies + 2e8 randoms (P(k) smoothed at 3 Mpc/h), 3500 Mpc/h box, "
                                   "N=1024 TSC interlaced, "
                                   "P_ell l=0,2,4 and P_4b in 100 bins of 0.005 to k=0.5, streamed moment meshes"},
            "data": "synthetic", **res}


def p4_study(args, F, torch, synth, dev, log):
    """The two hexadecapole estimators over many mocks (Sec. III.A, the
    comparison of Figs. P4LD and P4PTH, here on synthetic mocks): P_4 from the
    moment meshes (22 in the paper, 15 independent) and the split P_4b from
    those of the quadrupole (7, 6 independent), on the
    same catalogues.  Lognormal mocks of 2e5 galaxies (seeds 6000 + i) over
    one shared random catalogue of 1e7, 256^3 TSC interlaced, 45 bins of
    0.005 to k = 0.225.  Per bin: the bias ratio b_4 = <P_4b>/<P_4> with its
    standard error and the variance ratio sigma_4^2 = Var P_4b / Var P_4."""
    n = args.p4_study
    box = 3500.0
    gal0, ran, alpha0, observer, _ = synth.lognormal_mock(n_mesh=256, box=box, n_gal=2.0e5, n_ran=10_000_000,
                                                          seed=6000)
    r = F.device_catalog(ran, dev)
    n_ran = len(ran["w"])
    cfg = F.Config(n_grid=256, box=box, observer=observer, order=3, interlace=True, compensate=True, ell_max=4,
                   precision=32, pk_kmin=0.0, pk_dk=0.005, pk_nbins=45, max_objects=int(3e5) + n_ran)
    plan = F.Plan(cfg, device=dev)
    p4, p4b, k = [], [], None
    t0 = time.perf_counter()
    for i in range(n):
        g, _, a, _, _ = synth.lognormal_mock(n_mesh=256, box=box, n_gal=2.0e5, n_ran=n_ran, seed=6000 + i,
                                             ran_seed=6500, make_randoms=False) if i else (gal0, None, alpha0, None, None)
        out = plan.run(F.device_catalog(g, dev), r, a, bispectrum=False)
        p4.append(out["p4"])
        p4b.append(out["p4b"])
        k = out["k_eff"]
        if (i + 1) % 16 == 0:
            log(f"p4 study: {i + 1}/{n} mocks in {time.perf_counter() - t0:.0f} s")
    p4, p4b = np.asarray(p4), np.asarray(p4b)
    m4, m4b = p4.mean(0), p4b.mean(0)
    v4, v4b = p4.var(0, ddof=1), p4b.var(0, ddof=1)
    # standard error of the ratio of means (delta method, covariance of the two estimators included)
    c = np.array([np.cov(p4[:, j], p4b[:, j])[0, 1] for j in range(p4.shape[1])])
    b4 = m4b / m4
    b4_err = np.abs(b4) * np.sqrt((v4b / m4b**2 + v4 / m4**2 - 2 * c / (m4 * m4b)) / n)
    sel = k >= 0.02
    return {"metric": "hexadecapole estimators P_4 (all moments) vs split P_4b (quadrupole moments) over synthetic mocks",
            "mocks": n, "config": {"workload": "lognormal mocks 2e5 galaxies (seeds 6000+i) + one shared 1e7-random "
                                               "catalogue, 3500 Mpc/h box, 256^3 TSC interlaced, 45 bins of 0.005"},
            "data": "synthetic", "k": [float(v) for v in k],
            "b4": [float(v) for v in b4], "b4_err": [float(v) for v in b4_err],
            "sigma4_sq": [float(v) for v in v4b / v4],
            "summary_k_ge_0.02": {"b4_mean": float(np.mean(b4[sel])),
                                  "bins_b4_within_2_sigma_of_1": float(np.mean(np.abs(b4[sel] - 1) < 2 * b4_err[sel])),
                                  "sigma4_sq_median": float(np.median((v4b / v4)[sel])),
                                  "sigma4_sq_mean": float(np.mean((v4b / v4)[sel]))}}


def batch_study(args, F, torch, synth, dev, log):
    """Small meshes of a covariance run (many mocks over one survey, Sec.
    III.C): lognormal mocks of 2e5 galaxies (8 distinct, seeds 6000 + i,
    cycled) against one cached catalogue of 1e7 randoms, TSC interlaced,
    P_ell l = 0, 2, 4 in bins of 0.005 to min(0.225, 0.95 k_Nyquist), on
    64^3, 128^3 and 256^3 meshes (FP32).  Mocks resident in HBM, outputs left
    on the device; per mesh size the throughput of --batch-mocks mocks served
    (a) one at a time on one plan and stream (frsd_mesh_assign_cached +
    frsd_pk_multipoles), (b) on 3 plans with a stream each, round robin, and
    (c) in batches of 8 and 16 requests (frsd_pk_batch, one stream: one
    launch per kernel per batch), and (d) in batches of 8 alternating between
    two streams.  Each batched result is compared with the one-at-a-time
    result of the same mock, per multipole."""
    box = 3500.0
    n_ran = 10_000_000
    n_mock = 8
    t0 = time.perf_counter()
    gal0, ran, alpha0, observer, _ = synth.lognormal_mock(n_mesh=256, box=box, n_gal=2.0e5, n_ran=n_ran, seed=6000)
    mocks = [(gal0, alpha0)]
    for i in range(1, n_mock):
        g, _, a, _, _ = synth.lognormal_mock(n_mesh=256, box=box, n_gal=2.0e5, n_ran=n_ran, seed=6000 + i,
                                             ran_seed=6500, make_randoms=False)
        mocks.append((g, a))
    log(f"batch study: {n_mock} mocks in {time.perf_counter() - t0:.0f} s")
    r_dev = F.device_catalog(ran, dev)
    dev_mocks = [(F.device_catalog(g, dev), a) for g, a in mocks]
    K = args.batch_mocks
    results = {}
    for N in (int(v) for v in args.batch_n.split(",")):
        k_ny = math.pi * N / box
        nb = int(min(0.225, 0.95 * k_ny) / 0.005)
        cfg = F.Config(n_grid=N, box=box, observer=observer, order=3, interlace=True, compensate=True, ell_max=4,
                       precision=32, pk_kmin=0.0, pk_dk=0.005, pk_nbins=nb, max_objects=max(int(3e5), n_ran),
                       random_cache=True)
        streams = [torch.cuda.Stream(dev) for _ in range(3)]
        plans = [F.Plan(cfg, device=dev, stream=streams[0]) for _ in range(16)]
        n_more = 0 if args.batch_profile else 1
        side = [F.Plan(cfg, device=dev, stream=streams[k]) for k in (1, 2)][:2 * n_more]
        second = [F.Plan(cfg, device=dev, stream=streams[1]) for _ in range(8 * n_more)]  # batches on a second stream
        for pl in plans + side + second:
            pl.random_cache(r_dev)
        torch.cuda.synchronize()
        if args.batch_profile:
            time.sleep(0.5)  # a gap in a kernel trace between the caches and the batches

        def one_at_a_time(n):
            for i in range(n):
                g, a = dev_mocks[i % n_mock]
                plans[0].mesh_assign_cached(g, a)
                plans[0].pk()

        def round_robin(n):
            rr = [plans[0]] + side
            for i in range(n):
                g, a = dev_mocks[i % n_mock]
                rr[i % 3].mesh_assign_cached(g, a)
                rr[i % 3].pk()

        def batched(n, b):
            for i0 in range(0, n, b):
                idx = [(i0 + j) % n_mock for j in range(b)]
                F.pk_batch(plans[:b], [dev_mocks[i][0] for i in idx], None, [dev_mocks[i][1] for i in idx])

        def batched_two_streams(n):
            for q, i0 in enumerate(range(0, n, 8)):
                idx = [(i0 + j) % n_mock for j in range(8)]
                F.pk_batch(plans[:8] if q % 2 == 0 else second, [dev_mocks[i][0] for i in idx], None,
                           [dev_mocks[i][1] for i in idx])

        def timed(fn, *a):
            fn(*a)  # warm-up pass
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn(*a)
            torch.cuda.synchronize()
            return K / (time.perf_counter() - t)

        if args.batch_profile:  # batches of 16 only (a profiler run)
            results[str(N)] = {"batch16": timed(batched, K, 16)}
            log(f"batch study N={N}: batch16 {results[str(N)]['batch16']:.4g} mocks/s")
            del plans, side, second
            continue
        row = {"pk_nbins": nb, "workspace_gb_per_plan": plans[0].ws_bytes / 1e9,
               "one_at_a_time": timed(one_at_a_time, K), "three_streams": timed(round_robin, K)}
        for b in (8, 16):
            row[f"batch{b}"] = timed(batched, K, b)
        row["batch8_two_streams"] = timed(batched_two_streams, K)
        # per-kernel device time per mock (library HIP events, untimed passes of 16 mocks)
        for name, fn, a in (("one_at_a_time", one_at_a_time, (16,)), ("batch16", batched, (16, 16))):
            F.frsd_profile(True)
            F.frsd_profile_report()
            fn(*a)
            torch.cuda.synchronize()
            rep = F.frsd_profile_report()
            F.frsd_profile(False)
            row[f"kernel_ms_per_mock_{name}"] = {k: round(v[1] / 16, 4) for k, v in sorted(rep.items())}
        # batched results against one-at-a-time results of the same mocks
        ref = []
        for i in range(n_mock):
            g, a = dev_mocks[i]
            ref.append(plans[0].run_cached(g, a, bispectrum=False))
        outs = F.run_batch(plans[:n_mock], [m[0] for m in dev_mocks], None, [m[1] for m in dev_mocks])
        for key in ("p0", "p2", "p4"):
            row[f"{key}_max_diff_batch_vs_one_at_a_time"] = max(
                float(np.max(np.abs(outs[i][key] - ref[i][key])) / np.max(np.abs(ref[i][key]))) for i in range(n_mock))
        for pl in plans + side + second:
            assert pl.status() == 0
        log(f"batch study N={N}: " + ", ".join(f"{k} {v:.4g}" for k, v in row.items() if not isinstance(v, dict)))
        for k, v in row.items():
            if isinstance(v, dict):
                log(f"  {k}: " + ", ".join(f"{n} {t:.3f}" for n, t in v.items()))
        results[str(N)] = row
        del plans, side, second
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    served = None
    if not args.batch_profile and args.batch_requests > 0:
        served = batch_serving(args, F, torch, dev, log, dev_mocks, r_dev, observer, box, n_ran)
    return {"metric": "small-mesh covariance throughput (mocks/s): one at a time vs 3 streams vs batched requests",
            "unit": "mocks/s", "mocks_timed": K,
            "config": {"workload": "lognormal mocks 2e5 galaxies (8 distinct, seeds 6000+i, cycled) against one "
                                   "cached 1e7-random catalogue, 3500 Mpc/h box, TSC interlaced, P_ell l=0,2,4 in bins "
                                   "of 0.005 to min(0.225, 0.95 k_Ny), FP32"},
            "data": "synthetic", "results": results, "served": served}


def batch_serving(args, F, torch, dev, log, dev_mocks, r_dev, observer, box, n_ran):
    """Continuous batching of small meshes (paper_1506_02729_amd/serve.py):
    Poisson arrivals (--batch-rates per second: one rate for 64^3, one for
    128^3) of --batch-requests covariance mocks (the batch study's, cycled),
    served two ways by a BatchServer holding the random catalogue's spectra in
    every plan: per request (three groups of one plan, a stream each: a
    queued request takes the first free plan) and batched (two groups of 8
    plans, a stream each: a free group takes every queued request, up to 8,
    as one frsd_pk_batch, so requests that arrive while a batch runs form
    the next one).  Outputs go to page-locked host arrays and are copied out
    per request; latency runs from arrival to the poll that completes it."""
    from paper_1506_02729_amd.serve import BatchServer
    out = {}
    R = args.batch_requests
    for N, rate in zip((64, 128), (float(v) for v in args.batch_rates.split(","))):
        nb = int(min(0.225, 0.95 * math.pi * N / box) / 0.005)
        cfg = F.Config(n_grid=N, box=box, observer=observer, order=3, interlace=True, compensate=True, ell_max=4,
                       precision=32, pk_kmin=0.0, pk_dk=0.005, pk_nbins=nb, max_objects=max(int(3e5), n_ran),
                       random_cache=True)
        rng = np.random.Generator(np.random.PCG64(7000 + N))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, R))
        row = {}
        for mode, groups, size in (("per_request", 3, 1), ("batched", 2, 8)):
            server = BatchServer(cfg, groups=groups, group_size=size, device=dev, randoms=r_dev)
            torch.cuda.synchronize()
            lat = np.zeros(R)
            nxt = finished = 0
            t0 = time.perf_counter()
            while finished < R:
                now = time.perf_counter() - t0
                while nxt < R and arrivals[nxt] <= now:
                    g, a = dev_mocks[nxt % len(dev_mocks)]
                    server.submit(g, a).t_submit = t0 + arrivals[nxt]  # latency from the arrival
                    nxt += 1
                for req in server.poll():
                    lat[req.rid] = 1e3 * (req.t_done - req.t_submit)
                    finished += 1
            t_end = time.perf_counter() - t0
            row[mode] = {"mocks_per_s": R / (t_end - arrivals[0]), "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "mean_batch": float(np.mean(server.batch_sizes)),
                         "launch_groups": groups}
            log(f"batch serving N={N} {mode}: " + ", ".join(f"{k} {v:.4g}" for k, v in row[mode].items()))
            assert server.rejected() == 0
            del server
            torch.cuda.empty_cache()
        out[str(N)] = {"pk_nbins": nb, "arrival_rate_per_s": rate, **row}
    return {"requests": R, "results": out}


SERVE_SIZES = (256, 384, 512)


def serving(args, F, torch, synth, dev, log):
    """The served covariance workload: Poisson arrivals (exponential gaps of
    mean --mean-gap s) of lognormal mocks of uneven size -- N_g uniform in
    [3e5, 1.5e6], N_r = 50 N_g, taken as prefixes of shuffled pool catalogues
    (two galaxy mocks of 1.5e6 and 7.5e7 randoms over the same survey),
    with nbar and the FKP weight w = 1/(1 + nbar 1e4) rescaled to each
    request's N_g -- on meshes of 256^3, 384^3 or 512^3 (uniform), P_ell
    l = 0, 2, 4 to min(0.3, k_Nyquist) in bins of 0.005 and B_0 to k = 0.1
    (18 bins of 3 k_f).  The loop admits requests by HBM footprint: a queued
    request takes a free plan (workspace + stream) of its size, or a new one
    while the workspaces (exact sizes from the plan) stay within
    --hbm-budget-gb, or waits; requests in flight overlap on the device.
    Latency runs from arrival to the P_ell and B_0 arrays on the host.
    Compared with: the same requests one at a time on plain FP64 plans (a
    sample per size), and each size's first request recomputed alone (FP32)
    against its in-flight result."""
    from collections import deque
    box = 3500.0
    kf = 2 * math.pi / box
    n_gal_pool, n_ran_pool = 1.5e6, 75_000_000
    t0 = time.perf_counter()
    pool, ran, observer = synth.lognormal_pool(2, seed0=4100, n_mesh=512, box=box, n_gal=n_gal_pool,
                                               n_ran=n_ran_pool)
    vol = synth.survey_volume(1150.0, 1750.0, 60.0)

    def shuffled(c, seed):
        perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(c["w"]))
        return {k: v[perm] for k, v in c.items()}

    gals = [torch.as_tensor(shuffled(g, 4200 + i)["pos"]).to(dev) for i, (g, _) in enumerate(pool)]
    rand = torch.as_tensor(shuffled(ran, 4300)["pos"]).to(dev)
    ng_max = min(int(g.shape[0]) for g in gals)
    nr_all = int(rand.shape[0])
    log(f"serving: pool of {len(gals)} mocks ({ng_max}+ galaxies), {nr_all} randoms in {time.perf_counter() - t0:.1f} s")
    plans, nbins, cfgs, ws_bytes = {}, {}, {}, {}
    budget = args.hbm_budget_gb * 1e9
    for N in SERVE_SIZES:
        kny = math.pi * N / box
        nbins[N] = min(60, int(math.floor(kny / 0.005 - 1e-9)))
        cfgs[N] = {p: F.Config(n_grid=N, box=box, observer=observer, order=3, interlace=True, compensate=True,
                               ell_max=4, precision=p, pk_kmin=0.0, pk_dk=0.005, pk_nbins=nbins[N],
                               bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=18, bk_ell_max=0,
                               max_objects=ng_max + nr_all) for p in (32, 64)}
        h = F.frsd_plan_create(cfgs[N][32].to_c())
        ws_bytes[N] = F.frsd_plan_workspace_bytes(h)
        F.frsd_plan_destroy(h)
        plans[N] = [F.Plan(cfgs[N][32], device=dev, stream=torch.cuda.Stream(dev))]
    used = sum(ws_bytes[N] for N in SERVE_SIZES)
    if used > budget:
        raise SystemExit(f"--hbm-budget-gb {args.hbm_budget_gb} is below one workspace per size ({used / 1e9:.1f} GB)")
    rng = np.random.Generator(np.random.PCG64(4000))
    n = args.serve_requests
    arrive = np.cumsum(rng.exponential(args.mean_gap, n))
    n_of = rng.choice(np.array(SERVE_SIZES), n)
    ng_of = rng.integers(300_000, ng_max + 1, n)
    mock_of = rng.integers(0, len(gals), n)

    def catalogue(k, dtype=torch.float64):
        """Device catalogue of request k: prefixes of the pool positions, nbar and
        w rescaled to its galaxy count (constant over the survey)."""
        ng = int(ng_of[k])
        nr = min(50 * ng, nr_all)
        nbar = ng / vol
        w = 1.0 / (1.0 + nbar * 1.0e4)
        def cat(pos, m):
            return {"pos": pos[:m].to(dtype), "w": torch.full((m,), w, dtype=dtype, device=dev),
                    "nbar": torch.full((m,), nbar, dtype=dtype, device=dev)}
        return cat(gals[mock_of[k]], ng), cat(rand, nr), ng / nr

    def submit(pl, k):
        g, r, a = catalogue(k)
        pl.mesh_assign(g, r, a)
        pl.pk()
        pl.bk()

    def host_result(pl):
        out = {key: pl.pk_buf[key].cpu().numpy().copy() for key in ("n_modes", "p0", "p2", "p4", "s00")}
        out.update({"bk_" + key: pl.bk_buf[key].cpu().numpy().copy() for key in ("nt", "t0", "b0")})
        return out

    for N in SERVE_SIZES:  # one untimed request per plan: code objects loaded, tables resident
        submit(plans[N][0], 0)
    torch.cuda.synchronize()
    free = {id(pl): True for N in SERVE_SIZES for pl in plans[N]}
    queue, inflight, lat, sizes_done, results = deque(), [], [], [], {}
    keep = {int(np.nonzero(n_of == N)[0][0]) for N in SERVE_SIZES if np.any(n_of == N)}
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
                res = host_result(pl)
                lat.append(time.perf_counter() - t0 - arrive[k])
                sizes_done.append(int(n_of[k]))
                if k in keep:
                    results[k] = res
                inflight.remove(rec)
                free[id(pl)] = True
        for k in list(queue):
            N = int(n_of[k])
            pl = next((p for p in plans[N] if free[id(p)]), None)
            if pl is None and used + ws_bytes[N] <= budget:
                pl = F.Plan(cfgs[N][32], device=dev, stream=torch.cuda.Stream(dev))
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
    for N in SERVE_SIZES:
        for pl in plans[N]:
            assert pl.status() == 0
    n_plans = {str(N): len(plans[N]) for N in SERVE_SIZES}
    del plans
    torch.cuda.empty_cache()

    def max_rel(a, b, keys):
        return float(max(np.max(np.abs(a[k] - b[k])) / max(np.max(np.abs(b[k])), 1e-300) for k in keys))

    # each size's first request alone (FP32), against its in-flight result
    alone = {}
    for k in sorted(keep):
        pl = F.Plan(cfgs[int(n_of[k])][32], device=dev)
        submit(pl, k)
        torch.cuda.synchronize()
        ref = host_result(pl)
        assert np.array_equal(ref["n_modes"], results[k]["n_modes"]) and np.array_equal(ref["bk_nt"], results[k]["bk_nt"])
        alone[str(int(n_of[k]))] = max_rel(results[k], ref, ("p0", "p2", "p4", "bk_t0"))
        del pl
    # plain FP64, one request at a time: a sample of two requests per size
    fp64_ms, fp64_err = [], {}
    for N in SERVE_SIZES:
        idx = np.nonzero(n_of == N)[0][:2]
        if len(idx) == 0:
            continue
        pl64 = F.Plan(cfgs[N][64], device=dev)
        submit(pl64, int(idx[0]))          # untimed: code objects loaded
        torch.cuda.synchronize()
        for k in idx:
            t1 = time.perf_counter()
            submit(pl64, int(k))
            res64 = host_result(pl64)
            fp64_ms.append(1e3 * (time.perf_counter() - t1))
            if int(k) in results:
                fp64_err[str(N)] = max_rel(results[int(k)], res64, ("p0", "p2", "p4", "bk_t0"))
        del pl64
        torch.cuda.empty_cache()
    lat_ms = 1e3 * np.asarray(lat)
    sz = np.asarray(sizes_done)
    per_size = {str(N): {"requests": int((sz == N).sum()), "p50_ms": float(np.percentile(lat_ms[sz == N], 50)),
                         "p99_ms": float(np.percentile(lat_ms[sz == N], 99))} for N in SERVE_SIZES if (sz == N).any()}
    return {"workload": "served covariance run: lognormal mocks, N_g uniform in [3e5, 1.5e6], N_r = 50 N_g, nbar and "
                        "w rescaled per request, N uniform in {256, 384, 512}, Poisson arrivals, P_ell l=0,2,4 to "
                        "min(0.3, k_Ny), B_0 on 18 bins of 3 k_f (k <= 0.1)",
            "requests": n, "mean_gap_s": args.mean_gap, "mocks_per_s": n / elapsed,
            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
            "per_size": per_size, "hbm_budget_gb": args.hbm_budget_gb, "plans_per_size": n_plans,
            "workspace_gb": used / 1e9, "pk_bins": {str(N): nbins[N] for N in SERVE_SIZES},
            "alone_vs_in_flight_max_rel": alone,
            "fp64_one_at_a_time": {"requests": len(fp64_ms),
                                   "mocks_per_s": 1e3 / float(np.mean(fp64_ms)) if fp64_ms else None,
                                   "p50_ms": float(np.percentile(fp64_ms, 50)) if fp64_ms else None,
                                   "p99_ms": float(np.percentile(fp64_ms, 99)) if fp64_ms else None,
                                   "fp32_vs_fp64_max_rel": fp64_err},
            "dtype": "f32"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64, help="requests served in the timed closed loop")
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--mocks", type=int, default=8, help="distinct mocks in the pool, cycled")
    ap.add_argument("--streams", type=int, default=3,
                    help="requests in flight: one plan (workspace) and HIP stream each, default priority")
    ap.add_argument("--kernel-steps", type=int, default=8,
                    help="requests served one at a time after the timed loop, for per-kernel timings and the roofline")
    ap.add_argument("--quick", action="store_true", help="256^3 workload for development runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-random-cache", action="store_true", help="skip the closed loop with the random cache")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the served plan's launch parameters first and store them in the tuning cache")
    ap.add_argument("--no-tuning", action="store_true", help="library default launch parameters (ignore the cache)")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the served covariance run (Poisson arrivals, mixed mesh sizes); 0: skip it")
    ap.add_argument("--serve-only", action="store_true", help="run only the served covariance run")
    ap.add_argument("--p4-study", type=int, default=0,
                    help="run only the P_4 vs P_4b bias and variance study over this many synthetic mocks")
    ap.add_argument("--batch-study", action="store_true",
                    help="run only the small-mesh study: one at a time vs 3 streams vs batched requests")
    ap.add_argument("--batch-mocks", type=int, default=64, help="batch study: mocks per timed pass")
    ap.add_argument("--batch-n", default="64,128,256", help="batch study: mesh sides")
    ap.add_argument("--no-batch-study", action="store_true", help="skip the small-mesh batch study of the default run")
    ap.add_argument("--batch-rates", default="2000,2600",
                    help="batch study: Poisson arrival rates of the served run at 64^3 and 128^3 (1/s)")
    ap.add_argument("--batch-requests", type=int, default=1024, help="batch study: requests of the served run (0: skip)")
    ap.add_argument("--batch-profile", action="store_true", help="batch study: batches of 16 only")
    ap.add_argument("--large-mesh", action="store_true",
                    help="run only the 1024^3 streamed precision sweep (FP32 vs FP64 vs the stored oracle)")
    ap.add_argument("--mean-gap", type=float, default=0.5, help="served run: mean inter-arrival time (s)")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0,
                    help="served run: device memory for plan workspaces (admission by footprint)")
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
    if args.serve_only:
        print(json.dumps(serving(args, F, torch, synth, dev, log)), flush=True)
        return
    if args.large_mesh:
        print(json.dumps(large_mesh(args, F, torch, synth, dev, log)), flush=True)
        return
    if args.batch_study:
        print(json.dumps(batch_study(args, F, torch, synth, dev, log)), flush=True)
        return
    if args.p4_study > 0:
        print(json.dumps(p4_study(args, F, torch, synth, dev, log)), flush=True)
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
    from paper_1506_02729_amd import autotune
    def one(pl, it=iter(range(1 << 30))):  # one request on pl (autotuner runs)
        g, r, a = dev_mocks[next(it) % len(dev_mocks)]
        pl.mesh_assign(g, r, a)
        pl.pk()
        pl.bk()
    if args.autotune:
        autotune.tune(plan, one, torch.cuda.synchronize, path=autotune.DEFAULT_CACHE, log=log)
    tuning = None if args.no_tuning else [autotune.apply(pl) for pl in plans][0]
    log(f"tuning: {tuning if tuning else 'library defaults'}")
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

    M = plan.bk_grid
    assert f"M={M}" in wl["name"], (M, wl["name"])
    n_out = plan.ntri * 3
    ks = max(1, args.kernel_steps)
    n_obj_kern = float(np.mean([len(pool[i % len(pool)][0]["w"]) for i in range(ks)])) + len(ran["w"])
    geom = plan_geometry(cfg, M)
    col, xm = live_masks([pool[0][0]["pos"], ran["pos"]], cfg.n_grid, cfg.box)
    alg = algorithmic_traffic(geom, col, xm, n_obj_kern, N_SLOT_H512, 3 * cfg.bk_nbins, 4,
                              n_batch_pairs=F.frsd_plan_get_tuning(plan.handle)["pair_batch"])
    mfma_flops = 6.0 * n_out * M**3      # three bf16 split products of 2 flops per listed output and cell
    kernels = {}
    for k, (n, ms) in kern.items():
        avg = ms / n / 1e3
        e = {"launches": n, "total_ms": round(ms, 3), "avg_ms": round(ms / n, 4)}
        if k in alg:
            e["alg_bytes"] = int(alg[k])
            e["alg_GBps"] = round(alg[k] / avg / 1e9, 1)
            e["alg_hbm_frac"] = round(alg[k] / avg / 1e9 / HBM_PEAK_GBS, 4)
        ct = measured_traffic(k)
        if ct:
            e["counter_bytes"] = int(ct)
            e["counter_hbm_frac"] = round(ct / avg / 1e9 / HBM_PEAK_GBS, 4)
        if k == "triple":
            e["mfma_TFLOPs"] = round(mfma_flops / avg / 1e12, 1)
            e["mfma_frac"] = round(mfma_flops / avg / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4)
            e["fp32_equiv_frac"] = round(2.0 * n_out * M**3 / avg / 1e12 / FP32_VEC_PEAK_TFLOPS, 4)
        kernels[k] = e
    dom = max(kern, key=lambda k: kern[k][1])
    n_launch, tot_ms = kern[dom]
    avg_s = tot_ms / n_launch / 1e3
    if dom == "triple":
        roof = {"kernel": dom, "bound": "mfma", "achieved": mfma_flops / avg_s / 1e12, "peak": BF16_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "flops_per_launch": mfma_flops,
                "flops_rule": "6 x listed outputs (5416 triangles x 3 multipoles) x M^3: three bf16 hi/lo products "
                              "of 2 flops per output and cell",
                "fp32_equiv": {"achieved": 2.0 * n_out * M**3 / avg_s / 1e12, "peak": FP32_VEC_PEAK_TFLOPS,
                               "unit": "TFLOP/s"}}
    elif dom in alg:
        roof = {"kernel": dom, "bound": "hbm", "achieved": alg[dom] / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "bytes_per_launch": alg[dom]}
    else:
        roof = {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None}
    if roof["achieved"] is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["avg_launch_ms"] = avg_s * 1e3
    roof["traffic"] = measured_traffic(dom)
    del plan, last_plan, plans
    torch.cuda.empty_cache()

    # ---- served FP32 with the random catalogue cached ---------------------
    cached = None
    if not args.no_random_cache:
        cached = served_with_random_cache(args, F, torch, wl, dev_mocks, r_dev, observer, max_obj, nstream,
                                          (last, p32, b32), log)
        torch.cuda.empty_cache()

    # ---- plain FP64: one mock at a time ------------------------------------
    fp64 = None
    if not args.no_fp64 and args.fp64_steps > 0:
        cfg64 = make_config(F, wl, 64, observer, max_obj)
        plan64 = F.Plan(cfg64, device=dev)
        if args.autotune:
            autotune.tune(plan64, one, torch.cuda.synchronize, path=autotune.DEFAULT_CACHE, log=log)
        tuning64 = None if args.no_tuning else autotune.apply(plan64)
        log(f"fp64 tuning: {tuning64 if tuning64 else 'library defaults'}")
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
        fp64 = {"value": args.fp64_steps / e64, "unit": "mocks/s", "steps": args.fp64_steps, "tuning": tuning64,
                "ms_per_step": 1e3 * e64 / args.fp64_steps, "fp32_vs_fp64": cmp}
        del plan64
        torch.cuda.empty_cache()

    serve = None
    if args.serve_requests > 0:
        serve = serving(args, F, torch, synth, dev, log)
        torch.cuda.empty_cache()

    batches = None
    if not args.no_batch_study:
        # request batches on small meshes (the study of --batch-study at 64^3 and 128^3)
        bargs = argparse.Namespace(**{**vars(args), "batch_n": "64,128", "batch_profile": False})
        batches = batch_study(bargs, F, torch, synth, dev, log)
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
                   "tuning": tuning,
                   "precision": "fp32 served (closed loop), fp64 plain (one mock at a time)"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "note": "closed loop, enqueue to stream completion with --streams requests in flight; "
                               "arrival-to-result latency of the served covariance run is in serving"},
        "roofline": roof,
        "kernels": kernels,
        "fp32_vs_oracle": gold,
        "fp64_plain": fp64,
        "served_with_random_cache": cached,
        "serving": serve,
        "small_mesh_batches": batches,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
