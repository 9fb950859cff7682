"""Benchmark: rays/s deflected at N_* = 1e6 by the mixed-precision FMM, next
to the FP64 direct sum on the same GPU, at a stated relative error.

Workload (one "step"): 1e6 stars with power-law masses uniform in a disk of
convergence 0.4 (kappa_s = 0.2, gamma = 0.35), an 8192 x 8192 cell-centred ray
grid over the square inscribed in the disk; one lens_deflect call with no
plan, so each step runs the whole path: star quadtree build, P2M, M2M, the
downward pass and the fused evaluation, writing y [8192^2, 2] FP64.  Stars
are resident in HBM before the timed region; grid rays need no input bytes.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ...]

(K, W default per workload: 50 and 20 for the deflection benchmark.)

--workload map runs the high-magnification map instead: 5e6 equal-mass
stars (kappa_* = 0.1, kappa_s = 0.75, gamma = 0.05, mu = 50), a 16384^2 ray
grid over [-120,120] x [-60,60] shot into a 2000^2 int32 map over [-10,10]^2
(one lens_map call per step, mixed precision with p, leaf level and FP32 M2L
levels from the autotuner for a 1e-4 expected bin-reassignment rate).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s deflected at N_*=1e6 (mixed FMM vs FP64 direct) at stated rel. error"
PEAK_FP32_VECTOR = 157.3e12      # MI355X published FP32 vector peak, FLOP/s
PEAK_HBM = 8.0e12                # bytes/s
PAIR_FLOPS = 12                  # per near pair: 2 sub, |d|^2 (3), rcp (1), m*rcp (1), 2 FMA (4), + cvt free
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "eval_deflect_1e6_traffic.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def near_pairs(info, f, g):
    """Near-field pairs of one evaluation: sum over rays of the stars in the
    3x3 leaf neighbourhood of the ray's leaf box (counting only)."""
    import numpy as np
    L = info["leaf_level"]
    nb = 1 << L
    s = math.ldexp(info["root_side"], -L)

    def box(v, origin):
        t = (v - origin) / s
        return np.floor(np.clip(t, 0, nb - 1)).astype(np.int64)

    bx = box(f.xy[:, 0], info["root_x0"])
    by = box(f.xy[:, 1], info["root_y0"])
    cnt = np.bincount(by * nb + bx, minlength=nb * nb).reshape(nb, nb).astype(np.float64)
    pad = np.pad(cnt, 1)
    n3 = sum(pad[1 + dy:1 + dy + nb, 1 + dx:1 + dx + nb] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    rx = g.x0 + (np.arange(g.nx) + 0.5) * g.dx
    ry = g.y0 + (np.arange(g.ny) + 0.5) * g.dy
    cx = np.bincount(box(rx, info["root_x0"]), minlength=nb).astype(np.float64)
    cy = np.bincount(box(ry, info["root_y0"]), minlength=nb).astype(np.float64)
    return float(cy @ n3 @ cx)


PEAK_MFMA_FP32 = 157.3e12      # MI355X dense FP32 matrix, FLOP/s
PEAK_MFMA_FP64 = 78.6e12       # dense FP64 matrix


def stage_rooflines(info, f, g, p, stage_ms, fp32_levels=2):
    """Algorithmic work of the non-evaluation stages of one call against the
    roofline that bounds each (per call, from the stage profiler's times):
      * downward: M2L, 27 source boxes x p^2 complex MACs (8 real FLOPs) per
        target box of every level (the boxes that cover the ray grid), FP32
        MFMA on the finest fp32_levels levels, FP64 MFMA above; the peak is
        the two peaks weighted by the levels' FLOPs (the L2L the stage also
        runs is not counted);
      * upward: P2M, p complex MACs per star at each level formed from the
        stars, is small; the stage moves the sorted stars (24 B each) and
        writes the multipoles (16 p B per box): HBM;
      * tree: keys and values (8 B) read and written by each radix pass
        (3 passes for keys of 2L <= 24 bits), the stars gathered (24 B read,
        24 B written) and the leaf starts written (4 B per leaf box): HBM."""
    import math as _m
    L = info["leaf_level"]
    out = {}
    x0, y0, side = info["root_x0"], info["root_y0"], info["root_side"]
    gx0, gx1 = g.x0 + 0.5 * g.dx, g.x0 + (g.nx - 0.5) * g.dx
    gy0, gy1 = g.y0 + 0.5 * g.dy, g.y0 + (g.ny - 0.5) * g.dy
    f32 = f64 = 0.0
    boxes_total = 0
    for lv in range(2, L + 1):
        n = 1 << lv
        s = _m.ldexp(side, -lv)
        nx = min(n - 1, int((gx1 - x0) // s)) - max(0, int((gx0 - x0) // s)) + 1
        ny = min(n - 1, int((gy1 - y0) // s)) - max(0, int((gy0 - y0) // s)) + 1
        boxes = nx * ny
        boxes_total += n * n
        flops = boxes * 27 * 8.0 * p * p
        if lv > L - fp32_levels:
            f32 += flops
        else:
            f64 += flops
    t_dn = stage_ms.get("downward", float("nan")) * 1e-3
    peak_dn = (f32 + f64) / (f32 / PEAK_MFMA_FP32 + f64 / PEAK_MFMA_FP64)
    out["downward_m2l"] = {"bound": "mfma", "flops": f32 + f64, "achieved_tflops": (f32 + f64) / t_dn / 1e12,
                           "peak_tflops": peak_dn / 1e12, "frac": (f32 + f64) / t_dn / peak_dn}
    n_st = f.n
    up_bytes = n_st * 24.0 + boxes_total * 16.0 * p
    t_up = stage_ms.get("upward", float("nan")) * 1e-3
    out["upward"] = {"bound": "hbm", "bytes": up_bytes, "achieved_gbs": up_bytes / t_up / 1e9,
                     "peak_gbs": PEAK_HBM / 1e9, "frac": up_bytes / t_up / PEAK_HBM}
    passes = max(1, _m.ceil(2 * L / 8))
    tree_bytes = n_st * (16.0 * passes + 48.0) + 4.0 * (1 << (2 * L))
    t_tr = stage_ms.get("tree", float("nan")) * 1e-3
    out["tree"] = {"bound": "hbm", "bytes": tree_bytes, "achieved_gbs": tree_bytes / t_tr / 1e9,
                   "peak_gbs": PEAK_HBM / 1e9, "frac": tree_bytes / t_tr / PEAK_HBM}
    return out


def host_threads():
    """Threads for the CPU oracle: the cores this process may run on, capped
    by OMP_NUM_THREADS when set (a shared machine may grant each GPU a share of its
    host cores through it)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return min(n, omp) if omp > 0 else n


def host_desc():
    n_aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return (f"nproc {os.cpu_count()}, affinity {n_aff}, "
            f"OMP_NUM_THREADS {os.environ.get('OMP_NUM_THREADS', 'unset')}")


def ray_error_stats(y, y_ref, alpha_ref):
    """Relative l2 error of alpha, and the per-ray relative error
    |dalpha_k| / max(|alpha_k|, 1e-3 rms alpha): maximum and 99.9th percentile."""
    import numpy as np
    d = np.hypot(*(y - y_ref).T)
    a = np.hypot(*alpha_ref.T)
    r = d / np.maximum(a, 1e-3 * np.sqrt(np.mean(a * a)))
    return {"rel_l2": float(np.linalg.norm(y - y_ref) / np.linalg.norm(alpha_ref)),
            "ray_max": float(r.max()), "ray_p99.9": float(np.percentile(r, 99.9)),
            "max_abs_dy": float(np.abs(y - y_ref).max())}


def eval_source_hash():
    """Hash of what the evaluation kernel is compiled from: eval.hip, the
    device helpers and the EvalArgs declaration (the rest of the internal
    header does not change the kernel)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2211_00354_amd", "csrc")
    for fn in ("eval.hip", "device_common.h"):
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(fh.read())
    txt = open(os.path.join(csrc, "lens_internal.h")).read()
    i = txt.index("struct EvalArgs")
    h.update(txt[i:txt.index("};", i)].encode())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # defaults per workload (None): a deflection step takes ~1.2 ms, so 50
    # timed steps after 20 untimed ones (the GPU's clocks settle over the
    # first ~10) run in well under a second; an arc map takes ~4 s
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--leaf", type=int, default=0, help="leaf level (0 = the library's choice)")
    ap.add_argument("--tune", action="store_true", help="time leaf levels 9-11 and use the fastest")
    ap.add_argument("--p", type=int, default=12)
    ap.add_argument("--p-fp64", type=int, default=0,
                    help="order of the FP64 FMM run at the 1e-10 target (reported in extra); "
                         "0: the autotuner's order and leaf level for a 1e-10 per-ray error")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-direct", action="store_true", help="skip the FP64 direct comparator")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup+steps of the mixed FMM only (for rocprofv3)")
    ap.add_argument("--workload", choices=("deflect", "map", "ipm", "batch", "halo", "arc"),
                    default="deflect",
                    help="deflect: 1e6 stars, 8192^2 rays (the headline metric); "
                         "map: 5e6 stars, 16384^2 rays shot into a 2000^2 map (IRS); "
                         "ipm: the same field and grid, inverse polygon mapping; "
                         "batch: 64 fields of 1e4-2e5 stars, 2048^2 rays each, one graph; "
                         "halo: 1.575e7 halo particles, 4000^2 rays (deflect, tol 1e-5); "
                         "arc: 1.8e6 deflectors, 1.5e11 rays of a 15000x10 region, IPM map")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="with --profile-only: also run one device-to-device copy of this many "
                         "MiB, the reference for scaling FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args()
    dsteps, dwarm = {"deflect": (50, 20), "map": (20, 5), "ipm": (10, 3), "batch": (20, 5),
                     "halo": (20, 5), "arc": (1, 0)}[args.workload]
    if args.steps is None:
        args.steps = dsteps
    if args.warmup is None:
        args.warmup = dwarm
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the ray grid would shard into bands of rows, one per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2211_00354_amd as lf
    from paper_2211_00354_amd import _lib
    import workloads as wl

    torch.cuda.set_device(0)
    if args.workload in ("map", "ipm"):
        return bench_map(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload in ("halo", "arc"):
        return bench_application(args)
    log("generating workload")
    f, g = wl.powerlaw_disk()
    xy = torch.from_numpy(f.xy).cuda()
    m = torch.from_numpy(f.m).cuda()
    grid = lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
    y = torch.empty((g.n, 2), dtype=torch.float64, device="cuda")
    n_rays = g.n

    def run(prec="mixed", p=args.p, leaf=0, method="fmm"):
        lf.deflect(xy, m, grid=grid, kappa_s=f.kappa_s, gamma=f.gamma, precision=prec, p=p,
                   leaf_level=leaf, method=method, out=y)

    def timed(fn, reps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # leaf level: the library's cost model (leaf_level 0), or --leaf, or the
    # fastest of a few with --tune (outside the timed region)
    leaf = args.leaf
    if args.tune:
        best = None
        for L in (9, 10, 11):
            run(leaf=L)
            t = timed(lambda: run(leaf=L), 2)
            log(f"leaf level {L}: {t:.3f} ms")
            if best is None or t < best[0]:
                best = (t, L)
        leaf = best[1]
    log(f"leaf level {leaf or 'auto'}, p={args.p}")

    for _ in range(args.warmup):
        run(leaf=leaf)
    torch.cuda.synchronize()
    # timed region: repeated identical calls replay the library's captured
    # graph of the call (built during the warmup)
    t0 = time.perf_counter()
    ms = timed(lambda: run(leaf=leaf), args.steps)
    wall = time.perf_counter() - t0
    # per-call times of the same steps (an event pair around each call):
    # their median, outside the timed region above
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record()
        run(leaf=leaf)
        e1.record()
    torch.cuda.synchronize()
    per_call = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    ms_median = per_call[len(per_call) // 2]
    # the same steps once more with the stage profiler on (HIP events around
    # every stage on its stream; the profiler runs the calls eagerly), for the
    # evaluation kernel's duration
    _lib.profile_enable(True)
    ms_prof = timed(lambda: run(leaf=leaf), args.steps)
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    log(f"mixed FMM: {ms:.3f} ms/step ({wall:.2f} s wall for {args.steps} steps); "
        f"profiled eager steps {ms_prof:.3f} ms; stages {prof}")
    if args.profile_only:
        if args.calib_copy_mib:
            # known-size reference kernels for the FETCH_SIZE / WRITE_SIZE
            # counters: two fills write 2 x N bytes; the second evicts the
            # first from the 256 MB Infinity Cache; the sum then reads N bytes
            n = args.calib_copy_mib * (1 << 20) // 4
            a = torch.ones(n, dtype=torch.float32, device="cuda")
            b = torch.ones(n, dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            a.sum().item()
            del a, b
            log(f"calibration: 2 fills of {args.calib_copy_mib} MiB, one sum over "
                f"{args.calib_copy_mib} MiB")
        return

    value = n_rays / (ms * 1e-3)
    idx = g.strided(32, 16)
    y_mixed_sample = y[torch.from_numpy(idx).cuda()].cpu().numpy()

    # algorithmic work of the dominant kernel (fused evaluation)
    # the same tree the timed calls build (grid-aligned, same leaf level)
    plan = lf.Plan(xy, m, grid=grid, precision="mixed", p=args.p, leaf_level=leaf)
    info = plan.info()
    plan.close()
    leaf = info["leaf_level"]
    pairs = near_pairs(info, f, g)
    flops = PAIR_FLOPS * pairs + (8 * args.p + 2) * n_rays
    ev_ms, ev_n = prof.get("eval", (float("nan"), 1))
    ev_avg = ev_ms / max(ev_n, 1)
    achieved = flops / (ev_avg * 1e-3)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            t = json.load(open(TRAFFIC_FILE))
            if t.get("eval_source_hash") == eval_source_hash() and t.get("leaf_level") == leaf:
                traffic = t.get("hbm_bytes_per_launch")
        except Exception:
            traffic = None

    extra = {"leaf_level": leaf, "p": args.p, "near_pairs_per_ray": pairs / n_rays,
             "median_ms_per_call": ms_median, "median_rays_per_s": n_rays / (ms_median * 1e-3),
             "leaf_box_side": math.ldexp(info["root_side"], -leaf),
             "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in prof.items()},
             "eval_flops_per_launch": flops, "profiled_eager_ms_per_step": ms_prof}
    extra["stage_rooflines"] = stage_rooflines(info, f, g, args.p, extra["stage_ms_per_step"])

    # FP64 direct sum on the same GPU, on 128 full rows of the grid (rays/s is
    # exactly linear in the ray count for a direct sum)
    if not args.no_direct:
        sub = lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, 128)
        ysub = torch.empty((g.nx * 128, 2), dtype=torch.float64, device="cuda")
        fn = lambda: lf.deflect(xy, m, grid=sub, kappa_s=f.kappa_s, gamma=f.gamma,
                                method="direct", out=ysub)
        fn()
        dms = timed(fn, 2)
        direct = g.nx * 128 / (dms * 1e-3)
        extra["fp64_direct_rays_per_s"] = direct
        extra["mixed_fmm_speedup_vs_fp64_direct"] = value / direct
        log(f"FP64 direct: {dms:.1f} ms for {g.nx * 128} rays -> {direct:.3e} rays/s")
        # FP64 FMM at the same p, for context (two untimed calls first, so
        # that the timed ones replay the cached call graph like the mixed ones)
        for _ in range(2):
            run(prec="fp64", leaf=leaf)
        fms = timed(lambda: run(prec="fp64", leaf=leaf), 3)
        extra["fp64_fmm_rays_per_s"] = n_rays / (fms * 1e-3)
        yf = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        # FP64 FMM at the 1e-10 target: the autotuner's order and leaf level
        # for a 1e-10 per-ray error on its 256^2 sample (or --p-fp64)
        p_hi, leaf_hi = args.p_fp64, leaf
        if p_hi == 0:
            t_hi = lf.autotune(xy, m, grid, tol=1e-10, kappa_s=f.kappa_s, gamma=f.gamma,
                               precision="fp64")
            p_hi, leaf_hi = t_hi["p"], t_hi["leaf_level"]
            extra["fp64_fmm_1e-10_autotune"] = t_hi
        for _ in range(2):
            run(prec="fp64", p=p_hi, leaf=leaf_hi)
        fms_hi = timed(lambda: run(prec="fp64", p=p_hi, leaf=leaf_hi), 3)
        extra["fp64_fmm_1e-10"] = {"p": p_hi, "leaf_level": leaf_hi,
                                   "rays_per_s": n_rays / (fms_hi * 1e-3), "ms": fms_hi}
        yf_hi = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        log(f"FP64 FMM p={args.p}: {fms:.3f} ms; p={p_hi} leaf {leaf_hi}: {fms_hi:.3f} ms")
        run(leaf=leaf)   # restore the mixed output (not timed)

    cpu = None
    if not args.no_cpu:
        import oracle
        rays = g.rays(idx)
        nthr = host_threads()
        t1 = time.perf_counter()
        yo, ao, _ = oracle.deflect(f.xy, f.m, rays, f.kappa_s, f.gamma, nthreads=nthr)
        dt = time.perf_counter() - t1
        cpu = {"value": len(idx) / dt, "unit": "rays/s", "cores": nthr, "kind": "oracle",
               "sample": f"{len(idx)} rays (every 32nd row and column of the 8192^2 grid) "
                         f"against all 1e6 stars, FP64 direct sum, {dt:.1f} s on {nthr} threads "
                         f"({host_desc()})"}
        # one thread, for comparison with the paper's single core
        idx1 = idx[::64]
        t1 = time.perf_counter()
        oracle.deflect(f.xy, f.m, g.rays(idx1), f.kappa_s, f.gamma, nthreads=1)
        dt1 = time.perf_counter() - t1
        extra["cpu_oracle_1_thread"] = {"value": len(idx1) / dt1, "unit": "rays/s",
                                        "sample": f"{len(idx1)} rays, {dt1:.1f} s"}
        st = ray_error_stats(y_mixed_sample, yo, ao)
        extra["err_mixed_p%d" % args.p] = st
        extra["rel_l2_err_alpha_mixed"] = st["rel_l2"]
        if not args.no_direct:
            extra["err_fp64_fmm_p%d" % args.p] = ray_error_stats(yf, yo, ao)
            extra["fp64_fmm_1e-10"]["err"] = ray_error_stats(yf_hi, yo, ao)
        log(f"oracle: {dt:.1f} s on {nthr} threads ({host_desc()}), 1 thread "
            f"{len(idx1) / dt1:.1f} rays/s; mixed errors {st}")

    out = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64 mixed", "data": "synthetic",
        "config": {"workload": "N_*=1e6 power-law-mass disk (kappa_*=0.4, kappa_s=0.2, "
                               "gamma=0.35), 8192x8192 ray grid, mixed FMM p=%d" % args.p,
                   "n_stars": f.n, "n_rays": n_rays, "p": args.p, "leaf_level": leaf},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
                     "kernel": "k_eval (fused L2P + P2P + smooth term)",
                     "eval_ms_avg": ev_avg},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


MAP_METRIC = "rays/s shot into a 2000x2000 magnification map at N_*=5e6, mu=50 (mixed FMM)"
IPM_METRIC = ("corner rays/s mapped into a 2000x2000 IPM magnification map at N_*=5e6, mu=50 "
              "(mixed FMM)")


def bench_map(args):
    """High-magnification inverse ray shooting: one lens_map call per step."""
    import numpy as np
    import torch

    import paper_2211_00354_amd as lf
    from paper_2211_00354_amd import _lib
    import workloads as wl

    log("generating workload")
    f, g, mp = wl.high_magnification()
    xy = torch.from_numpy(f.xy).cuda()
    m = torch.from_numpy(f.m).cuda()
    grid = lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
    md = lf.MapDesc(mp.y1min, mp.y2min, mp.side, mp.npix)
    # p, leaf level and FP32 levels from the autotuner for a 1e-4 expected
    # bin-reassignment rate (outside the timed region)
    t0 = time.perf_counter()
    tuned = lf.autotune(xy, m, grid, map=md, tol=1e-4, kappa_s=f.kappa_s, gamma=f.gamma,
                        leaf_level=args.leaf)
    tune_s = time.perf_counter() - t0
    log(f"autotune: {tuned} in {tune_s:.2f} s")
    p, fl, args.leaf = tuned["p"], tuned["fp32_levels"], tuned["leaf_level"]
    counts = torch.zeros((mp.npix, mp.npix), dtype=torch.int32, device="cuda")
    kw = dict(kappa_s=f.kappa_s, gamma=f.gamma, precision="mixed", p=p, fp32_levels=fl,
              leaf_level=args.leaf)

    ipm = args.workload == "ipm"
    mu = torch.zeros((mp.npix, mp.npix), dtype=torch.float64, device="cuda")

    def step():
        if ipm:
            mu.zero_()
            lf.ipm_map(xy, m, grid=grid, map=md, mu=mu, **kw)
        else:
            counts.zero_()
            lf.irs_map(xy, m, grid=grid, map=md, counts=counts, **kw)

    def timed_steps():
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    for _ in range(args.warmup):
        step()
    ms = timed_steps()   # graph replays of the call
    _lib.profile_enable(True)
    ms_prof = timed_steps()   # eager, with HIP events around every stage
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    log(f"map: {ms:.3f} ms/step; profiled eager steps {ms_prof:.3f} ms; stages {prof}")
    if args.profile_only:
        return
    value = g.n / (ms * 1e-3)
    plan = lf.Plan(xy, m, grid=grid, kappa_s=f.kappa_s, gamma=f.gamma, precision="mixed", p=p,
                   leaf_level=args.leaf, fp32_levels=fl)
    info = plan.info()
    leaf = info["leaf_level"]
    pairs = near_pairs(info, f, g)
    flops = PAIR_FLOPS * pairs + (8 * p + 2) * g.n
    ev_ms, ev_n = prof.get("eval" if ipm else "eval_map", (float("nan"), 1))
    ev_avg = ev_ms / max(ev_n, 1)
    achieved = flops / (ev_avg * 1e-3)
    extra = {"leaf_level": leaf, "p": p, "fp32_levels": fl, "autotune": tuned, "autotune_s": tune_s,
             "near_pairs_per_ray": pairs / g.n,
             "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in prof.items()},
             "eval_flops_per_launch": flops,
             "map_mean": float(mu.mean()) if ipm else float(counts.double().mean()),
             "profiled_eager_ms_per_step": ms_prof}
    cpu = None
    if not args.no_cpu:
        import oracle
        idx = g.strided(512, 256)
        rays = g.rays(idx)
        ys = lf.deflect(rays=torch.from_numpy(rays).cuda(), plan=plan, kappa_s=f.kappa_s,
                        gamma=f.gamma).cpu().numpy()
        nthr = host_threads()
        t1 = time.perf_counter()
        yo, ao, _ = oracle.deflect(f.xy, f.m, rays, f.kappa_s, f.gamma, nthreads=nthr)
        dt = time.perf_counter() - t1
        cpu = {"value": len(idx) / dt, "unit": "rays/s", "cores": nthr, "kind": "oracle",
               "sample": f"{len(idx)} rays (every 512th row and column of the 16384^2 grid) "
                         f"against all 5e6 stars, FP64 direct sum, {dt:.1f} s"}
        S = mp.npix / mp.side
        off = np.array([mp.y1min, mp.y2min])
        moved = int(np.count_nonzero(np.any(np.floor((ys - off) * S) != np.floor((yo - off) * S), 1)))
        extra["rel_l2_err_alpha_mixed"] = float(np.linalg.norm(ys - yo) / np.linalg.norm(ao))
        extra["bin_reassignment_estimate"] = float(np.abs(ys - yo).sum(1).mean() * S)
        extra["bins_moved_in_sample"] = f"{moved}/{len(idx)}"
        log(f"oracle: {dt:.1f} s on {nthr} threads; reassignment estimate "
            f"{extra['bin_reassignment_estimate']:.2e}")
    plan.close()
    if ipm:
        ip_ms, ip_n = prof.get("ipm", (float("nan"), 1))
        extra["ipm_kernel_ms"] = ip_ms / max(ip_n, 1)
    out = {
        "metric": IPM_METRIC if ipm else MAP_METRIC, "value": value, "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64 mixed", "data": "synthetic",
        "config": {"workload": "N_*=5e6 equal masses (kappa_*=0.1, kappa_s=0.75, gamma=0.05), "
                               "16384x16384 rays into a 2000x2000 %s map, mixed FMM p=%d"
                               % ("IPM" if ipm else "IRS", p),
                   "n_stars": f.n, "n_rays": g.n, "p": p, "leaf_level": leaf},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": None,
                     "kernel": ("k_eval (fused L2P + P2P + smooth term), corners for IPM" if ipm else
                                "k_eval (fused L2P + P2P + smooth term + binning)"),
                     "eval_ms_avg": ev_avg},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


BATCH_METRIC = "rays/s shot into 64 independent 512x512 maps (one captured graph, mixed FMM)"


def bench_batch(args):
    """64 star fields (N_* log-uniform in [1e4, 2e5], kappa_* in [0.05, 0.6],
    gamma in [0, 0.6]), 2048^2 rays and a 512^2 map each, all in one
    lens_map_batched call (one captured graph); p, leaf level and FP32 levels
    tuned per field for a 1e-4 expected bin-reassignment rate when the graph
    is built (outside the timed region)."""
    import numpy as np
    import torch

    import paper_2211_00354_amd as lf
    from paper_2211_00354_amd import _lib
    import workloads as wl

    log("generating workload")
    cases = wl.field_batch()
    fields, grids, maps = [], [], []
    for f, g, mp in cases:
        fields.append((torch.from_numpy(f.xy).cuda(), torch.from_numpy(f.m).cuda(), f.kappa_s, f.gamma))
        grids.append(lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny))
        maps.append(lf.MapDesc(mp.y1min, mp.y2min, mp.side, mp.npix))
    counts = [torch.zeros((mp.npix, mp.npix), dtype=torch.int32, device="cuda") for mp in maps]
    n_rays = sum(g.nx * g.ny for g in grids)
    t0 = time.perf_counter()
    lf.irs_map_batched(fields, grids, maps, counts=counts, p=0, tol=1e-4)   # tunes, captures
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(f"tuning + capture + first replay: {build_s:.2f} s")

    def step():
        for c in counts:
            c.zero_()
        lf.irs_map_batched(fields, grids, maps, counts=counts, p=0, tol=1e-4)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = n_rays / (ms * 1e-3)
    log(f"batch: {ms:.3f} ms/step -> {value:.3e} rays/s")
    extra = {"fields": len(cases), "tune_capture_s": build_s,
             "n_stars": [int(f.n) for f, _, _ in cases][:8] + ["..."]}
    cpu = None
    if not args.no_cpu:
        import oracle
        # the oracle's deflection of a strided sample of field 0's rays
        f, g, mp = cases[0]
        idx = g.strided(4, 2)
        nthr = host_threads()
        t1 = time.perf_counter()
        oracle.deflect(f.xy, f.m, g.rays(idx), f.kappa_s, f.gamma, nthreads=nthr)
        dt = time.perf_counter() - t1
        cpu = {"value": len(idx) / dt, "unit": "rays/s", "cores": nthr, "kind": "oracle",
               "sample": f"{len(idx)} rays of field 0 (N_*={f.n}) against all its stars, FP64 "
                         f"direct sum, {dt:.1f} s"}
    out = {
        "metric": BATCH_METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64 mixed", "data": "synthetic",
        "config": {"workload": "64 fields, N_* log-uniform in [1e4, 2e5], kappa_* U[0.05,0.6], "
                               "gamma U[0,0.6], 2048x2048 rays and a 512x512 map each, one graph",
                   "n_rays": n_rays},
        "roofline": None,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


APP_METRIC = {
    "halo": "rays/s deflected by a 1.575e7-particle halo (mixed FMM, order chosen for 1e-5)",
    "arc": "rays/s mapped by IPM over a 15000x10 anamorphic region (1.8e6 deflectors, mu=4200)",
}


def bench_application(args):
    """The two application workloads, one whole call per step (plan built
    inside the call).  halo: lens_deflect of 4000^2 rays through 1.575e7
    particles, mixed precision, order and leaf level from the autotuner for
    a 1e-5 per-ray error (tuned outside the timed region).  arc: one
    lens_map_ipm call over 1.5e11 rays (passes of 2^28 rays), mixed
    precision, p = 24 with every M2L level in FP64."""
    import numpy as np
    import torch

    import paper_2211_00354_amd as lf
    from paper_2211_00354_amd import _lib
    import workloads as wl

    log("generating workload")
    halo = args.workload == "halo"
    if halo:
        f, g = wl.synthetic_halo()
    else:
        f, g, mp = wl.anamorphic_arc()
    xy = torch.from_numpy(f.xy).cuda()
    m = torch.from_numpy(f.m).cuda()
    grid = lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
    extra = {}
    if halo:
        t0 = time.perf_counter()
        tuned = lf.autotune(xy, m, grid, tol=1e-5, kappa_s=f.kappa_s, gamma=f.gamma)
        extra["autotune"], extra["autotune_s"] = tuned, time.perf_counter() - t0
        log(f"autotune: {tuned}")
        kw = dict(kappa_s=f.kappa_s, gamma=f.gamma, precision="mixed", p=tuned["p"],
                  leaf_level=tuned["leaf_level"], fp32_levels=tuned["fp32_levels"])
        y = torch.empty((g.n, 2), dtype=torch.float64, device="cuda")

        def step():
            lf.deflect(xy, m, grid=grid, out=y, **kw)
        desc = ("1.575e7 halo particles (dark matter, gas, stars, 128 black holes; Einstein "
                "radius ~30), 4000x4000 rays over [-45,45]^2, mixed FMM p=%d" % kw["p"])
    else:
        md = lf.MapDesc(mp.y1min, mp.y2min, mp.side, mp.npix)
        kw = dict(kappa_s=f.kappa_s, gamma=f.gamma, precision="mixed", p=24, fp32_levels=-1)
        mu = torch.zeros((mp.npix, mp.npix), dtype=torch.float64, device="cuda")

        def step():
            mu.zero_()
            lf.ipm_map(xy, m, grid=grid, map=md, mu=mu, **kw)
        desc = ("1.8e6 deflectors of 0.2 (kappa_*=0.0064) in a 15000-diameter disk, macro "
                "mu=4200 (axis ratio 1500), 15000000x10000 rays over 15000x10 into a 4000x4000 "
                "IPM map of 0.001 pixels, mixed FMM p=24, FP64 M2L")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    _lib.profile_enable(True)
    step()
    torch.cuda.synchronize()
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    extra["stage_ms_one_step"] = {k: v[0] for k, v in prof.items()}
    value = g.n / (ms * 1e-3)
    log(f"{args.workload}: {ms:.3f} ms/step -> {value:.3e} rays/s; stages {extra['stage_ms_one_step']}")
    if not halo:
        extra["map_mean_mu"] = float(mu.mean())
        extra["mu_macro"] = f.meta["mu_macro"]
    cpu = None
    if not args.no_cpu:
        import oracle
        rng = np.random.default_rng(5)
        idx = g.strided(128, 61) if halo else rng.integers(0, g.n, 1000)
        rays = g.rays(idx)
        plan = lf.Plan(xy, m, grid=grid, **kw)
        ys = lf.deflect(rays=torch.from_numpy(rays).cuda(), plan=plan, kappa_s=f.kappa_s,
                        gamma=f.gamma).cpu().numpy()
        plan.close()
        nthr = host_threads()
        t1 = time.perf_counter()
        yo, ao, _ = oracle.deflect(f.xy, f.m, rays, f.kappa_s, f.gamma, nthreads=nthr)
        dt = time.perf_counter() - t1
        cpu = {"value": len(idx) / dt, "unit": "rays/s", "cores": nthr, "kind": "oracle",
               "sample": f"{len(idx)} rays of the grid against all {f.n} deflectors, FP64 "
                         f"direct sum, {dt:.1f} s"}
        if halo:
            extra["ray_error"] = ray_error_stats(ys, yo, ao)
        else:
            S = mp.npix / mp.side
            extra["bin_reassignment_estimate"] = float(np.abs(ys - yo).sum(1).mean() * S)
    out = {
        "metric": APP_METRIC[args.workload], "value": value, "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64 mixed", "data": "synthetic",
        "config": {"workload": desc, "n_stars": f.n, "n_rays": g.n},
        "roofline": None, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
