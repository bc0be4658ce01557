"""Benchmark: ACR setup + CG solve to a 1e-8 relative residual on the
127^3 variable-coefficient Poisson workload, mixed precision vs FP64.

One step = the whole hot path on one batch of synthetic input: assembly,
geometry, level-by-level H-matrix cyclic reduction (setup) and the
ACR-preconditioned CG solve to ||b - A x|| / ||b|| <= 1e-8.  Inputs are
resident in HBM before the timed region starts.

Workload (seeded, synthetic): 127^3 interior grid (2,048,383 unknowns),
kappa piecewise constant on 8^3 sub-cubes with values 10^U(-3,3), f ~
U(-1,1), eps = 1e-4, eta = 2, leaf size 32.

Timed: W warmup steps then K steps in the headline precision (mixed: FP32
factors, FP64 leaf inversion / truncation cores / Krylov); then K steps in
FP64 for the mixed-vs-FP64 speedup.  `value` is the mean mixed-precision
seconds per step (lower is better).

Also printed (same JSON line):
  roofline      -- the dominant kernel of the H-arithmetic steps (ALU
                   bound): algorithmic flops per launch / mean launch
                   duration (HIP events on its stream), against 78.6
                   TFLOP/s (truncating kernel, FP64 cores) or 157.3 TFLOP/s
                   (accumulate-only kernel, FP32 products);
                   roofline_second_kernel -- the other one
  apply_roofline-- the preconditioner application (HBM bound):
                   algorithmic bytes per apply / apply time vs 8 TB/s, for
                   the mixed handle (apply_roofline_fp64: the FP64 one)
  cpu_baseline  -- the CPU FP64 oracle on a bounded sample (same recipe at
                   23^3, ~20 s), projected to 127^3 by the N log^2 N setup
                   complexity; rank 0, N=1 only.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
METRIC = "ACR setup+solve secs to 1e-8 resid, 127^3 Poisson; mixed vs FP64 GPU speedup"


# HBM traffic of the accumulation kernel from rocprofv3 --pmc FETCH_SIZE /
# WRITE_SIZE passes (profiles/accum_kernel_traffic.json), valid only for the
# kernel source it was measured on.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "accum_kernel_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1712_08872_amd", "csrc", f) for f in ("k_harith.hip", "hprog.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """Bytes per launch of `kernel` from the committed counter record, or
    None when it is absent or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec.get("kernels", {}).get(kernel, {}).get("traffic_bytes_per_launch")


def kernel_roofline(name, launches, seconds, flops, peak):
    """Algorithmic flops per launch over the mean launch duration (HIP
    events around every launch on its stream)."""
    launches = max(launches, 1)
    per_s = seconds / launches
    per_f = flops / launches
    tf = per_f / per_s / 1e12 if per_s > 0 else 0.0
    traffic = measured_traffic(name)
    return {"bound": "alu", "achieved": round(tf, 4), "peak": peak, "unit": "TFLOP/s", "frac": round(tf / peak, 6),
            "traffic": round(traffic) if traffic is not None else None, "kernel": name, "launches": launches,
            "mean_launch_ms": round(per_s * 1e3, 4), "flops_per_launch": per_f,
            "total_seconds": round(seconds, 3)}


def copy_probe(mib):
    """A plain device copy of known size, for calibrating FETCH_SIZE /
    WRITE_SIZE (rocprofv3 --pmc ... -- python bench.py --copy-probe MIB)."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}), flush=True)


def _inputs(n, seed_offset=0):
    import synth
    k = synth.kappa_subcubes(n, 11 + 2 * seed_offset)
    f = synth.rhs_uniform(n ** 3, 12 + 2 * seed_offset)
    return k, f


def gpu_step(acr, torch, n, kap, f, precision, eps, rtol):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = acr.acr_setup(n, n, n, acr.POISSON_HARMONIC, kappa=kap, eps=eps, eta=2.0, leaf_size=32,
                      precision=precision)
    t1 = time.perf_counter()
    x, info = acr.krylov_solve(h, f, method=acr.CG, rtol=rtol, maxit=500)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st = acr.acr_stats(h)
    return h, x, {"seconds": t2 - t0, "setup_s": t1 - t0, "solve_s": t2 - t1, "iters": info["iters"],
                  "relres": info["relres_true"], "stats": st}


def apply_roofline(acr, torch, h, f, reps=5):
    stream = torch.cuda.current_stream()
    z = torch.empty_like(f)
    acr.acr_apply(h, f, z)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        acr.acr_apply(h, f, z, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    b = acr.acr_stats(h)["bytes_per_apply"]
    gbs = b / t / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "ms_per_apply": round(t * 1e3, 3),
            "bytes_per_apply": b}


def cpu_baseline(n_sample=23, n_full=127, eps=1e-4):
    """The oracle (numpy/scipy FP64, single BLAS thread) on the same recipe
    at n_sample^3, projected to n_full^3 with the N log^2 N setup cost."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
        cores = 1
    except Exception:
        cores = len(os.sched_getaffinity(0))
    import numpy as np  # noqa: F401
    from oracle import assembly, hacr, krylov
    kap, f = _inputs(n_sample)
    S = assembly.stencil7("poisson", n_sample, n_sample, n_sample, kappa=kap)
    A = assembly.to_sparse(S, n_sample, n_sample, n_sample)
    t0 = time.perf_counter()
    H = hacr.HACR(S, n_sample, n_sample, n_sample, eps=eps, eta=2.0, leaf=32)
    x, info = krylov.pcg(lambda v: A @ v, f, H.apply, tol=1e-8)
    t = time.perf_counter() - t0
    Ns, Nf = n_sample ** 3, n_full ** 3
    scale = (Nf * math.log2(Nf) ** 2) / (Ns * math.log2(Ns) ** 2)
    return {"value": round(t * scale, 1), "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"oracle setup+PCG on the same recipe at {n_sample}^3 ({t:.1f} s, {info['iters']} iters), "
                      f"projected x{scale:.0f} by N log^2 N to {n_full}^3",
            "sample_seconds": round(t, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--n", type=int, default=127)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the plane-sharded multi-GPU "
              f"path is not built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    os.environ["ACR_KERNEL_TIMING"] = "1"
    import torch
    import paper_1712_08872_amd as acr
    n = args.n
    kap_np, f_np = _inputs(n)
    kap = torch.from_numpy(kap_np.reshape(-1)).cuda()
    f = torch.from_numpy(f_np).cuda()
    torch.cuda.synchronize()
    for w in range(args.warmup):
        h, _, r = gpu_step(acr, torch, n, kap, f, acr.MIXED_FP32, args.eps, args.rtol)
        del h
        print(f"[bench] warmup {w}: {r['seconds']:.2f} s", file=sys.stderr, flush=True)
    mixed, fp64 = [], []
    last = None
    for k in range(args.steps):
        if last is not None:
            del last
            last = None
        h, x, r = gpu_step(acr, torch, n, kap, f, acr.MIXED_FP32, args.eps, args.rtol)
        mixed.append(r)
        print(f"[bench] mixed step {k}: {r['seconds']:.2f} s (setup {r['setup_s']:.2f}, solve {r['solve_s']:.3f}, "
              f"{r['iters']} iters)", file=sys.stderr, flush=True)
        last = h
    st = mixed[-1]["stats"]
    aroof = apply_roofline(acr, torch, last, f)
    del last
    aroof64 = None
    if not args.no_fp64:
        for k in range(args.steps):
            h, _, r = gpu_step(acr, torch, n, kap, f, acr.FP64, args.eps, args.rtol)
            fp64.append(r)
            print(f"[bench] fp64 step {k}: {r['seconds']:.2f} s (setup {r['setup_s']:.2f}, "
                  f"solve {r['solve_s']:.3f}, {r['iters']} iters)", file=sys.stderr, flush=True)
            if k == args.steps - 1:
                aroof64 = apply_roofline(acr, torch, h, f)
            del h
    t_mixed = sum(r["seconds"] for r in mixed) / len(mixed)
    t_fp64 = sum(r["seconds"] for r in fp64) / len(fp64) if fp64 else None
    # H-arithmetic kernels (ALU bound): the truncating kernel (FP64 Gram
    # matrices and cores) and the accumulate-only kernel (FP32 products with
    # FP32 factors); `roofline` is the one with the larger total time
    kt = kernel_roofline("accum_kernel", st["accum_launches"], st["accum_seconds"], st["accum_flops"],
                         FP64_VECTOR_PEAK_TFLOPS)
    kd = kernel_roofline("accum_dense_kernel", st["dense_launches"], st["dense_seconds"], st["dense_flops"],
                         FP32_VECTOR_PEAK_TFLOPS)
    roof, roof2 = (kt, kd) if st["accum_seconds"] >= st["dense_seconds"] else (kd, kt)
    out = {"metric": METRIC, "value": round(t_mixed, 3), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(t_mixed * 1e3, 1), "higher_is_better": False,
           "scaling": "strong", "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
           "config": {"workload": f"variable-coefficient Poisson {n}^3, 8^3 sub-cube kappa 10^U(-3,3), "
                                  f"eps={args.eps:g}, eta=2, leaf 32, CG to {args.rtol:g}",
                      "n": n, "unknowns": n ** 3, "precision": "mixed FP32 factors / FP64 Krylov"},
           "mixed_s": round(t_mixed, 3), "fp64_s": round(t_fp64, 3) if t_fp64 else None,
           "speedup_mixed_vs_fp64": round(t_fp64 / t_mixed, 3) if t_fp64 else None,
           "mixed_setup_s": round(mixed[-1]["setup_s"], 3), "mixed_solve_s": round(mixed[-1]["solve_s"], 4),
           "mixed_iters": mixed[-1]["iters"], "mixed_relres": mixed[-1]["relres"],
           "fp64_setup_s": round(fp64[-1]["setup_s"], 3) if fp64 else None,
           "fp64_solve_s": round(fp64[-1]["solve_s"], 4) if fp64 else None,
           "fp64_iters": fp64[-1]["iters"] if fp64 else None,
           "max_rank": st["max_rank_all"], "factor_GB": round(st["bytes_factors"] / 1e9, 2),
           "roofline": roof, "roofline_second_kernel": roof2, "apply_roofline": aroof,
           "apply_roofline_fp64": aroof64}
    if not args.no_cpu and int(os.environ.get("RANK", "0")) == 0:
        out["cpu_baseline"] = cpu_baseline(eps=args.eps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
