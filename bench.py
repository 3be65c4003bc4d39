"""Throughput of the whole GDSW hot path on one MI355X.

One step = gdsw_setup (index maps, local LU factorizations, GDSW basis,
Galerkin recursion, coarsest factorization) + gdsw_solve (FGMRES(30) to a
relative residual of 1e-8 preconditioned by the three-level method) +
gdsw_destroy, on a seeded 32x16x16 die-like voxel channel (Q2-P1disc, Carreau
nu0 = 1, lambda = 1, n = 0.5, 2^3-voxel parts, 2x2x2 subregions).  The matrix
and the right-hand side are resident in HBM before the timed region.

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of one level-1 local-solve launch on this workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a 1 GiB copy (profiles/local_solve_die32x16x16.md), valid only for the
# local-solve kernel source it was measured on.
LOCAL_SOLVE_TRAFFIC = {"bytes": 3.993e9, "source_hash": "935223e387098f25", "precision": "fp64"}


def local_solve_source_hash():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2606_01433_amd", "csrc", "apply.hip")).read()
    a, b = src.index("// Local solves w_i"), src.index("__global__ void k_scatter_sum")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]
FP64_MFMA_TFLOPS = 78.6
FP32_MFMA_TFLOPS = 157.3


def workload(args):
    from harness import die_problem
    return die_problem(32, 16, 16, seed=args.seed, nu0=1.0, lam=1.0, n_exp=0.5, levels=3)


def cpu_baseline(P, gpu_iterations, budget_its=4):
    """Oracle (FP64 NumPy/SciPy, single thread): full setup, then a few FGMRES iterations, extrapolated."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    import oracle
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        H = oracle.setup(P)
        t1 = time.perf_counter()
        K = P.K()
        _, info = oracle.fgmres(lambda v: K @ v, lambda v: oracle.apply(H, v), P.b, tol=1e-8, max_it=budget_its)
        t2 = time.perf_counter()
    per_it = (t2 - t1) / max(1, info["iterations"])
    t_solve = (t1 - t0) + per_it * gpu_iterations
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle setup of the full workload ({t1 - t0:.1f} s) + {info['iterations']} FGMRES "
                       f"iterations ({per_it:.2f} s each), extrapolated to the GPU's {gpu_iterations} iterations")}


def serving_bench(seed=0, n_requests=24):
    """Poisson stream of Picard-step solves over a pool of seeded dies: FP32-factor serving with
    concurrent slots vs. plain FP64 one at a time on the same arrival times."""
    import numpy as np
    from harness import die_problem
    from paper_2606_01433_amd.serving import Server, Request, summarize
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    pool = []
    for nx, ny, nz in [(16, 16, 16), (32, 16, 16), (48, 24, 24), (64, 32, 32)]:
        for q in range(2):
            n_exp = float(rng.uniform(0.3, 0.9))
            lam = float(10.0 ** rng.uniform(-1.0, 1.0))
            # four levels on the larger dies keep the coarsest dense problem at order ~2k
            levels = 3 if nx * ny * nz <= 8192 else 4
            pool.append(die_problem(nx, ny, nz, seed=seed + q, nu0=1.0, lam=lam, n_exp=n_exp, levels=levels))
    picks = rng.integers(0, len(pool), n_requests)
    # service time of the plain FP64 path, one request at a time (also warms every size up)
    srv = Server(max_active=1)
    t0 = time.perf_counter()
    for k, P in enumerate(pool):
        srv.submit(Request(-1 - k, P, tol=1e-8)).wait()
    t_mean = (time.perf_counter() - t0) / len(pool)
    srv.close()
    rate = 1.5 / t_mean
    gaps = rng.exponential(1.0 / rate, n_requests)

    def stream(server, **opts):
        reqs = []
        t_start = time.perf_counter()
        t_next = t_start
        for k in range(n_requests):
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            reqs.append(server.submit(Request(k, pool[int(picks[k])], arrival=time.perf_counter(), **opts)))
            t_next += gaps[k]
        server.drain(reqs)
        t_end = time.perf_counter()
        server.close()
        return reqs, summarize(reqs, t_start, t_end)

    base_reqs, base = stream(Server(max_active=1), tol=1e-8)
    srv = Server(budget_bytes=200 * 2 ** 30, max_active=4)
    mix_reqs, mixed = stream(srv, tol=1e-8, precision="mixed")
    mixed["peak_active"] = srv.peak_active
    err = max(float(np.linalg.norm(m.x - b_.x) / np.linalg.norm(b_.x)) for m, b_ in zip(mix_reqs, base_reqs))
    return {"requests": n_requests, "arrival_rate_hz": rate,
            "pool": "seeded dies 16x16x16, 32x16x16, 48x24x24, 64x32x32 (two each); Carreau n ~ U[0.3,0.9], "
                    "lambda = 10^U[-1,1]; three levels up to 32x16x16, four above; FGMRES(30) to 1e-8",
            "serving_fp32_factors_4_slots": mixed, "fp64_one_at_a_time": base,
            "max_rel_diff_fp32_vs_fp64_solution": err}


def mixed_precision_leg(P, step, x64, t64, n_steps=3):
    """The same step with FP32 local factors and bases (FP64 Krylov, residuals and coarsest solve),
    against the FP64 GPU path just timed: step time, iterations, error, FP32 factor rate."""
    import numpy as np
    import torch
    step(False, "mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        x, info, st = step(True, "mixed")
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / n_steps
    xh, x64h = x.cpu().numpy(), x64.cpu().numpy()
    launches = st["local_solve_launches"]
    return {"solves_per_s": 1.0 / T, "ms_per_step": T * 1e3, "speedup_vs_fp64": t64 / T,
            "ms_setup": st["ms_total"], "ms_solve": info["ms_total"], "iterations": info["iterations"],
            "true_rel_residual": float(np.linalg.norm(P.K() @ xh - P.b) / np.linalg.norm(P.b)),
            "rel_diff_vs_fp64_gpu_solution": float(np.linalg.norm(xh - x64h) / np.linalg.norm(x64h)),
            "level1_local_solve_gbs": (st["local_solve_bytes"] / (st["ms_local_solve"] / launches * 1e-3) / 1e9
                                       if launches else None),
            "factor": {"flops_level1": st["factor_flops"][0], "ms_factor_all_levels": st["ms_factor"],
                       "tflops_level1_lower_bound": st["factor_flops"][0] / (st["ms_factor"] * 1e-3) / 1e12,
                       "peak_tflops": FP32_MFMA_TFLOPS}}


def solve_only_bench(P, Kdev, b, precision, n_solves=5):
    """Setup amortized: several solves on one context, eager applies vs captured hipGraph applies."""
    import torch
    from paper_2606_01433_amd import gdsw
    out = {}
    for graph in (False, True):
        with gdsw.Context(P, K=Kdev, tol=1e-8, precision=precision, graph=graph) as ctx:
            ctx.solve(b)                     # warm-up (captures the graphs in graph mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n_solves):
                x, info = ctx.solve(b)
            torch.cuda.synchronize()
            out["graph" if graph else "eager"] = {"ms_per_solve": (time.perf_counter() - t0) / n_solves * 1e3,
                                                  "solves_per_s": n_solves / (time.perf_counter() - t0)}
            if not graph:
                out["spmv"] = spmv_roofline(ctx, P, b)
    return out


def spmv_roofline(ctx, P, x, calls=50):
    """y = K x through the library, timed with HIP events on the launching stream: algorithmic bytes
    (CSR values and int32 columns, int64 row pointers, x once, y) over the mean duration."""
    import torch
    y = torch.empty_like(x)
    ctx.spmv(x, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(calls):
        ctx.spmv(x, out=y)
    e1.record()
    e1.synchronize()
    us = e0.elapsed_time(e1) / calls * 1e3
    nbytes = 12.0 * len(P.col) + 8.0 * (P.n + 1) + 16.0 * P.n
    return {"bound": "hbm", "achieved": nbytes / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_call": nbytes, "us_per_call": us}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is not part of this build",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2606_01433_amd import gdsw
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(args.copy_calibration * (1 << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 8}))
        return
    gdsw.load_library()
    P = workload(args)
    dev = torch.device("cuda", 0)
    Kdev = (torch.as_tensor(P.rowptr, device=dev), torch.as_tensor(P.col, device=dev),
            torch.as_tensor(P.val, device=dev))
    b = torch.as_tensor(P.b, device=dev)
    stream = torch.cuda.current_stream()

    def step(profile, precision=args.precision):
        ctx = gdsw.Context(P, K=Kdev, tol=1e-8, precision=precision, profile=profile, stream=stream)
        x, info = ctx.solve(b, stream=stream)
        st = ctx.stats()
        ctx.close()
        return x, info, st

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    infos, stats = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, info, st = step(True)
        infos.append(info)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T = (t1 - t0) / args.steps
    res = float(np.linalg.norm(P.K() @ x.cpu().numpy() - P.b) / np.linalg.norm(P.b))
    launches = sum(s["local_solve_launches"] for s in stats)
    ms_ls = sum(s["ms_local_solve"] for s in stats)
    bytes_per_launch = stats[0]["local_solve_bytes"]
    achieved = bytes_per_launch / (ms_ls / launches * 1e-3) / 1e9 if launches else 0.0
    st0 = stats[0]
    iters = infos[-1]["iterations"]
    traffic = None
    if (local_solve_source_hash() == LOCAL_SOLVE_TRAFFIC["source_hash"]
            and args.precision == LOCAL_SOLVE_TRAFFIC["precision"] and args.seed == 0):
        traffic = LOCAL_SOLVE_TRAFFIC["bytes"]
    out = {
        "metric": "Stokes solves/s to 1e-8 rel. residual",
        "value": 1.0 / T,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 local factors / f64 Krylov",
        "data": "synthetic (seeded die-like voxel channel, Carreau viscosity at a seeded linearization point)",
        "config": {"workload": "three-level FP64 monolithic GDSW + FGMRES(30) to 1e-8, 32x16x16 voxel die "
                               "(~20% masked), Q2-P1disc, Carreau nu0=1 lambda=1 n=0.5, 2^3-voxel parts, overlap 1",
                   "n_dofs": int(P.n), "nnz": int(len(P.col)), "parts": st0["parts"][:st0["levels"]],
                   "level_dofs": st0["n"][:st0["levels"]], "iterations": iters,
                   "local_solve_waves_per_matrix": st0["ls_waves"][:st0["levels"] - 1],
                   "true_rel_residual": res, "precision": args.precision,
                   "ms_setup": st0["ms_total"], "ms_solve": infos[-1]["ms_total"],
                   "ms_setup_phases": {"host_maps": st0["ms_maps"], "host_prep": st0["ms_extract"],
                                       "factor": st0["ms_factor"],
                                       "basis_galerkin": st0["ms_basis"], "coarsest": st0["ms_coarse"]},
                   "setup_timeline_ms": {
                       "note": "GPU events, ms after the setup's first event: [begin, end]",
                       "factor": [[round(a, 2), round(b, 2)] for a, b in st0["tl_factor"][:st0["levels"] - 1]],
                       "basis_galerkin": [[round(a, 2), round(b, 2)] for a, b in st0["tl_basis"][:st0["levels"] - 1]],
                       "coarsest": [round(x, 2) for x in st0["tl_coarsest"]]}},
        "roofline": {"kernel": "k_local_solve (level-1 batched pivoted LU forward/backward substitution)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_per_launch, "launches": launches,
                     "avg_launch_us": ms_ls / launches * 1e3 if launches else None},
        "factor": {"flops_level1": st0["factor_flops"][0], "ms_factor_all_levels": st0["ms_factor"],
                   "tflops_level1_lower_bound": st0["factor_flops"][0] / (st0["ms_factor"] * 1e-3) / 1e12,
                   "peak_tflops": FP64_MFMA_TFLOPS if args.precision == "fp64" else FP32_MFMA_TFLOPS},
    }
    out["solve_only"] = solve_only_bench(P, Kdev, b, args.precision)
    if args.precision == "fp64":
        out["mixed_precision"] = mixed_precision_leg(P, step, x, T)
    if not args.no_serving:
        out["serving"] = serving_bench(args.seed)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
