"""Throughput of the whole GDSW hot path on one MI355X.

Headline: one step = gdsw_setup (index maps, local LU factorizations, GDSW
basis, Galerkin recursion, coarsest factorization) + gdsw_solve (FGMRES(150) to
a relative residual of 1e-8) + gdsw_destroy, on the batching workload: a
seeded 96x48x48 die-like voxel channel (Q2-P1disc, Carreau nu0 = 1, lambda =
10, n = 0.4; level-1 parts of 2 or 3 voxels per axis, about 21k of them; four
levels), FP32 local factors and bases, FP64 Krylov / residuals / coarsest
solve, restricted combination, autotuned local solves and LU variants.  The matrix and the
right-hand side are resident in HBM before the timed region.

Further objects on the same JSON line: the level-1 local-solve roofline, the
whole-apply roofline, the event-timed level-1 LU kernel rate, setup-amortized
solves (eager against captured graphs) with the SpMV roofline, the precision
workload (64x32x32 die, three levels, FP64 against FP32 factors), the
three-level FP64 32x16x16 die, the serving stream, and the oracle on the host.

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
FP64_MFMA_TFLOPS = 78.6
FP32_MFMA_TFLOPS = 157.3

# FGMRES restart length of every solve to 1e-8 here.  The paper names none; the whole Krylov basis of the
# largest workload (2 x 151 vectors of 4.75M doubles, 11.5 GB) fits in HBM, so these solves do not restart
# (the library's default of 30 is reported beside the headline).
RESTART = 150

# HBM traffic of one level-1 local-solve launch per workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs scaled by a plain 1 GiB device copy (profiles/), valid only for the local-solve kernel source it
# was measured on (hash of that part of apply.hip) and for the precision and seed it was taken with.
LOCAL_SOLVE_TRAFFIC = {
    ("die32x16x16", "fp64"): {"bytes": 2.612e9, "source_hash": "53d5f1ed57d9cc29"},
    ("die96x48x48", "mixed"): {"bytes": 50.440e9, "source_hash": "53d5f1ed57d9cc29"},
}

WORKLOADS = {
    # batching workload (headline): four levels, uneven 2/3-voxel parts, FP32 factors
    "die96x48x48": dict(shape=(96, 48, 48), nu0=1.0, lam=10.0, n_exp=0.4, levels=4, frac3=0.1),
    # precision workload: same operator as the 32x16x16 die on 64x32x32, three levels
    "die64x32x32": dict(shape=(64, 32, 32), nu0=1.0, lam=1.0, n_exp=0.5, levels=3, frac3=0.0),
    # three-level FP64 workload
    "die32x16x16": dict(shape=(32, 16, 16), nu0=1.0, lam=1.0, n_exp=0.5, levels=3, frac3=0.0),
}


def local_solve_source_hash():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2606_01433_amd", "csrc", "apply.hip")).read()
    a = src.index("// Local solves w_i")
    b = src.index("// ---------------------------------------------------------------------------\n// Local solves of KC")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_problem(name, seed=0):
    from harness import die_problem
    w = WORKLOADS[name]
    nx, ny, nz = w["shape"]
    t0 = time.perf_counter()
    P = die_problem(nx, ny, nz, seed=seed, nu0=w["nu0"], lam=w["lam"], n_exp=w["n_exp"], levels=w["levels"],
                    frac3=w["frac3"])
    say(f"{name}: assembled in {time.perf_counter() - t0:.1f} s, n = {P.n}, nnz = {len(P.col)}, parts {P.n_parts}")
    return P


def describe(name, precision):
    w = WORKLOADS[name]
    nx, ny, nz = w["shape"]
    parts = "2- or 3-voxel parts per axis (3 with probability 0.1)" if w["frac3"] else "2^3-voxel parts"
    prec = "FP64" if precision == "fp64" else "FP32 local factors and bases, FP64 Krylov/residuals/coarsest"
    return (f"{w['levels']}-level monolithic GDSW, restricted (RAS) combination, {prec}, FGMRES({RESTART}) to 1e-8; "
            f"{nx}x{ny}x{nz} seeded voxel die (~20% masked), Q2-P1disc, Carreau nu0={w['nu0']:g} "
            f"lambda={w['lam']:g} n={w['n_exp']:g}, {parts}, overlap 1")


class Runner:
    """Device copies of one problem and the setup + solve + destroy step on them."""

    def __init__(self, P, stream):
        import torch
        dev = torch.device("cuda", 0)
        self.P = P
        self.K = (torch.as_tensor(P.rowptr, device=dev), torch.as_tensor(P.col, device=dev),
                  torch.as_tensor(P.val, device=dev))
        self.b = torch.as_tensor(P.b, device=dev)
        self.stream = stream
        self.Kh = P.K().tocsr()

    def context(self, **opts):
        from paper_2606_01433_amd import gdsw
        o = dict(tol=1e-8, restart=RESTART)
        o.update(opts)
        return gdsw.Context(self.P, K=self.K, stream=self.stream, **o)

    def step(self, **opts):
        ctx = self.context(**opts)
        x, info = ctx.solve(self.b, stream=self.stream)
        st = ctx.stats()
        ctx.close()
        return x, info, st

    def true_residual(self, x):
        import numpy as np
        xh = x.cpu().numpy()
        return float(np.linalg.norm(self.P.b - self.Kh @ xh) / np.linalg.norm(self.P.b))

    def timed_steps(self, steps, warmup, **opts):
        import torch
        for _ in range(warmup):
            self.step(**opts)
        torch.cuda.synchronize()
        infos, stats = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            x, info, st = self.step(**opts)
            infos.append(info)
            stats.append(st)
        torch.cuda.synchronize()
        T = (time.perf_counter() - t0) / steps
        return T, x, infos, stats


def local_solve_roofline(stats, traffic_key, precision, seed):
    launches = sum(s["local_solve_launches"] for s in stats)
    ms_ls = sum(s["ms_local_solve"] for s in stats)
    bytes_per_launch = stats[0]["local_solve_bytes"]
    achieved = bytes_per_launch / (ms_ls / launches * 1e-3) / 1e9 if launches else 0.0
    traffic = None
    rec = LOCAL_SOLVE_TRAFFIC.get((traffic_key, precision))
    if rec and rec["source_hash"] == local_solve_source_hash() and seed == 0:
        traffic = rec["bytes"]
    return {"kernel": "k_local_solve_wg (level-1 batched pivoted-LU forward/backward substitution, "
                      + ("FP64" if precision == "fp64" else "FP32") + " factors)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_launch": bytes_per_launch,
            "launches": launches, "avg_launch_us": ms_ls / launches * 1e3 if launches else None}


def local_solve_levels(stats):
    """Event-timed local solves of every Schwarz level (levels >= 2 run on a side stream beside the
    level-1 solves, so their rate is that of a shared GPU)."""
    out = []
    L = stats[0]["levels"]
    for l in range(8):
        launches = sum(s["local_solve_launches_level"][l] for s in stats)
        if not launches:
            continue
        ms = sum(s["ms_local_solve_level"][l] for s in stats) / launches
        b = stats[0]["local_solve_bytes_level"][l]
        out.append({"level": l + 1, "avg_launch_us": ms * 1e3, "bytes_per_launch": b,
                    "achieved_gbs": b / (ms * 1e-3) / 1e9, "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS})
    return out


def lu_rate(stats, precision):
    """Level-1 LU flops sum (2/3) n_i^3 over the event-timed level-1 LU kernels (median over steps).
    The flop count is the dense factorization's; the trailing updates skip tiles whose product is an
    exact zero, so this is a dense-equivalent rate."""
    import numpy as np
    ms = float(np.median([s["ms_lu"][0] for s in stats]))
    fl = stats[0]["factor_flops"][0]
    peak = FP64_MFMA_TFLOPS if precision == "fp64" else FP32_MFMA_TFLOPS
    tf = fl / (ms * 1e-3) / 1e12
    return {"flops_level1": fl, "ms_lu_kernels_level1": ms, "achieved_tflops": tf, "peak_tflops": peak,
            "frac": tf / peak, "bound": "mfma",
            "note": "dense-equivalent rate: (2/3) n^3 per block over the event-timed level-1 LU launches on "
                    "their stream (the rank-128 updates skip exact-zero tiles); the basis / Galerkin / coarse "
                    "chain runs concurrently on other streams"}


def apply_roofline(run, precision, n_apply=10):
    """Whole apply of eq. (2.2): the library's algorithmic bytes over the event-timed apply (all levels,
    side streams joined)."""
    import torch
    from harness import random_vector
    ctx = run.context(precision=precision)
    r = torch.as_tensor(random_vector(run.P.n, 3), device="cuda")
    z = torch.empty_like(r)
    with torch.cuda.stream(run.stream):
        ctx.apply(r, out=z, stream=run.stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(run.stream)
        for _ in range(n_apply):
            ctx.apply(r, out=z, stream=run.stream)
        e1.record(run.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / n_apply
    A = ctx.stats()["apply_bytes"]
    ctx.close()
    return {"bound": "hbm", "achieved": A / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": A / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_per_apply": A, "ms_per_apply": ms}


def spmv_roofline(ctx, P, x, stream, calls=50):
    """y = K x through the library, timed with HIP events on the launching stream: algorithmic bytes
    (CSR values, int32 columns read once per group of three rows that share them, int64 row pointers,
    x once, y; the library's count) over the mean duration; the plain CSR bytes (every row's columns)
    beside them."""
    import torch
    y = torch.empty_like(x)
    ctx.spmv(x, out=y, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(calls):
        ctx.spmv(x, out=y, stream=stream)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) / calls * 1e3
    csr_bytes = 12.0 * len(P.col) + 8.0 * (P.n + 1) + 16.0 * P.n
    nbytes = float(ctx.stats()["spmv_bytes"]) or csr_bytes
    return {"bound": "hbm", "achieved": nbytes / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_call": nbytes, "us_per_call": us,
            "plain_csr_bytes": csr_bytes, "plain_csr_gbs": csr_bytes / (us * 1e-6) / 1e9}


def solve_only(run, precision, n_solves, tune=False):
    """Setup amortized: solves on one context, eager applies against captured hipGraph applies."""
    import torch
    out = {}
    for graph in (False, True):
        ctx = run.context(precision=precision, graph=graph, tune=tune)
        ctx.solve(run.b, stream=run.stream)                 # warm-up (captures the graphs in graph mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_solves):
            x, info = ctx.solve(run.b, stream=run.stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n_solves
        out["graph" if graph else "eager"] = {"ms_per_solve": dt * 1e3, "solves_per_s": 1.0 / dt,
                                              "iterations": info["iterations"]}
        if not graph:
            out["spmv"] = spmv_roofline(ctx, run.P, run.b, run.stream)
        ctx.close()
    return out


def many_solve_leg(run, precision, ks=(1, 8, 32), tol=1e-1, reps=3):
    """The low-accuracy many-solve regime (section 3: the solver as a coarse solver invoked many times
    to a 1e-1 reduction): one setup, then batches of k right-hand sides solved in lockstep with one
    multi-right-hand-side apply per iteration (k = 1: plain gdsw_solve), setup amortized."""
    import numpy as np
    import torch
    from harness import random_vector
    ctx = run.context(precision=precision, tol=tol)
    out = {"tol": tol, "workload": f"setup once, FGMRES({RESTART}) to a 1e-1 relative residual per right-hand side"}
    kmax = max(ks)
    B = torch.as_tensor(np.stack([random_vector(run.P.n, 100 + q) for q in range(kmax)]), device="cuda")
    for k in ks:
        Bk = B[:k].contiguous()
        if k == 1:
            ctx.solve(Bk[0], stream=run.stream)
        else:
            ctx.solve_multi(Bk, stream=run.stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if k == 1:
                _, info = ctx.solve(Bk[0], stream=run.stream)
                its = [info["iterations"]]
            else:
                _, infos = ctx.solve_multi(Bk, stream=run.stream)
                its = [i["iterations"] for i in infos]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        # the preconditioner alone on k vectors
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        Z = torch.empty_like(Bk)
        if k == 1:
            ctx.apply(Bk[0], out=Z[0], stream=run.stream)
        else:
            ctx.apply_multi(Bk, out=Z, stream=run.stream)
        e0.record(run.stream)
        for _ in range(5):
            if k == 1:
                ctx.apply(Bk[0], out=Z[0], stream=run.stream)
            else:
                ctx.apply_multi(Bk, out=Z, stream=run.stream)
        e1.record(run.stream)
        e1.synchronize()
        ms_apply = e0.elapsed_time(e1) / 5
        out[f"k{k}"] = {"solves_per_s": k / dt, "ms_per_batch": dt * 1e3, "iterations": its,
                        "ms_apply_batch": ms_apply, "ms_apply_per_rhs": ms_apply / k}
    ctx.close()
    out["speedup_k32_vs_k1"] = out[f"k{kmax}"]["solves_per_s"] / out["k1"]["solves_per_s"]
    return out


def ablation(stream, seed=0, steps=2):
    """Mirror of Table 1 on seeded dies: 2, 3 and 4 levels at two part counts, FGMRES to 1e-8 (the
    preconditioner role) and to a 1e-1 reduction (the coarse-solver role); Effic_rel as the paper defines
    it (one GPU for every run, so the rank ratio is 1), T0 = three levels on the smaller die.  Also the
    overlap of two node layers and the additive combination of eq. (2.2)."""
    import numpy as np
    from harness import die_problem
    from paper_2606_01433_amd.metrics import effic_rel
    rows = []
    for shape in ((24, 12, 12), (32, 16, 16)):
        for levels in (2, 3, 4):
            P = die_problem(*shape, seed=seed, nu0=1.0, lam=1.0, n_exp=0.5, levels=levels)
            run = Runner(P, stream)
            for tol in (1e-8, 1e-1):
                T, x, infos, stats = run.timed_steps(steps, 1, tol=tol)
                st = stats[0]
                rows.append({"die": "x".join(map(str, shape)), "n_dofs": int(P.n), "levels": levels, "tol": tol,
                             "parts": st["parts"][:st["levels"]], "coarsest": st["n"][st["levels"] - 1],
                             "ms_per_step": T * 1e3, "ms_setup": st["ms_total"], "ms_solve": infos[-1]["ms_total"],
                             "iterations": infos[-1]["iterations"], "converged": bool(infos[-1]["converged"])})
                say("ablation", rows[-1]["die"], levels, tol, rows[-1]["iterations"], f"{T * 1e3:.1f} ms")
            del run
    for tol in (1e-8, 1e-1):
        base = [r for r in rows if r["die"] == "24x12x12" and r["levels"] == 3 and r["tol"] == tol][0]
        for r in rows:
            if r["tol"] == tol:
                r["effic_rel"] = effic_rel(r["ms_per_step"], r["n_dofs"], 1, base["ms_per_step"], base["n_dofs"], 1)
    extra = []
    P = die_problem(32, 16, 16, seed=seed, nu0=1.0, lam=1.0, n_exp=0.5, levels=3)
    run = Runner(P, stream)
    T, x, infos, stats = run.timed_steps(steps, 1, overlap=2)
    extra.append({"variant": "overlap 2 node layers, 3 levels, 32x16x16", "ms_per_step": T * 1e3,
                  "iterations": infos[-1]["iterations"], "max_local_order": stats[0]["max_ni"][0],
                  "converged": bool(infos[-1]["converged"])})
    for levels in (2, 3):
        Pl = P if levels == 3 else die_problem(32, 16, 16, seed=seed, nu0=1.0, lam=1.0, n_exp=0.5, levels=2)
        runl = Runner(Pl, stream)
        T, x, infos, stats = runl.timed_steps(1, 0, combine="additive", max_it=400)
        extra.append({"variant": f"additive combination, {levels} levels, 32x16x16", "ms_per_step": T * 1e3,
                      "iterations": infos[-1]["iterations"], "converged": bool(infos[-1]["converged"]),
                      "rel_residual": infos[-1]["rel_residual"]})
    return {"table1_mirror": rows, "variants": extra}


def multigrid_leg(stream, seed=0, steps=2, precision="fp64"):
    """Section 3's second role (Table 1, bottom): two-grid geometric multigrid for the refined 32x16x16 die
    (64x32x32 voxels) whose coarse problem, the 32x16x16 die, is solved by FGMRES preconditioned by the
    three-level GDSW method to a 1e-1 reduction; smoother: damped one-level restricted Schwarz on the fine
    2^3-voxel parts (2 pre, 2 post); FGMRES(150) on the fine system with the cycle as preconditioner to
    1e-8.  A step = both setups + the solve + destroy."""
    import numpy as np
    import torch
    from harness import die_problem
    from harness.problems import prolongation
    from paper_2606_01433_amd import gdsw
    t0 = time.perf_counter()
    Pc = die_problem(32, 16, 16, seed=seed, nu0=1.0, lam=1.0, n_exp=0.5, levels=3)
    Pf = die_problem(32, 16, 16, seed=seed, nu0=1.0, lam=1.0, n_exp=0.5, levels=2, refine=2)
    P = prolongation(Pc, Pf)
    say(f"multigrid pair assembled in {time.perf_counter() - t0:.1f} s: fine n = {Pf.n}, coarse n = {Pc.n}")
    rf, rc = Runner(Pf, stream), Runner(Pc, stream)

    def step():
        fine = rf.context(no_coarse=True, tol=1e-8, precision=precision)
        coarse = rc.context(tol=1e-1, precision=precision)
        mg = gdsw.MultiGrid(fine, coarse, P, nu_pre=2, nu_post=2, omega=1.0, stream=stream)
        x, info = mg.solve(rf.b, stream=stream)
        cnt = mg.counts()
        stf, stc = fine.stats(), coarse.stats()
        mg.close()
        fine.close()
        coarse.close()
        return x, info, cnt, stf, stc

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x, info, cnt, stf, stc = step()
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / steps
    return {"workload": f"two-grid geometric multigrid, {precision} factors: fine = refined 32x16x16 die "
                        f"(64x32x32 voxels, {Pf.n} dofs, one-level restricted Schwarz smoother on "
                        f"{stf['parts'][0]} parts, 2 + 2 steps), coarse = the 32x16x16 die ({Pc.n} dofs, "
                        f"three-level GDSW, FGMRES to 1e-1); FGMRES({RESTART}) to 1e-8 on the fine system",
            "solves_per_s": 1.0 / T, "ms_per_step": T * 1e3, "outer_iterations": info["iterations"],
            "coarse_iterations_per_cycle": cnt["coarse_iterations"] / max(1, cnt["cycles"]),
            "true_rel_residual": rf.true_residual(x), "ms_solve": info["ms_total"],
            "ms_setup_fine_smoother": stf["ms_total"], "ms_setup_coarse_gdsw": stc["ms_total"]}


def workload_leg(name, precision, steps, warmup, stream, seed=0, P=None):
    """setup + solve + destroy steps of one workload in one precision."""
    P = make_problem(name, seed) if P is None else P
    run = Runner(P, stream)
    T, x, infos, stats = run.timed_steps(steps, warmup, precision=precision, profile=True)
    st = stats[0]
    return run, x, {
        "workload": describe(name, precision), "n_dofs": int(P.n), "nnz": int(len(P.col)),
        "solves_per_s": 1.0 / T, "ms_per_step": T * 1e3, "steps": steps,
        "iterations": infos[-1]["iterations"], "true_rel_residual": run.true_residual(x),
        "parts": st["parts"][:st["levels"]], "level_dofs": st["n"][:st["levels"]],
        "ms_setup": st["ms_total"], "ms_solve": infos[-1]["ms_total"],
        "roofline_local_solve": local_solve_roofline(stats, name, precision, seed),
        "lu_kernels": lu_rate(stats, precision)}


def serving_bench(seed=0, n_requests=16, loads=(0.5, 0.8, 0.95), partial_path=None):
    """Poisson streams of Picard-step solves over seeded dies of 7 sizes (16^3 .. 64x32x32) with Carreau
    n ~ U[0.3, 0.9] and lambda = 10^U[-1, 1]: FP32-factor serving with 4 slots against FP64 with 4 slots
    and FP64 one at a time, at arrival rates rho x the FP64 one-at-a-time capacity."""
    import numpy as np
    from harness import die_problem
    from paper_2606_01433_amd.serving import Server, Request, summarize
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    pool = []
    for k, nx in enumerate((16, 24, 32, 40, 48, 56, 64)):
        ny = max(16, nx // 2)
        n_exp = float(rng.uniform(0.3, 0.9))
        lam = float(10.0 ** rng.uniform(-1.0, 1.0))
        levels = 3 if nx * ny * ny <= 16 * 16 * 16 * 2 else 4
        pool.append(die_problem(nx, ny, ny, seed=seed + k, nu0=1.0, lam=lam, n_exp=n_exp, levels=levels))
    say("serving pool assembled:", [p.n for p in pool])
    # service time of the plain FP64 path, one request at a time (also warms every size up)
    srv = Server(max_active=1)
    t0 = time.perf_counter()
    for k, P in enumerate(pool):
        srv.submit(Request(-1 - k, P, tol=1e-8)).wait()
    t_mean = (time.perf_counter() - t0) / len(pool)
    srv.close()
    capacity = 1.0 / t_mean

    def stream(server, picks, gaps, **opts):
        reqs = []
        t_start = time.perf_counter()
        t_next = t_start
        for k in range(len(picks)):
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            reqs.append(server.submit(Request(k, pool[int(picks[k])], arrival=time.perf_counter(), **opts)))
            t_next += gaps[k]
            if (k + 1) % 20 == 0:
                say(f"  submitted {k + 1}/{len(picks)}")
        for k, r in enumerate(reqs):          # progress while the backlog drains
            r.wait()
            say(f"  completed {k + 1}/{len(reqs)} ({(r.latency or 0) * 1e3:.0f} ms)")
        t_end = time.perf_counter()
        server.close()
        return reqs, summarize(reqs, t_start, t_end)

    out = {"requests_per_load": n_requests, "fp64_one_at_a_time_capacity_hz": capacity,
           "pool": "seeded dies nx in {16,24,32,40,48,56,64}, ny = nz = max(16, nx/2); Carreau n ~ U[0.3,0.9], "
                   f"lambda = 10^U[-1,1]; three levels up to 32x16x16, four above; FGMRES({RESTART}) to 1e-8; "
                   "FP32 slots admitted against a 200 GB footprint budget",
           "loads": {}}
    for rho in loads:
        picks = rng.integers(0, len(pool), n_requests)
        gaps = rng.exponential(1.0 / (rho * capacity), n_requests)
        say(f"serving rho = {rho}")
        srv32 = Server(budget_bytes=200 * 2 ** 30, max_active=4)
        r32, s32 = stream(srv32, picks, gaps, tol=1e-8, restart=RESTART, precision="mixed")
        s32["peak_active"] = srv32.peak_active
        srv64 = Server(budget_bytes=200 * 2 ** 30, max_active=4)
        r64, s64 = stream(srv64, picks, gaps, tol=1e-8, restart=RESTART)
        s64["peak_active"] = srv64.peak_active
        _, s1 = stream(Server(max_active=1), picks, gaps, tol=1e-8, restart=RESTART)
        pairs = [(a, b_) for a, b_ in zip(r32, r64) if a.x is not None and b_.x is not None]
        err = max([float(np.linalg.norm(a.x - b_.x) / np.linalg.norm(b_.x)) for a, b_ in pairs] or [float("nan")])
        for name_, rs in (("fp32_factors_4_slots", r32), ("fp64_4_slots", r64)):
            msgs = sorted({str(r.error)[:200] for r in rs if r.error is not None})
            if msgs:
                say(f"  {name_}: failed requests: {msgs}")
        out["loads"][str(rho)] = {"arrival_rate_hz": rho * capacity, "fp32_factors_4_slots": s32,
                                  "fp64_4_slots": s64, "fp64_one_at_a_time": s1,
                                  "max_rel_diff_fp32_vs_fp64_solution": err}
        if partial_path:
            with open(partial_path, "a") as f:
                f.write(json.dumps({"rho": rho, **out["loads"][str(rho)]}) + "\n")
    return out


def cpu_baseline(P, gpu_iterations_here, scale_to=None, budget_its=None):
    """The oracle (FP64 NumPy/SciPy) on the host: its full three-level setup and FGMRES solve of the
    32x16x16 die, with BLAS limited to one thread and with all host cores; optionally extrapolated
    linearly in the number of dofs (and in the iteration count) to the headline workload."""
    from threadpoolctl import threadpool_limits, threadpool_info
    import oracle
    K = P.K()
    res = {}
    for label, limit in (("single", 1), ("all", None)):
        with threadpool_limits(limits=limit):
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
            t0 = time.perf_counter()
            H = oracle.setup(P)
            t1 = time.perf_counter()
            _, info = oracle.fgmres(lambda v: K @ v, lambda v: oracle.apply(H, v), P.b, tol=1e-8,
                                    restart=RESTART, max_it=budget_its or 1000)
            t2 = time.perf_counter()
        res[label] = dict(setup=t1 - t0, per_it=(t2 - t1) / max(1, info["iterations"]), its=info["iterations"],
                          threads=threads)
        say(f"oracle {label}: setup {t1 - t0:.1f} s, {info['iterations']} its in {t2 - t1:.1f} s ({threads} threads)")
    out = {"kind": "oracle", "host_cpu_count": os.cpu_count()}
    for label in ("single", "all"):
        r = res[label]
        t_here = r["setup"] + r["per_it"] * gpu_iterations_here
        entry = {"solves_per_s_32x16x16": 1.0 / t_here, "cores": r["threads"], "ms_setup": r["setup"] * 1e3,
                 "ms_per_iteration": r["per_it"] * 1e3, "iterations": r["its"]}
        if scale_to:
            f = scale_to["n"] / P.n
            entry["solves_per_s_extrapolated"] = 1.0 / (f * r["setup"] + f * r["per_it"] * scale_to["iterations"])
        out[label] = entry
    main = out["single"]
    out["value"] = main["solves_per_s_extrapolated"] if scale_to else main["solves_per_s_32x16x16"]
    out["unit"] = "solves/s"
    out["cores"] = main["cores"]
    out["sample"] = (f"oracle's full three-level setup + complete FGMRES({RESTART}) solve to 1e-8 of the 32x16x16 die "
                     f"({P.n} dofs; {res['single']['its']} iterations)"
                     + (f", extrapolated linearly in dofs ({scale_to['n']}) and iterations "
                        f"({scale_to['iterations']}) to the headline workload" if scale_to else ""))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--headline", default="die96x48x48", choices=list(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="headline precision (default: mixed for die96x48x48, fp64 otherwise)")
    ap.add_argument("--no-legs", action="store_true", help="headline only (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=16)
    ap.add_argument("--serving-only", action="store_true", help="only the serving streams")
    ap.add_argument("--serving-loads", default="0.5,0.8,0.95", help="comma-separated rho values")
    ap.add_argument("--serving-partial", default=None, help="append each load's result to this file")
    ap.add_argument("--ablation", action="store_true", help="only the Table 1 mirror (levels, overlap, combination)")
    ap.add_argument("--multigrid-only", action="store_true", help="only the multigrid-role leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is not part of this build",
              file=sys.stderr)
        sys.exit(2)
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
    stream = torch.cuda.current_stream()
    if args.ablation:
        print(json.dumps(ablation(stream, args.seed)), flush=True)
        return
    if args.multigrid_only:
        print(json.dumps(multigrid_leg(stream, args.seed)), flush=True)
        return
    if args.serving_only:
        loads = tuple(float(x) for x in args.serving_loads.split(","))
        print(json.dumps(serving_bench(args.seed, n_requests=args.serving_requests, loads=loads,
                                       partial_path=args.serving_partial)), flush=True)
        return
    name = args.headline
    precision = args.precision or ("mixed" if name == "die96x48x48" else "fp64")
    P = make_problem(name, args.seed)
    run = Runner(P, stream)
    tune = "all" if name == "die96x48x48" else False
    say("headline steps")
    T, x, infos, stats = run.timed_steps(args.steps, args.warmup, precision=precision, profile=True, tune=tune)
    st0 = stats[0]
    res = run.true_residual(x)
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
        "dtype": "f64" if precision == "fp64" else "f32 local factors / f64 Krylov",
        "data": "synthetic (seeded die-like voxel channel, Carreau viscosity at a seeded linearization point)",
        "config": {"workload": describe(name, precision) + (", autotuned local solves and LU variants" if tune else ""),
                   "n_dofs": int(P.n), "nnz": int(len(P.col)), "parts": st0["parts"][:st0["levels"]],
                   "level_dofs": st0["n"][:st0["levels"]], "iterations": infos[-1]["iterations"],
                   "second_gram_schmidt_passes": infos[-1]["reorthogonalizations"],
                   "local_solve_waves_per_matrix": st0["ls_waves"][:st0["levels"] - 1],
                   "true_rel_residual": res, "precision": precision,
                   "ms_setup": float(sum(s["ms_total"] for s in stats) / len(stats)),
                   "ms_solve": float(sum(i["ms_total"] for i in infos) / len(infos)),
                   "ms_setup_phases": {"host_maps": st0["ms_maps"], "host_prep": st0["ms_extract"],
                                       "factor": st0["ms_factor"], "basis_galerkin": st0["ms_basis"],
                                       "coarsest": st0["ms_coarse"]},
                   "factor_bytes": st0["factor_bytes"][:st0["levels"] - 1],
                   "lu_variant_per_level": st0["lu_variant"][:st0["levels"] - 1]},
        "roofline": local_solve_roofline(stats, name, precision, args.seed),
        "factor": lu_rate(stats, precision),
        "local_solves_per_level": local_solve_levels(stats),
    }
    say(f"headline {1.0 / T:.3f} solves/s, {infos[-1]['iterations']} its, residual {res:.2e}")
    if not args.no_legs:
        say("headline with the library's default restart")
        T30, _, infos30, _ = run.timed_steps(1, 0, precision=precision, tune=tune, restart=30)
        out["headline_restart30"] = {"solves_per_s": 1.0 / T30, "ms_per_step": T30 * 1e3,
                                     "iterations": infos30[-1]["iterations"], "restarts": infos30[-1]["restarts"],
                                     "ms_solve": infos30[-1]["ms_total"]}
    if not args.no_legs:
        say("whole-apply roofline")
        out["apply"] = apply_roofline(run, precision)
        say("solve only")
        out["solve_only"] = solve_only(run, precision, n_solves=1, tune=tune)
        del run, P
        say("precision workload 64x32x32")
        P64 = make_problem("die64x32x32", args.seed)
        r64, x64, leg64 = workload_leg("die64x32x32", "fp64", 2, 1, stream, args.seed, P=P64)
        _, x32, leg32 = workload_leg("die64x32x32", "mixed", 2, 1, stream, args.seed, P=P64)
        import numpy as np
        a, b_ = x32.cpu().numpy(), x64.cpu().numpy()
        leg32["rel_diff_vs_fp64_solution"] = float(np.linalg.norm(a - b_) / np.linalg.norm(b_))
        leg32["speedup_vs_fp64"] = leg32["solves_per_s"] / leg64["solves_per_s"]
        out["precision_64x32x32"] = {"fp64": leg64, "fp32_factors": leg32,
                                     "apply_fp64": apply_roofline(r64, "fp64"),
                                     "apply_fp32_factors": apply_roofline(r64, "mixed")}
        del r64, P64
        say("three-level FP64 32x16x16")
        P32 = make_problem("die32x16x16", args.seed)
        r32, _, leg = workload_leg("die32x16x16", "fp64", 5, 2, stream, args.seed, P=P32)
        leg["solve_only"] = solve_only(r32, "fp64", n_solves=5)
        out["fp64_32x16x16"] = leg
        say("many-solve regime (multi-right-hand-side solves)")
        out["many_solve_32x16x16"] = many_solve_leg(r32, "fp64")
        say("multigrid role (two-grid, GDSW coarse solver)")
        out["multigrid_64x32x32"] = multigrid_leg(stream, args.seed)
        if not args.no_serving:
            out["serving"] = serving_bench(args.seed, n_requests=args.serving_requests)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(P32, leg["iterations"],
                                               scale_to={"n": out["config"]["n_dofs"],
                                                         "iterations": out["config"]["iterations"]}
                                               if name != "die32x16x16" else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
