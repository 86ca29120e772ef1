"""Benchmark of the MI355X restarted-PDHG solver.

Default line: the large sparse QP (n = 1e7 R+ columns, m = 5e6 rows, 5.1e7
nonzeros with power-law column degrees, 10% slack columns; Q sparse with 3e7
nonzeros), the one workload whose working set (~3.5 GB) is far larger than
the caches, so the HBM roofline is the bound.  One step = one solve from a
cold start over a fixed budget of outer iterations (--budget, default 256;
every row of the hot path runs: A^T product, Jacobi projected-BB inner loop
with the P product, A product and dual update, reflected-Halpern update,
restarts, device KKT checks).  The method does not reach 1e-4 on this
instance within minutes, so the line reports iterations/s over the budget and
the relative KKT reached; time to tolerance is reported for the mixed-cone
workload among the variants.  Setup (rescaling, A^T, power iteration) is
outside the timed region; problem data is resident in HBM when timing starts.

Variants (default line): FP32 bulk on the same instance and budget, the
mixed-cone SOCP/QCQP solve to 1e-6 in FP64 and FP32 bulk, and the batch of
4096 portfolio QPs against a per-instance loop.  --workload selects another
workload as the main line (mixed_cone, fisher, tiny_qp, portfolio_batch,
fisher_warm, mlp_train, fisher_paper --buyers N).

cpu_baseline: the oracle as it stands, one thread, on the first outer
iterations of the same instance, run in a child process started before the
GPU work (its setup, which is not timed, overlaps the GPU runs).

Prints one JSON line.  `--gpus N` with N > 1 is rejected: the solver runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
BF16_DENSE_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix-core peak

# HBM traffic of one solve_kernel launch on the default workload, from two
# rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE scaled by the factors
# that make a 256 MiB device copy read and write 256 MiB), as a dict with the
# workload, grid, iterations per launch, the kernel sources' sha256 and
# bytes_per_launch.  Valid only for the recorded kernel sources, grid and
# iteration count; otherwise (and while None) the bench reports null.
MEASURED_TRAFFIC = {
    "workload": "large_sparse_qp", "grid": 512, "iterations": 256,
    "sources_sha256": "ada668ab3d6c519d6e411bf50b7f4fc254eddc242767f17a5bab3e6c08f8bb37",
    # FETCH_SIZE 3,561,594,958.7 KiB x 1.99974 (copy calibration) + WRITE_SIZE
    # 478,528,850.6 KiB x 1.0, per 256-iteration launch of solve_kernel_lin
    # (degree coordinate order)
    "bytes_per_launch": 7783200183547.8,
}
KERNEL_SOURCES = ("solver.hip", "cones.hpp", "common.hpp", "api.cpp", "host_setup.cpp")


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_09159_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()
METRIC = "time-to-1e-6 rel KKT (s) + PDHG iters/s; FP32/batched/warm vs plain FP64"


def workload(name):
    from instances import synth
    if name == "mixed_cone":
        return synth.mixed_cone(seed=0), "mixed-cone SOCP/QCQP n=1e5 m=5e4"
    if name == "tiny_qp":
        return synth.tiny_qp(0), "tiny QP n=200 m=100"
    if name == "fisher":
        return synth.fisher(seed=1_000_001), "Fisher market 1000 buyers x 500 goods (EXP)"
    if name == "large_sparse_qp":
        return synth.large_sparse_qp(seed=0), "large sparse QP n=1e7 m=5e6"
    if name == "portfolio_batch":
        return synth.portfolio_batch(4096), "4096 portfolio QPs n~U[50,2000] k~U[5,20]"
    raise ValueError(name)


def method_bytes_model(prob, iters, inner_total, checks):
    """Algorithmic HBM bytes of the method over `iters` outer iterations
    with `inner_total` projected-BB steps and `checks` KKT checks: every
    product reads its matrix once (FP64 value + int32 column, 12 bytes per
    nonzero, and 4 bytes per row pointer), its input vector once (an ideal
    gather) and writes its output once; A z is kept by recurrence.
        A^T product + prox input     12 nnz(A) + 4n + 8m + 16n
        A product + dual candidate   12 nnz(A) + 4m + 8n + 40m
        reflected-Halpern update     32n + 64m
        diagonal prox                32n
        each JBB inner step          12 nnz(P) + 16 r n + 92n
    so 24 nnz(A) + 60n + 116m per outer iteration plus the prox; a check
    adds one A^T product and one Q product (12 nnz(P) + 16 r n + 16n)."""
    n, m = prob.n, prob.m
    nnzA = prob.A.nnz
    nnzP = 0 if prob.P is None else prob.P.nnz
    r = 0 if prob.R is None else prob.R.shape[0]
    diag_q = r == 0 and (prob.P is None or np.all(prob.P.tocoo().row == prob.P.tocoo().col))
    b_at = 12 * nnzA + 4 * n + 8 * m + 16 * n
    b_a = 12 * nnzA + 4 * m + 8 * n + 40 * m
    b_halpern = 32 * n + 64 * m
    b_q = 12 * nnzP + 16 * r * n + 16 * n
    prox = iters * 32 * n if diag_q else inner_total * (12 * nnzP + 16 * r * n + 92 * n)
    return iters * (b_at + b_a + b_halpern) + prox + checks * (b_at + b_q)


def bytes_model(prob, iters, inner_total, checks):
    """Algorithmic HBM bytes of the solver kernel for `iters` outer
    iterations with `inner_total` projected-BB steps in total (FP64 values,
    int32 column indices, int64 row pointers; every matrix read once per use,
    every vector read or written once per pass, ideal gathers)."""
    n, m = prob.n, prob.m
    nnzA = prob.A.nnz
    nnzP = 0 if prob.P is None else prob.P.nnz
    r = 0 if prob.R is None else prob.R.shape[0]
    nc = sum(d for k, s, d, a in prob.cones if k not in ("free", "nonneg"))
    spmv_at = 12 * nnzA + 8 * (n + 1) + 8 * m
    spmv_a = 12 * nnzA + 8 * (m + 1) + 8 * n
    spmv_p = (12 * nnzP + 8 * (n + 1) + 8 * n) if nnzP else 0
    diag_q = r == 0 and (prob.P is None or np.all(prob.P.tocoo().row == prob.P.tocoo().col))
    p6 = spmv_a + 72 * m + 32 * n
    if diag_q:
        per_iter = spmv_at + 33 * n + 24 * nc + p6
        inner_bytes = 0
    else:
        per_iter = spmv_at + spmv_p + 8 * r * n + 57 * n + 32 * nc + 8 * r * nc + p6
        first = iters                                     # one first step per iteration
        inner_bytes = max(inner_total - first, 0) * (spmv_p + 16 * r * n + 121 * n + 16 * nc)
    check_bytes = checks * (spmv_at + spmv_p + 8 * r * n + 41 * n + 24 * nc + 40 * m + 32 * n)
    return iters * per_iter + inner_bytes + check_bytes


def footprint_bytes(prob):
    """Device working set of one solve: A and A^T (values, int32 columns,
    int64 row pointers), P, the dense factor R, and the iteration vectors
    (about 17 of length n and 8 of length m, FP64)."""
    nnz = prob.A.nnz
    by = 2 * 12.0 * nnz + 8.0 * (prob.m + 1) + 8.0 * (prob.n + 1)
    if prob.P is not None:
        by += 12.0 * prob.P.nnz + 8.0 * (prob.n + 1)
    if prob.R is not None:
        by += 8.0 * prob.R.size
    return by + 8.0 * (17 * prob.n + 8 * prob.m)


def same_footprint_context(prob, s_per_iter, reps=20):
    """Per-iteration time and the bandwidth of a plain device copy whose
    source and destination together span the solve's working set: for a
    cache-resident instance this, not the 8 TB/s HBM peak, is what a
    bandwidth-bound kernel of the same footprint could reach."""
    import torch
    fb = footprint_bytes(prob)
    half = max(int(fb // 16), 1)             # FP64 elements in each of src and dst
    src = torch.ones(half, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return {"us_per_iteration": 1e6 * s_per_iter, "footprint_bytes": fb,
            "same_footprint_copy_GBs": 2.0 * 8.0 * half / t / 1e9}


def log(msg):
    """Progress of the phases, on stderr (the JSON line goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def cpu_baseline(prob, budget_s=15.0):
    """The oracle as it stands, single thread, on the first outer iterations
    of the same instance; iterations/s."""
    from threadpoolctl import threadpool_limits
    from oracle import pdhg
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        S = pdhg.setup(prob, pdhg.Settings())
        t_setup = time.perf_counter() - t0
        log(f"oracle setup done ({t_setup:.1f} s)")
        iters = 2
        while True:
            t0 = time.perf_counter()
            r = pdhg.solve(prob, pdhg.Settings(max_iter=iters), S=S)
            dt = time.perf_counter() - t0
            log(f"oracle: {r.iterations} outer iterations in {dt:.1f} s")
            if dt >= 0.6 * budget_s or iters >= 100000 or r.status != "MAX_ITER":
                break
            grow = min(max(1.25, budget_s / max(dt, 1e-3)), 8.0)
            iters = int(min(iters * grow, 100000))
    return dict(value=r.iterations / dt, unit="PDHG iters/s", cores=1, kind="oracle",
                host_cores=host_cores(),
                sample=f"first {r.iterations} outer iterations of the same instance "
                       f"({dt:.1f}s, {r.inner_iterations} inner steps; setup {t_setup:.1f}s "
                       f"excluded); NumPy/SciPy FP64, BLAS pinned to 1 thread")


def start_cpu_child(args):
    """The cpu_baseline leg in a child process (no GPU use), so the oracle's
    setup overlaps the GPU runs; returns the Popen handle."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", "--workload", args.workload,
           "--cpu-budget", str(args.cpu_budget)]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, env=env, text=True)


def finish_cpu_child(proc):
    out, _ = proc.communicate()
    if proc.returncode != 0:
        return {"error": f"oracle child exited with {proc.returncode}"}
    return json.loads(out.strip().splitlines()[-1])


def bench_batch(args, probs, wname):
    """Batched portfolio QPs: one graph-replayed persistent launch for all
    instances against a host loop of single-instance pdhcg_solve calls (the
    plain FP64 solver, each launch on its own cooperative grid) at the same
    tolerance.  Step sizes of the loop handles are taken from the batch so both
    run the same iterations."""
    import torch
    import paper_2608_09159_amd as pkg
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    h = pkg.setup_batch(probs, tol=args.tol, time_kernels=1, stream=stream.cuda_stream)
    setup_s = time.perf_counter() - t0
    etas = [h.scaling(i)["eta"] for i in range(len(probs))]
    for _ in range(args.warmup):
        h.solve()
    torch.cuda.synchronize()
    walls, runs = [], []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        runs.append(h.solve())
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    h.free()
    last = runs[-1]
    iters = sum(r["iterations"] for r in last)
    inner = sum(r["inner_iterations"] for r in last)
    ksum = [r[0]["kernel_s"] for r in runs]
    wall = float(np.median(walls))
    kmed = float(np.median(ksum))
    alg = sum(bytes_model(p, r["iterations"], r["inner_iterations"],
                          math.ceil(r["iterations"] / 64) + r["restarts"] + 1)
              for p, r in zip(probs, last))
    st = [r["status"] for r in last]
    # per-instance loop (sample of instances when --loop-sample < count)
    k = min(args.loop_sample, len(probs))
    idx = np.linspace(0, len(probs) - 1, k).round().astype(int) if k < len(probs) else np.arange(len(probs))
    hs = [pkg.setup(probs[i], tol=args.tol, a_norm=0.998 / etas[i], stream=stream.cuda_stream)
          for i in idx]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop_iters = 0
    for hh in hs:
        loop_iters += hh.solve()["iterations"]
    torch.cuda.synchronize()
    loop_wall = (time.perf_counter() - t0) * len(probs) / k
    for hh in hs:
        hh.free()
    out = {
        "metric": METRIC,
        "value": iters / wall,
        "unit": "PDHG iters/s (summed over instances)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wname, "instances": len(probs), "sum_n": int(sum(p.n for p in probs)),
                   "tol": args.tol, "precision": "fp64"},
        "time_to_tol_s": wall,
        "statuses": {s: st.count(s) for s in sorted(set(st))},
        "iterations_total": iters, "inner_total": inner,
        "setup_s": setup_s,
        "loop_baseline": {"time_to_tol_s": loop_wall, "instances_timed": int(k),
                          "iterations_total_timed": int(loop_iters),
                          "kind": "host loop of pdhcg_solve (one handle per instance)"},
        "speedup_vs_loop": loop_wall / wall,
        "roofline": {"bound": "hbm", "achieved": alg / kmed / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg / kmed / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "batch_kernel (graph: reset + batch + gather)",
                     "kernel_avg_launch_ms": 1e3 * kmed, "launch": [last[0]["grid_dim"], last[0]["block_dim"]]},
    }
    return out


def fp32_variant(prob, args, t64, g64):
    """The same solve in FP32-bulk mode with the FP64 polish, timed like the
    FP64 solve; error of its result against the FP64 GPU result."""
    import torch
    import paper_2608_09159_amd as pkg
    stream = torch.cuda.current_stream()
    h = pkg.setup(prob, tol=args.tol, precision="fp32", time_kernels=1, stream=stream.cuda_stream)
    for _ in range(args.warmup):
        h.solve()
    torch.cuda.synchronize()
    walls, r = [], None
    for _ in range(args.steps):
        t0 = time.perf_counter()
        r = h.solve()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    h.free()
    t32 = float(np.median(walls))
    return {"time_to_tol_s": t32, "speedup_vs_fp64": t64 / t32, "status": r["status"],
            "iterations": r["iterations"], "polish_iterations": r["polish_iterations"],
            "rel_kkt": max(r["rel_primal"], r["rel_dual"], r["rel_gap"]),
            "x_rel_err_vs_fp64": float(np.linalg.norm(r["x"] - g64["x"]) / np.linalg.norm(g64["x"])),
            "obj_rel_diff_vs_fp64": abs(r["primal_obj"] - g64["primal_obj"]) / max(1.0, abs(g64["primal_obj"]))}


def bench_warm(args):
    """Learned warm start on the Fisher family (1000 buyers x 500 goods):
    label a reduced training set with batched solves, train the network with
    the library's BF16 matrix-core kernels, then solve held-out seeds cold and
    warm-started to the same tolerance."""
    from paper_2608_09159_amd import warmstart as W
    fam = W.FisherFamily()
    ntr = args.train_instances
    model, info = W.build_and_train(fam, list(range(1, ntr + 1)), tol=args.tol, epochs=args.epochs,
                                    lr=args.lr, log=log)
    log(f"trained: loss {info['loss'][0]:.4f} -> {info['loss'][-1]:.4f}")
    try:
        ev = W.evaluate(model, fam, list(range(1_000_001, 1_000_001 + args.eval_instances)), tol=args.tol,
                        timed=args.timed, log=log)
    finally:
        model.free()
    out = {
        "metric": METRIC, "value": ev["speedup_median"], "unit": "median wall-clock speedup warm vs cold",
        "n_gpus": 1, "steps": args.eval_instances, "warmup": 0,
        "ms_per_step": 1e3 * ev["warm_time_median_s"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 solve, bf16/fp32 network", "data": "synthetic",
        "config": {"workload": "learned warm start, Fisher market 1000 buyers x 500 goods",
                   "train_instances": ntr, "train_instances_note": "reduced from 20,000 (labelling budget)",
                   "network": [51000, 512, 512, 56500], "epochs": args.epochs, "lr": args.lr,
                   "held_out": args.eval_instances, "tol": args.tol},
        "train": {k: v for k, v in info.items() if k != "loss"},
        "train_loss_first_last": [info["loss"][0], info["loss"][-1]],
        "eval": ev,
    }
    print(json.dumps(out), flush=True)


def mlp_step_bytes(dims, B):
    """Algorithmic HBM bytes of one training step: every operand read and
    every result written once (BF16 activations, signals and weight copies,
    FP32 input conversion, output, weight gradients and Adam state).  Split-K
    partial tiles are implementation traffic and not counted."""
    L = len(dims) - 1
    by = 4.0 * B * dims[0] + 2.0 * B * dims[0]                  # input to BF16
    for l in range(L):
        a, b = dims[l], dims[l + 1]
        out = 4.0 * B * b if l == L - 1 else 2.0 * B * b
        by += 2.0 * B * a + 2.0 * a * b + out                    # forward
    dl = dims[-1]
    by += 4.0 * B * dl + 4.0 * B * dl + 2.0 * B * dl             # loss and dZ_L
    for l in range(L - 1, -1, -1):
        a, b = dims[l], dims[l + 1]
        by += 2.0 * B * a + 2.0 * B * b + 4.0 * a * b            # dW = H^T dZ
        by += 2.0 * B * b + 4.0 * b                              # db
        if l > 0:
            by += 2.0 * B * b + 2.0 * a * b + 2.0 * B * a + 2.0 * B * a   # dH, mask, dZ_{l-1}
    params = sum(a * b + b for a, b in zip(dims[:-1], dims[1:]))
    by += 30.0 * params                                          # Adam: w, g, m, v in; w, m, v, BF16 w out
    return by


def bench_mlp(args):
    """Training steps of the full-size warm-start network (51,000 -> 512 ->
    512 -> 56,500, batch 256) on synthetic data: the BF16 matrix-core GEMMs,
    epilogues and Adam.  FLOPs counted: 6 x batch x sum of layer products
    (forward, and the two backward products)."""
    import torch
    import paper_2608_09159_amd as pkg
    dims, B = [51000, 512, 512, 56500], 256
    rng = np.random.default_rng(0)
    net = pkg.MLP(dims, B)
    for l, (a, b) in enumerate(zip(dims[:-1], dims[1:])):
        net.set_params(l, (rng.standard_normal((a, b)) * np.sqrt(2.0 / a)).astype(np.float32),
                       np.zeros(b, np.float32))
    X = torch.randn(B, dims[0], device="cuda")
    Y = torch.randn(B, dims[-1], device="cuda")
    for _ in range(args.warmup):
        net.train_step(X, Y, lr=1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(X, Y, lr=1e-4)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    net.free()
    flops = 6.0 * B * sum(a * b for a, b in zip(dims[:-1], dims[1:]))
    tf = flops * args.steps / wall / 1e12
    step_bytes = mlp_step_bytes(dims, B)
    gbs = step_bytes * args.steps / wall / 1e9
    out = {"metric": "warm-start network training throughput", "value": tf, "unit": "TFLOP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)",
           "data": "synthetic", "config": {"workload": "warm-start network 51000-512-512-56500, batch 256"},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                        "algorithmic_bytes_per_step": step_bytes,
                        "mfma_tflops": tf, "mfma_frac": tf / BF16_DENSE_PEAK_TFLOPS,
                        "note": "whole train step (GEMMs, split-K reductions, epilogues, Adam) per wall "
                                "time; at the HBM peak the step's bytes take about 9x longer than its FLOPs "
                                "at the BF16 matrix-core peak, so HBM is the bound"}}
    print(json.dumps(out), flush=True)


def timed_solves(prob, args, budget, precision="fp64", verbose=0):
    """Setup, warm-up and the timed solves of one instance on torch's current
    stream; returns (runs, wall seconds of the timed solves, setup seconds)."""
    import torch
    import paper_2608_09159_amd as pkg
    stream = torch.cuda.current_stream()
    extra = {"max_iter": budget} if budget > 0 else {}
    t0 = time.perf_counter()
    h = pkg.setup(prob, tol=args.tol, time_kernels=1, stream=stream.cuda_stream, precision=precision,
                  verbose=verbose, **extra)
    setup_s = time.perf_counter() - t0
    log(f"setup done ({setup_s:.1f} s, {precision})")
    for _ in range(args.warmup):
        w = h.solve()
        log(f"warm-up solve: {w['status']} {w['iterations']} it in {w['solve_s']:.2f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [h.solve() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h.free()
    return runs, wall, setup_s


def solver_kernel_name(prob, precision, grid):
    """The library's solver kernel for this solve: FP32 bulk, one workgroup,
    the implementation-form features (row bounds, boxes, fixed-middle EXP),
    or, without cone blocks, the cone-free kernel at two workgroups per CU."""
    kinds = {k for k, _, _, _ in prob.cones}
    ext = getattr(prob, "row_lo", None) is not None or bool(kinds & {"box", "exp1"})
    cones = bool(kinds & {"soc", "rsoc", "exp", "pow", "exp1"})
    if precision == "fp32":
        return "solve_kernel_f32" + ("" if cones else "_lin") + ("_ext" if ext else "")
    if grid == 1:
        return "solve_kernel_one_ext" if ext else "solve_kernel_one"
    if ext:
        return "solve_kernel_ext" if cones else "solve_kernel_lin_ext"
    return "solve_kernel" if cones else "solve_kernel_lin"


def rel_kkt(r):
    return max(r["rel_primal"], r["rel_dual"], r["rel_gap"])


def fp32_budget_variant(prob, args, budget, wall64, last64):
    """FP32 bulk on the same instance and iteration budget: time per
    iteration against FP64, the relative KKT reached, and the distance of
    its iterate from the FP64 one at the same iteration count."""
    runs, wall, _ = timed_solves(prob, args, budget, precision="fp32")
    r = runs[-1]
    return {"iterations": r["iterations"], "time_per_iteration_ms": 1e3 * wall / sum(x["iterations"] for x in runs),
            "speedup_per_iteration_vs_fp64": wall64 / wall,
            "rel_kkt": rel_kkt(r), "rel_kkt_fp64": rel_kkt(last64), "status": r["status"],
            "x_rel_err_vs_fp64": float(np.linalg.norm(r["x"] - last64["x"]) / max(np.linalg.norm(last64["x"]), 1e-300)),
            "kernel_ms_per_iteration": 1e3 * sum(x["kernel_s"] for x in runs) / sum(x["iterations"] for x in runs)}


def mixed_cone_variant(args):
    """The mixed-cone SOCP/QCQP instance solved to the tolerance in FP64 and
    in FP32 bulk with the FP64 polish."""
    prob, wname = workload("mixed_cone")
    runs, wall, _ = timed_solves(prob, args, 0)
    t64 = wall / args.steps
    out = {"workload": wname, "time_to_tol_s": t64, "iterations": runs[-1]["iterations"],
           "inner_iterations": runs[-1]["inner_iterations"], "status": runs[-1]["status"],
           "rel_kkt": rel_kkt(runs[-1]), "iters_per_s": sum(r["iterations"] for r in runs) / wall,
           "kernel_ms_per_solve": 1e3 * sum(r["kernel_s"] for r in runs) / args.steps}
    out["fp32_bulk"] = fp32_variant(prob, args, t64, runs[-1])
    return out


# the paper's single-GPU Fisher times (one H100 80 GB, precision not stated),
# seconds to relative KKT 1e-4 and 1e-6, by buyer count
FISHER_PAPER_H100_S = {1_000: (0.36, 0.85), 10_000: (0.69, 0.77), 100_000: (4.43, 4.77),
                       1_000_000: (46.65, 48.32), 10_000_000: (231.94, 241.53)}


def bench_fisher_paper(args):
    """Paper-shaped Fisher market (buyers --buyers; goods and density of the
    paper's instance table, U[0.1, 1.1] valuations and budgets, supplies
    0.2 n): FP64 solves to 1e-4 and to 1e-6 from a cold start, each timed
    over --steps runs after --warmup, next to the paper's own times."""
    import torch
    import paper_2608_09159_amd as pkg
    from instances import synth
    t0 = time.perf_counter()
    prob = synth.fisher_paper(args.buyers)
    log(f"fisher_paper n={args.buyers}: generated ({time.perf_counter() - t0:.1f} s), "
        f"N={prob.n} M={prob.m} nnz={prob.A.nnz}")
    out = {"workload": f"Fisher market, paper shape, {args.buyers} buyers x {prob.meta['n_goods']} goods",
           "N": prob.n, "M": prob.m, "edges": int(prob.meta["edges"]), "nnz_A": int(prob.A.nnz)}
    for tol in (1e-4, 1e-6):
        a2 = argparse.Namespace(**{**vars(args), "tol": tol})
        runs, wall, setup_s = timed_solves(prob, a2, 0, verbose=1 if prob.n > 1_000_000 else 0)
        r = runs[-1]
        out[f"tol_{tol:g}"] = {"time_to_tol_s": wall / args.steps, "iterations": r["iterations"],
                               "status": r["status"], "rel_kkt": rel_kkt(r), "setup_s": setup_s,
                               "kernel_s": r["kernel_s"],
                               "iters_per_s": sum(x["iterations"] for x in runs) / wall}
        log(f"tol {tol:g}: {r['status']} {r['iterations']} it, {wall / args.steps:.3f} s")
    paper = FISHER_PAPER_H100_S.get(args.buyers)
    if paper:
        out["paper_h100_s"] = {"tol_1e-04": paper[0], "tol_1e-06": paper[1],
                               "hardware": "one H100 80 GB, precision not stated"}
    return out


# the ablation variants: settings on top of the defaults (reflected Halpern,
# Jacobi inner metric, monotone adaptive inner tolerance, cone-preserving
# block scaling)
ABLATION_VARIANTS = [
    ("default", {}),
    ("no_jacobi", {"inner": "euclid"}),
    ("fixed_eps_in_1e-6", {"eps_in0": 1e-6, "eps_min": 1e-6}),
    ("fixed_eps_in_1e-9", {"eps_in0": 1e-9, "eps_min": 1e-9}),
    ("averaged", {"scheme": "avg"}),
    ("rescaled_cone", {"cone_scaling": "rescaled"}),
]


def sgm(values, shift=10.0):
    """Shifted geometric mean with shift 10."""
    v = np.asarray(values, dtype=float)
    return float(np.exp(np.mean(np.log(v + shift))) - shift)


def bench_ablation(args):
    """Synthetic analogue of the paper's inner-accuracy ablation (App.
    "Ablation: Inner Accuracy and Preconditioning"), widened to the averaged
    scheme and the rescaled-cone mode: every variant solves the ten tiny QPs
    (seeds 0-9, sparse general Q) and the mixed-cone instance (diagonal plus
    low-rank Q) to --tol from a cold start, with a --time-limit per solve.
    Reported per variant and family: solved count, SGM10 of solve time and
    of outer iterations, total inner steps."""
    import torch
    import paper_2608_09159_amd as pkg
    from instances import synth
    families = [("tiny QP n=200 m=100 (seeds 0-9)", [synth.tiny_qp(s) for s in range(10)]),
                ("mixed-cone SOCP/QCQP n=1e5 m=5e4", [synth.mixed_cone(seed=0)])]
    out = {"workload": "ablation", "tol": args.tol, "time_limit_s": args.time_limit, "families": {}}
    stream = torch.cuda.current_stream()
    for fname, probs in families:
        h = pkg.setup(probs[0], tol=args.tol, stream=stream.cuda_stream)
        h.solve()                             # first-launch costs, outside the timings
        h.free()
        rows = {}
        for vname, kw in ABLATION_VARIANTS:
            times, its, inner, solved = [], [], 0, 0
            for p in probs:
                h = pkg.setup(p, tol=args.tol, time_limit=args.time_limit, max_iter=10_000_000,
                              stream=stream.cuda_stream, **kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = h.solve()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                h.free()
                solved += r["status"] == "OPTIMAL"
                times.append(dt if r["status"] == "OPTIMAL" else args.time_limit)
                its.append(r["iterations"])
                inner += r["inner_iterations"]
                if dt > 2.0:
                    log(f"  {p.name} {vname}: {r['status']} {r['iterations']} it in {dt:.1f} s")
            rows[vname] = {"solved": solved, "of": len(probs), "time_sgm10_s": sgm(times),
                           "iter_sgm10": sgm(its), "inner_total": int(inner), "settings": kw}
            log(f"ablation {fname} {vname}: {solved}/{len(probs)} solved, "
                f"SGM10 {rows[vname]['time_sgm10_s']:.4f} s, {rows[vname]['iter_sgm10']:.0f} it, "
                f"{inner} inner")
        out["families"][fname] = rows
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large_sparse_qp")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--budget", type=int, default=-1,
                    help="outer iterations per step (0: run to the tolerance; default: 256 for the "
                         "large sparse QP, 0 otherwise)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32-bulk, mixed-cone and batched comparisons of the default line")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--loop-sample", type=int, default=4096,
                    help="portfolio_batch: instances timed in the per-instance loop baseline")
    ap.add_argument("--train-instances", type=int, default=1024,
                    help="fisher_warm: training instances labelled by the solver")
    ap.add_argument("--eval-instances", type=int, default=128, help="fisher_warm: held-out seeds")
    ap.add_argument("--timed", type=int, default=16, help="fisher_warm: held-out seeds timed one by one")
    ap.add_argument("--epochs", type=int, default=100, help="fisher_warm: training epochs")
    ap.add_argument("--lr", type=float, default=1e-4, help="fisher_warm: Adam learning rate")
    ap.add_argument("--buyers", type=int, default=100_000, help="fisher_paper: buyer count")
    ap.add_argument("--time-limit", type=float, default=20.0, help="ablation: seconds per solve")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.cpu_child:
        prob, _ = workload(args.workload)
        log("oracle child: instance generated")
        print(json.dumps(cpu_baseline(prob, args.cpu_budget)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not supported "
              "(the 2-D partition across GPUs is design-only).", file=sys.stderr)
        sys.exit(2)
    budget = args.budget if args.budget >= 0 else (256 if args.workload == "large_sparse_qp" else 0)
    child = None
    if not args.no_cpu and args.workload in ("large_sparse_qp", "mixed_cone", "fisher", "tiny_qp"):
        child = start_cpu_child(args)

    import torch
    import paper_2608_09159_amd as pkg

    if not os.path.exists(pkg.lib_path()):
        from paper_2608_09159_amd import build
        build.build()
    if args.workload == "fisher_warm":
        bench_warm(args)
        return
    if args.workload == "mlp_train":
        bench_mlp(args)
        return
    if args.workload == "fisher_paper":
        print(json.dumps(bench_fisher_paper(args)), flush=True)
        return
    if args.workload == "ablation":
        print(json.dumps(bench_ablation(args)), flush=True)
        return
    prob, wname = workload(args.workload)
    if args.workload == "portfolio_batch":
        print(json.dumps(bench_batch(args, prob, wname)), flush=True)
        return
    if args.calibrate_copy:
        src = torch.ones(32 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"{wname}: instance generated")
    runs, wall, setup_s = timed_solves(prob, args, budget)
    log(f"{wname}: {args.steps} timed solves in {wall:.2f} s (setup {setup_s:.1f} s)")
    iters = sum(r["iterations"] for r in runs)
    inner = sum(r["inner_iterations"] for r in runs)
    ksum = sum(r["kernel_s"] for r in runs)
    launches = sum(r["kernel_launches"] for r in runs)
    grid = runs[-1]["grid_dim"]
    traffic = None
    mt = MEASURED_TRAFFIC
    if (mt is not None and args.workload == mt["workload"] and kernel_sources_hash() == mt["sources_sha256"]
            and grid == mt["grid"] and all(r["iterations"] == mt["iterations"] for r in runs)):
        traffic = mt["bytes_per_launch"]
    checks = sum(math.ceil(r["iterations"] / 64) + r["restarts"] + 1 for r in runs)
    alg_bytes = method_bytes_model(prob, iters, inner, checks)
    achieved = alg_bytes / ksum / 1e9
    last = runs[-1]
    reached = last["status"] == "OPTIMAL"
    out = {
        "metric": METRIC,
        "value": iters / wall,
        "unit": "PDHG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wname, "n": prob.n, "m": prob.m, "nnz_A": int(prob.A.nnz),
                   "nnz_P": int(prob.P.nnz) if prob.P is not None else 0,
                   "tol": args.tol, "precision": "fp64",
                   "outer_iterations_per_step": budget if budget > 0 else "to tolerance"},
        "time_to_tol_s": wall / args.steps if reached else None,
        "iterations_per_solve": iters / args.steps,
        "inner_per_solve": inner / args.steps,
        "status": last["status"],
        "rel_kkt": rel_kkt(last),
        "rel_primal": last["rel_primal"], "rel_dual": last["rel_dual"], "rel_gap": last["rel_gap"],
        "setup_s": setup_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
                     "kernel": solver_kernel_name(prob, "fp64", grid), "kernel_avg_launch_ms": 1e3 * ksum / launches,
                     "launch": [grid, runs[-1]["block_dim"]],
                     "algorithmic_bytes_per_iteration": alg_bytes / iters,
                     "bytes_model": "method (A, A^T, P read once per product, ideal gathers)"},
    }
    ctx = same_footprint_context(prob, ksum / iters)
    ctx["kernel_pass_bytes_per_iteration"] = bytes_model(prob, iters, inner, checks) / iters
    out["context"] = ctx
    if not args.no_variants and args.workload == "large_sparse_qp":
        out["variants"] = {"fp32_bulk": fp32_budget_variant(prob, args, budget, wall, last)}
        log("fp32 bulk variant done")
        del prob
        out["variants"]["mixed_cone"] = mixed_cone_variant(args)
        log("mixed-cone variant done")
        bargs = argparse.Namespace(**{**vars(args), "loop_sample": 128})
        bw, bname = workload("portfolio_batch")
        bo = bench_batch(bargs, bw, bname)
        out["variants"]["batched"] = {
            "workload": bname, "time_to_tol_s": bo["time_to_tol_s"],
            "loop_time_to_tol_s": bo["loop_baseline"]["time_to_tol_s"],
            "loop_instances_timed": bo["loop_baseline"]["instances_timed"],
            "speedup_vs_loop": bo["speedup_vs_loop"], "statuses": bo["statuses"],
            "iters_per_s": bo["value"], "roofline_frac": bo["roofline"]["frac"]}
        log("batched variant done")
    elif not args.no_variants and args.workload == "mixed_cone":
        out["variants"] = {"fp32_bulk": fp32_variant(prob, args, wall / args.steps, last)}
    if child is not None:
        log("waiting for the oracle child")
        out["cpu_baseline"] = finish_cpu_child(child)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
