"""Benchmark: mixed-precision MGRIT on one MI355X, with the plain FP64 method and the other forms beside it.

Headline workload (--workload mixed-511, the default): 511 x 511 interior nodes, 4096 graded steps
t_n = (n / N)^2 (time-dependent propagators), beta, gamma ~ U(0.55, 0.95) from seed 3, K = 1, T = 1,
coarsening m = 8, levels 4096 -> 512 -> 64 (the last solved by sequential stepping); F ~ N(0,1) per node and
step, psi_0 ~ U[0,1] (numpy PCG64, seed 3), resident on the GPU before timing.  One step = one MGRIT solve
to the stop test (C-point residual 1e-8 of the first one; CG to 1e-9 relative on level 0, 5e-3 on the coarse
levels), `opt` coarse propagator, fast-diagonalisation preconditioner with BF16 products, mixed precision:
FP64 outer residuals and refinement, FP32 inner PCG with the operator by FP32 FFTs (1024 points).  The
result must agree with FP64 sequential stepping on the GPU (CG 1e-13, itself tied to the CPU oracle by the
GPU tests) to relative l2 <= 1e-8.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mixed-511 | vcycle-255] [--no-cpu] ...

The K timed solves run without instrumentation; one more solve after them is instrumented with HIP events
around every kernel of a CG iteration (and each preconditioner application), which gives the per-kernel
figures of the `roofline` block.  Beside the headline, `forms` times other forms of the same
solver on the same workload (one instrumented warm-up solve, then one timed solve each): the plain FP64
method (FP64 matrix-core Toeplitz products, FP64 preconditioner products), FP64 with the FFT operator, and
the mixed forms with the inner operator on the FP32 matrix cores and as split-BF16 products.  Then
sequential stepping, a context run on the 255 x 255 x 1024 V-cycle workload (MGRIT vs parareal vs sequential
stepping), the many-instance and serving workloads, and the CPU oracle on a bounded sample.  One JSON line
on stdout; progress on stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "space-time DOF/s at 1e-8 rel. error vs FP64 sequential"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}      # MI355X dense TFLOP/s (matrix; FP64/FP32 vector alike)
HBM_PEAK_GBPS = 8000.0

# kernel classes of the library's instrumentation (include/mgrit.h, MGRIT_PROF_*)
OP64_T64, OP64_T32, OP32_T64, OP32_T32, OP_BF16, PRECOND, UPD64, DIR64, UPD32, DIR32 = range(10)

# options shared by every timed MGRIT form
BASE = dict(max_levels=3, coarse="opt", cg_rtol=1e-9, cg_rtol_coarse=5e-3, cg_maxit=100000, tol_abs=0.0,
            tol_rel=1e-8, max_iter=40)
HEADLINE = dict(precision="mixed", precond="fd-bf16", op="auto")
FORMS = {
    # plain FP64: Toeplitz products on the FP64 matrix cores, preconditioner products in FP64: no FFT, no BF16
    "fp64-dense": dict(precision="fp64", precond="fd", op="dense"),
    # FP64 with the operator by FP64 FFTs and FP64 preconditioner products
    "fp64-fft": dict(precision="fp64", precond="fd", op="fft"),
    # mixed precision with the dense operator: FP64 outer products on the FP64 matrix cores, inner on the FP32 ones
    "mixed-dense-fp32": dict(precision="mixed", precond="fd-bf16", op="dense"),
    # the same with the inner Toeplitz products as split-BF16 products on the BF16 matrix cores
    "mixed-dense-bf16": dict(precision="mixed-bf16", precond="fd-bf16", op="dense"),
}
REF_OPTS = dict(cg_rtol=1e-13, cg_maxit=100000, precond="fd-bf16")     # FP64 sequential reference
SEQ_CG_RTOL = 3e-10          # sequential stepping at a CG tolerance whose error meets 1e-8


def note(msg):
    """Progress of a long run on stderr (stdout carries only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def fft_flops(nx, ny):
    """Flops of one operator application by FFT as the kernels compute them: per direction ceil(lines / 2)
    packed line pairs, each one forward and one inverse transform of L points (L = 512: a radix-8 DFT (56 flops)
    and two twiddled ones (78 + 56) per lane, 64 lanes: 20736; L = 1024: a radix-16 DFT (192) and two passes of
    two twiddled radix-8 DFTs (268 each): 46592) and the spectral combination at L / 2 + 64 frequencies (half
    the spectrum plus one row, the other half being conjugates): 59 flops each in the x pass (unpacking 16,
    kernel and mass coefficients 11, the two outputs 32) and 48 in the y pass (no coefficients)."""
    L = 512 if 2 * max(nx, ny) - 1 <= 512 else 1024
    tflops = 20736 if L == 512 else 46592
    freq = L // 2 + 64
    return float(((ny + 1) // 2) * (2 * tflops + 59 * freq) + ((nx + 1) // 2) * (2 * tflops + 48 * freq)), L


def kernel_models(nx, ny, fft, precond):
    """Per kernel class: (name, bound, dtype peak key, work per slice application, unit).  Work is the
    algorithmic count: flops of the dense Toeplitz products (6 n_x^2 n_y + 6 n_x n_y^2) for the tiled operator,
    the FFT flops above for the FFT operator, 4 n_x n_y (n_x + n_y) for the four preconditioner products, and
    the bytes each vector kernel must move (x, r, p, q read and x, r written; z, p read and p written)."""
    dense = 6.0 * nx * nx * ny + 6.0 * nx * ny * ny
    ff, L = fft_flops(nx, ny)
    n2 = float(nx * ny)
    pc = 4.0 * nx * ny * (nx + ny)
    pc_name = "k_fdb_gemm x4 (preconditioner, BF16 products)" if precond == "fd-bf16" else \
        "k_fd_gemm x4 (preconditioner, FP64 products)"
    m = {
        OP64_T64: (f"k_fft_line<double,0,2> + <double,1,2> (operator by {L}-point FFTs, FP64)", "alu", "fp64", ff,
                   "TFLOP/s") if fft else ("k_prop_apply<64,2> (operator, FP64 matrix cores)", "mfma", "fp64", dense,
                                           "TFLOP/s"),
        OP64_T32: ("k_prop_apply<32,2> (operator, FP64 matrix cores, 32-node tiles)", "mfma", "fp64", dense, "TFLOP/s"),
        OP32_T64: (f"k_fft_line32<0,2> + <1,2> (inner operator by {L}-point FFTs, FP32)", "alu", "fp32", ff,
                   "TFLOP/s") if fft else ("k_apply32<64> (inner operator, FP32 matrix cores)", "mfma", "fp32", dense,
                                           "TFLOP/s"),
        OP32_T32: ("k_apply32<32> (inner operator, FP32 matrix cores, 32-node tiles)", "mfma", "fp32", dense,
                   "TFLOP/s"),
        OP_BF16: ("k_apply_bf16 (inner operator, split-BF16 products: 3 BF16 MFMA passes per algorithmic flop)",
                  "mfma", "bf16", dense, "TFLOP/s"),
        PRECOND: (pc_name, "mfma", "bf16" if precond == "fd-bf16" else "fp64", pc, "TFLOP/s"),
        UPD64: ("k_cg_update (x += alpha p, r -= alpha q; FP64)", "hbm", None, 48.0 * n2, "GB/s"),
        DIR64: ("k_cg_direction (p = z + beta p; FP64)", "hbm", None, 24.0 * n2, "GB/s"),
        UPD32: ("k_mx_update (d += alpha p, r -= alpha q; FP32)", "hbm", None, 24.0 * n2, "GB/s"),
        DIR32: ("k_mx_direction (p = z + beta p; FP32)", "hbm", None, 12.0 * n2, "GB/s"),
    }
    return m


def read_kernels(solver, nx, ny, fft, precond):
    """Per-class figures of the instrumented solve(s): average launch time and achieved rate vs its peak."""
    models = kernel_models(nx, ny, fft, precond)
    out = []
    for cls in range(10):
        ms, n, sl = solver.profile_read(cls)
        if n == 0 or ms <= 0:
            continue
        name, bound, peak_key, work, unit = models[cls]
        per_launch = work * sl / n
        sec = ms * 1e-3 / n
        if unit == "TFLOP/s":
            achieved, peak = per_launch / sec / 1e12, PEAK[peak_key]
        else:
            achieved, peak = per_launch / sec / 1e9, HBM_PEAK_GBPS
        out.append({"class": cls, "kernel": name, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                    "frac": achieved / peak, "avg_launch_us": sec * 1e6, "launches": n,
                    "slice_applies_per_launch": sl / n, "work_per_slice_apply": work, "total_ms": ms})
    return sorted(out, key=lambda k: -k["total_ms"])


def timed_solves(solver, Fd, pd, U, n):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = rc = None
    for _ in range(n):
        _, st, rc = solver.solve(Fd, pd, out=U)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(n, 1), st, rc


def instrumented_solve(solver, Fd, pd, U):
    solver.profile(True)
    _, st, rc = solver.solve(Fd, pd, out=U)
    return st, rc


def rel_err(U, Uref, shape):
    import torch
    return float(torch.linalg.norm(U.view(shape) - Uref) / torch.linalg.norm(Uref))


def run_form(mgrit, common, m, opts, Fd, pd, U, Uref, shape, nx, ny, fft_fits):
    """One instrumented warm-up solve (kernel figures), then one timed solve."""
    o = dict(BASE, **opts)
    with mgrit.Solver(*common, m=m, **o) as s:
        st, rc = instrumented_solve(s, Fd, pd, U)
        fft = o["op"] == "fft" or (o["op"] == "auto" and fft_fits)
        kern = read_kernels(s, nx, ny, fft, o["precond"])
        s.profile(False)
        sec, st, rc = timed_solves(s, Fd, pd, U, 1)
    dof = nx * ny * (shape[0] - 1)
    return {"dof_per_s": dof / sec, "ms_per_step": sec * 1e3, "rel_l2_err": rel_err(U, Uref, shape),
            "mgrit_iterations": st.iterations, "cg_iterations": st.cg_iterations, "refinements": st.refinements,
            "rc": rc, "options": o, "kernels": kern[:6]}


def context_vcycle_255(mgrit, wl, torch):
    """MGRIT (the headline's options) vs parareal (two levels, F-relaxation, the same coarse propagator and
    coarsening) vs sequential stepping on the 255 x 255 x 1024 uniform V-cycle workload."""
    W = wl.FP64_VCYCLE_255
    t = wl.uniform_grid(W["Nt"])
    nx, ny, Nt = W["Mx"] - 1, W["My"] - 1, W["Nt"]
    F, psi0 = wl.random_inputs(W["seed"], Nt, nx, ny)
    Fd, pd = torch.from_numpy(F).cuda(), torch.from_numpy(psi0).cuda()
    common = (W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"], t)
    shape = (Nt + 1, ny, nx)
    with mgrit.Solver(*common, m=W["m"], **REF_OPTS) as ref:
        Uref, _, _ = ref.sequential(Fd, pd)
    U = torch.empty((Nt + 1) * nx * ny, dtype=torch.float64, device="cuda")
    out = {"workload": W["name"]}
    # parareal takes the L-stable backward-Euler coarse step: with the two Crank-Nicolson steps of `opt` its
    # coarse factor tends to +1 on stiff modes, where F-relaxation alone gives it no damping
    for name, extra in (("mgrit", {}), ("parareal", dict(max_levels=2, relax="F", coarse="be", max_iter=80))):
        o = dict(BASE, **HEADLINE)
        o.update(extra)
        with mgrit.Solver(*common, m=W["m"], **o) as s:
            timed_solves(s, Fd, pd, U, 1)
            sec, st, rc = timed_solves(s, Fd, pd, U, 1)
        out[name] = {"dof_per_s": nx * ny * Nt / sec, "ms_per_step": sec * 1e3, "rel_l2_err": rel_err(U, Uref, shape),
                     "iterations": st.iterations, "rc": rc, "levels": 2 if extra else 3,
                     "relax": o["relax"] if "relax" in o else "FCF", "coarse": o["coarse"]}
    with mgrit.Solver(*common, m=W["m"], **dict(HEADLINE, cg_rtol=SEQ_CG_RTOL, cg_maxit=100000)) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Useq, _, _ = s.sequential(Fd, pd, out=U)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
    out["sequential"] = {"dof_per_s": nx * ny * Nt / sec, "ms_per_step": sec * 1e3, "cg_rtol": SEQ_CG_RTOL,
                         "rel_l2_err": rel_err(U, Uref, shape)}
    out["note"] = ("paper (Table 7 and Section 4.3, 512 Xeon cores, 128^2 x 8192): MGRIT 4.6x and parareal 2.0x "
                   "over sequential stepping")
    return out


def serving(mgrit, wl, torch, n_requests, rate, nt_scale, max_concurrent, budget_gb):
    """Replay the first n_requests arrivals of the seeded Poisson stream through the server; latency =
    finish - arrival (queueing included)."""
    trace = wl.serving_stream(5, n_requests, rate, nt_scale=nt_scale)
    dev = [wl.device_inputs(r["input_seed"], r["Nt"], r["nx"], r["ny"]) for r in trace]
    torch.cuda.synchronize()
    opts = dict(BASE, **HEADLINE)
    handles = []
    with mgrit.Server(int(budget_gb * (1 << 30)), max_concurrent=max_concurrent) as srv:
        t0 = time.perf_counter()             # just after the server's own clock started: latencies err high
        for r, (F, p) in zip(trace, dev):
            delay = r["arrival"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            handles.append(srv.submit(F, p, r["beta"], r["gamma"], r["Kx"], r["Ky"], r["nx"] + 1, r["ny"] + 1,
                                      r["t"], m=8, **opts))
        infos = [h.wait()[1] for h in handles]
    lat = np.array([i.finish_s - r["arrival"] for i, r in zip(infos, trace)])
    span = max(i.finish_s for i in infos)
    dof = sum(r["nx"] * r["ny"] * r["Nt"] for r in trace)
    return {"requests": n_requests, "arrival_rate_per_s": rate, "max_concurrent": max_concurrent,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_queue_s": float(np.mean([i.start_s - i.submit_s for i in infos])),
            "throughput_dof_per_s": dof / span, "all_converged": all(i.rc == 0 for i in infos),
            "trace": (f"first {n_requests} arrivals of the seed-5 Poisson stream at {rate:g}/s: n_x, n_y ~ U{{63..1023}}, "
                      f"N_t ~ U{{128..8192}} divided by {nt_scale} (multiple of 8), beta, gamma ~ U(0.55, 0.95), K = 1, "
                      f"m = 8; F ~ N(0,1), psi_0 ~ U[0,1] drawn on the GPU; the headline's options")}


def many_instance(mgrit, wl, torch, n_problems, max_concurrent):
    """Independent problems of uneven sizes submitted at once; aggregate DOF/s."""
    probs = wl.many_problem_set(4, n_problems)
    dev = [wl.device_inputs(r["input_seed"], r["Nt"], r["nx"], r["ny"]) for r in probs]
    torch.cuda.synchronize()
    opts = dict(BASE, **HEADLINE)
    t0 = time.perf_counter()
    with mgrit.Server(200 << 30, max_concurrent=max_concurrent) as srv:
        hs = [srv.submit(F, p, r["beta"], r["gamma"], r["Kx"], r["Ky"], r["nx"] + 1, r["ny"] + 1, r["t"], m=r["m"],
                         **opts) for r, (F, p) in zip(probs, dev)]
        infos = [h.wait()[1] for h in hs]
    dt = time.perf_counter() - t0
    dof = sum(r["nx"] * r["ny"] * r["Nt"] for r in probs)
    return {"problems": n_problems, "max_concurrent": max_concurrent, "dof_per_s": dof / dt, "seconds": dt,
            "all_converged": all(i.rc == 0 for i in infos),
            "set": (f"first {n_problems} of the seed-4 set: n ~ U{{127..383}} square, N_t ~ U{{256..2048}}, "
                    f"m in {{4, 8, 16}}, beta, gamma ~ U(0.55, 0.95), K = 1; the headline's options")}


def many_same_mesh(mgrit, wl, torch, n_problems, n):
    """Independent problems on one mesh: one group (their sweeps in shared launches) against the server
    (concurrent solves on 4 streams) and against one solve after another; aggregate DOF/s each, and the
    largest difference between a problem's group and solo results."""
    probs = wl.many_same_mesh(6, n_problems, n=n)
    dev = [wl.device_inputs(r["input_seed"], r["Nt"], r["nx"], r["ny"]) for r in probs]
    dof = sum(r["nx"] * r["ny"] * r["Nt"] for r in probs)
    opts = dict(BASE, **HEADLINE)
    out = {"problems": n_problems, "n": n,
           "set": (f"seed 6: {n_problems} problems on one {n} x {n} mesh, N_t ~ U{{256..2048}} (multiple of 8), m = 8, "
                   f"beta, gamma ~ U(0.55, 0.95), K = 1; the headline's options")}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with mgrit.Group([dict(beta=r["beta"], gamma=r["gamma"], Kx=r["Kx"], Ky=r["Ky"], t=r["t"]) for r in probs],
                     n + 1, n + 1, m=8, **opts) as g:
        g.solve([F for F, _ in dev], [p for _, p in dev])          # cold: set-up and first solve
        torch.cuda.synchronize()
        cold = time.perf_counter() - t0
        t0 = time.perf_counter()
        Ug, stg, rc = g.solve([F for F, _ in dev], [p for _, p in dev])
        torch.cuda.synchronize()
        out["group"] = {"dof_per_s": dof / (time.perf_counter() - t0), "rc": rc,
                        "dof_per_s_with_setup": dof / cold,
                        "mgrit_iterations": [st.iterations for st in stg]}
    Us = []
    t0 = time.perf_counter()
    for r, (F, p) in zip(probs, dev):
        with mgrit.Solver(r["beta"], r["gamma"], r["Kx"], r["Ky"], n + 1, n + 1, r["t"], m=8, **opts) as s:
            U, st, rc = s.solve(F, p)
            Us.append(U)
    torch.cuda.synchronize()
    out["one_after_another"] = {"dof_per_s": dof / (time.perf_counter() - t0),
                                "note": "includes each solve's set-up"}
    out["max_rel_diff_group_vs_solo"] = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                                            for a, b in zip(Ug, Us))
    t0 = time.perf_counter()
    with mgrit.Server(200 << 30, max_concurrent=4) as srv:
        hs = [srv.submit(F, p, r["beta"], r["gamma"], r["Kx"], r["Ky"], n + 1, n + 1, r["t"], m=8, **opts)
              for r, (F, p) in zip(probs, dev)]
        infos = [h.wait()[1] for h in hs]
    out["server_4_streams"] = {"dof_per_s": dof / (time.perf_counter() - t0),
                               "all_converged": all(i.rc == 0 for i in infos), "note": "includes each solve's set-up"}
    t0 = time.perf_counter()
    with mgrit.Server(200 << 30, max_concurrent=4, group_limit=8) as srv:
        hs = [srv.submit(F, p, r["beta"], r["gamma"], r["Kx"], r["Ky"], n + 1, n + 1, r["t"], m=8, **opts)
              for r, (F, p) in zip(probs, dev)]
        infos = [h.wait()[1] for h in hs]
    out["server_4_streams_groups_of_8"] = {
        "dof_per_s": dof / (time.perf_counter() - t0), "all_converged": all(i.rc == 0 for i in infos),
        "group_sizes": sorted(set(i.group_size for i in infos)),
        "note": "queued requests of one mesh taken into group solves of up to 8; includes set-up"}
    return out


def cpu_baseline(W, t, F, psi0, steps, start):
    """The CPU oracle as it stands: sequential stepping over `steps` steps of the time grid from step `start`."""
    from oracle import fem, propagator
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    prob = fem.Problem(W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"])
    op = fem.Operator(prob)
    solver = propagator.CGSolver(op, BASE["cg_rtol"], 100000)
    ts = t[start: start + steps + 1] - t[start]
    t0 = time.perf_counter()
    propagator.sequential(op, solver, ts, F[start: start + steps], psi0)
    dt = time.perf_counter() - t0
    return {"value": prob.nx * prob.ny * steps / dt, "unit": "DOF/s", "cores": int(cores), "kind": "oracle",
            "sample": f"sequential time stepping (the result MGRIT converges to) over steps {start + 1}..{start + steps} "
                      f"of the {len(t) - 1}-step grid, plain CG rtol {BASE['cg_rtol']:g}, numpy FP64 on the host; "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed-511",
                    help="mixed-511 (511 x 511 x 4096 graded, the default) | vcycle-255 (255 x 255 x 1024 uniform)")
    ap.add_argument("--forms", default="all", help="comma list of " + ", ".join(FORMS) + " | all | none")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-context", action="store_true", help="skip the 255 x 255 MGRIT / parareal / sequential run")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving trace and the many-instance set")
    ap.add_argument("--serving-requests", type=int, default=16)
    ap.add_argument("--serving-nt-scale", type=int, default=8)
    ap.add_argument("--many", type=int, default=32, help="problems of the many-instance set")
    ap.add_argument("--precision", default=None, help="override the headline's precision")
    ap.add_argument("--op", default=None, help="override the headline's operator (auto | dense | fft)")
    ap.add_argument("--precond", default=None, help="override the headline's preconditioner (fd | fd-bf16 | none)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--skip-reference", action="store_true",
                    help="headline solves only (no reference, forms or extras): for profiler runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per run: the time-sharded multi-GPU form is not implemented; "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        from paper_1805_06688_amd import profiling
        profiling.copy(512)
        return
    from paper_1805_06688_amd import mgrit, workloads as wl

    if args.workload == "mixed-511":
        W = wl.mixed_511()
        t = wl.graded_grid(W["Nt"])
    elif args.workload == "vcycle-255":
        W = wl.FP64_VCYCLE_255
        t = wl.uniform_grid(W["Nt"])
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    head = dict(HEADLINE)
    if args.precision:
        head["precision"] = args.precision
    if args.op:
        head["op"] = args.op
    if args.precond:
        head["precond"] = args.precond
    nx, ny, Nt = W["Mx"] - 1, W["My"] - 1, W["Nt"]
    shape = (Nt + 1, ny, nx)
    fft_fits = 2 * max(nx, ny) - 1 <= 1024
    F, psi0 = wl.random_inputs(W["seed"], Nt, nx, ny)
    torch.cuda.set_device(0)
    Fd = torch.from_numpy(F).cuda()
    pd = torch.from_numpy(psi0).cuda()
    common = (W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"], t)
    note(f"inputs ready: {W['name']}")

    Uref = None
    if not args.skip_reference:
        with mgrit.Solver(*common, m=W["m"], **REF_OPTS) as ref:      # outside every timed region
            Uref, _, _ = ref.sequential(Fd, pd)
        torch.cuda.synchronize()
        note("FP64 sequential reference done")

    U = torch.empty((Nt + 1) * nx * ny, dtype=torch.float64, device="cuda")
    hopts = dict(BASE, **head)
    s = mgrit.Solver(*common, m=W["m"], **hopts)
    for i in range(args.warmup):
        s.solve(Fd, pd, out=U)
    note("warm-up done")
    per_step, st, rc = timed_solves(s, Fd, pd, U, args.steps)
    note(f"timed solves done: {per_step * 1e3:.1f} ms each")
    # kernel figures: one more solve, instrumented (events around each launch stay out of the timed ones)
    instrumented_solve(s, Fd, pd, U)
    fft = head["op"] == "fft" or (head["op"] == "auto" and fft_fits)
    kern = read_kernels(s, nx, ny, fft, head["precond"])
    s.profile(False)
    levels = s.levels()
    err = None if Uref is None else rel_err(U, Uref, shape)
    s.close()

    dof = nx * ny * Nt
    dom = kern[0]
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{W['name']}.json")
    if os.path.exists(tfile):
        from paper_1805_06688_amd import profiling
        with open(tfile) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == profiling.source_hash() and tr.get("class") == dom["class"]:
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": dom["bound"], "kernel": dom["kernel"], "achieved": dom["achieved"], "peak": dom["peak"],
                "unit": dom["unit"], "frac": dom["frac"], "traffic": traffic,
                "avg_launch_ms": dom["avg_launch_us"] * 1e-3, "launches": dom["launches"],
                "slice_applies_per_launch": dom["slice_applies_per_launch"],
                "work_per_slice_apply": dom["work_per_slice_apply"],
                "measured": "HIP events around each launch on the solver's stream, in one solve after the timed ones",
                "kernels": kern}
    out = {"metric": METRIC, "value": dof / per_step, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": per_step * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None,
           "dtype": ("f64" if head["precision"] == "fp64" else "f64+f32") +
                    ("+bf16" if head["precond"] == "fd-bf16" or head["precision"] == "mixed-bf16" else ""),
           "data": "synthetic",
           "config": {"workload": W["name"], "nx": nx, "ny": ny, "Nt": Nt, "beta": W["beta"], "gamma": W["gamma"],
                      "Kx": W["Kx"], "Ky": W["Ky"], "m": W["m"], "levels": levels, "relax": "FCF",
                      "coarse": hopts["coarse"], "precond": hopts["precond"], "cg_rtol": hopts["cg_rtol"],
                      "cg_rtol_coarse": hopts["cg_rtol_coarse"], "tol_rel": hopts["tol_rel"],
                      "precision": hopts["precision"], "operator": hopts["op"],
                      "coarse_level_passes": ("wholly FP32 (right-hand side and initial residual in FP32 from the "
                                              "FP64 data, one refinement step) at the coarse CG tolerance"
                                              if hopts["precision"] != "fp64" and (hopts["op"] == "fft" or (
                                                  hopts["op"] == "auto" and fft_fits)) else "as level 0"),
                      "mgrit_iterations": st.iterations, "phi_per_solve": st.phi_applications,
                      "cg_iterations_per_solve": st.cg_iterations, "refinements_per_solve": st.refinements,
                      "rel_l2_err_vs_fp64_sequential": err, "parallelism": "time (MGRIT), one GPU"},
           "roofline": roofline}

    if not args.skip_reference:
        names = list(FORMS) if args.forms == "all" else ([] if args.forms == "none" else args.forms.split(","))
        forms = {}
        for name in names:
            if name not in FORMS:
                raise SystemExit(f"unknown form {name}")
            if FORMS[name]["op"] == "fft" and not fft_fits:
                continue
            forms[name] = run_form(mgrit, common, W["m"], FORMS[name], Fd, pd, U, Uref, shape, nx, ny, fft_fits)
            note(f"form {name}: {forms[name]['dof_per_s'] / 1e6:.1f} M DOF/s, error {forms[name]['rel_l2_err']:.2e}")
        forms["headline:" + head["precision"] + "-" + head["op"]] = {
            "dof_per_s": dof / per_step, "ms_per_step": per_step * 1e3, "rel_l2_err": err,
            "mgrit_iterations": st.iterations, "options": hopts}
        out["forms"] = forms
        # sequential stepping with the headline's spatial solver at a CG tolerance that meets the bar
        with mgrit.Solver(*common, m=W["m"], **dict(head, cg_rtol=SEQ_CG_RTOL, cg_maxit=100000)) as sq:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sq.sequential(Fd, pd, out=U)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
        out["sequential"] = {"dof_per_s": dof / sec, "ms_per_step": sec * 1e3, "cg_rtol": SEQ_CG_RTOL,
                             "precision": head["precision"], "rel_l2_err": rel_err(U, Uref, shape)}
        note(f"sequential stepping: {dof / sec / 1e6:.1f} M DOF/s")
    del U
    if not args.skip_reference and not args.no_context:
        out["context"] = context_vcycle_255(mgrit, wl, torch)
        note("context run (255 x 255: MGRIT, parareal, sequential) done")
    if not args.skip_reference and not args.no_serving:
        del Fd, Uref
        torch.cuda.empty_cache()
        out["many_instance"] = many_instance(mgrit, wl, torch, args.many, 4)
        note("many-instance set done")
        out["many_instance_same_mesh"] = many_same_mesh(mgrit, wl, torch, args.many, 127)
        note("same-mesh set done (group, one after another, server)")
        out["serving"] = serving(mgrit, wl, torch, args.serving_requests, 20.0, args.serving_nt_scale, 4, 200)
        note("serving trace done")
    if not args.no_cpu and not args.skip_reference:
        out["cpu_baseline"] = cpu_baseline(W, t, F, psi0, 160 if nx > 300 else 200, Nt // 2)
    print(json.dumps(out), flush=True)
    if args.skip_reference:
        return
    if not (err <= 1e-8 and rc == 0):
        print(f"accuracy target missed: rel_l2_err={err:.3e} rc={rc}", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
