"""Benchmark: FP64 multilevel MGRIT V-cycle on one MI355X.

Workload: 255 x 255 interior nodes, beta = 0.75, gamma = 0.85, K_x = 2, K_y = 1,
T = 1, 1024 uniform steps, coarsening m = 8 (levels 1024 -> 128 -> 16, the
16-point level solved by sequential stepping),
F ~ N(0,1) per node and step and psi_0 ~ U[0,1] from seed 2, all FP64 and
resident on the GPU before timing.  One step = one full MGRIT solve to the
stop test; the result is checked against FP64 sequential stepping on the GPU
(CG to rtol 1e-13) and must agree to relative l2 <= 1e-8.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Prints one JSON line.  The operator kernel (the CG matrix-vector product) is
timed with HIP events inside the library over the timed region; its algorithmic
work is the six dense Toeplitz products, 6 n_x^2 n_y + 6 n_x n_y^2 flops per
slice application.
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
FP64_PEAK_TFLOPS = 78.6          # MI355X dense FP64 (matrix and vector)
FP32_PEAK_TFLOPS = 157.3         # MI355X dense FP32 (matrix)
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_prop_apply64_fp64_vcycle_255_traffic.json")
FFT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fft_line_vcycle_255_traffic.json")


def note(msg):
    """Progress of a long run on stderr (stdout carries only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_baseline(W, t, F, psi0, steps, cg_rtol):
    """The CPU oracle as it stands: sequential stepping over the first `steps` steps."""
    import numpy as np
    from oracle import fem, propagator
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    prob = fem.Problem(W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"])
    op = fem.Operator(prob)
    solver = propagator.CGSolver(op, cg_rtol, 100000)
    t0 = time.perf_counter()
    propagator.sequential(op, solver, t[: steps + 1], F[:steps], psi0)
    dt = time.perf_counter() - t0
    return {"value": prob.nx * prob.ny * steps / dt, "unit": "DOF/s", "cores": int(cores), "kind": "oracle",
            "sample": f"sequential time stepping (the result MGRIT converges to) over the first {steps} of "
                      f"{len(t) - 1} steps, CG rtol {cg_rtol:g}, numpy FP64 on the host; {dt:.1f} s"}


SOLVE_OPTS = dict(coarse="opt", precond="fd-bf16", cg_rtol=1e-9, cg_rtol_coarse=5e-3, precision="mixed",
                  cg_maxit=100000, tol_abs=0.0, tol_rel=1e-8, max_iter=40, max_levels=3)


def serving(mgrit, wl, torch, n_requests, rate, max_concurrent, budget_gb):
    """Replay a seeded Poisson trace through the server; latency = finish - arrival."""
    trace = wl.serving_trace(5, n_requests, rate)
    dev = [(torch.from_numpy(r["F"]).cuda(), torch.from_numpy(r["psi0"]).cuda()) for r in trace]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    handles = []
    with mgrit.Server(int(budget_gb * (1 << 30)), max_concurrent=max_concurrent) as srv:
        for r, (F, p) in zip(trace, dev):
            delay = r["arrival"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            handles.append((srv.submit(F, p, r["beta"], r["gamma"], r["Kx"], r["Ky"], r["nx"] + 1, r["ny"] + 1,
                                       r["t"], m=8, **SOLVE_OPTS), time.perf_counter() - t0))
        done = [(h.wait()[1], sub) for h, sub in handles]
    span = max(i.finish_s for i, _ in done) - min(i.submit_s for i, _ in done)
    lat = np.array([i.finish_s - i.submit_s for i, _ in done])
    dof = sum(r["nx"] * r["ny"] * r["Nt"] for r in trace)
    ok = all(i.rc == 0 for i, _ in done)
    return {"requests": n_requests, "arrival_rate_per_s": rate, "max_concurrent": max_concurrent,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_queue_s": float(np.mean([i.start_s - i.submit_s for i, _ in done])),
            "throughput_dof_per_s": dof / span, "all_converged": ok,
            "trace": "seed 5: Poisson arrivals; n_x, n_y ~ U{63..255}, N_t ~ U{64..512} (multiple of 8), "
                     "beta, gamma ~ U(0.55, 0.95), K = 1, m = 8; mixed precision with FP64 stop tests (CG 1e-9, "
                     "coarse levels 5e-3, MGRIT stop 1e-8 rel.)"}


def many_instance(mgrit, wl, torch, n_problems, max_concurrent):
    """Independent problems of uneven sizes submitted at once; aggregate DOF/s."""
    probs = wl.many_problems(4, n_problems)
    dev = [(torch.from_numpy(r["F"]).cuda(), torch.from_numpy(r["psi0"]).cuda()) for r in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with mgrit.Server(200 << 30, max_concurrent=max_concurrent) as srv:
        hs = [srv.submit(F, p, r["beta"], r["gamma"], r["Kx"], r["Ky"], r["nx"] + 1, r["ny"] + 1, r["t"], m=r["m"],
                         **SOLVE_OPTS) for r, (F, p) in zip(probs, dev)]
        infos = [h.wait()[1] for h in hs]
    dt = time.perf_counter() - t0
    dof = sum(r["nx"] * r["ny"] * r["Nt"] for r in probs)
    return {"problems": n_problems, "max_concurrent": max_concurrent, "dof_per_s": dof / dt, "seconds": dt,
            "all_converged": all(i.rc == 0 for i in infos),
            "set": "seed 4: n ~ U{127..255} square, N_t ~ U{64..256}, m in {4, 8, 16}, beta, gamma ~ U(0.55, 0.95)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--coarse", default="opt")
    # CG tolerance of the paper's spatial solves (1e-9 relative); MGRIT stops once the C-point residual
    # norm has dropped by 1e-8, which leaves the error against FP64 sequential stepping at about 4e-9
    ap.add_argument("--cg-rtol", type=float, default=1e-9)
    ap.add_argument("--tol-rel", type=float, default=1e-8)
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="steps of the CPU oracle sample (0: 200 at 255 x 255, 25 at 511 x 511)")
    ap.add_argument("--workload", default="vcycle-255",
                    help="vcycle-255 (255 x 255 x 1024 uniform, the benchmark) | mixed-511 (511 x 511 x 4096 graded)")
    ap.add_argument("--precond", default="fd-bf16")
    ap.add_argument("--max-levels", type=int, default=3)
    ap.add_argument("--tile", default="auto", help="operator tile policy: auto | rule | 64 | 32")
    ap.add_argument("--precision", default="mixed", help="fp64 | mixed | mixed-coarse")
    ap.add_argument("--graphs", action="store_true", help="replay CG iteration pairs as HIP graphs")
    ap.add_argument("--relax", default="FCF", help="relaxation on level 0: F | FCF")
    ap.add_argument("--coarse-relax", default=None, help="relaxation on levels >= 1: F | FCF (default: FCF)")
    ap.add_argument("--op", default="auto", help="operator: dense (matrix-core Toeplitz products) | fft | auto")
    ap.add_argument("--inner-rtol", type=float, default=0.0, help="mixed precision: inner FP32 tolerance floor")
    ap.add_argument("--cg-rtol-coarse", type=float, default=5e-3,
                    help="CG tolerance on the coarse levels (0: --cg-rtol)")
    ap.add_argument("--cg-adapt", type=float, default=0.0,
                    help="CG rtol of MGRIT iteration k = clamp(cg_adapt x relative residual, cg_rtol, 1e-4)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving trace and the many-instance batch")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--skip-reference", action="store_true",
                    help="time MGRIT only (no sequential reference, no accuracy check): for profiler runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (the time-sharded form is not implemented); "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    if args.calibrate_copy:
        from paper_1805_06688_amd import profiling
        profiling.copy(512)
        return
    from paper_1805_06688_amd import mgrit, workloads as wl

    if args.workload == "vcycle-255":
        W = wl.FP64_VCYCLE_255
        t = wl.uniform_grid(W["Nt"], W["T"])
    elif args.workload == "mixed-511":
        W = wl.mixed_511()
        t = wl.graded_grid(W["Nt"], W["T"])
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    nx, ny, Nt = W["Mx"] - 1, W["My"] - 1, W["Nt"]
    if args.cpu_steps <= 0:
        args.cpu_steps = 200 if nx <= 255 else 25
    F, psi0 = wl.random_inputs(W["seed"], Nt, nx, ny)
    torch.cuda.set_device(0)
    Fd = torch.from_numpy(F).cuda()
    pd = torch.from_numpy(psi0).cuda()
    common = (W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"], t)
    note(f"inputs ready: {W['name']}")

    Uref, seq_s, seq_err = None, None, None
    if not args.skip_reference:
        # FP64 sequential reference (outside the timed region)
        with mgrit.Solver(*common, m=W["m"], cg_rtol=1e-13, cg_maxit=100000, precond=args.precond) as ref:
            Uref, _, _ = ref.sequential(Fd, pd)
        note("FP64 sequential reference done")
        torch.cuda.synchronize()
        # sequential stepping at the benchmark CG tolerance, for comparison
        with mgrit.Solver(*common, m=W["m"], cg_rtol=args.cg_rtol, cg_maxit=100000, precond=args.precond) as sq:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Useq, _, _ = sq.sequential(Fd, pd)
            torch.cuda.synchronize()
            seq_s = time.perf_counter() - t0
        seq_err = float(torch.linalg.norm(Useq - Uref) / torch.linalg.norm(Uref))
        note("sequential stepping at the benchmark tolerance done")
        del Useq

    stream = None
    if args.graphs:                       # graph capture needs a stream of its own
        import ctypes
        side = torch.cuda.Stream()
        stream = ctypes.c_void_p(side.cuda_stream)
    torch.cuda.synchronize()
    s = mgrit.Solver(*common, stream=stream, m=W["m"], max_levels=args.max_levels, coarse=args.coarse, cg_rtol=args.cg_rtol,
                     cg_maxit=100000,
                     tol_abs=0.0, tol_rel=args.tol_rel, max_iter=40, precond=args.precond,
                     cg_rtol_adapt=args.cg_adapt, tile=args.tile, cg_rtol_coarse=args.cg_rtol_coarse,
                     precision=args.precision, inner_rtol=args.inner_rtol, graphs=args.graphs, op=args.op,
                     coarse_relax=args.coarse_relax, relax=args.relax)
    U = torch.empty((Nt + 1) * nx * ny, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        s.solve(Fd, pd, out=U)
    torch.cuda.synchronize()
    note("warm-up done")
    s.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st, rc = s.solve(Fd, pd, out=U)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    note(f"timed solves done: {elapsed / args.steps * 1e3:.1f} ms each")
    prof = [s.profile_read(v) for v in (0, 1, 2, 3)]
    s.profile(False)
    levels = s.levels()
    err = None if Uref is None else float(torch.linalg.norm(U.view(Nt + 1, ny, nx) - Uref) / torch.linalg.norm(Uref))
    s.close()

    # the plain FP64 form of the same solver (same options, FP64 inner solves), beside the chosen form
    forms = None
    if args.precision != "fp64" and not args.skip_reference:
        with mgrit.Solver(*common, m=W["m"], max_levels=args.max_levels, coarse=args.coarse, cg_rtol=args.cg_rtol,
                          cg_maxit=100000, tol_abs=0.0, tol_rel=args.tol_rel, max_iter=40, precond=args.precond,
                          cg_rtol_coarse=args.cg_rtol_coarse, op=args.op, coarse_relax=args.coarse_relax,
                          relax=args.relax) as s64:
            U64 = torch.empty_like(U)
            s64.solve(Fd, pd, out=U64)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                _, st64, rc64 = s64.solve(Fd, pd, out=U64)
            torch.cuda.synchronize()
            t64 = (time.perf_counter() - t1) / args.steps
        note("FP64 form done")
        err64 = float(torch.linalg.norm(U64.view(Nt + 1, ny, nx) - Uref) / torch.linalg.norm(Uref))
        forms = {"fp64": {"dof_per_s": nx * ny * Nt / t64, "ms_per_step": t64 * 1e3, "rel_l2_err": err64,
                          "mgrit_iterations": st64.iterations, "rc": rc64},
                 args.precision: {"dof_per_s": nx * ny * Nt / (elapsed / args.steps),
                                  "ms_per_step": elapsed / args.steps * 1e3, "rel_l2_err": err}}
        del U64

    dof = nx * ny * Nt
    per_step = elapsed / args.steps
    fft = args.op == "fft" or (args.op == "auto" and 2 * max(nx, ny) - 1 <= 1024)
    if fft:
        # one operator application by FFT: per direction ceil(n_lines / 2) packed output pairs, each one
        # forward and one inverse transform of L points and the spectral combination with the three
        # kernels (76 flops per frequency).  Transform flops as the kernel computes them, per lane:
        # L = 512: a radix-8 DFT (56) and two twiddled ones (78 + 56 each), 64 lanes: 20736;
        # L = 1024: a radix-16 DFT (192) and two passes of two twiddled radix-8 DFTs (268 each): 46592
        L = 512 if 2 * max(nx, ny) - 1 <= 512 else 1024
        tflops = 20736 if L == 512 else 46592
        flops_per_apply = float(((ny + 1) // 2 + (nx + 1) // 2) * (2 * tflops + 76 * L))
        names = ["k_fft_line<double,0,2> + <double,1,2> (CG operator by FFT, x and y passes, FP64)", "",
                 "k_fft_line32<0,2> + <1,2> (inner CG operator of mixed precision by FFT, FP32)", ""]
        bound = "alu"
        peaks = [FP64_PEAK_TFLOPS, FP64_PEAK_TFLOPS, FP32_VECTOR_PEAK_TFLOPS, FP32_VECTOR_PEAK_TFLOPS]
        tfile = FFT_TRAFFIC_FILE
    else:
        # dense Toeplitz products: three factors per direction, 2 n flops per entry and factor
        flops_per_apply = 6.0 * nx * nx * ny + 6.0 * nx * ny * ny
        names = ["k_prop_apply<64,2> (CG operator, FP64 MFMA, 64-point tiles)",
                 "k_prop_apply<32,2> (CG operator, FP64 MFMA, 32-point tiles)",
                 "k_apply32<64> (inner CG operator of mixed precision, FP32 MFMA, 64-point tiles)",
                 "k_apply32<32> (inner CG operator of mixed precision, FP32 MFMA, 32-point tiles)"]
        bound = "mfma"
        peaks = [FP64_PEAK_TFLOPS, FP64_PEAK_TFLOPS, FP32_PEAK_TFLOPS, FP32_PEAK_TFLOPS]
        tfile = TRAFFIC_FILE

    def achieved(v):
        ms, n, sl = prof[v]
        return flops_per_apply * sl / (ms * 1e-3) / 1e12 if ms > 0 else None

    from paper_1805_06688_amd import profiling
    # dominant kernel: the operator variant with the most kernel time
    v0 = max(range(4), key=lambda v: prof[v][0])
    traffic = None
    if os.path.exists(tfile) and args.workload == "vcycle-255":      # the counters were taken on that workload
        with open(tfile) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == profiling.source_hash() and tr.get("variant") == v0:
            traffic = tr.get("bytes_per_launch")
    ms0, n0, sl0 = prof[v0]
    a0 = achieved(v0)
    roofline = {"bound": bound, "kernel": names[v0], "achieved": a0, "peak": peaks[v0], "unit": "TFLOP/s",
                "frac": a0 / peaks[v0] if a0 else None, "traffic": traffic,
                "avg_launch_ms": ms0 / n0 if n0 else None, "launches": n0,
                "slice_applies_per_launch": sl0 / n0 if n0 else None, "flops_per_slice_apply": flops_per_apply,
                "other_variants": [{"kernel": names[v].split(" (")[0], "achieved_tflops": achieved(v),
                                    "launches": prof[v][1], "total_ms": prof[v][0],
                                    "avg_launch_ms": prof[v][0] / prof[v][1] if prof[v][1] else None}
                                   for v in range(4) if v != v0 and prof[v][1]]}
    if fft and sl0:
        # the same launches against HBM: bytes the operator must move (read v, write the result)
        word = 8 if v0 < 2 else 4
        byt = 2.0 * word * nx * ny * sl0 / n0
        roofline["hbm_view"] = {"algorithmic_bytes_per_launch": byt,
                                "achieved_GBps": byt / (ms0 / n0 * 1e-3) / 1e9, "peak_GBps": HBM_PEAK_GBPS}
    out = {"metric": METRIC, "value": dof / per_step, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": per_step * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": ("f64" if args.precision == "fp64" else "f64+f32") + ("+bf16" if args.precond == "fd-bf16" else ""), "data": "synthetic",
           "config": {"workload": W["name"], "nx": nx, "ny": ny, "Nt": Nt, "beta": W["beta"], "gamma": W["gamma"],
                      "Kx": W["Kx"], "Ky": W["Ky"], "m": W["m"], "levels": levels, "relax": args.relax,
                      "coarse": args.coarse, "precond": args.precond, "cg_rtol": args.cg_rtol,
                      "tol_rel": args.tol_rel, "cg_rtol_adapt": args.cg_adapt, "tile": args.tile,
                      "cg_rtol_coarse": args.cg_rtol_coarse, "precision": args.precision,
                      "inner_rtol": args.inner_rtol, "refinements_per_solve": st.refinements,
                      "graphs": args.graphs, "operator": args.op,
                      "coarse_relax": args.coarse_relax or "FCF",
                      "mgrit_iterations": st.iterations, "phi_per_solve": st.phi_applications,
                      "cg_iterations_per_solve": st.cg_iterations, "rel_l2_err_vs_fp64_sequential": err,
                      "sequential_dof_per_s": dof / seq_s if seq_s else None, "sequential_rel_l2_err": seq_err,
                      "parallelism": "time (MGRIT), one GPU"},
           "roofline": roofline}
    if forms:
        out["forms"] = forms
    if not args.no_serving and not args.skip_reference:
        out["serving"] = serving(mgrit, wl, torch, 32, 4.0, 4, 64)
        out["many_instance"] = many_instance(mgrit, wl, torch, 16, 4)
    if not args.no_cpu and not args.skip_reference:
        out["cpu_baseline"] = cpu_baseline(W, t, F, psi0, args.cpu_steps, args.cg_rtol)
    print(json.dumps(out), flush=True)
    if args.skip_reference:
        return
    if not (err <= 1e-8 and rc == 0):
        print(f"accuracy target missed: rel_l2_err={err:.3e} rc={rc}", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
