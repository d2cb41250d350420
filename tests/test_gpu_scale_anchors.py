"""The benchmark's references tied to the CPU oracle at the benchmark geometries.

The benchmark measures its error against FP64 sequential stepping on the GPU (CG to a relative
residual of 1e-13, fast-diagonalisation preconditioner with BF16 products), because the oracle
cannot step 1024 or 4096 steps of these grids in seconds.  Here that reference is compared with the
oracle's sequential stepping (plain CG to 1e-14, eq. chp-02-03) over stretches of the same time grids:
the first 48 steps of the 255 x 255 uniform grid, and 8 steps at the start and 12 in the middle of the
511 x 511 graded grid (t_n = (n/N)^2, where the steps are 2.4e-4 long).  Each step solves to 1e-13
relative residual with a condition number of B_n below 1e3 here, so the reference must agree with the
oracle to 1e-10, a hundredth of the benchmark's accuracy bar.  A serving request, run with the
benchmark's mixed-precision options, is compared with the oracle at that bar (1e-8).
"""
import numpy as np
import pytest

from oracle import fem, propagator
from paper_1805_06688_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REF_OPTS = dict(cg_rtol=1e-13, cg_maxit=100000, precond="fd-bf16")      # the benchmark's FP64 reference


def _mg():
    from paper_1805_06688_amd import mgrit
    return mgrit


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _anchor(W, t, seed):
    mg = _mg()
    prob = fem.Problem(W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"])
    op = fem.Operator(prob)
    N = len(t) - 1
    F, psi0 = wl.random_inputs(seed, N, prob.nx, prob.ny)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14, 100000), t, F, psi0)
    with mg.Solver(W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"], t, m=4, **REF_OPTS) as s:
        U, st, rc = s.sequential(dev(F), dev(psi0))
        U = U.cpu().numpy()
    assert rc == 0 and st.phi_applications == N
    err = rel(U, ref)
    print(f"{W['name']}: {N} steps, GPU FP64 reference vs oracle {err:.3e}")
    assert err <= 1e-10, err


def test_fp64_reference_255_uniform_matches_oracle():
    W = wl.FP64_VCYCLE_255
    _anchor(W, wl.uniform_grid(W["Nt"])[:49], W["seed"])


def test_fp64_reference_511_graded_start_matches_oracle():
    W = wl.mixed_511()
    _anchor(W, wl.graded_grid(W["Nt"])[:9], W["seed"])


def test_fp64_reference_511_graded_middle_matches_oracle():
    """Steps 2049..2060 of the graded grid (the propagators depend on the step lengths only)."""
    W = wl.mixed_511()
    t = wl.graded_grid(W["Nt"])[2048:2061]
    _anchor(W, t - t[0], W["seed"])


def test_serving_requests_match_oracle():
    """Three requests in flight at once, with the benchmark's mixed-precision options, each against the
    oracle's sequential stepping at the accuracy bar of the mixed form."""
    mg = _mg()
    reqs = [(70, 63, 48, 0.6, 0.9), (95, 64, 64, 0.8, 0.7), (63, 100, 40, 0.9, 0.55)]
    opts = dict(m=8, coarse="opt", precond="fd-bf16", cg_rtol=1e-9, cg_rtol_coarse=5e-3, precision="mixed",
                cg_maxit=100000, tol_abs=0.0, tol_rel=1e-8, max_iter=40, max_levels=3)
    inputs, handles = [], []
    with mg.Server(8 << 30, max_concurrent=3) as srv:
        for k, (Mx, My, Nt, beta, gamma) in enumerate(reqs):
            t = wl.uniform_grid(Nt)
            F, psi0 = wl.random_inputs(500 + k, Nt, Mx - 1, My - 1)
            inputs.append((t, F, psi0))
            handles.append(srv.submit(dev(F), dev(psi0), beta, gamma, 1.0, 1.0, Mx, My, t, **opts))
        outs = [h.wait() for h in handles]
    for (Mx, My, Nt, beta, gamma), (t, F, psi0), (U, info) in zip(reqs, inputs, outs):
        assert info.rc == 0
        prob = fem.Problem(beta, gamma, 1.0, 1.0, Mx, My)
        op = fem.Operator(prob)
        ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14, 100000), t, F, psi0)
        err = rel(U.cpu().numpy(), ref)
        print(f"request {Mx - 1}x{My - 1}x{Nt}: {info.stats.iterations} MGRIT iterations, error {err:.3e}")
        assert err <= 1e-8, err
