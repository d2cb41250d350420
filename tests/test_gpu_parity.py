"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerance: relative l2 <= 1e-10 for FP64 results of solves (both sides run CG
to rtol 1e-14; the remaining gap is the conditioning of B_n times rounding);
<= 1e-13 (relative to the largest entry) for a single operator application.
"""
import math

import numpy as np
import pytest

from oracle import fem, manufactured as mf, mgrit as omgrit, propagator
from paper_1805_06688_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mg():
    from paper_1805_06688_amd import mgrit
    return mgrit


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


GEOMS = [  # beta, gamma, Kx, Ky, Mx, My, domain
    (0.7, 0.8, 1.0, 1.0, 32, 32, (0, 1, 0, 1)),          # one tile, padded
    (0.75, 0.85, 2.0, 1.0, 96, 78, (0, 1, 0, 1)),        # 2 x 2 tiles, ragged both ways
    (0.55, 0.95, 3.0, 7.5, 131, 65, (0, 2, -1, 1)),      # 3 x 2 tiles, ragged, non-unit domain
    (0.95, 0.6, 0.5, 2.0, 65, 160, (0, 1, 0, 3)),        # exactly one tile + 1 in x
]


@pytest.mark.parametrize("geo", GEOMS)
def test_apply_matches_oracle(geo):
    beta, gamma, Kx, Ky, Mx, My, dom = geo
    mg = _mg()
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My, *dom)
    op = fem.Operator(prob)
    S = 5
    v = wl.random_slices(11, S, prob.nx, prob.ny)
    add = wl.random_slices(12, S, prob.nx, prob.ny)
    theta = np.array([0.0, 1e-3, 0.5, -0.25, 7.0])
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, wl.uniform_grid(8), domain=dom, m=2, op="dense") as s:
        for sign, use_add in ((1.0, False), (-1.0, True)):
            out = host(s.apply(theta, dev(v), sign=sign, add=dev(add) if use_add else None))
            for k in range(S):
                ref = sign * (op.apply_M(v[k]) + theta[k] * op.apply_A(v[k])) + (add[k] if use_add else 0.0)
                assert np.abs(out[k] - ref).max() <= 1e-13 * np.abs(ref).max(), (k, sign)


def test_apply_host_memory_and_empty():
    mg = _mg()
    prob = fem.Problem(0.7, 0.8, 1.0, 1.0, 40, 30)
    op = fem.Operator(prob)
    v = wl.random_slices(3, 2, prob.nx, prob.ny)
    with mg.Solver(0.7, 0.8, 1.0, 1.0, 40, 30, wl.uniform_grid(4), m=2) as s:
        out = s.apply([0.3, 0.0], v)                    # numpy in, numpy out
        for k in range(2):
            ref = op.apply_M(v[k]) + [0.3, 0.0][k] * op.apply_A(v[k])
            assert np.abs(out[k] - ref).max() <= 1e-13 * np.abs(ref).max()
        s.apply(np.zeros(0), np.zeros(0))                # zero slices is a no-op


@pytest.mark.parametrize("geo", GEOMS[:3])
def test_propagate_level0_matches_oracle(geo):
    beta, gamma, Kx, Ky, Mx, My, dom = geo
    mg = _mg()
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My, *dom)
    op = fem.Operator(prob)
    t = wl.random_grid(12, 5)
    steps = [1, 4, 7, 12]
    u = wl.random_slices(21, len(steps), prob.nx, prob.ny)
    F = wl.random_slices(22, len(steps), prob.nx, prob.ny)
    solver = propagator.CGSolver(op, 1e-14, 20000)
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, t, domain=dom, m=2, cg_rtol=1e-14, cg_maxit=20000, op="dense") as s:
        out = host(s.propagate(0, steps, dev(u), dev(F)))
    for i, k in enumerate(steps):
        ref = propagator.cn_step(op, solver, t[k] - t[k - 1], u[i], F[i])
        assert rel(out[i], ref) <= 1e-10, (i, k, rel(out[i], ref))


@pytest.mark.parametrize("coarse,opk", [("cn", "dense"), ("be", "dense"), ("cn2", "dense"), ("opt", "dense"),
                                        ("cn", "fft"), ("opt", "fft")])
def test_propagate_coarse_level_matches_oracle(coarse, opk):
    mg = _mg()
    beta, gamma, Kx, Ky, Mx, My = 0.75, 0.85, 2.0, 1.0, 70, 66
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My)
    op = fem.Operator(prob)
    t = wl.random_grid(32, 9)
    m = 4
    osolver = omgrit.MGRIT(op, t, m, max_levels=3, coarse=coarse, cg_rtol=1e-14)
    steps = [1, 3, 8]
    u = wl.random_slices(31, 3, prob.nx, prob.ny)
    g = wl.random_slices(32, 3, prob.nx, prob.ny)
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, t, m=m, max_levels=3, coarse=coarse, cg_rtol=1e-14, op=opk) as s:
        assert s.levels() == [32, 8, 2]
        out = host(s.propagate(1, steps, dev(u), dev(g)))
        out_nog = host(s.propagate(1, steps, dev(u)))
    for i, k in enumerate(steps):
        ref = osolver.psi(1, k, u[i])
        assert rel(out_nog[i], ref) <= 1e-10
        assert rel(out[i], ref + g[i]) <= 1e-10


def _random_problem(seed, Nt, beta=0.7, gamma=0.8, Mx=40, My=34, Kx=1.0, Ky=1.0):
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My)
    t = wl.random_grid(Nt, seed)
    F, psi0 = wl.random_inputs(seed, Nt, prob.nx, prob.ny)
    return prob, t, F, psi0


def test_sequential_matches_oracle():
    mg = _mg()
    prob, t, F, psi0 = _random_problem(1, 20)
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    with mg.Solver(prob.beta, prob.gamma, 1.0, 1.0, prob.Mx, prob.My, t, m=4, cg_rtol=1e-14) as s:
        U, st, _ = s.sequential(dev(F), dev(psi0))
        U = host(U)
    assert rel(U, ref) <= 1e-10
    assert st.phi_applications == 20


CASES = [  # m, levels, relax, coarse, Nt
    (4, 2, "FCF", "cn", 32),
    (2, 4, "FCF", "be", 24),
    (3, 3, "FCF", "cn2", 29),          # Nt not a multiple of m: trailing F-points
    (4, 3, "F", "be", 37),
    (4, 3, "FCF", "opt", 34),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("iters", [1, 2, 3])
def test_mgrit_iterates_match_oracle(case, iters):
    """The iterate after k MGRIT iterations (plus final F-relaxation) equals the oracle's, step for step."""
    m, levels, relax, coarse, Nt = case
    mg = _mg()
    prob, t, F, psi0 = _random_problem(7 + Nt, Nt)
    op = fem.Operator(prob)
    U0 = wl.random_slices(99, Nt + 1, prob.nx, prob.ny)
    o = omgrit.MGRIT(op, t, m, max_levels=levels, relax=relax, coarse=coarse, cg_rtol=1e-14)
    ref = o.iterate(F, psi0, iters, U0=U0)
    with mg.Solver(prob.beta, prob.gamma, 1.0, 1.0, prob.Mx, prob.My, t, m=m, max_levels=levels, relax=relax,
                   coarse=coarse, cg_rtol=1e-14) as s:
        assert s.levels() == [lv.N for lv in o.levels]
        U, st, _ = s.iterate(dev(F), dev(psi0), iters, U_init=dev(U0))
        U = host(U)
    assert rel(U, ref) <= 1e-10, rel(U, ref)


@pytest.mark.parametrize("case", CASES[:3] + CASES[4:])
def test_mgrit_solve_reaches_sequential(case):
    m, levels, relax, coarse, Nt = case
    mg = _mg()
    prob, t, F, psi0 = _random_problem(3, Nt)
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    o = omgrit.MGRIT(op, t, m, max_levels=levels, relax=relax, coarse=coarse, cg_rtol=1e-14)
    _, oit, oconv, ohist = o.solve(F, psi0, tol=1e-9, max_iter=50, return_history=True)
    with mg.Solver(prob.beta, prob.gamma, 1.0, 1.0, prob.Mx, prob.My, t, m=m, max_levels=levels, relax=relax,
                   coarse=coarse, cg_rtol=1e-14, tol_abs=1e-9, max_iter=50) as s:
        U, st, rc = s.solve(dev(F), dev(psi0))
        U = host(U)
    assert rc == 0 and st.converged == 1
    assert st.iterations == oit
    hist = st.history()
    assert np.allclose(hist, ohist[: len(hist)], rtol=1e-6, atol=1e-12 * ohist[0])   # rounding-level tail
    assert rel(U, ref) <= 1e-10


def test_manufactured_two_level_workload():
    """31 x 31 nodes, beta 0.7, gamma 0.8, K = 1, 64 uniform steps, two-level FCF m = 4,
    u = x^2(1-x)^2 y^2(1-y)^2 e^{-t}: MGRIT equals sequential stepping and the L2 error is O(h^2)."""
    mg = _mg()
    W = wl.FP64_TWOLEVEL_31
    M = W["Mx"]
    prob = fem.Problem(W["beta"], W["gamma"], W["Kx"], W["Ky"], M, M)
    op = fem.Operator(prob)
    t = wl.uniform_grid(W["Nt"])
    F = mf.load_vectors(t, W["beta"], W["gamma"], W["Kx"], W["Ky"], M, amp=W["amp"])
    psi0 = mf.nodal_psi0(M, amp=W["amp"])
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    with mg.Solver(W["beta"], W["gamma"], W["Kx"], W["Ky"], M, M, t, m=W["m"], max_levels=W["levels"],
                   cg_rtol=1e-14, tol_abs=1e-13, max_iter=40) as s:
        U, st, rc = s.solve(dev(F), dev(psi0))
        U = host(U)
    assert rc == 0
    assert st.iterations <= math.ceil(16 / 2)          # finite termination bound for two levels
    assert rel(U, ref) <= 1e-10
    err = mf.l2_error(U[-1], 1.0, M, amp=W["amp"])
    assert err < 2e-5


def test_zero_data_gives_zero_and_noconv_code():
    mg = _mg()
    prob, t, F, psi0 = _random_problem(4, 16)
    with mg.Solver(prob.beta, prob.gamma, 1.0, 1.0, prob.Mx, prob.My, t, m=4, cg_rtol=1e-14, max_iter=1,
                   tol_abs=0.0) as s:
        U, st, rc = s.solve(dev(np.zeros_like(F)), dev(np.zeros_like(psi0)))
        assert not torch.any(U != 0)
        U, st, rc = s.solve(dev(F), dev(psi0))
        assert rc == mg.ENOCONV and st.converged == 0 and st.iterations == 1


def test_full_size_apply_and_step_sampled():
    """Benchmark geometry (255 x 255, beta 0.75, gamma 0.85, K = (2, 1)): operator and one step on sampled slices."""
    mg = _mg()
    W = wl.FP64_VCYCLE_255
    prob = fem.Problem(W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"])
    op = fem.Operator(prob)
    t = wl.uniform_grid(W["Nt"])
    u = wl.random_slices(5, 3, prob.nx, prob.ny)
    F = wl.random_slices(6, 3, prob.nx, prob.ny)
    with mg.Solver(W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"], t, m=W["m"], cg_rtol=1e-14, op="dense") as s:
        theta = np.array([0.5 / 1024, 4.0 / 1024, 0.0])
        out = host(s.apply(theta, dev(u)))
        steps = [1, 500, 1024]
        prop = host(s.propagate(0, steps, dev(u), dev(F)))
    for k in range(3):
        ref = op.apply_M(u[k]) + theta[k] * op.apply_A(u[k])
        assert np.abs(out[k] - ref).max() <= 1e-13 * np.abs(ref).max()
    solver = propagator.CGSolver(op, 1e-14, 20000)
    ref = propagator.cn_step(op, solver, t[1] - t[0], u[0], F[0])
    assert rel(prop[0], ref) <= 1e-10


@pytest.mark.parametrize("level,coarse,pc", [(0, "cn", "fd"), (1, "opt", "fd"), (1, "be", "fd"), (0, "cn", "fd-bf16"),
                                             (1, "opt", "fd-bf16")])
def test_preconditioned_propagate_matches_oracle(level, coarse, pc):
    """PCG with the fast-diagonalisation preconditioner (FP64 or BF16 products) converges to the same
    propagator as plain CG."""
    mg = _mg()
    beta, gamma, Kx, Ky, Mx, My = 0.65, 0.9, 2.0, 0.5, 97, 70
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My)
    op = fem.Operator(prob)
    t = wl.random_grid(24, 13)
    o = omgrit.MGRIT(op, t, 4, max_levels=3, coarse=coarse, cg_rtol=1e-14)
    steps = [1, 2, 5] if level else [1, 9, 24]
    u = wl.random_slices(41, 3, prob.nx, prob.ny)
    g = wl.random_slices(42, 3, prob.nx, prob.ny)
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, t, m=4, max_levels=3, coarse=coarse, cg_rtol=1e-14,
                   precond=pc, op="dense") as s:
        out = host(s.propagate(level, steps, dev(u), dev(g)))
    solver = propagator.CGSolver(op, 1e-14, 20000)
    for i, k in enumerate(steps):
        if level == 0:
            ref = propagator.cn_step(op, solver, t[k] - t[k - 1], u[i], g[i])
        else:
            ref = o.psi(1, k, u[i]) + g[i]
        assert rel(out[i], ref) <= 1e-10, (i, rel(out[i], ref))


@pytest.mark.parametrize("iters,pc", [(1, "fd"), (3, "fd"), (2, "fd-bf16")])
def test_preconditioned_mgrit_iterates_match_oracle(iters, pc):
    mg = _mg()
    prob, t, F, psi0 = _random_problem(5, 40, beta=0.75, gamma=0.85, Mx=70, My=66, Kx=2.0, Ky=1.0)
    op = fem.Operator(prob)
    U0 = wl.random_slices(98, 41, prob.nx, prob.ny)
    o = omgrit.MGRIT(op, t, 4, max_levels=3, coarse="opt", cg_rtol=1e-14)
    ref = o.iterate(F, psi0, iters, U0=U0)
    with mg.Solver(prob.beta, prob.gamma, 2.0, 1.0, prob.Mx, prob.My, t, m=4, max_levels=3, coarse="opt",
                   cg_rtol=1e-14, precond=pc) as s:
        U, st, _ = s.iterate(dev(F), dev(psi0), iters, U_init=dev(U0))
        U = host(U)
    assert rel(U, ref) <= 1e-10
    assert st.cg_iterations / st.phi_applications < 30


def test_adaptive_cg_tolerance_reaches_sequential():
    """Loose CG tolerances in early MGRIT iterations (tightening with the residual) keep the fixed point."""
    mg = _mg()
    prob, t, F, psi0 = _random_problem(6, 48, beta=0.75, gamma=0.85, Mx=66, My=70, Kx=2.0, Ky=1.0)
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    with mg.Solver(prob.beta, prob.gamma, 2.0, 1.0, prob.Mx, prob.My, t, m=4, max_levels=3, coarse="opt",
                   precond="fd", cg_rtol=1e-13, cg_rtol_adapt=1e-3, tol_abs=0.0, tol_rel=1e-12, max_iter=30) as s:
        U, st, rc = s.solve(dev(F), dev(psi0))
        U = host(U)
    assert rc == 0
    assert rel(U, ref) <= 1e-10


def test_warm_start_keeps_fixed_point_and_saves_iterations():
    """Starting CG from the previous iterate at the target point changes only the CG iteration count."""
    mg = _mg()
    prob, t, F, psi0 = _random_problem(8, 64, beta=0.75, gamma=0.85, Mx=66, My=60, Kx=2.0, Ky=1.0)
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    out = {}
    for warm in (False, True):
        with mg.Solver(prob.beta, prob.gamma, 2.0, 1.0, prob.Mx, prob.My, t, m=4, max_levels=3, coarse="opt",
                       precond="fd", cg_rtol=1e-13, tol_abs=0.0, tol_rel=1e-12, max_iter=30, warm_start=warm) as s:
            U, st, rc = s.solve(dev(F), dev(psi0))
            assert rc == 0
            out[warm] = (host(U), st.cg_iterations, st.iterations)
    assert rel(out[True][0], ref) <= 1e-10 and rel(out[False][0], ref) <= 1e-10
    assert out[True][2] == out[False][2]
    assert out[True][1] < 0.8 * out[False][1]


@pytest.mark.parametrize("pc", ["none", "fd", "fd-bf16"])
def test_tile_policy_changes_speed_only(pc):
    """64- and 32-node operator tiles (forced, by rule or autotuned) give bitwise the same solve."""
    mg = _mg()
    prob, t, F, psi0 = _random_problem(9, 32, beta=0.7, gamma=0.9, Mx=97, My=70, Kx=1.5, Ky=1.0)
    out = {}
    for tile in ("64", "32", "rule", "auto"):
        with mg.Solver(prob.beta, prob.gamma, 1.5, 1.0, prob.Mx, prob.My, t, m=4, max_levels=3, coarse="opt",
                       precond=pc, cg_rtol=1e-12, tol_abs=0.0, tol_rel=1e-10, max_iter=30, tile=tile,
                       op="dense") as s:
            U, st, rc = s.solve(dev(F), dev(psi0))
            assert rc == 0
            out[tile] = (U.clone(), st.cg_iterations, st.iterations, st.history())
    base = out["64"]
    for tile, (U, cg, its, hist) in out.items():
        assert torch.equal(U, base[0]), tile
        assert (cg, its, hist) == base[1:], tile
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    assert rel(host(base[0]), ref) <= 1e-9


def test_loose_coarse_cg_keeps_fixed_point():
    """Coarse-level propagators solved to a loose CG tolerance change the corrections, not the fixed point."""
    mg = _mg()
    prob, t, F, psi0 = _random_problem(10, 64, beta=0.8, gamma=0.7, Mx=70, My=58, Kx=1.0, Ky=2.0)
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    its = {}
    for rc_coarse in (0.0, 1e-3):
        with mg.Solver(prob.beta, prob.gamma, 1.0, 2.0, prob.Mx, prob.My, t, m=4, max_levels=3, coarse="opt",
                       precond="fd-bf16", cg_rtol=1e-13, cg_rtol_coarse=rc_coarse, tol_abs=0.0, tol_rel=1e-12,
                       max_iter=40) as s:
            U, st, rc = s.solve(dev(F), dev(psi0))
            assert rc == 0
            assert rel(host(U), ref) <= 1e-10, rc_coarse
            its[rc_coarse] = (st.iterations, st.cg_iterations)
    assert its[1e-3][1] < its[0.0][1]


@pytest.mark.parametrize("level,coarse,pc", [(0, "cn", "fd-bf16"), (1, "opt", "fd-bf16"), (0, "cn", "none"),
                                             (1, "be", "none")])
def test_mixed_precision_propagate_matches_oracle(level, coarse, pc):
    """Iterative refinement with FP32 inner PCG reaches the FP64 propagator."""
    mg = _mg()
    beta, gamma, Kx, Ky, Mx, My = 0.7, 0.85, 1.0, 2.0, 90, 75
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My)
    op = fem.Operator(prob)
    t = wl.random_grid(16, 21)
    o = omgrit.MGRIT(op, t, 4, max_levels=3, coarse=coarse, cg_rtol=1e-14)
    steps = [1, 3, 4] if level else [1, 8, 16]
    u = wl.random_slices(51, 3, prob.nx, prob.ny)
    g = wl.random_slices(52, 3, prob.nx, prob.ny)
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, t, m=4, max_levels=3, coarse=coarse, cg_rtol=1e-13,
                   precond=pc, precision="mixed", op="dense") as s:
        out = host(s.propagate(level, steps, dev(u), dev(g)))
    solver = propagator.CGSolver(op, 1e-14, 20000)
    for i, k in enumerate(steps):
        if level == 0:
            ref = propagator.cn_step(op, solver, t[k] - t[k - 1], u[i], g[i])
        else:
            ref = o.psi(1, k, u[i]) + g[i]
        assert rel(out[i], ref) <= 1e-10, (i, rel(out[i], ref))


@pytest.mark.parametrize("pc", ["fd-bf16", "none"])
def test_loose_mixed_pass_meets_its_tolerance(pc):
    """A mixed-precision pass at a CG tolerance of 1e-4 or looser forms its right-hand side and initial
    residual in FP32 (from the FP64 data) and settles in one refinement step; its result still meets the
    stop criterion ||b - B x|| <= rtol ||b||, b = C u + F, evaluated in FP64 by the oracle."""
    mg = _mg()
    beta, gamma, Kx, Ky, Mx, My = 0.65, 0.9, 1.5, 1.0, 80, 70
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My)
    op = fem.Operator(prob)
    t = wl.random_grid(17, 9)
    steps = [1, 4, 8]
    u = wl.random_slices(61, 3, prob.nx, prob.ny)
    f = wl.random_slices(62, 3, prob.nx, prob.ny)
    rtol = 2e-3
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, t, m=4, cg_rtol=rtol, precond=pc, precision="mixed") as s:
        out = host(s.propagate(0, steps, dev(u), dev(f)))
    for i, k in enumerate(steps):
        tau = t[k] - t[k - 1]
        b = op.apply_C(u[i], tau) + f[i]
        r = b - op.apply_B(out[i], tau)
        assert np.linalg.norm(r) <= 1.01 * rtol * np.linalg.norm(b), (i, np.linalg.norm(r) / np.linalg.norm(b))


@pytest.mark.parametrize("precision", ["mixed", "mixed-coarse"])
def test_mixed_precision_solve_reaches_sequential(precision):
    mg = _mg()
    prob, t, F, psi0 = _random_problem(12, 64, beta=0.75, gamma=0.85, Mx=72, My=66, Kx=2.0, Ky=1.0)
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    with mg.Solver(prob.beta, prob.gamma, 2.0, 1.0, prob.Mx, prob.My, t, m=4, max_levels=3, coarse="opt",
                   precond="fd-bf16", cg_rtol=1e-13, cg_rtol_coarse=1e-3, tol_abs=0.0, tol_rel=1e-12, max_iter=40,
                   precision=precision) as s:
        U, st, rc = s.solve(dev(F), dev(psi0))
        assert rc == 0
        assert st.refinements > 0
        assert rel(host(U), ref) <= 1e-10
        Useq, st2, _ = s.sequential(dev(F), dev(psi0))
        assert rel(host(Useq), ref) <= 1e-10
        assert (st2.refinements > 0) == (precision == "mixed")


def test_mixed_precision_zero_data():
    mg = _mg()
    prob, t, F, psi0 = _random_problem(4, 16)
    with mg.Solver(prob.beta, prob.gamma, 1.0, 1.0, prob.Mx, prob.My, t, m=4, max_levels=2, precision="mixed",
                   precond="fd-bf16") as s:
        U, st, rc = s.solve(dev(np.zeros_like(F)), dev(np.zeros_like(psi0)))
        assert not torch.any(U != 0) and not torch.isnan(U).any()
        assert st.refinements == 0


@pytest.mark.parametrize("precision,pc", [("fp64", "fd-bf16"), ("fp64", "none"), ("mixed", "fd-bf16")])
def test_graph_replay_matches_direct_launches(precision, pc):
    """Pairs of CG iterations replayed as captured HIP graphs give bitwise the results of direct launches, on
    every replay (three solves per handle, with other GPU work and synchronisation between them)."""
    import ctypes
    mg = _mg()
    prob, t, F, psi0 = _random_problem(13, 32, beta=0.7, gamma=0.9, Mx=80, My=60, Kx=1.0, Ky=1.5)
    Fd, pd = dev(F), dev(psi0)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    res = {}
    for graphs in (False, True):
        outs = []
        with mg.Solver(prob.beta, prob.gamma, 1.0, 1.5, prob.Mx, prob.My, t, stream=ctypes.c_void_p(side.cuda_stream),
                       m=4, max_levels=3, coarse="opt", precond=pc, precision=precision, cg_rtol=1e-12,
                       cg_rtol_coarse=1e-3, tol_abs=0.0, tol_rel=1e-10, max_iter=30, graphs=graphs) as s:
            for rep in range(3):
                U, st, rc = s.solve(Fd, pd)
                side.synchronize()
                assert rc == 0
                outs.append((U.clone(), st.cg_iterations, st.iterations))
                junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
                torch.cuda.synchronize()
                assert torch.isfinite(junk)
        res[graphs] = outs
    for (Ua, ca, ia), (Ub, cb, ib) in zip(res[False], res[True]):
        assert torch.equal(Ua, Ub) and ca == cb and ia == ib


@pytest.mark.parametrize("geo", GEOMS)
def test_fft_operator_apply_matches_oracle(geo):
    """The operator by circulant-embedded FFTs equals the dense Toeplitz products to rounding."""
    beta, gamma, Kx, Ky, Mx, My, dom = geo
    mg = _mg()
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My, *dom)
    op = fem.Operator(prob)
    S = 5
    v = wl.random_slices(11, S, prob.nx, prob.ny)
    add = wl.random_slices(12, S, prob.nx, prob.ny)
    theta = np.array([0.0, 1e-3, 0.5, -0.25, 7.0])
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, wl.uniform_grid(8), domain=dom, m=2, op="fft") as s:
        for sign, use_add in ((1.0, False), (-1.0, True)):
            out = host(s.apply(theta, dev(v), sign=sign, add=dev(add) if use_add else None))
            for k in range(S):
                ref = sign * (op.apply_M(v[k]) + theta[k] * op.apply_A(v[k])) + (add[k] if use_add else 0.0)
                assert np.abs(out[k] - ref).max() <= 1e-13 * np.abs(ref).max(), (k, sign)


@pytest.mark.parametrize("level,coarse,precision", [(0, "cn", "fp64"), (1, "opt", "fp64"), (0, "cn", "mixed"),
                                                    (1, "opt", "mixed")])
def test_fft_operator_propagate_matches_oracle(level, coarse, precision):
    mg = _mg()
    beta, gamma, Kx, Ky, Mx, My = 0.65, 0.9, 2.0, 0.5, 97, 70
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My)
    op = fem.Operator(prob)
    t = wl.random_grid(24, 13)
    o = omgrit.MGRIT(op, t, 4, max_levels=3, coarse=coarse, cg_rtol=1e-14)
    steps = [1, 2, 5] if level else [1, 9, 24]
    u = wl.random_slices(41, 3, prob.nx, prob.ny)
    g = wl.random_slices(42, 3, prob.nx, prob.ny)
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, t, m=4, max_levels=3, coarse=coarse, cg_rtol=1e-13,
                   precond="fd-bf16", precision=precision, op="fft") as s:
        out = host(s.propagate(level, steps, dev(u), dev(g)))
    solver = propagator.CGSolver(op, 1e-14, 20000)
    for i, k in enumerate(steps):
        ref = propagator.cn_step(op, solver, t[k] - t[k - 1], u[i], g[i]) if level == 0 else o.psi(1, k, u[i]) + g[i]
        assert rel(out[i], ref) <= 1e-10, (i, rel(out[i], ref))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fft_operator_solve_reaches_sequential(precision):
    mg = _mg()
    prob, t, F, psi0 = _random_problem(14, 64, beta=0.75, gamma=0.85, Mx=72, My=66, Kx=2.0, Ky=1.0)
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    with mg.Solver(prob.beta, prob.gamma, 2.0, 1.0, prob.Mx, prob.My, t, m=4, max_levels=3, coarse="opt",
                   precond="fd-bf16", cg_rtol=1e-13, cg_rtol_coarse=1e-3, tol_abs=0.0, tol_rel=1e-12, max_iter=40,
                   precision=precision, op="fft") as s:
        U, st, rc = s.solve(dev(F), dev(psi0))
        assert rc == 0
        assert rel(host(U), ref) <= 1e-10


def test_fft_operator_full_size_sampled():
    """255 x 255 (the largest FFT grid, 19 x 19 workgroups per pass, ragged last one): a batch of 130 slices
    through the FFT operator equals the tiled operator (itself checked against the oracle)."""
    mg = _mg()
    W = wl.FP64_VCYCLE_255
    nx = W["Mx"] - 1
    v = dev(wl.random_slices(7, 130, nx, nx))
    theta = np.linspace(-1.0, 3.0, 130)
    common = (W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"], wl.uniform_grid(16))
    with mg.Solver(*common, m=4, op="fft") as s:
        a = s.apply(theta, v)
    with mg.Solver(*common, m=4, op="dense") as s:
        b = s.apply(theta, v)
    err = float((a - b).abs().max() / b.abs().max())
    assert err <= 1e-13, err


def test_coarse_f_relaxation_keeps_fixed_point():
    """F-relaxation on the coarse levels (FCF on level 0) changes the convergence, not the solution."""
    mg = _mg()
    prob, t, F, psi0 = _random_problem(15, 64, beta=0.7, gamma=0.8, Mx=60, My=52, Kx=1.0, Ky=1.0)
    op = fem.Operator(prob)
    ref = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    with mg.Solver(prob.beta, prob.gamma, 1.0, 1.0, prob.Mx, prob.My, t, m=4, max_levels=3, coarse="opt",
                   precond="fd-bf16", cg_rtol=1e-13, tol_abs=0.0, tol_rel=1e-12, max_iter=40,
                   coarse_relax="F") as s:
        U, st, rc = s.solve(dev(F), dev(psi0))
    assert rc == 0
    assert rel(host(U), ref) <= 1e-10


@pytest.mark.parametrize("opk", ["auto", "dense"])
def test_mixed_511_full_size_sampled(opk):
    """The 511 x 511 mixed-precision geometry (graded grid of 4096 steps; dense operator, FP32 matrix cores in
    the inner solves): operator on sampled slices against the oracle; propagator steps of the mixed form equal
    the FP64 form, and the oracle's operator confirms the FP64 step by its residual."""
    mg = _mg()
    W = wl.mixed_511()
    prob = fem.Problem(W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"])
    op = fem.Operator(prob)
    t = wl.graded_grid(W["Nt"])
    u = wl.random_slices(7, 3, prob.nx, prob.ny)
    F = wl.random_slices(8, 3, prob.nx, prob.ny)
    steps = [1, 2048, 4096]
    common = (W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"], t)
    opts = dict(m=W["m"], max_levels=3, coarse="opt", precond="fd-bf16", cg_rtol=1e-12, op=opk)
    with mg.Solver(*common, precision="fp64", **opts) as s:
        theta = np.array([0.5 * (t[1] - t[0]), 0.5 * (t[-1] - t[-2]), 0.0])
        out = host(s.apply(theta, dev(u)))
        p64 = host(s.propagate(0, steps, dev(u), dev(F)))
    with mg.Solver(*common, precision="mixed", **opts) as s:
        p32 = host(s.propagate(0, steps, dev(u), dev(F)))
    for k in range(3):
        ref = op.apply_M(u[k]) + theta[k] * op.apply_A(u[k])
        assert np.abs(out[k] - ref).max() <= 1e-13 * np.abs(ref).max()
    for i, k in enumerate(steps):
        tau = t[k] - t[k - 1]
        rhs = op.apply_M(u[i]) - 0.5 * tau * op.apply_A(u[i]) + F[i]
        res = op.apply_M(p64[i]) + 0.5 * tau * op.apply_A(p64[i]) - rhs
        assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(rhs), (k, np.linalg.norm(res) / np.linalg.norm(rhs))
        assert rel(p32[i], p64[i]) <= 1e-10, (k, rel(p32[i], p64[i]))


@pytest.mark.parametrize("cg_rtol,cg_coarse,tol_rel", [(3e-10, 1e-3, 1e-9), (1e-9, 5e-3, 1e-8)])
def test_mixed_511_mgrit_reaches_fp64_sequential(cg_rtol, cg_coarse, tol_rel):
    """511 x 511, graded grid (128 steps here), mixed-precision MGRIT against FP64 sequential stepping:
    relative l2 <= 1e-8 (the bar of the mixed form), also at the benchmark's tolerances (CG 1e-9, MGRIT
    stop 1e-8, coarse-level CG 5e-3)."""
    mg = _mg()
    W = wl.mixed_511()
    Nt = 128
    t = wl.graded_grid(Nt)
    n = W["Mx"] - 1
    F, psi0 = wl.random_inputs(W["seed"], Nt, n, n)
    common = (W["beta"], W["gamma"], W["Kx"], W["Ky"], W["Mx"], W["My"], t)
    with mg.Solver(*common, m=W["m"], precond="fd-bf16", cg_rtol=1e-13) as s:
        ref, _, _ = s.sequential(dev(F), dev(psi0))
    with mg.Solver(*common, m=W["m"], max_levels=3, coarse="opt", precond="fd-bf16", precision="mixed",
                   cg_rtol=cg_rtol, cg_rtol_coarse=cg_coarse, tol_abs=0.0, tol_rel=tol_rel, max_iter=40) as s:
        U, st, rc = s.solve(dev(F), dev(psi0))
    assert rc == 0
    err = float(torch.linalg.norm(U - ref) / torch.linalg.norm(ref))
    print(f"511 mixed MGRIT cg_rtol={cg_rtol:g} coarse {cg_coarse:g} tol_rel={tol_rel:g}: {st.iterations} iterations, "
          f"error {err:.3e}")
    assert err <= 1e-8, err


@pytest.mark.parametrize("Mx,My,expect_fft", [(257, 40, True), (258, 40, True), (40, 513, True), (514, 33, False)])
def test_operator_at_the_fft_size_limits(Mx, My, expect_fft):
    """n = 256 is the largest grid line of the 512-point transforms (2n - 1 <= 512) and n = 512 of the 1024-point
    ones; one more node falls back to the dense products under op = auto.  All sides of the limits match the
    oracle."""
    mg = _mg()
    prob = fem.Problem(0.6, 0.9, 1.0, 2.0, Mx, My)
    op = fem.Operator(prob)
    v = wl.random_slices(21, 3, prob.nx, prob.ny)
    theta = np.array([0.0, 0.01, 3.0])
    with mg.Solver(0.6, 0.9, 1.0, 2.0, Mx, My, wl.uniform_grid(4), m=2) as s:
        out = host(s.apply(theta, dev(v)))
    for k in range(3):
        ref = op.apply_M(v[k]) + theta[k] * op.apply_A(v[k])
        assert np.abs(out[k] - ref).max() <= 1e-13 * np.abs(ref).max(), k
    if not expect_fft:
        with pytest.raises(mg.MgritError):
            mg.Solver(0.6, 0.9, 1.0, 2.0, Mx, My, wl.uniform_grid(4), m=2, op="fft")
