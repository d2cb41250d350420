"""Pins of the oracle's MGRIT (Algorithm 3.1, Lemma 3.1, Theorem 3.2)."""
import math

import numpy as np
import pytest

from oracle import analysis, fem, manufactured as mf, mgrit, propagator


def _setup(N=32, seed=0, grid="random", beta=0.7, gamma=0.8, Mx=10, My=9):
    rng = np.random.default_rng(seed)
    p = fem.Problem(beta, gamma, 1.0, 1.0, Mx, My)
    op = fem.Operator(p)
    if grid == "random":
        t = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, N - 1)]))
    else:
        t = mf.uniform_grid(N)
    F = rng.standard_normal((N, p.ny, p.nx))
    psi0 = rng.uniform(0, 1, (p.ny, p.nx))
    ch = propagator.CholeskySolver(op)
    Useq = propagator.sequential(op, ch, t, F, psi0)
    return p, op, t, F, psi0, ch, Useq


@pytest.mark.parametrize("coarse", ["cn", "be", "cn2", "opt"])
@pytest.mark.parametrize("m,levels", [(4, 2), (2, 5), (3, 3)])
def test_mgrit_reaches_sequential(coarse, m, levels):
    """The fixed point of MGRIT is sequential stepping, whatever the coarse propagator."""
    if coarse == "opt" and m % 2:
        with pytest.raises(ValueError):
            mgrit.MGRIT(fem.Operator(fem.Problem(0.7, 0.8, 1, 1, 5, 5)), np.linspace(0, 1, 10), m, coarse="opt")
        return
    p, op, t, F, psi0, ch, Useq = _setup(N=31)
    mg = mgrit.MGRIT(op, t, m, max_levels=levels, coarse=coarse, solver=ch)
    U, it, conv = mg.solve(F, psi0, tol=1e-10, max_iter=60)
    assert conv
    assert np.linalg.norm(U - Useq) <= 1e-10 * np.linalg.norm(Useq)


def test_f_relaxation_only_converges():
    p, op, t, F, psi0, ch, Useq = _setup()
    mg = mgrit.MGRIT(op, t, 4, max_levels=3, relax="F", coarse="be", solver=ch)
    U, it, conv = mg.solve(F, psi0, tol=1e-10, max_iter=60)
    assert conv and np.linalg.norm(U - Useq) <= 1e-10 * np.linalg.norm(Useq)


@pytest.mark.parametrize("coarse", ["cn", "be"])
def test_two_level_finite_termination(coarse):
    """Two-level FCF: after ceil(Nc/2) iterations every C-point is exact (consequence of Lemma 3.1,
    whose error is zero at C-points 0 and m and moves two intervals per iteration)."""
    p, op, t, F, psi0, ch, Useq = _setup(N=40, beta=0.95, gamma=0.9, Mx=12, My=12)
    m = 4
    Nc = 10
    mg = mgrit.MGRIT(op, t, m, max_levels=2, coarse=coarse, solver=ch)
    U = mg.iterate(F, psi0, math.ceil(Nc / 2))
    assert np.abs(U - Useq).max() <= 1e-12 * np.abs(Useq).max()
    U = mg.iterate(F, psi0, math.ceil(Nc / 2) - 2)
    assert np.abs(U - Useq).max() > 1e-8 * np.abs(Useq).max()


@pytest.mark.parametrize("levels", [2, 3])
def test_ideal_coarse_propagator_is_exact_in_one_iteration(levels):
    """With Psi^Delta equal to the product of the m fine propagators the bracket of Lemma 3.1 vanishes."""
    p, op, t, F, psi0, ch, Useq = _setup(N=36)
    mg = mgrit.MGRIT(op, t, 3, max_levels=levels, coarse="ideal", solver=ch)
    U = mg.iterate(F, psi0, 1)
    assert np.abs(U - Useq).max() <= 1e-12 * np.abs(Useq).max()


def test_lemma31_error_formula():
    """Measured C-point error after one two-level iteration = the sum of Lemma 3.1 (non-uniform grid)."""
    rng = np.random.default_rng(3)
    p = fem.Problem(0.8, 0.65, 2.0, 0.5, 5, 5)
    op = fem.Operator(p)
    N, m = 16, 4
    t = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, N - 1)]))
    F = rng.standard_normal((N, p.ny, p.nx))
    psi0 = rng.uniform(0, 1, (p.ny, p.nx))
    ch = propagator.CholeskySolver(op)
    Useq = propagator.sequential(op, ch, t, F, psi0)
    U0 = Useq + rng.standard_normal(Useq.shape)
    U0[0] = psi0
    mg = mgrit.MGRIT(op, t, m, max_levels=2, coarse="cn", solver=ch)
    U1 = mg.iterate(F, psi0, 1, U0=U0)
    E_before = (Useq - U0)[::m].reshape(N // m + 1, -1)
    E_after = (Useq - U1)[::m].reshape(N // m + 1, -1)
    fine, coarse = analysis.dense_propagators(op, t, m)
    pred = analysis.lemma31_error(fine, coarse, m, E_before)
    assert np.abs(E_after[:2]).max() <= 1e-12 * np.abs(E_before).max()
    assert np.allclose(E_after, pred, rtol=0, atol=1e-10 * np.abs(pred).max())


@pytest.mark.parametrize("beta,gamma,M,N,m", [(0.6, 0.7, 8, 64, 2), (0.6, 0.7, 16, 256, 2), (0.95, 0.65, 8, 64, 2)])
def test_theorem32_bound_holds(beta, gamma, M, N, m):
    """Measured ratios of successive residual norms never exceed the theoretical upper bound eq. (equ-03-11)."""
    p = fem.Problem(beta, gamma, 2.0, 0.5, M, M)
    op = fem.Operator(p)
    t = mf.uniform_grid(N)
    F = mf.load_vectors(t, beta, gamma, 2.0, 0.5, M)
    bound = analysis.tub(analysis.generalized_sigma(op), t, m)
    mg = mgrit.MGRIT(op, t, m, max_levels=2, coarse="cn", solver=propagator.CholeskySolver(op))
    U0 = np.random.default_rng(0).uniform(-1, 1, (N + 1, p.ny, p.nx))
    _, _, _, hist = mg.solve(F, mf.nodal_psi0(M), tol=1e-14, max_iter=8, U0=U0, return_history=True)
    ratios = np.array(hist[1:]) / np.array(hist[:-1])
    assert np.all(ratios <= bound)


def test_tub_closed_form_m2():
    """Uniform grid, m = 2, one mode z = tau sigma, Nc = 2 (geometric factor 1): eq. (equ-03-03) reduces to
    lambda^2 |lambda^2 - mu| = 2 z^3 (2-z)^2 / ((2+z)^4 (1+z)) by direct algebra."""
    t = np.linspace(0, 4, 5)             # tau = 1
    for z in (0.05, 2.0 / 3.0, 1.7):
        val = analysis.tub(np.array([z]), t, 2)
        closed = 2 * z ** 3 * (2 - z) ** 2 / ((2 + z) ** 4 * (1 + z))
        assert math.isclose(val, closed, rel_tol=1e-9)   # lambda^2 - mu cancels to O(z^3)


def test_trailing_f_points_and_levels():
    p, op, t, F, psi0, ch, Useq = _setup(N=37)
    mg = mgrit.MGRIT(op, t, 4, max_levels=10, coarse="be", solver=ch)
    assert [lv.N for lv in mg.levels] == [37, 9, 2]
    U, it, conv = mg.solve(F, psi0, tol=1e-10, max_iter=60)
    assert conv and np.linalg.norm(U - Useq) <= 1e-10 * np.linalg.norm(Useq)


def test_cg_inside_mgrit():
    p, op, t, F, psi0, ch, Useq = _setup(N=24)
    mg = mgrit.MGRIT(op, t, 4, max_levels=3, coarse="be", cg_rtol=1e-14)
    U, it, conv = mg.solve(F, psi0, tol=1e-9, max_iter=60)
    assert conv and np.linalg.norm(U - Useq) <= 1e-11 * np.linalg.norm(Useq)


def test_opt_factors_reproduce_two_fine_steps():
    """With two fine steps per coarse step the opt factors are exactly those two steps (any lengths)."""
    for taus in ([0.25, 0.25], [0.1, 0.37], [0.9, 0.05]):
        short, long_ = mgrit.opt_factors(taus)
        assert math.isclose(short, min(taus), rel_tol=1e-12) and math.isclose(long_, max(taus), rel_tol=1e-12)


def test_opt_m2_two_level_exact_in_one_iteration():
    p, op, t, F, psi0, ch, Useq = _setup(N=30)
    mg = mgrit.MGRIT(op, t, 2, max_levels=2, coarse="opt", solver=ch)
    U = mg.iterate(F, psi0, 1)
    assert np.abs(U - Useq).max() <= 1e-12 * np.abs(Useq).max()


@pytest.mark.parametrize("M", [4, 8, 64])
def test_opt_factor_matches_ideal_asymptotics(M):
    """Per mode: R(y) = prod CN factors equals the ideal ((2 - y/M)/(2 + y/M))^M to O(y^2) at 0 and to O(1/y^2)
    at infinity (uniform fine steps)."""
    short, long_ = mgrit.opt_factors(np.full(M, 1.0 / M))
    R = lambda y: (2 - short * y) / (2 + short * y) * (2 - long_ * y) / (2 + long_ * y)
    ideal = lambda y: ((2 - y / M) / (2 + y / M)) ** M
    for y in (1e-3, 1e-4):
        assert abs(R(y) - ideal(y)) < 2 * y * y
    for y in (1e6, 1e7):
        assert abs(R(y) - ideal(y)) * y < 1e-2 * 4 * M * M
    assert abs(R(1e9) - 1) * 1e9 == pytest.approx(4 * M * M, rel=1e-3)


def test_opt_converges_fast_on_stiff_problem():
    """tau sigma_max ~ 80: the paper's coarse propagator barely contracts, opt by more than 50x per iteration."""
    p, op, t, F, psi0, ch, Useq = _setup(N=64, grid="uniform", Mx=32, My=32, beta=0.75, gamma=0.85)
    errs = {}
    for coarse in ("cn", "opt"):
        mg = mgrit.MGRIT(op, t, 8, max_levels=2, coarse=coarse, solver=ch)
        errs[coarse] = [np.linalg.norm(mg.iterate(F, psi0, k) - Useq) / np.linalg.norm(Useq) for k in (1, 2)]
    assert errs["cn"][1] > 0.5 * errs["cn"][0]          # the paper's coarse step barely contracts here
    assert errs["opt"][1] < errs["opt"][0] / 50 and errs["opt"][0] < 1e-2
