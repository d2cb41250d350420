"""Pins of the oracle's time stepping (eq. chp-02-03, eq. equ-03-05) and Example 4.1."""
import math

import numpy as np
import pytest

import golden_tables
from oracle import analysis, fem, manufactured as mf, propagator


def _problem(seed=0):
    p = fem.Problem(0.7, 0.8, 1.0, 1.0, 9, 8)
    rng = np.random.default_rng(seed)
    return p, fem.Operator(p), rng


def test_cg_propagator_equals_cholesky():
    p, op, rng = _problem()
    t = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 7)]))
    F = rng.standard_normal((8, p.ny, p.nx))
    psi0 = rng.uniform(0, 1, (p.ny, p.nx))
    U1 = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    U2 = propagator.sequential(op, propagator.CholeskySolver(op), t, F, psi0)
    assert np.linalg.norm(U1 - U2) <= 1e-12 * np.linalg.norm(U2)


def test_zero_rhs_gives_zero():
    p, op, rng = _problem()
    x, it = propagator.cg(op.apply_M, np.zeros((p.ny, p.nx)), rng.standard_normal((p.ny, p.nx)), 1e-12, 100)
    assert it == 0 and not np.any(x)


@pytest.mark.parametrize("tau", [0.01, 0.3, 5.0])
def test_propagator_eigenvalues(tau):
    """eq. (equ-03-05): eig(Psi) = (2 - tau sigma)/(2 + tau sigma), |.| < 1 (Lemma 3.3), sigma > 0 (Lemma 3.2)."""
    p = fem.Problem(0.85, 0.6, 2.0, 0.5, 6, 7)
    op = fem.Operator(p)
    sigma = analysis.generalized_sigma(op)
    assert sigma.min() > 0
    M, A = op.assembled_M(), op.assembled_A()
    Psi = np.linalg.solve(M + 0.5 * tau * A, M - 0.5 * tau * A)
    lam = np.sort(np.linalg.eigvals(Psi).real)
    pred = np.sort(analysis.cn_factor(tau, sigma))
    assert np.allclose(lam, pred, atol=1e-10)
    assert np.abs(pred).max() < 1


def test_source_matches_numerical_riesz_derivative():
    """The f of Example 4.1 equals u_t - K_x d^2b u/d|x|^2b - K_y d^2g u/d|y|^2g with the Riemann-Liouville
    derivatives evaluated by quadrature.  For w(s) = (s - s^2)^2 (w(0) = w'(0) = 0) differentiating
    under the integral gives D_L^(2r) w(z) = 1/Gamma(2-2r) int_0^z q^(1-2r) w''(z - q) dq."""
    import mpmath
    beta, gamma, Kx, Ky = 0.7, 0.85, 2.0, 0.5
    w = lambda s: (s - s * s) ** 2
    w2 = lambda s: 2 - 12 * s + 12 * s * s

    def rl_left(z, r):
        return mpmath.quad(lambda q: q ** (1 - 2 * r) * w2(z - q), [0, z]) / mpmath.gamma(2 - 2 * r)

    def riesz(z, r):                       # -(D_L + D_R)/(2 cos(r pi)); D_R at z is D_L of w(1-s) at 1-z
        return -(rl_left(z, r) + rl_left(1 - z, r)) / (2 * mpmath.cos(r * mpmath.pi))

    with mpmath.workdps(30):
        for (x, y) in [(0.3, 0.6), (0.71, 0.22)]:
            u = 10 * w(x) * w(y)                # t = 0, u_t = -u
            f_num = -u - Kx * 10 * w(y) * riesz(x, beta) - Ky * 10 * w(x) * riesz(y, gamma)
            f_printed = mf.source_g(x, y, beta, gamma, Kx, Ky, 10.0)
            assert abs(float(f_num) - f_printed) <= 1e-10 * abs(f_printed)


def _table_errors(name, grid, K, max_N):
    out = []
    for beta, gamma, M, N, e in golden_tables.load(name):
        if N > max_N:
            continue
        p = fem.Problem(beta, gamma, K[0], K[1], M, M)
        op = fem.Operator(p)
        t = grid(N)
        F = mf.load_vectors(t, beta, gamma, K[0], K[1], M)
        U = propagator.sequential(op, propagator.CholeskySolver(op), t, F, mf.nodal_psi0(M))
        out.append((beta, gamma, M, e, mf.l2_error(U[-1], 1.0, M)))
    return out


def _check_table(rows):
    """Values within the band left by the paper's unstated load quadrature; O(h^2 + tau^2) rates."""
    for beta, gamma, M, printed, ours in rows:
        assert 0.88 * printed <= ours <= 1.02 * printed, (beta, gamma, M, printed, ours)
    by = {}
    for beta, gamma, M, printed, ours in rows:
        by.setdefault((beta, gamma), []).append((M, ours))
    for key, seq in by.items():
        seq.sort()
        for (M0, e0), (M1, e1) in zip(seq, seq[1:]):
            rate = math.log(e0 / e1) / math.log(M1 / M0)
            assert 1.7 < rate < 2.3, (key, M0, M1, rate)


def test_table1_uniform_tau_h():
    _check_table(_table_errors("table1_errors.txt", mf.uniform_grid, (2.0, 0.5), 64))


def test_table2_uniform_tau_h3():
    _check_table(_table_errors("table2_errors.txt", mf.uniform_grid, (3.0, 7.5), 4096))


def test_table3_piecewise_uniform():
    _check_table(_table_errors("table3_errors.txt", lambda N: mf.piecewise_uniform_grid(N, 2.0 ** -6), (3.0, 7.5), 64))


def test_table4_piecewise_uniform_h3():
    _check_table(_table_errors("table4_errors.txt", lambda N: mf.piecewise_uniform_grid(N, 2.0 ** -8), (2.0, 0.5), 4096))


def test_piecewise_uniform_grid_shape():
    t = mf.piecewise_uniform_grid(16, 2.0 ** -6)
    s = 2 * 2.0 ** -6 * math.log(16)
    assert len(t) == 17 and t[0] == 0 and abs(t[-1] - 1) < 1e-15
    assert abs(t[4] - s) < 1e-15 and abs(t[12] - (1 - s)) < 1e-15
    assert len(set(np.round(np.diff(t), 14))) == 2
