"""Pins of the oracle's space discretisation (Section 2) against independent routes."""
import math

import numpy as np
import pytest

import fe_weakform
from oracle import fem, toeplitz


@pytest.mark.parametrize("beta,gamma,Mx,My,b,d", [
    (0.6, 0.95, 6, 5, 1.0, 1.3),
    (0.75, 0.55, 5, 7, 2.0, 1.0),
    (0.95, 0.7, 5, 5, 1.0, 1.0),
])
def test_stiffness_equals_weak_form_quadrature(beta, gamma, Mx, My, b, d):
    """Printed Toeplitz entries x c_x (and the P_pi form of A_y) = quadrature of eq. (chp-02-07)."""
    p = fem.Problem(beta, gamma, 1.0, 1.0, Mx, My, 0.0, b, 0.0, d)
    op = fem.Operator(p)
    Ax = fe_weakform.stiffness_matrix_x(Mx, My, p.hx, p.hy, beta)
    Ay = fe_weakform.stiffness_matrix_y(Mx, My, p.hx, p.hy, gamma)
    assert np.abs(op.assembled_Ax() - Ax).max() <= 1e-10 * np.abs(Ax).max()
    assert np.abs(op.assembled_Ay() - Ay).max() <= 1e-10 * np.abs(Ay).max()


def test_mass_equals_element_assembly():
    p = fem.Problem(0.7, 0.8, 1.0, 1.0, 6, 5, 0.0, 1.5, 0.0, 1.0)
    op = fem.Operator(p)
    ref = fe_weakform.mass_matrix(6, 5, p.hx, p.hy)
    assert np.allclose(op.assembled_M(), ref, rtol=0, atol=1e-15)


def test_rho_one_reduces_to_five_point_laplacian():
    """At rho = 1 the sequences give A_1 = -4 tridiag(-1, 2, -1), A_2 = 0 and c_x A_1 = (h_y/h_x) tridiag(-1,2,-1)."""
    n = 9
    A1, A2 = toeplitz.toeplitz_factors(1.0, n)
    lap = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    assert np.allclose(A1, -4.0 * lap, atol=1e-13)
    assert np.allclose(A2, 0.0, atol=1e-13)
    hx, hy = 0.1, 0.25
    c = toeplitz.stiffness_scale(1.0, hx, hy)
    assert math.isclose(c, -hy / (4 * hx), rel_tol=1e-14)


def test_subdiagonal_formula_is_shifted_superdiagonal():
    """The two printed general formulas of A_2 satisfy w_m = u_{m+1}; the diagonal/first off-diagonal are special."""
    for rho in (0.55, 0.8, 0.95):
        u = toeplitz.a2_upper_sequence(rho, 40)
        w = toeplitz.a2_lower_sequence(rho, 39)
        assert np.allclose(w[1:], u[2:], rtol=1e-15, atol=0)


def test_extended_precision_needed_for_tails():
    """Plain FP64 evaluation of the general A_1 formula loses the tail; the oracle keeps it.

    Reference: the same difference computed in exact-ish binomial-series form
    sum_k coef_k (l+k)^e for large l via mpmath at 80 digits.
    """
    import mpmath
    rho, l = 0.55, 1000
    t = toeplitz.a1_sequence(rho, l + 1)[l]
    with mpmath.workdps(80):
        r = mpmath.mpf(rho)
        e3, e4 = 3 - 2 * r, 4 - 2 * r
        L = mpmath.mpf(l)
        ref = (4 * e4 * (-(L - 1) ** e3 + 2 * L ** e3 - (L + 1) ** e3)
               - 2 * (L - 2) ** e4 + 4 * (L - 1) ** e4 - 4 * (L + 1) ** e4 + 2 * (L + 2) ** e4)
    assert abs(t - float(ref)) <= 1e-15 * abs(float(ref))
    e3, e4 = 3 - 2 * rho, 4 - 2 * rho
    L = float(l)
    naive = (4 * e4 * (-(L - 1) ** e3 + 2 * L ** e3 - (L + 1) ** e3)
             - 2 * (L - 2) ** e4 + 4 * (L - 1) ** e4 - 4 * (L + 1) ** e4 + 2 * (L + 2) ** e4)
    assert abs(naive - float(ref)) > 1e-3 * abs(float(ref))


def test_sequence_decay_and_signs():
    """Off-diagonal entries of A_1 are positive and decay like l^(-1-2 rho) (the kernel |x|^(-1-2rho))."""
    rho = 0.75
    t = toeplitz.a1_sequence(rho, 400)
    assert t[0] < 0 and np.all(t[1:] > 0)
    ratio = t[399] / t[199]
    assert abs(ratio - (399 / 199) ** (-1 - 2 * rho)) < 0.01


@pytest.mark.parametrize("beta,gamma", [(0.6, 0.7), (0.95, 0.55)])
def test_symmetric_positive_definite(beta, gamma):
    """Lemma 3.2 ingredients: M_h, A_x, A_y, A_h symmetric positive definite."""
    p = fem.Problem(beta, gamma, 2.0, 0.5, 7, 6)
    op = fem.Operator(p)
    for K in (op.assembled_M(), op.assembled_Ax(), op.assembled_Ay(), op.assembled_A()):
        assert np.allclose(K, K.T, rtol=0, atol=1e-13 * np.abs(K).max())
        assert np.linalg.eigvalsh(K).min() > 0


def test_matrix_free_equals_assembled():
    rng = np.random.default_rng(1)
    p = fem.Problem(0.65, 0.9, 1.5, 0.7, 8, 6, 0.0, 1.0, 0.0, 2.0)
    op = fem.Operator(p)
    V = rng.standard_normal((3, p.ny, p.nx))
    for fn, K in ((op.apply_M, op.assembled_M()), (op.apply_Ax, op.assembled_Ax()),
                  (op.apply_Ay, op.assembled_Ay()), (op.apply_A, op.assembled_A())):
        out = fn(V)
        ref = (K @ V.reshape(3, -1).T).T.reshape(V.shape)
        assert np.allclose(out, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_problem_validation():
    for bad in [dict(beta=0.5), dict(beta=1.0), dict(gamma=0.4), dict(Kx=0.0), dict(Mx=1)]:
        kw = dict(beta=0.7, gamma=0.8, Kx=1.0, Ky=1.0, Mx=4, My=4)
        kw.update(bad)
        with pytest.raises(ValueError):
            fem.Problem(**kw)
