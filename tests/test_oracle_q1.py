"""Pins of the oracle's bilinear (Q1) tensor-product variant (oracle/q1.py)."""
import math

import numpy as np
import pytest

from oracle import fem, mgrit as omgrit, propagator, q1
from paper_1805_06688_amd import workloads as wl


@pytest.mark.parametrize("rho", [0.6, 0.75, 0.95])
@pytest.mark.parametrize("h", [1.0 / 16, 1.0 / 7])
def test_1d_stiffness_equals_fourier_quadrature(rho, h):
    """The closed form (kink pairs and Beta integrals) against a quadrature of the Fourier form
    (1/pi) int xi^(2 rho) |phi^|^2 cos(xi d) d xi of the same bilinear form."""
    a = q1.stiffness_1d_entries(rho, 8, h)
    for l in range(8):
        assert abs(a[l] - q1.fourier_entry(rho, l, h)) <= 1e-9 * abs(a[0]), l


def test_rho_one_gives_the_linear_element_laplacian():
    """At rho = 1 the Riesz derivative is d^2/dx^2 and a(l) the stiffness 1/h tridiag(-1, 2, -1)."""
    h = 0.1
    a = q1.stiffness_1d_entries(1.0, 6, h)
    assert np.allclose(a, [2 / h, -1 / h, 0, 0, 0, 0], atol=1e-12 / h)


def _q1_element_mass(Mx, My, hx, hy):
    """Textbook bilinear-element mass, assembled cell by cell with a 2 x 2 Gauss rule (exact here)."""
    nx, ny = Mx - 1, My - 1
    g = np.array([-1.0, 1.0]) / math.sqrt(3.0)
    pts = [(0.5 * (1 + a), 0.5 * (1 + b)) for a in g for b in g]
    M = np.zeros((nx * ny, nx * ny))
    for j in range(My):
        for k in range(Mx):
            corners = [(k, j), (k + 1, j), (k, j + 1), (k + 1, j + 1)]
            for (s, t) in pts:
                phi = [(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t]
                w = 0.25 * hx * hy
                for a, (xa, ya) in enumerate(corners):
                    if not (0 < xa < Mx and 0 < ya < My):
                        continue
                    for b, (xb, yb) in enumerate(corners):
                        if 0 < xb < Mx and 0 < yb < My:
                            M[(xa - 1) + (ya - 1) * nx, (xb - 1) + (yb - 1) * nx] += w * phi[a] * phi[b]
    return M


def test_q1_mass_is_the_bilinear_element_mass():
    prob = fem.Problem(0.7, 0.8, 1.0, 1.0, 7, 5, 0.0, 2.0, -1.0, 1.0)
    op = q1.Q1Operator(prob)
    assert np.allclose(op.assembled_M(), _q1_element_mass(7, 5, prob.hx, prob.hy), atol=1e-15)


def test_q1_apply_equals_kronecker_assembly_and_is_spd():
    prob = fem.Problem(0.65, 0.9, 2.0, 0.5, 9, 7)
    op = q1.Q1Operator(prob)
    V = np.random.default_rng(0).standard_normal((prob.ny, prob.nx))
    A, M = op.assembled_A(), op.assembled_M()
    assert np.allclose(A @ V.ravel(), op.apply_A(V).ravel(), rtol=1e-13, atol=1e-12 * np.abs(A).max())
    assert np.allclose(M @ V.ravel(), op.apply_M(V).ravel(), rtol=1e-13, atol=1e-16)
    assert np.allclose(A, A.T) and np.linalg.eigvalsh(A).min() > 0 and np.linalg.eigvalsh(M).min() > 0
    assert np.linalg.eigvalsh(op.Ax).min() > 0


def test_q1_cg_step_equals_cholesky_and_mgrit_terminates():
    prob = fem.Problem(0.75, 0.85, 2.0, 1.0, 10, 9)
    op = q1.Q1Operator(prob)
    t = wl.random_grid(16, 3)
    F, psi0 = wl.random_inputs(3, 16, prob.nx, prob.ny)
    U1 = propagator.sequential(op, propagator.CGSolver(op, 1e-14), t, F, psi0)
    U2 = propagator.sequential(op, propagator.CholeskySolver(op), t, F, psi0)
    assert np.linalg.norm(U1 - U2) <= 1e-12 * np.linalg.norm(U2)
    o = omgrit.MGRIT(op, t, 4, max_levels=2, coarse="be", solver=propagator.CholeskySolver(op))
    U = o.iterate(F, psi0, 2)              # N_c = 4 coarse intervals: exact after ceil(4 / 2) iterations
    assert np.linalg.norm(U - U2) <= 1e-12 * np.linalg.norm(U2)
