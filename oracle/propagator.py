"""Time propagators Phi_n and sequential time stepping.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; not part of the product path).

* Eq. (chp-02-03): [M_h + tau_n/2 A_h] U_n = F_n + [M_h - tau_n/2 A_h] U_{n-1},
  tau_n = t_n - t_{n-1}, A_h = K_x A_x + K_y A_y, U_0 = nodal values of psi_0.
* Eq. (equ-03-01): the same step written as U_n = Psi_n U_{n-1} + G_n with
  G_n = [M_h + tau_n/2 A_h]^{-1} F_n; the inverse is a spatial solve.
* Section 3.2 (implementation details): every spatial solve is conjugate
  gradients without preconditioner, stopped on the Euclidean norm of the
  residual relative to the right-hand side.

Readings (the paper does not say): the CG start vector is the propagated
state u itself; a zero right-hand side returns the zero vector (the exact
solution) without iterating.
"""
import numpy as np


def cg(apply, b, x0, rtol, maxit):
    """Plain conjugate gradients on an SPD operator.

    Stops when ||r||_2 <= rtol ||b||_2 (r the recursively updated residual)
    or after maxit iterations.  Returns (x, iterations).
    """
    b = np.asarray(b, dtype=np.float64)
    bb = float(np.vdot(b, b))
    if bb == 0.0:
        return np.zeros_like(b), 0
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply(x)
    p = r.copy()
    rr = float(np.vdot(r, r))
    it = 0
    while rr > rtol * rtol * bb and it < maxit:
        q = apply(p)
        alpha = rr / float(np.vdot(p, q))
        x += alpha * p
        r -= alpha * q
        rr_new = float(np.vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


class CGSolver:
    """Solves with B(theta) = M_h + theta A_h by CG, counting iterations."""

    def __init__(self, op, rtol=1e-14, maxit=5000):
        self.op, self.rtol, self.maxit = op, rtol, maxit
        self.iterations = 0
        self.solves = 0

    def solve(self, theta, b, x0):
        x, it = cg(lambda v: self.op.apply_M(v) + theta * self.op.apply_A(v), b, x0, self.rtol, self.maxit)
        self.iterations += it
        self.solves += 1
        return x


class CholeskySolver:
    """Dense Cholesky solves with B(theta) (small grids), cached per theta."""

    def __init__(self, op):
        import scipy.linalg
        self._sl = scipy.linalg
        self.M = op.assembled_M()
        self.A = op.assembled_A()
        self._cache = {}
        self.solves = 0
        self.iterations = 0

    def solve(self, theta, b, x0=None):
        f = self._cache.get(theta)
        if f is None:
            f = self._sl.cho_factor(self.M + theta * self.A)
            self._cache[theta] = f
        self.solves += 1
        shape = b.shape
        return self._sl.cho_solve(f, b.reshape(-1)).reshape(shape)


def cn_step(op, solver, tau, u, F=None):
    """One step of eq. (chp-02-03): solve B U_n = C U_{n-1} + F_n (F may be None = 0)."""
    rhs = op.apply_C(u, tau)
    if F is not None:
        rhs = rhs + F
    return solver.solve(0.5 * tau, rhs, u)


def sequential(op, solver, t, F, psi0):
    """Sequential time stepping U_n = Phi_n(U_{n-1}), n = 1..N.

    t: N+1 time points; F: [N, n_y, n_x] load vectors F_1..F_N (None = zero);
    psi0: [n_y, n_x].  Returns U: [N+1, n_y, n_x].
    """
    t = np.asarray(t, dtype=np.float64)
    N = len(t) - 1
    U = np.empty((N + 1,) + np.shape(psi0))
    U[0] = psi0
    for n in range(1, N + 1):
        U[n] = cn_step(op, solver, t[n] - t[n - 1], U[n - 1], None if F is None else F[n - 1])
    return U
