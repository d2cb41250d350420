"""Multigrid reduction in time (Algorithm 3.1) for the block bidiagonal system (ode-03).

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; not part of the product path).

Section 3.1: the system A U = G with unit diagonal blocks and sub-diagonal
blocks -Psi_n.  With coarsening factor m the C-points are t_{m i}; FCF
relaxation is F-, then C-, then F-relaxation; restriction is injection at the
C-points; interpolation is injection followed by F-relaxation; the hierarchy
is built recursively (Algorithm 3.1, steps 1-4).  Remark 3.1: on the finest
level the correction touches C-points only, and the F-points are brought up
to date by the relaxation of the next iteration (or a final F-relaxation).
Eq. (equ-03-02): the coarse propagator re-discretises eq. (chp-02-03) with
the coarse step t~_j - t~_{j-1}.

Readings (where the paper is silent or ambiguous):
* levels are counted as l = 0..L-1 with level L-1 solved by sequential
  stepping (two-level = two levels); coarsening stops when the next level
  would hold fewer than two intervals, or at max_levels;
* when N_l is not a multiple of m the C-points are the multiples of m and
  the trailing F-points are only F-relaxed; N_{l+1} = floor(N_l / m);
* linear correction scheme: step 3 starts the coarse level from zero and the
  coarse right-hand side is the injected residual in the G (solution) space,
  r_k = Phi_{km}(U_{km-1}) - U_{km};
* stop test: the residual is taken after the level-0 relaxation at the
  C-points, and its norm is sqrt(h_x h_y sum_k ||r_k||_2^2) ("discrete L^2"),
  compared with an absolute tolerance; when it passes the iterate is returned
  as it stands (it is F-consistent); when max_iter is reached the C-point
  correction is followed by a final F-relaxation;
* coarse propagator: "cn" is eq. (equ-03-02).  Also available: "be"
  (backward Euler with the coarse step), "cn2" (two Crank-Nicolson half
  steps), "ideal" (the product of the fine propagators over the coarse
  step, i.e. the exact Schur complement) and "opt", a product of two
  Crank-Nicolson steps whose lengths are chosen so that, mode by mode
  (eq. equ-03-05), it agrees with the ideal propagator to first order in
  tau~ sigma and in the stiff limit tau~ sigma -> infinity (see
  opt_factors).  The choice changes the convergence speed, never the fixed
  point, which is sequential stepping.
"""
import numpy as np

from .propagator import CGSolver


COARSE_KINDS = ("cn", "be", "cn2", "ideal", "opt")


def opt_factors(taus):
    """Step lengths of the two Crank-Nicolson factors of the "opt" coarse propagator.

    taus: the level-0 steps tau_n inside one coarse step (an even number of them),
    tau~ = sum tau_n.  Per mode (eq. equ-03-05, y = tau~ sigma) the ideal coarse
    propagator is prod_n (2 - tau_n sigma)/(2 + tau_n sigma), which behaves as
    1 - y for small y and as 1 - c/y with c = 4 tau~ sum_n 1/tau_n for large y.
    A product (a1 - y)/(a1 + y) * (a2 - y)/(a2 + y) behaves as 1 - 2 y (1/a1 + 1/a2)
    and 1 - 2 (a1 + a2)/y, so a1 + a2 = c/2 and 1/a1 + 1/a2 = 1/2: a1, a2 are the
    roots of s^2 - (c/2) s + c = 0 (real since c >= 16).  The factor (a - y)/(a + y)
    is a Crank-Nicolson step of length 2 tau~ / a.  Returns (short step, long step).
    """
    taus = np.asarray(taus, dtype=np.float64)
    if len(taus) % 2:
        raise ValueError("the opt coarse propagator needs an even number of fine steps")
    T = float(taus.sum())
    c = 4.0 * T * float(np.sum(1.0 / taus))
    d = np.sqrt(c * c / 16.0 - c)
    a1, a2 = c / 4.0 + d, c / 4.0 - d
    return 2.0 * T / a1, 2.0 * T / a2


class _Level:
    def __init__(self, fine_index):
        self.fine_index = np.asarray(fine_index)     # level-0 index of each point
        self.N = len(fine_index) - 1
        self.G = None                                 # [N+1, ny, nx] at levels >= 1


class MGRIT:
    def __init__(self, op, t, m, max_levels=30, relax="FCF", coarse="cn", solver=None,
                 cg_rtol=1e-14, cg_maxit=5000):
        if m < 2:
            raise ValueError("coarsening factor m must be >= 2")
        if relax not in ("F", "FCF"):
            raise ValueError("relax must be 'F' or 'FCF'")
        if coarse not in COARSE_KINDS:
            raise ValueError("unknown coarse propagator")
        if max_levels < 2:
            raise ValueError("need at least two levels")
        if coarse == "opt" and m % 2:
            raise ValueError("the opt coarse propagator needs an even coarsening factor")
        self.op = op
        self.t = np.asarray(t, dtype=np.float64)
        self.m, self.relax_kind, self.coarse = m, relax, coarse
        self.solver = solver if solver is not None else CGSolver(op, cg_rtol, cg_maxit)
        N = len(self.t) - 1
        self.levels = [_Level(np.arange(N + 1))]
        while len(self.levels) < max_levels:
            prev = self.levels[-1]
            Nc = prev.N // m
            if Nc < 2:
                break
            self.levels.append(_Level(prev.fine_index[: Nc * m + 1: m]))
        if len(self.levels) < 2:
            raise ValueError("time grid too short for one coarsening")
        self.phi_calls = 0

    # ---- propagators -------------------------------------------------------------------------
    def _cn(self, tau, u, F=None):
        rhs = self.op.apply_C(u, tau)
        if F is not None:
            rhs = rhs + F
        return self.solver.solve(0.5 * tau, rhs, u)

    def psi(self, l, k, u):
        """Homogeneous propagator of level l from point k-1 to point k."""
        lev = self.levels[l]
        i0, i1 = lev.fine_index[k - 1], lev.fine_index[k]
        tau = self.t[i1] - self.t[i0]
        if l == 0 or self.coarse == "cn":
            return self._cn(tau, u)
        if self.coarse == "be":
            return self.solver.solve(tau, self.op.apply_M(u), u)
        if self.coarse == "cn2":
            v = self._cn(0.5 * tau, u)
            return self._cn(0.5 * tau, v)
        if self.coarse == "opt":
            short, long_ = opt_factors(np.diff(self.t[i0:i1 + 1]))
            v = self._cn(short, u)
            return self._cn(long_, v)
        v = u                                  # "ideal": fine steps i0+1 .. i1
        for n in range(i0 + 1, i1 + 1):
            v = self._cn(self.t[n] - self.t[n - 1], v)
        return v

    def phi(self, l, k, u):
        """Affine propagator Phi^(l)_k(u) = Psi^(l)_k u + G^(l)_k."""
        self.phi_calls += 1
        if l == 0:
            tau = self.t[k] - self.t[k - 1]
            return self._cn(tau, u, None if self.F is None else self.F[k - 1])
        return self.psi(l, k, u) + self.levels[l].G[k]

    # ---- relaxation and transfer ---------------------------------------------------------
    def f_relax(self, l, U):
        N, m = self.levels[l].N, self.m
        for c in range(0, N + 1, m):           # every C-point starts an interval of F-points
            for k in range(c + 1, min(c + m, N + 1)):
                U[k] = self.phi(l, k, U[k - 1])

    def c_relax(self, l, U):
        N, m = self.levels[l].N, self.m
        for k in range(m, (N // m) * m + 1, m):
            U[k] = self.phi(l, k, U[k - 1])

    def relax(self, l, U):
        self.f_relax(l, U)
        if self.relax_kind == "FCF":
            self.c_relax(l, U)
            self.f_relax(l, U)

    def residual(self, l, U):
        """Injected C-point residual r_k = Phi_{km}(U_{km-1}) - U_{km}, k = 0..N_{l+1} (r_0 = 0)."""
        m = self.m
        Nc = self.levels[l + 1].N
        r = np.zeros((Nc + 1,) + U.shape[1:])
        for k in range(1, Nc + 1):
            r[k] = self.phi(l, k * m, U[k * m - 1]) - U[k * m]
        return r

    def coarsest_solve(self, l, E):
        E[0] = self.levels[l].G[0]
        for k in range(1, self.levels[l].N + 1):
            E[k] = self.phi(l, k, E[k - 1])

    def cycle(self, l, U):
        """Steps 1-4 of Algorithm 3.1 on level l >= 1 (U holds the zero start)."""
        if l == len(self.levels) - 1:
            self.coarsest_solve(l, U)
            return
        self.relax(l, U)
        self.levels[l + 1].G = self.residual(l, U)
        E = np.zeros_like(self.levels[l + 1].G)
        self.cycle(l + 1, E)
        U[:: self.m][: E.shape[0]] += E
        self.f_relax(l, U)                     # interpolation: injection + F-relaxation

    # ---- driver ------------------------------------------------------------------------------
    def solve(self, F, psi0, tol=1e-9, max_iter=100, U0=None, return_history=False):
        """Run V-cycles until the level-0 residual norm drops below tol.

        F: [N, ny, nx] level-0 loads (None = zero); psi0: [ny, nx];
        U0: optional initial space-time iterate [N+1, ny, nx] (its slice 0 is
        replaced by psi0).  Returns (U, iterations, converged[, history]).
        """
        self.F = None if F is None else np.asarray(F, dtype=np.float64)
        N = self.levels[0].N
        shape = (N + 1,) + np.shape(psi0)
        U = np.zeros(shape) if U0 is None else np.array(U0, dtype=np.float64, copy=True)
        U[0] = psi0
        h = self.op.prob.hx * self.op.prob.hy
        hist = []
        converged = False
        it = 0
        while it < max_iter:
            self.relax(0, U)
            r = self.residual(0, U)
            norm = float(np.sqrt(h * np.sum(r * r)))
            hist.append(norm)
            if norm < tol:
                converged = True
                break
            it += 1
            self.levels[1].G = r
            E = np.zeros_like(r)
            self.cycle(1, E)
            U[:: self.m][: E.shape[0]] += E
        if not converged:
            self.f_relax(0, U)
        out = (U, it, converged)
        return out + (hist,) if return_history else out

    def iterate(self, F, psi0, iterations, U0=None):
        """Exactly `iterations` cycles (relax, residual, coarse solve, C-point correction)
        followed by a final F-relaxation; no stop test.  Returns U."""
        self.F = None if F is None else np.asarray(F, dtype=np.float64)
        N = self.levels[0].N
        U = np.zeros((N + 1,) + np.shape(psi0)) if U0 is None else np.array(U0, dtype=np.float64, copy=True)
        U[0] = psi0
        for _ in range(iterations):
            self.relax(0, U)
            r = self.residual(0, U)
            self.levels[1].G = r
            E = np.zeros_like(r)
            self.cycle(1, E)
            U[:: self.m][: E.shape[0]] += E
        self.f_relax(0, U)
        return U
