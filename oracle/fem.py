"""Space discretisation: mass matrix M_h and fractional stiffness A_x^beta, A_y^gamma.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; not part of the product path).

Follows Section 2, eq. (chp-02-03) and the block forms printed after it:

* unknowns are the interior nodes, ordered x fastest: node (i, j) with
  i = 0..n_x-1 (x), j = 0..n_y-1 (y), n_x = M_beta - 1, n_y = M_gamma - 1;
* M_h = (h_x h_y / 12) * blocktridiag(M_2^T, M_1, M_2), n_y blocks of size n_x,
  M_1 = tridiag(1, 6, 1), M_2 = identity plus first super-diagonal;
* A_x^beta = c_x * blocktridiag((A_2^beta)^T, A_1^beta, A_2^beta), n_y blocks;
* A_y^gamma = c_y * P_pi^T blocktridiag((A_2^gamma)^T, A_1^gamma, A_2^gamma) P_pi,
  n_x blocks of size n_y, where P_pi reorders x-fastest into y-fastest;
* c_x = h_x^(1-2beta) h_y / (2 cos(beta pi) Gamma(5-2beta)),
  c_y = h_x h_y^(1-2gamma) / (2 cos(gamma pi) Gamma(5-2gamma)),
  h_x = (b-a)/M_beta, h_y = (d-c)/M_gamma.

Two forms are provided: ``assembled_*`` builds the matrices literally from the
printed block structure (including the permutation index list pi), for small
grids; ``apply_*`` applies the same block rows to a grid array without forming
the matrix (block row j of a block-tridiagonal matrix times the vector), for
grids up to the benchmark size.  Arrays of grid values have shape
[..., n_y, n_x] (x fastest), the same memory order as the paper's vectors.
"""
import numpy as np

from . import toeplitz


class Problem:
    """Problem statement of eqs. (1.1)-(1.3) plus the spatial mesh size."""

    def __init__(self, beta, gamma, Kx, Ky, Mx, My, a=0.0, b=1.0, c=0.0, d=1.0):
        if not (0.5 < beta < 1.0 and 0.5 < gamma < 1.0):
            raise ValueError("orders must satisfy 1/2 < beta, gamma < 1")
        if Kx <= 0 or Ky <= 0:
            raise ValueError("diffusion coefficients must be positive")
        if Mx < 2 or My < 2 or not (a < b and c < d):
            raise ValueError("bad mesh or domain")
        self.beta, self.gamma, self.Kx, self.Ky = float(beta), float(gamma), float(Kx), float(Ky)
        self.Mx, self.My = int(Mx), int(My)
        self.a, self.b, self.c, self.d = float(a), float(b), float(c), float(d)
        self.nx, self.ny = self.Mx - 1, self.My - 1
        self.hx = (self.b - self.a) / self.Mx
        self.hy = (self.d - self.c) / self.My

    @property
    def ndof(self):
        return self.nx * self.ny

    def nodes(self):
        """Interior node coordinates as arrays [n_y, n_x]."""
        x = self.a + self.hx * np.arange(1, self.Mx)
        y = self.c + self.hy * np.arange(1, self.My)
        return np.meshgrid(x, y, indexing="xy")


class Operator:
    """M_h and A_h = K_x A_x + K_y A_y for one Problem."""

    def __init__(self, prob):
        self.prob = prob
        p = prob
        self.A1x, self.A2x = toeplitz.toeplitz_factors(p.beta, p.nx)
        self.A1y, self.A2y = toeplitz.toeplitz_factors(p.gamma, p.ny)
        self.cx = toeplitz.stiffness_scale(p.beta, p.hx, p.hy)
        self.cy = toeplitz.stiffness_scale(p.gamma, p.hy, p.hx)
        self.mass_scale = p.hx * p.hy / 12.0

    # ---- block-row application (matrix free) -------------------------------------------
    @staticmethod
    def _blocktridiag_rows(V, D, U):
        """Apply blocktridiag(U^T, D, U) to V[..., nblk, bs]: out_j = D v_j + U v_{j+1} + U^T v_{j-1}."""
        out = V @ D.T
        up = V @ U.T          # U v_k for every block k
        lo = V @ U            # U^T v_k for every block k
        out[..., :-1, :] += up[..., 1:, :]
        out[..., 1:, :] += lo[..., :-1, :]
        return out

    def apply_M(self, V):
        """M_h v for grid arrays V[..., n_y, n_x]."""
        V = np.asarray(V, dtype=np.float64)
        out = 6.0 * V
        out[..., :, :-1] += V[..., :, 1:]      # M_1 off-diagonals
        out[..., :, 1:] += V[..., :, :-1]
        # block (j, j+1) = M_2 = I + S: v_{j+1}[i] + v_{j+1}[i+1]
        out[..., :-1, :] += V[..., 1:, :]
        out[..., :-1, :-1] += V[..., 1:, 1:]
        # block (j+1, j) = M_2^T: v_{j-1}[i] + v_{j-1}[i-1]
        out[..., 1:, :] += V[..., :-1, :]
        out[..., 1:, 1:] += V[..., :-1, :-1]
        return self.mass_scale * out

    def apply_Ax(self, V):
        """A_x^beta v: blocks run over y (rows of V), each block acts along x."""
        V = np.asarray(V, dtype=np.float64)
        return self.cx * self._blocktridiag_rows(V, self.A1x, self.A2x)

    def apply_Ay(self, V):
        """A_y^gamma v through the permutation: transpose to y-fastest, apply blocks over x, transpose back."""
        V = np.asarray(V, dtype=np.float64)
        Vt = np.swapaxes(V, -1, -2)                       # P_pi v as an [n_x, n_y] array
        Wt = self._blocktridiag_rows(Vt, self.A1y, self.A2y)
        return self.cy * np.swapaxes(Wt, -1, -2)          # P_pi^T (...)

    def apply_A(self, V):
        """A_h v = K_x A_x v + K_y A_y v."""
        return self.prob.Kx * self.apply_Ax(V) + self.prob.Ky * self.apply_Ay(V)

    def apply_B(self, V, tau):
        """(M_h + tau/2 A_h) v, the left-hand matrix of eq. (chp-02-03)."""
        return self.apply_M(V) + 0.5 * tau * self.apply_A(V)

    def apply_C(self, V, tau):
        """(M_h - tau/2 A_h) v, the right-hand matrix of eq. (chp-02-03)."""
        return self.apply_M(V) - 0.5 * tau * self.apply_A(V)

    # ---- literal assembly (small grids) --------------------------------------------------
    @staticmethod
    def _assemble_blocktridiag(D, U, nblk):
        bs = D.shape[0]
        K = np.zeros((nblk * bs, nblk * bs))
        for j in range(nblk):
            K[j * bs:(j + 1) * bs, j * bs:(j + 1) * bs] = D
            if j + 1 < nblk:
                K[j * bs:(j + 1) * bs, (j + 1) * bs:(j + 2) * bs] = U
                K[(j + 1) * bs:(j + 2) * bs, j * bs:(j + 1) * bs] = U.T
        return K

    def permutation(self):
        """P_pi from the index list pi (1-based in the paper): x-index groups of y-runs."""
        nx, ny = self.prob.nx, self.prob.ny
        pi = []
        for i in range(1, nx + 1):                 # group for x-index i
            for j in range(ny):                    # i, i + (M_beta-1), ..., i + (M_beta-1)(M_gamma-2)
                pi.append(i + j * nx)
        P = np.zeros((nx * ny, nx * ny))
        for row, col in enumerate(pi):
            P[row, col - 1] = 1.0
        return P

    def assembled_M(self):
        nx, ny = self.prob.nx, self.prob.ny
        M1 = 6.0 * np.eye(nx) + np.eye(nx, k=1) + np.eye(nx, k=-1)
        M2 = np.eye(nx) + np.eye(nx, k=1)
        return self.mass_scale * self._assemble_blocktridiag(M1, M2, ny)

    def assembled_Ax(self):
        return self.cx * self._assemble_blocktridiag(self.A1x, self.A2x, self.prob.ny)

    def assembled_Ay(self):
        P = self.permutation()
        return self.cy * P.T @ self._assemble_blocktridiag(self.A1y, self.A2y, self.prob.nx) @ P

    def assembled_A(self):
        return self.prob.Kx * self.assembled_Ax() + self.prob.Ky * self.assembled_Ay()
