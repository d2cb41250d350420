"""Independent evaluation of the fractional bilinear form on P1 hat functions.

Pin for the oracle's stiffness matrices (not part of the oracle): the entry
of A_x^beta between nodes P and Q is, by eq. (chp-02-07),

  1/(2 cos(beta pi)) * int_c^d [ (D_L^beta phi_P, D_R^beta phi_Q) + (D_R^beta phi_P, D_L^beta phi_Q) ] dy,

the inner products taken along the horizontal line at height y.  On such a
line a hat function is piecewise linear with kinks z_k and slope jumps c_k,
so phi = sum_k c_k (x - z_k)_+ = sum_k c_k (z_k - x)_+.  The Riemann-Liouville
derivatives of order beta of these ramps are (x - z)_+^(1-beta)/Gamma(2-beta)
and (z - x)_+^(1-beta)/Gamma(2-beta), and the Beta integral gives

  (D_L^beta phi_P, D_R^beta phi_Q) = sum_{k,l} c^P_k c^Q_l (z_l - z_k)_+^(3-2beta) / Gamma(4-2beta).

The y integral is done numerically (adaptive QUADPACK) strip by strip.  This
route shares nothing with the printed closed forms of the Toeplitz entries.
"""
import math

import numpy as np
import scipy.integrate


def _line_trace(p, q, j, s, M, h):
    """Kinks and values of the hat of grid node (p, q) on the line y = y_j + s h_y (strip j).

    The mesh cell [x_k, x_k+1] x [y_j, y_j+1] is cut by the diagonal (x_k, y_j)-(x_k+1, y_j+1).
    Returns breakpoints z (including both domain ends) and the trace values there.
    """
    def nodal(k, jj):
        return 1.0 if (k == p and jj == q) else 0.0

    z, v = [], []
    for k in range(M + 1):
        z.append(k * h)
        v.append((1 - s) * nodal(k, j) + s * nodal(k, j + 1))
        if k < M:
            z.append((k + s) * h)
            v.append((1 - s) * nodal(k, j) + s * nodal(k + 1, j + 1))
    return np.array(z), np.array(v)


def _slope_jumps(z, v):
    dz = np.diff(z)
    slopes = np.where(dz > 0, np.diff(v) / np.where(dz > 0, dz, 1.0), 0.0)
    full = np.concatenate([[0.0], slopes, [0.0]])
    return np.diff(full)                  # jump at every breakpoint


def line_form(P, Q, j, s, M, h, rho):
    """(D_L phi_P, D_R phi_Q) + (D_R phi_P, D_L phi_Q) on the line y = y_j + s h."""
    z, vP = _line_trace(P[0], P[1], j, s, M, h)
    _, vQ = _line_trace(Q[0], Q[1], j, s, M, h)
    cP, cQ = _slope_jumps(z, vP), _slope_jumps(z, vQ)
    D = z[None, :] - z[:, None]             # D[k, l] = z_l - z_k
    K = np.where(D > 0, np.abs(D) ** (3 - 2 * rho), 0.0)
    return float(cP @ K @ cQ + cQ @ K @ cP) / math.gamma(4 - 2 * rho)


def stiffness_entry_x(P, Q, Mx, My, h_x, h_y, rho):
    """A_x^rho entry between grid nodes P = (p, q) and Q (1-based interior grid indices, Mx x My mesh)."""
    M = Mx
    total = 0.0
    for j in range(My):                     # strips [y_j, y_j+1]
        if not ({j, j + 1} & {P[1]}) or not ({j, j + 1} & {Q[1]}):
            continue
        val, _ = scipy.integrate.quad(lambda s: line_form(P, Q, j, s, M, h_x, rho), 0.0, 1.0,
                                      epsabs=1e-15, epsrel=1e-13, limit=200)
        total += val * h_y
    return total / (2.0 * math.cos(rho * math.pi))


def stiffness_matrix_x(Mx, My, h_x, h_y, rho):
    """Full A_x^rho by quadrature, x-fastest ordering of the (Mx-1)(My-1) interior nodes."""
    nx, ny = Mx - 1, My - 1
    nodes = [(i + 1, j + 1) for j in range(ny) for i in range(nx)]
    A = np.zeros((nx * ny, nx * ny))
    for a, P in enumerate(nodes):
        for b, Q in enumerate(nodes):
            if b < a:
                continue
            if abs(P[1] - Q[1]) > 1:
                continue
            A[a, b] = A[b, a] = stiffness_entry_x(P, Q, Mx, My, h_x, h_y, rho)
    return A


def stiffness_matrix_y(Mx, My, h_x, h_y, rho):
    """A_y^rho by quadrature: the diagonal cut is symmetric under x <-> y, so swap the roles."""
    nx, ny = Mx - 1, My - 1
    Ax_swapped = stiffness_matrix_x(My, Mx, h_y, h_x, rho)   # acts on y-fastest ordering
    perm = np.array([i * ny + j for j in range(ny) for i in range(nx)])  # x-fastest index -> y-fastest index
    return Ax_swapped[np.ix_(perm, perm)]


def mass_matrix(Mx, My, h_x, h_y):
    """Textbook P1 mass matrix assembled from element matrices (area/12) * [[2,1,1],[1,2,1],[1,1,2]]."""
    nx, ny = Mx - 1, My - 1
    K = np.zeros((nx * ny, nx * ny))
    loc = (0.5 * h_x * h_y / 12.0) * (np.ones((3, 3)) + np.eye(3))
    for j in range(My):
        for k in range(Mx):
            for tri in (((k, j), (k + 1, j), (k + 1, j + 1)), ((k, j), (k + 1, j + 1), (k, j + 1))):
                idx = [(x - 1) + (y - 1) * nx if 0 < x < Mx and 0 < y < My else -1 for x, y in tri]
                for a in range(3):
                    for b in range(3):
                        if idx[a] >= 0 and idx[b] >= 0:
                            K[idx[a], idx[b]] += loc[a, b]
    return K
