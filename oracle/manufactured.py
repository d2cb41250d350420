"""Example 4.1: manufactured solution, its load vectors and the L^2 error at T.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; not part of the product path).

Example 4.1 fixes u(x, y, t) = A e^{-t} (x - x^2)^2 (y - y^2)^2 on (0,1)^2 with
A = 10, and prints the source f; here the amplitude A is a parameter (the
f printed in the paper scales linearly with it).  f = e^{-t} g(x, y) with

  g = -A (x-x^2)^2 (y-y^2)^2
      + A K_x (y-y^2)^2 / cos(beta pi) * [ (x^{2-2b} + (1-x)^{2-2b}) / Gamma(3-2b)
              - 6 (x^{3-2b} + (1-x)^{3-2b}) / Gamma(4-2b) + 12 (x^{4-2b} + (1-x)^{4-2b}) / Gamma(5-2b) ]
      + (the same in y with K_y, gamma).

Load vector, eq. (chp-02-03): F_n,j = int_{t_{n-1}}^{t_n} (f, phi_j) dt.  The paper
uses an unspecified quadrature; reading taken here: the time integral is
exact, (e^{-t_{n-1}} - e^{-t_n}) (g, phi_j), and (g, phi_j) is a Duffy-collapsed
Gauss-Legendre rule on every triangle.  The error column ||error||_0 of
Tables 1-4 is the continuous L^2(Omega) norm of u(T) - u_h(T), u_h the
piecewise-linear interpolant of the nodal values, integrated per triangle.

Triangulation (Section 2, read from the 7-point mass stencil): every mesh
cell [x_k, x_k+1] x [y_j, y_j+1] is cut by the diagonal from (x_k, y_j) to
(x_k+1, y_j+1).
"""
import math

import numpy as np


def exact_u(x, y, t, amp=10.0):
    return amp * np.exp(-t) * (x - x * x) ** 2 * (y - y * y) ** 2


def source_g(x, y, beta, gamma, Kx, Ky, amp=10.0):
    """Spatial factor g of f = e^{-t} g, as printed in Example 4.1."""
    def bracket(z, r):
        e = 2.0 - 2.0 * r
        return ((z ** e + (1 - z) ** e) / math.gamma(3 - 2 * r)
                - 6.0 * (z ** (e + 1) + (1 - z) ** (e + 1)) / math.gamma(4 - 2 * r)
                + 12.0 * (z ** (e + 2) + (1 - z) ** (e + 2)) / math.gamma(5 - 2 * r))
    px = (x - x * x) ** 2
    py = (y - y * y) ** 2
    return (-amp * px * py
            + amp * Kx * py / math.cos(beta * math.pi) * bracket(x, beta)
            + amp * Ky * px / math.cos(gamma * math.pi) * bracket(y, gamma))


def _triangle_rule(q):
    """Points (barycentric l1, l2, l3) and weights (sum 1/2) on the reference triangle."""
    g, w = np.polynomial.legendre.leggauss(q)
    s = 0.5 * (g + 1.0)
    ws = 0.5 * w
    S, T = np.meshgrid(s, s, indexing="ij")
    W = np.outer(ws, ws) * (1.0 - S)            # Duffy map (s, t) -> (s, (1-s) t)
    xi = S.ravel()
    eta = ((1.0 - S) * T).ravel()
    return np.stack([1.0 - xi - eta, xi, eta], axis=1), W.ravel()


def _triangles(M):
    """Vertex index triples (k, j) of all triangles of the M x M mesh on the unit square."""
    tris = []
    for j in range(M):
        for k in range(M):
            tris.append(((k, j), (k + 1, j), (k + 1, j + 1)))
            tris.append(((k, j), (k + 1, j + 1), (k, j + 1)))
    return np.array(tris)                          # [ntri, 3, 2]


def load_spatial(beta, gamma, Kx, Ky, M, amp=10.0, q=12):
    """(g, phi_j) for every interior node of the M x M mesh of (0,1)^2, as [M-1, M-1] (y rows, x cols)."""
    h = 1.0 / M
    bary, w = _triangle_rule(q)
    tris = _triangles(M)
    V = tris.astype(np.float64) * h                 # [ntri, 3, 2] coordinates
    P = np.einsum("qv,tvd->tqd", bary, V)           # [ntri, nq, 2]
    gv = source_g(P[..., 0], P[..., 1], beta, gamma, Kx, Ky, amp)
    area = 0.5 * h * h
    out = np.zeros((M + 1, M + 1))                  # [y, x] including boundary nodes
    for v in range(3):
        contrib = 2.0 * area * (gv * bary[None, :, v] * w[None, :]).sum(axis=1)
        np.add.at(out, (tris[:, v, 1], tris[:, v, 0]), contrib)
    return out[1:M, 1:M]


def load_vectors(t, beta, gamma, Kx, Ky, M, amp=10.0, q=12):
    """F_n, n = 1..N, as [N, M-1, M-1]."""
    t = np.asarray(t, dtype=np.float64)
    G = load_spatial(beta, gamma, Kx, Ky, M, amp, q)
    fac = np.exp(-t[:-1]) - np.exp(-t[1:])
    return fac[:, None, None] * G[None, :, :]


def nodal_psi0(M, amp=10.0):
    x = np.arange(1, M) / M
    X, Y = np.meshgrid(x, x, indexing="xy")
    return exact_u(X, Y, 0.0, amp)


def l2_error(U_T, T, M, amp=10.0, q=8):
    """||u(., T) - u_h(., T)||_{L^2(Omega)} with u_h the P1 interpolant of interior values U_T [M-1, M-1]."""
    h = 1.0 / M
    full = np.zeros((M + 1, M + 1))
    full[1:M, 1:M] = U_T
    bary, w = _triangle_rule(q)
    tris = _triangles(M)
    V = tris.astype(np.float64) * h
    P = np.einsum("qv,tvd->tqd", bary, V)
    nod = full[tris[:, :, 1], tris[:, :, 0]]        # [ntri, 3]
    uh = nod @ bary.T                               # [ntri, nq]
    ue = exact_u(P[..., 0], P[..., 1], T, amp)
    area = 0.5 * h * h
    return float(math.sqrt((2.0 * area * ((ue - uh) ** 2 * w[None, :]).sum(axis=1)).sum()))


def uniform_grid(N, T=1.0):
    return np.linspace(0.0, T, N + 1)


def piecewise_uniform_grid(N, eps, T=1.0):
    """Section 4.1: N/4 steps on [0, s], N/2 on [s, T-s], N/4 on [T-s, T], s = 2 eps ln N."""
    if N % 4:
        raise ValueError("N must be a multiple of 4")
    s = 2.0 * eps * math.log(N)
    a = np.linspace(0.0, s, N // 4 + 1)
    b = np.linspace(s, T - s, N // 2 + 1)
    c = np.linspace(T - s, T, N // 4 + 1)
    return np.concatenate([a, b[1:], c[1:]])
