"""Seeded synthetic inputs shaped like the paper's workloads.

Only random numbers and time grids: no arithmetic of the method lives here,
so the HIP path and the CPU oracle can both be fed from this module.

Recipes (numpy PCG64, ``default_rng(seed)``):
* load vectors F_n ~ N(0, 1) i.i.d. per interior node and step, shape [Nt, n_y, n_x];
* initial values psi_0 ~ U[0, 1] per interior node, shape [n_y, n_x];
* time grids: uniform t_n = n T / N; graded t_n = T (n / N)^2; piecewise-uniform
  with N/4, N/2, N/4 equal steps on [0, s], [s, T-s], [T-s, T], s = 2 eps ln N
  (Section 4.1).
"""
import math

import numpy as np


def uniform_grid(N, T=1.0):
    return np.linspace(0.0, T, N + 1)


def graded_grid(N, T=1.0):
    return T * (np.arange(N + 1, dtype=np.float64) / N) ** 2


def piecewise_uniform_grid(N, eps, T=1.0):
    if N % 4:
        raise ValueError("N must be a multiple of 4")
    s = 2.0 * eps * math.log(N)
    a = np.linspace(0.0, s, N // 4 + 1)
    b = np.linspace(s, T - s, N // 2 + 1)
    c = np.linspace(T - s, T, N // 4 + 1)
    return np.concatenate([a, b[1:], c[1:]])


def random_grid(N, seed, T=1.0):
    rng = np.random.default_rng(seed)
    inner = np.sort(rng.uniform(0.0, T, N - 1))
    return np.concatenate([[0.0], inner, [T]])


def random_inputs(seed, Nt, nx, ny):
    """(F [Nt, ny, nx] ~ N(0,1), psi0 [ny, nx] ~ U[0,1]) from one seed."""
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((Nt, ny, nx))
    psi0 = rng.uniform(0.0, 1.0, (ny, nx))
    return F, psi0


def random_slices(seed, S, nx, ny):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((S, ny, nx))


# The benchmark workload: 255 x 255 interior nodes, beta = 0.75, gamma = 0.85,
# K_x = 2, K_y = 1, T = 1, 1024 uniform steps, V-cycle with m = 8; F ~ N(0,1),
# psi_0 ~ U[0,1] from seed 2.
FP64_VCYCLE_255 = dict(name="vcycle-255x255x1024-uniform", beta=0.75, gamma=0.85, Kx=2.0, Ky=1.0, Mx=256, My=256,
                       Nt=1024, T=1.0, m=8, seed=2)

# The small correctness workload: 31 x 31 nodes, beta = 0.7, gamma = 0.8, K = 1,
# 64 uniform steps, two-level FCF with m = 4, manufactured solution
# u = x^2 (1-x)^2 y^2 (1-y)^2 e^{-t}.
FP64_TWOLEVEL_31 = dict(name="fp64-twolevel-31x31x64", beta=0.7, gamma=0.8, Kx=1.0, Ky=1.0, Mx=32, My=32, Nt=64,
                        T=1.0, m=4, levels=2, amp=1.0)


# The mixed-precision workload: 511 x 511 nodes, 4096 graded steps t_n = (n / N)^2 (time-dependent
# propagators), beta, gamma ~ U(0.55, 0.95) from seed 3, K = 1, m = 8; F ~ N(0,1), psi_0 ~ U[0,1].
def mixed_511(seed=3):
    rng = np.random.default_rng(seed)
    beta, gamma = (float(v) for v in rng.uniform(0.55, 0.95, 2))
    return dict(name="mixed-511x511x4096-graded", beta=beta, gamma=gamma, Kx=1.0, Ky=1.0, Mx=512, My=512, Nt=4096,
                T=1.0, m=8, seed=seed)


def device_inputs(seed, Nt, nx, ny, device="cuda"):
    """(F [Nt, ny, nx] ~ N(0,1), psi0 [ny, nx] ~ U[0,1]) drawn on the GPU by torch's Philox generator from one
    seed: the same distributions as random_inputs for workloads too large to draw on the host."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    F = torch.randn((Nt, ny, nx), dtype=torch.float64, device=device, generator=g)
    psi0 = torch.rand((ny, nx), dtype=torch.float64, device=device, generator=g)
    return F, psi0


def serving_stream(seed, n_requests, rate=20.0, n_range=(63, 1023), nt_range=(128, 8192), nt_scale=1, m=8):
    """The serving workload: Poisson arrivals (rate per second) of solves with n_x, n_y ~ U{n_range}
    independently, N_t ~ U{nt_range} (then divided by nt_scale and rounded down to a multiple of m, at least
    2 m), beta, gamma ~ U(0.55, 0.95), K = 1, T = 1, uniform grid.  Returns the first n_requests arrivals as
    dicts (arrival time, sizes, orders, grid, and the seed of their F, psi_0 for device_inputs)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate)
        nx, ny = (int(v) for v in rng.integers(n_range[0], n_range[1] + 1, 2))
        Nt = max(2 * m, int(rng.integers(nt_range[0], nt_range[1] + 1)) // nt_scale // m * m)
        beta, gamma = (float(v) for v in rng.uniform(0.55, 0.95, 2))
        out.append(dict(arrival=t, nx=nx, ny=ny, Nt=Nt, beta=beta, gamma=gamma, Kx=1.0, Ky=1.0,
                        t=uniform_grid(Nt), input_seed=seed * 100000 + k))
    return out


def many_problem_set(seed, n_problems, n_range=(127, 383), nt_range=(256, 2048), ms=(4, 8, 16)):
    """The many-instance workload: independent problems with n ~ U{n_range} square, N_t ~ U{nt_range}
    (rounded down to a multiple of the drawn m), m from ms, beta, gamma ~ U(0.55, 0.95), K = 1, uniform grid;
    F, psi_0 from device_inputs with each problem's input_seed."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_problems):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        m = int(rng.choice(ms))
        Nt = max(2 * m, int(rng.integers(nt_range[0], nt_range[1] + 1)) // m * m)
        beta, gamma = (float(v) for v in rng.uniform(0.55, 0.95, 2))
        out.append(dict(nx=n, ny=n, Nt=Nt, m=m, beta=beta, gamma=gamma, Kx=1.0, Ky=1.0, t=uniform_grid(Nt),
                        input_seed=seed * 100000 + k))
    return out


def many_same_mesh(seed, n_problems, n=127, nt_range=(256, 2048), m=8):
    """Independent problems on one n x n mesh: N_t ~ U{nt_range} (a multiple of m), beta, gamma ~ U(0.55, 0.95),
    K = 1, uniform grid; F, psi_0 from device_inputs with each problem's input_seed."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_problems):
        Nt = max(2 * m, int(rng.integers(nt_range[0], nt_range[1] + 1)) // m * m)
        beta, gamma = (float(v) for v in rng.uniform(0.55, 0.95, 2))
        out.append(dict(nx=n, ny=n, Nt=Nt, m=m, beta=beta, gamma=gamma, Kx=1.0, Ky=1.0, t=uniform_grid(Nt),
                        input_seed=seed * 100000 + 50000 + k))
    return out


def serving_trace(seed, n_requests, rate, n_range=(63, 255), nt_range=(64, 512), m=8):
    """Poisson arrivals (rate per second) of solves with n_x, n_y ~ U{n_range}, N_t ~ U{nt_range}
    (a multiple of m), beta, gamma ~ U(0.55, 0.95), K = 1, T = 1, uniform grid; F ~ N(0,1), psi_0 ~ U[0,1].
    Returns a list of dicts with the arrival time and every input (host arrays)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate)
        nx, ny = (int(v) for v in rng.integers(n_range[0], n_range[1] + 1, 2))
        Nt = int(rng.integers(nt_range[0], nt_range[1] + 1)) // m * m
        beta, gamma = (float(v) for v in rng.uniform(0.55, 0.95, 2))
        F, psi0 = random_inputs(seed * 1000 + k, Nt, nx, ny)
        out.append(dict(arrival=t, nx=nx, ny=ny, Nt=Nt, beta=beta, gamma=gamma, Kx=1.0, Ky=1.0, F=F, psi0=psi0,
                        t=uniform_grid(Nt)))
    return out


def many_problems(seed, n_problems, n_range=(127, 255), nt_range=(64, 256), ms=(4, 8, 16)):
    """Independent problems of uneven sizes (seeded): n ~ U{n_range} square, N_t ~ U{nt_range} (a multiple
    of the drawn m), m from ms, beta, gamma ~ U(0.55, 0.95), K = 1; F ~ N(0,1), psi_0 ~ U[0,1]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_problems):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        m = int(rng.choice(ms))
        Nt = max(2 * m, int(rng.integers(nt_range[0], nt_range[1] + 1)) // m * m)
        beta, gamma = (float(v) for v in rng.uniform(0.55, 0.95, 2))
        F, psi0 = random_inputs(seed * 1000 + k, Nt, n, n)
        out.append(dict(nx=n, ny=n, Nt=Nt, m=m, beta=beta, gamma=gamma, Kx=1.0, Ky=1.0, F=F, psi0=psi0,
                        t=uniform_grid(Nt)))
    return out
