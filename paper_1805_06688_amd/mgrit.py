"""Thin ctypes binding of libmgrit.so (the C ABI in include/mgrit.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Arrays are either torch tensors on the GPU (passed as device pointers, work
ordered on the current torch stream) or numpy arrays (host memory, copied in
and out by the library).  There is no CPU fallback: importing this module
fails when the library has not been built.
"""
import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmgrit.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, EDIVERGED = 0, -1, -2, -3, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
RELAX = {"F": 0, "FCF": 1}
COARSE = {"cn": 0, "be": 1, "cn2": 2, "opt": 3}
PRECISION = {"fp64": 0, "mixed": 1, "mixed-coarse": 2, "mixed-bf16": 3}
PRECOND = {"none": 0, "fd": 1, "fd-bf16": 2}
TILE = {"auto": 0, "rule": 1, "64": 2, "32": 3}
OPERATOR = {"auto": 0, "dense": 1, "fft": 2}
ELEMENT = {"p1": 0, "q1": 1}


class _Problem(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("gamma", ctypes.c_double), ("Kx", ctypes.c_double),
                ("Ky", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("d", ctypes.c_double), ("Mx", ctypes.c_int), ("My", ctypes.c_int), ("Nt", ctypes.c_int),
                ("t", ctypes.POINTER(ctypes.c_double))]


class _Options(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("max_levels", ctypes.c_int), ("relax", ctypes.c_int),
                ("coarse", ctypes.c_int), ("precision", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("tol_abs", ctypes.c_double), ("tol_rel", ctypes.c_double), ("cg_rtol", ctypes.c_double),
                ("cg_maxit", ctypes.c_int), ("precond", ctypes.c_int), ("cg_rtol_adapt", ctypes.c_double),
                ("warm_start", ctypes.c_int),
                ("divergence_factor", ctypes.c_double), ("tile_policy", ctypes.c_int),
                ("cg_rtol_coarse", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("graphs", ctypes.c_int), ("op", ctypes.c_int), ("coarse_relax", ctypes.c_int),
                ("element", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("levels", ctypes.c_int),
                ("phi_applications", ctypes.c_longlong), ("cg_iterations", ctypes.c_longlong),
                ("residual_history", ctypes.c_double * 64), ("refinements", ctypes.c_longlong)]

    def history(self):
        n = min(64, self.iterations + 1)
        return [self.residual_history[i] for i in range(n)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("rc", ctypes.c_int), ("stats", Stats), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("finish_s", ctypes.c_double), ("bytes", ctypes.c_size_t),
                ("group_size", ctypes.c_int)]


SYMBOLS = ("mgrit_default_options", "mgrit_setup", "mgrit_setup_group", "mgrit_solve", "mgrit_solve_group",
           "mgrit_iterate", "mgrit_sequential", "mgrit_propagate", "mgrit_apply", "mgrit_apply_noalloc",
           "mgrit_apply_f32", "mgrit_rhs_f32", "mgrit_residual_f32", "mgrit_sequences", "mgrit_levels",
           "mgrit_destroy", "mgrit_last_error", "mgrit_toeplitz_sequences", "mgrit_stiffness_scale",
           "mgrit_profile_enable", "mgrit_profile_read", "mgrit_fd_stiffness_entry", "mgrit_fd_eigen",
           "mgrit_fd_eigen_consistent", "mgrit_footprint", "mgrit_device_bytes", "mgrit_server_create",
           "mgrit_server_set_group_limit", "mgrit_server_submit", "mgrit_server_wait", "mgrit_server_poll",
           "mgrit_server_destroy")


def load_library(path=_LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1805_06688_amd.build`")
    lib = ctypes.CDLL(path)
    P, c_int, c_dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.mgrit_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.mgrit_default_options.restype = None
    lib.mgrit_setup.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Options), P, ctypes.POINTER(P)]
    lib.mgrit_setup.restype = c_int
    lib.mgrit_setup_group.argtypes = [ctypes.POINTER(_Problem), c_int, ctypes.POINTER(_Options), P, ctypes.POINTER(P)]
    lib.mgrit_setup_group.restype = c_int
    lib.mgrit_solve_group.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), c_int,
                                      ctypes.POINTER(Stats)]
    lib.mgrit_solve_group.restype = c_int
    lib.mgrit_solve.argtypes = [P, P, P, P, P, c_int, ctypes.POINTER(Stats)]
    lib.mgrit_solve.restype = c_int
    lib.mgrit_iterate.argtypes = [P, P, P, P, c_int, P, c_int, ctypes.POINTER(Stats)]
    lib.mgrit_iterate.restype = c_int
    lib.mgrit_sequential.argtypes = [P, P, P, P, c_int, ctypes.POINTER(Stats)]
    lib.mgrit_sequential.restype = c_int
    lib.mgrit_propagate.argtypes = [P, c_int, ctypes.POINTER(c_int), c_int, P, P, P, c_int]
    lib.mgrit_propagate.restype = c_int
    lib.mgrit_apply.argtypes = [P, c_int, ctypes.POINTER(c_dbl), c_dbl, P, P, P, c_int]
    lib.mgrit_apply.restype = c_int
    lib.mgrit_apply_noalloc.argtypes = [P, c_int, P, c_dbl, P, P, P]
    lib.mgrit_apply_noalloc.restype = c_int
    lib.mgrit_apply_f32.argtypes = [P, c_int, ctypes.POINTER(c_dbl), P, P, c_int]
    lib.mgrit_apply_f32.restype = c_int
    lib.mgrit_rhs_f32.argtypes = [P, c_int, ctypes.POINTER(c_dbl), P, P, P, c_int]
    lib.mgrit_rhs_f32.restype = c_int
    lib.mgrit_residual_f32.argtypes = [P, c_int, ctypes.POINTER(c_dbl), P, P, P, c_int]
    lib.mgrit_residual_f32.restype = c_int
    lib.mgrit_sequences.argtypes = [P, ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl),
                                    ctypes.POINTER(c_dbl)]
    lib.mgrit_sequences.restype = c_int
    lib.mgrit_levels.argtypes = [P, ctypes.POINTER(c_int), c_int]
    lib.mgrit_levels.restype = c_int
    lib.mgrit_destroy.argtypes = [P]
    lib.mgrit_destroy.restype = None
    lib.mgrit_toeplitz_sequences.argtypes = [c_dbl, c_int, ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl),
                                             ctypes.POINTER(c_dbl)]
    lib.mgrit_toeplitz_sequences.restype = None
    lib.mgrit_stiffness_scale.argtypes = [c_dbl, c_dbl, c_dbl]
    lib.mgrit_stiffness_scale.restype = c_dbl
    lib.mgrit_profile_enable.argtypes = [P, c_int]
    lib.mgrit_profile_enable.restype = c_int
    lib.mgrit_profile_read.argtypes = [P, c_int, ctypes.POINTER(c_dbl), ctypes.POINTER(ctypes.c_longlong),
                                       ctypes.POINTER(ctypes.c_longlong)]
    lib.mgrit_profile_read.restype = c_int
    lib.mgrit_fd_stiffness_entry.argtypes = [c_dbl, c_dbl, c_dbl, c_int]
    lib.mgrit_fd_stiffness_entry.restype = c_dbl
    lib.mgrit_fd_eigen.argtypes = [c_dbl, c_int, c_dbl, c_dbl, ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl)]
    lib.mgrit_fd_eigen.restype = c_int
    lib.mgrit_fd_eigen_consistent.argtypes = lib.mgrit_fd_eigen.argtypes
    lib.mgrit_fd_eigen_consistent.restype = c_int
    lib.mgrit_footprint.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Options), c_int,
                                    ctypes.POINTER(ctypes.c_size_t)]
    lib.mgrit_footprint.restype = c_int
    lib.mgrit_device_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.mgrit_device_bytes.restype = c_int
    lib.mgrit_server_create.argtypes = [ctypes.c_size_t, c_int, ctypes.POINTER(P)]
    lib.mgrit_server_create.restype = c_int
    lib.mgrit_server_set_group_limit.argtypes = [P, c_int]
    lib.mgrit_server_set_group_limit.restype = c_int
    lib.mgrit_server_submit.argtypes = [P, ctypes.POINTER(_Problem), ctypes.POINTER(_Options), P, P, P, c_int,
                                        ctypes.POINTER(ctypes.c_longlong)]
    lib.mgrit_server_submit.restype = c_int
    lib.mgrit_server_wait.argtypes = [P, ctypes.c_longlong, ctypes.POINTER(RequestInfo)]
    lib.mgrit_server_wait.restype = c_int
    lib.mgrit_server_poll.argtypes = [P, ctypes.c_longlong, ctypes.POINTER(c_int)]
    lib.mgrit_server_poll.restype = c_int
    lib.mgrit_server_destroy.argtypes = [P]
    lib.mgrit_server_destroy.restype = None
    lib.mgrit_last_error.argtypes = []
    lib.mgrit_last_error.restype = ctypes.c_char_p
    return lib


_lib = load_library()


class MgritError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise MgritError(rc, _lib.mgrit_last_error().decode())
    return rc


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, mem, count, fp32=False):
    """Raw pointer of an FP64 (FP32) array with at least `count` elements in the expected memory space."""
    if x is None:
        return None
    if _is_torch(x):
        import torch
        if mem != MEM_DEVICE or not x.is_cuda:
            raise ValueError("mixing host and device arrays in one call")
        if x.dtype != (torch.float32 if fp32 else torch.float64) or not x.is_contiguous():
            raise ValueError(f"device arrays must be contiguous {'float32' if fp32 else 'float64'} tensors")
        if x.numel() < count:
            raise ValueError(f"array has {x.numel()} elements, {count} needed")
        return ctypes.c_void_p(x.data_ptr())
    if mem != MEM_HOST:
        raise ValueError("mixing host and device arrays in one call")
    if x.dtype != (np.float32 if fp32 else np.float64) or not x.flags["C_CONTIGUOUS"]:
        raise ValueError(f"host arrays must be C-contiguous {'float32' if fp32 else 'float64'}")
    if x.size < count:
        raise ValueError(f"array has {x.size} elements, {count} needed")
    return ctypes.c_void_p(x.ctypes.data)


def _mem_of(x):
    return MEM_DEVICE if _is_torch(x) else MEM_HOST


def toeplitz_sequences(rho, n):
    """Host-side generating sequences (t, u, w) of A_1^rho and A_2^rho, as the library builds them."""
    t, u, w = np.empty(n), np.empty(n), np.empty(n)
    dp = ctypes.POINTER(ctypes.c_double)
    _lib.mgrit_toeplitz_sequences(float(rho), int(n), t.ctypes.data_as(dp), u.ctypes.data_as(dp),
                                  w.ctypes.data_as(dp))
    return t, u, w


def stiffness_scale(rho, h_par, h_perp):
    return _lib.mgrit_stiffness_scale(float(rho), float(h_par), float(h_perp))


def fd_stiffness_entry(rho, h, K, l):
    return _lib.mgrit_fd_stiffness_entry(float(rho), float(h), float(K), int(l))


def fd_eigen(rho, n, h, K, consistent=False):
    """Generalised eigenpairs of the 1-D (K, M) pair of the preconditioner: (V [n, n], lambda [n]); M = h I, or
    h/6 tridiag(1, 4, 1) with consistent=True."""
    V = np.empty((n, n))
    lam = np.empty(n)
    dp = ctypes.POINTER(ctypes.c_double)
    fn = _lib.mgrit_fd_eigen_consistent if consistent else _lib.mgrit_fd_eigen
    rc = fn(float(rho), int(n), float(h), float(K), V.ctypes.data_as(dp), lam.ctypes.data_as(dp))
    if rc != 0:
        raise MgritError(rc, "eigen-iteration failed")
    return V, lam


def default_options():
    o = _Options()
    _lib.mgrit_default_options(ctypes.byref(o))
    return o


def make_problem(beta, gamma, Kx, Ky, Mx, My, t, domain=(0.0, 1.0, 0.0, 1.0)):
    """(ctypes problem struct, the time grid array it points to)."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    p = _Problem(beta, gamma, Kx, Ky, domain[0], domain[1], domain[2], domain[3], int(Mx), int(My), len(t) - 1,
                 t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return p, t


def make_options(m=8, max_levels=30, relax="FCF", coarse="cn", precision="fp64", max_iter=100, tol_abs=1e-9,
                 tol_rel=0.0, cg_rtol=1e-9, cg_maxit=10000, precond="none", cg_rtol_adapt=0.0, warm_start=True,
                 divergence_factor=0.0, tile="auto", cg_rtol_coarse=0.0, inner_rtol=0.0, graphs=False,
                 op="auto", coarse_relax=None, element="p1"):
    o = default_options()
    o.element = ELEMENT[element]
    o.coarse_relax = -1 if coarse_relax is None else RELAX[coarse_relax]
    o.op = OPERATOR[op]
    o.graphs = 1 if graphs else 0
    o.inner_rtol = float(inner_rtol)
    o.tile_policy = TILE[str(tile)]
    o.cg_rtol_coarse = float(cg_rtol_coarse)
    o.m, o.max_levels, o.max_iter, o.cg_maxit = int(m), int(max_levels), int(max_iter), int(cg_maxit)
    o.relax, o.coarse, o.precision = RELAX[relax], COARSE[coarse], PRECISION[precision]
    o.precond = PRECOND[precond]
    o.cg_rtol_adapt = float(cg_rtol_adapt)
    o.warm_start = 1 if warm_start else 0
    o.tol_abs, o.tol_rel = float(tol_abs), float(tol_rel)
    o.cg_rtol, o.divergence_factor = float(cg_rtol), float(divergence_factor)
    return o


def footprint(beta, gamma, Kx, Ky, Mx, My, t, mem=MEM_DEVICE, **opts):
    p, _t = make_problem(beta, gamma, Kx, Ky, Mx, My, t)
    o = make_options(**opts)
    b = ctypes.c_size_t()
    _check(_lib.mgrit_footprint(ctypes.byref(p), ctypes.byref(o), int(mem), ctypes.byref(b)))
    return b.value


class Solver:
    """One problem (eqs. 1.1-1.3 on a time grid) set up on the GPU."""

    def __init__(self, beta, gamma, Kx, Ky, Mx, My, t, domain=(0.0, 1.0, 0.0, 1.0), stream=None, **opts):
        self._h = None
        p, self._t = make_problem(beta, gamma, Kx, Ky, Mx, My, t, domain)
        o = make_options(**opts)
        if stream is None:
            stream = self._torch_stream()
        h = ctypes.c_void_p()
        _check(_lib.mgrit_setup(ctypes.byref(p), ctypes.byref(o), stream, ctypes.byref(h)))
        self._h = h
        self.nx, self.ny, self.Nt = int(Mx) - 1, int(My) - 1, len(self._t) - 1

    @staticmethod
    def _torch_stream():
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return None

    @property
    def slice_size(self):
        return self.nx * self.ny

    def close(self):
        if self._h is not None:
            _lib.mgrit_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _out(self, like, count, out):
        if out is not None:
            return out
        if _is_torch(like):
            import torch
            return torch.empty(count, dtype=torch.float64, device=like.device)
        return np.empty(count, dtype=np.float64)

    def _shape(self, arr, n):
        return arr.reshape(n, self.ny, self.nx)

    def solve(self, F, psi0, U_init=None, out=None, allow_noconv=True):
        """MGRIT V-cycles to the tolerance.  Returns (U [Nt+1, ny, nx], Stats, return code)."""
        return self._run(_lib.mgrit_solve, F, psi0, U_init, out, None, allow_noconv)

    def iterate(self, F, psi0, iterations, U_init=None, out=None):
        return self._run(_lib.mgrit_iterate, F, psi0, U_init, out, int(iterations), False)

    def sequential(self, F, psi0, out=None):
        return self._run(_lib.mgrit_sequential, F, psi0, None, out, None, False, seq=True)

    def _run(self, fn, F, psi0, U_init, out, iterations, allow_noconv, seq=False):
        mem = _mem_of(psi0)
        n = self.slice_size
        U = self._out(psi0, (self.Nt + 1) * n, out)
        st = Stats()
        args = [self._h, _ptr(F, mem, self.Nt * n), _ptr(psi0, mem, n)]
        if not seq:
            args.append(_ptr(U_init, mem, (self.Nt + 1) * n))
        if iterations is not None:
            args.append(iterations)
        args += [_ptr(U, mem, (self.Nt + 1) * n), mem, ctypes.byref(st)]
        rc = _check(fn(*args), allow=(ENOCONV, EDIVERGED) if allow_noconv else ())
        return self._shape(U, self.Nt + 1), st, rc

    def propagate(self, level, steps, u_in, g=None, out=None):
        steps = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
        S = len(steps)
        mem = _mem_of(u_in)
        n = self.slice_size
        U = self._out(u_in, S * n, out)
        _check(_lib.mgrit_propagate(self._h, int(level), steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), S,
                                    _ptr(u_in, mem, S * n), _ptr(g, mem, S * n), _ptr(U, mem, S * n), mem))
        return self._shape(U, S)

    def apply(self, theta, v, sign=1.0, add=None, out=None):
        theta = np.ascontiguousarray(np.atleast_1d(np.asarray(theta, dtype=np.float64)))
        S = len(theta)
        mem = _mem_of(v)
        n = self.slice_size
        U = self._out(v, S * n, out)
        _check(_lib.mgrit_apply(self._h, S, theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(sign),
                                _ptr(v, mem, S * n), _ptr(add, mem, S * n), _ptr(U, mem, S * n), mem))
        return self._shape(U, S)

    def apply_noalloc(self, theta, v, sign=1.0, add=None, out=None):
        """mgrit_apply_noalloc: as apply() with device arrays only (theta a float64 CUDA tensor); the work is
        enqueued on the handle's stream and nothing is allocated by the library."""
        S, n = theta.numel(), self.slice_size
        U = self._out(v, S * n, out)
        _check(_lib.mgrit_apply_noalloc(self._h, S, _ptr(theta, MEM_DEVICE, S), float(sign),
                                        _ptr(v, MEM_DEVICE, S * n), _ptr(add, MEM_DEVICE, S * n),
                                        _ptr(U, MEM_DEVICE, S * n)))
        return self._shape(U, S)

    def _out32(self, like, count, out):
        if out is not None:
            return out
        if _is_torch(like):
            import torch
            return torch.empty(count, dtype=torch.float32, device=like.device)
        return np.empty(count, dtype=np.float32)

    def apply_f32(self, theta, v, out=None):
        """FP32 inner operator: out[s] = M v[s] + theta[s] A v[s] with FP32 v and out (mixed-precision handles)."""
        theta = np.ascontiguousarray(np.atleast_1d(np.asarray(theta, dtype=np.float64)))
        S, mem, n = len(theta), _mem_of(v), self.slice_size
        U = self._out32(v, S * n, out)
        _check(_lib.mgrit_apply_f32(self._h, S, theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    _ptr(v, mem, S * n, True), _ptr(U, mem, S * n, True), mem))
        return self._shape(U, S)

    def rhs_f32(self, theta, u, f=None, out=None):
        """FP32 right-hand side b[s] = M u[s] + theta[s] A u[s] + f[s] from FP64 u, f (FFT operator)."""
        theta = np.ascontiguousarray(np.atleast_1d(np.asarray(theta, dtype=np.float64)))
        S, mem, n = len(theta), _mem_of(u), self.slice_size
        U = self._out32(u, S * n, out)
        _check(_lib.mgrit_rhs_f32(self._h, S, theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  _ptr(u, mem, S * n), _ptr(f, mem, S * n), _ptr(U, mem, S * n, True), mem))
        return self._shape(U, S)

    def residual_f32(self, theta, x, b, out=None):
        """FP32 residual r[s] = b[s] - (M x[s] + theta[s] A x[s]) from FP64 x and FP32 b (FFT operator)."""
        theta = np.ascontiguousarray(np.atleast_1d(np.asarray(theta, dtype=np.float64)))
        S, mem, n = len(theta), _mem_of(x), self.slice_size
        U = self._out32(x, S * n, out)
        _check(_lib.mgrit_residual_f32(self._h, S, theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       _ptr(x, mem, S * n), _ptr(b, mem, S * n, True), _ptr(U, mem, S * n, True),
                                       mem))
        return self._shape(U, S)

    def sequences(self):
        sx = np.empty(3 * self.nx)
        sy = np.empty(3 * self.ny)
        cx, cy = ctypes.c_double(), ctypes.c_double()
        dp = ctypes.POINTER(ctypes.c_double)
        _check(_lib.mgrit_sequences(self._h, sx.ctypes.data_as(dp), sy.ctypes.data_as(dp), ctypes.byref(cx),
                                    ctypes.byref(cy)))
        return sx, sy, cx.value, cy.value

    def profile(self, on=True):
        _check(_lib.mgrit_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, variant=0):
        """(kernel ms, launches, slice applications) of one kernel class of the instrumentation (MGRIT_PROF_*:
        0/1 FP64 operator 64/32 tiles or FFT, 2/3 FP32 operator, 4 split-BF16 operator, 5 preconditioner,
        6/7 FP64 CG update/direction, 8/9 FP32 update/direction)."""
        ms, n, sl = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_longlong()
        _check(_lib.mgrit_profile_read(self._h, int(variant), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(sl)))
        return ms.value, n.value, sl.value

    def device_bytes(self):
        b = ctypes.c_size_t()
        _check(_lib.mgrit_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    def levels(self):
        buf = (ctypes.c_int * 64)()
        L = _lib.mgrit_levels(self._h, buf, 64)
        return [buf[i] - 1 for i in range(L)]


class Group:
    """Several problems on one mesh whose sweeps share kernel launches (mgrit_setup_group).

    problems: list of dicts with beta, gamma, Kx, Ky and t (each its own time grid); Mx, My and the domain are
    common."""

    def __init__(self, problems, Mx, My, domain=(0.0, 1.0, 0.0, 1.0), stream=None, **opts):
        self._h = None
        made = [make_problem(q["beta"], q["gamma"], q["Kx"], q["Ky"], Mx, My, q["t"], domain) for q in problems]
        self._ts = [t for _, t in made]
        arr = (_Problem * len(made))(*[p for p, _ in made])
        o = make_options(**opts)
        if stream is None:
            stream = Solver._torch_stream()
        h = ctypes.c_void_p()
        _check(_lib.mgrit_setup_group(arr, len(made), ctypes.byref(o), stream, ctypes.byref(h)))
        self._h = h
        self.nx, self.ny = int(Mx) - 1, int(My) - 1
        self.Nts = [len(t) - 1 for t in self._ts]

    def close(self):
        if self._h is not None:
            _lib.mgrit_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, Fs, psi0s, outs=None, allow_noconv=True):
        """Solve all problems: returns ([U_p [Nt_p+1, ny, nx]], [Stats], return code)."""
        P = len(self.Nts)
        mem = _mem_of(psi0s[0])
        n = self.nx * self.ny
        if outs is None:
            outs = []
            for Nt, p0 in zip(self.Nts, psi0s):
                if _is_torch(p0):
                    import torch
                    outs.append(torch.empty((Nt + 1) * n, dtype=torch.float64, device=p0.device))
                else:
                    outs.append(np.empty((Nt + 1) * n))
        PA = ctypes.c_void_p * P
        f = PA(*[_ptr(F, mem, Nt * n) if F is not None else None for F, Nt in zip(Fs, self.Nts)])
        p0 = PA(*[_ptr(x, mem, n) for x in psi0s])
        u = PA(*[_ptr(x, mem, (Nt + 1) * n) for x, Nt in zip(outs, self.Nts)])
        st = (Stats * P)()
        rc = _check(_lib.mgrit_solve_group(self._h, f, p0, u, mem, st), allow=(ENOCONV, EDIVERGED) if allow_noconv else ())
        return [x.reshape(Nt + 1, self.ny, self.nx) for x, Nt in zip(outs, self.Nts)], list(st), rc


class Request:
    """A submitted solve; keeps its arrays alive until it has finished."""

    def __init__(self, server, rid, arrays, U, shape):
        self._server, self.id, self._arrays, self.U, self._shape = server, rid, arrays, U, shape

    def done(self):
        d = ctypes.c_int()
        _check(_lib.mgrit_server_poll(self._server._s, self.id, ctypes.byref(d)))
        return bool(d.value)

    def wait(self):
        info = RequestInfo()
        _check(_lib.mgrit_server_wait(self._server._s, self.id, ctypes.byref(info)))
        self._arrays = None
        return self.U.reshape(self._shape), info


class Server:
    """Admission by device-memory footprint, concurrent solves on separate streams (C ABI mgrit_server_*)."""

    def __init__(self, device_budget_bytes, max_concurrent=4, group_limit=1):
        self._s = None
        s = ctypes.c_void_p()
        _check(_lib.mgrit_server_create(ctypes.c_size_t(int(device_budget_bytes)), int(max_concurrent),
                                        ctypes.byref(s)))
        self._s = s
        _check(_lib.mgrit_server_set_group_limit(s, int(group_limit)))

    def submit(self, F, psi0, beta, gamma, Kx, Ky, Mx, My, t, domain=(0.0, 1.0, 0.0, 1.0), out=None, **opts):
        p, tt = make_problem(beta, gamma, Kx, Ky, Mx, My, t, domain)
        o = make_options(**opts)
        mem = _mem_of(psi0)
        n = (int(Mx) - 1) * (int(My) - 1)
        Nt = len(tt) - 1
        if out is None:
            if _is_torch(psi0):
                import torch
                out = torch.empty((Nt + 1) * n, dtype=torch.float64, device=psi0.device)
            else:
                out = np.empty((Nt + 1) * n)
        if mem == MEM_DEVICE:
            # the server's stream waits for no other: finish the work that wrote the inputs first
            import torch
            torch.cuda.current_stream(psi0.device).synchronize()
        rid = ctypes.c_longlong()
        _check(_lib.mgrit_server_submit(self._s, ctypes.byref(p), ctypes.byref(o), _ptr(F, mem, Nt * n),
                                        _ptr(psi0, mem, n), _ptr(out, mem, (Nt + 1) * n), mem, ctypes.byref(rid)))
        return Request(self, rid.value, (F, psi0, tt), out, (Nt + 1, int(My) - 1, int(Mx) - 1))

    def close(self):
        if self._s is not None:
            _lib.mgrit_server_destroy(self._s)
            self._s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()
