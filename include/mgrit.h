/*
 * C ABI of the MI355X (gfx950) MGRIT solver for the 2-D Riesz space-fractional
 * diffusion equation discretised by linear finite elements in space and time
 * (Yue, Shu, Xu, Bu, Pan: "Parallel-in-Time with Fully Finite Element Multigrid
 * for 2-D Space-fractional Diffusion Equations", arXiv 1805.06688).
 *
 * Problem (eqs. 1.1-1.3): u_t = K_x d^{2b}u/d|x|^{2b} + K_y d^{2g}u/d|y|^{2g} + f on
 * (a,b) x (c,d), u = 0 on the boundary, u(., 0) = psi_0, 1/2 < beta, gamma < 1.
 * One time step (eq. chp-02-03):
 *     [M_h + tau_n/2 A_h] U_n = F_n + [M_h - tau_n/2 A_h] U_{n-1},  A_h = K_x A_x + K_y A_y,
 * with M_h, A_x, A_y the block matrices printed in Section 2.  The space-time
 * system (eq. ode-03) is solved by MGRIT (Algorithm 3.1) with FCF- or
 * F-relaxation; every spatial solve is conjugate gradients (Section 3.2).
 *
 * Layout of every grid array ("slice"): n_y rows of n_x doubles, x fastest
 * (the paper's node order), n_x = Mx - 1, n_y = My - 1 interior nodes.
 * Space-time arrays are [count][n_y][n_x], contiguous.
 *
 * Memory: `mem` = MGRIT_MEM_DEVICE means every array pointer is a device
 * pointer valid on the handle's stream; MGRIT_MEM_HOST means host memory
 * (copied in and out inside the call).  The caller owns every array; inputs are
 * only read.  A handle owns its device memory and is not thread-safe; distinct
 * handles are independent.  All work is ordered on the stream given at setup
 * (NULL = the default stream); calls return after the stream has finished.
 *
 * Return codes: MGRIT_OK (0); negative = error, nothing written except where
 * stated; positive = finished without meeting the tolerance, outputs written.
 * mgrit_last_error() returns a thread-local message for the last failure.
 */
#ifndef MGRIT_H
#define MGRIT_H

#ifdef __cplusplus
extern "C" {
#endif

#define MGRIT_OK          0
#define MGRIT_EINVAL     (-1)   /* invalid argument (ranges below)                       */
#define MGRIT_ENOMEM     (-2)   /* device or host allocation failed                      */
#define MGRIT_EHIP       (-3)   /* a HIP runtime call failed                             */
#define MGRIT_ENOCONV     1     /* max_iter reached; last iterate written, stats filled  */
#define MGRIT_EDIVERGED   2     /* residual grew beyond divergence_factor x initial      */

#define MGRIT_MEM_HOST    0
#define MGRIT_MEM_DEVICE  1

#define MGRIT_RELAX_F     0
#define MGRIT_RELAX_FCF   1

/* Coarse-level propagator (levels >= 1).  CN is eq. (equ-03-02): Crank-Nicolson
 * with the coarse step.  BE: backward Euler with the coarse step.  CN2: two
 * Crank-Nicolson half steps.  OPT: two Crank-Nicolson steps of lengths
 * 2 tau~/a1 and 2 tau~/a2, a1,2 = c/4 +- sqrt(c^2/16 - c), c = 4 tau~ sum 1/tau_n
 * over the level-0 steps inside the coarse step; per mode of eq. (equ-03-05) it
 * agrees with the product of the fine propagators to first order in tau~ sigma
 * and in the stiff limit (needs an even m).  The choice changes the
 * convergence rate only; the fixed point is sequential stepping in every case. */
#define MGRIT_COARSE_CN   0
#define MGRIT_COARSE_BE   1
#define MGRIT_COARSE_CN2  2
#define MGRIT_COARSE_OPT  3

#define MGRIT_PREC_FP64   0   /* every operator application in FP64 (FP64 MFMA)        */
/* MIXED: each propagator solve by iterative refinement.  The right-hand side,
 * the iterate and its residual r = b - B x stay FP64 and the stop test is the
 * FP64 one (||r|| <= rtol ||b||); each refinement step solves B d = r / ||r||
 * by PCG in FP32 (operator on the FP32 matrix cores, FP32 vectors, FP64
 * reductions) to the relative tolerance max(rtol ||b|| / ||r||, inner_rtol).
 * The solution is the FP64 one to the CG tolerance; a refinement step whose
 * inner target was the pass tolerance itself (rtol ||b|| / ||r|| >= 10 x
 * inner_rtol, e.g. the last step) is accepted without recomputing the FP64
 * residual.  Passes whose CG tolerance is 1e-4 or looser (the coarse levels at
 * the usual cg_rtol_coarse) run wholly in FP32 with the FFT operator: right-hand
 * side and initial residual from the FP64 data rounded on load, one refinement
 * step (FP32 rounding, ~1e-7 of ||b||, is far below such a tolerance).
 * MIXED_COARSE: FP64 on level 0 (and in sequential stepping), MIXED on the
 * coarse levels.  Both take precond NONE or FD_BF16. */
#define MGRIT_PREC_MIXED        1
#define MGRIT_PREC_MIXED_COARSE 2
/* MIXED_BF16: MIXED with the inner operator's Toeplitz products on the BF16
 * matrix cores: every FP32 operand is split into two BF16 parts, x = x_hi +
 * x_lo + O(2^-18 x), and a v is taken as a_hi v_hi + a_hi v_lo + a_lo v_hi with
 * FP32 accumulation (relative error of each product below 3 x 2^-18, about the
 * inner tolerance); the mass stencil, the vectors and every FP64 step are those
 * of MIXED.  The refinement recovers the FP64 solution as in MIXED. */
#define MGRIT_PREC_MIXED_BF16   3

/* Preconditioner of the spatial CG solves (Section 3.2 uses none).  FD: exact
 * inverse of a Kronecker-structured approximation of the step matrix (lumped
 * mass, cross-lumped stiffness), applied by fast diagonalisation (see
 * mgrit_fd_eigen); it changes the iteration count only, not the solution the
 * solver converges to. */
#define MGRIT_PRECOND_NONE    0
#define MGRIT_PRECOND_FD      1
/* FD_BF16: the same preconditioner with its four dense products in BF16 on the
 * matrix cores (FP32 accumulation); the operator, residuals and iterates stay
 * FP64, so the solution is the FP64 one. */
#define MGRIT_PRECOND_FD_BF16 2

/* How the operator M_h + theta A_h is applied.  DENSE: the Toeplitz products
 * as dense contractions on the matrix cores (tiled kernels).  FFT: each
 * Toeplitz product along a grid line as a circulant convolution of length 512
 * (n_x, n_y <= 256) or 1024 (n_x, n_y <= 512; EINVAL beyond) by FFT,
 * O(n^2 log n) per slice instead of O(n^3); results agree with DENSE to
 * rounding.  AUTO: FFT where it applies, else DENSE. */
#define MGRIT_OP_AUTO  0
#define MGRIT_OP_DENSE 1
#define MGRIT_OP_FFT   2

/* Tile edge of the operator kernels (64 or 32 nodes).  AUTO times both on the
 * first batch of each width and keeps the faster; RULE takes 64 when the batch
 * holds at least 512 such tiles.  The choice changes speed only: results are
 * bitwise the same (dot products are summed per 32 x 32 block in a fixed order). */
#define MGRIT_TILE_AUTO  0
#define MGRIT_TILE_RULE  1
#define MGRIT_TILE_64    2
#define MGRIT_TILE_32    3

/* Space discretisation.  P1: linear elements on the triangulated mesh, the
 * matrices of Section 2 (the paper's scheme).  Q1: bilinear elements on the
 * same rectangles, whose matrices are Kronecker products of 1-D linear-element
 * matrices, M_h = M_y (x) M_x and A_h = K_x M_y (x) A_x + K_y A_y (x) M_x, with
 * M = h/6 tridiag(1, 4, 1) and the dense Toeplitz 1-D fractional stiffness
 * A[i][j] = h^(1-2rho) / (2 cos(rho pi) Gamma(4-2rho)) g(|i-j|) of
 * mgrit_fd_stiffness_entry (K = 1).  With Q1 the FD preconditioner is the
 * exact inverse of the step matrix (consistent 1-D mass, unweighted
 * stiffness), so each propagator solve converges in one PCG iteration: the
 * fast-diagonalisation propagator. */
#define MGRIT_ELEMENT_P1 0
#define MGRIT_ELEMENT_Q1 1

typedef struct {
    double beta, gamma;     /* fractional orders, 1/2 < beta, gamma < 1 (eq. 1.1)        */
    double Kx, Ky;          /* diffusion coefficients, > 0                               */
    double a, b, c, d;      /* domain (a,b) x (c,d), a < b, c < d                        */
    int Mx, My;             /* mesh intervals per direction (h_x = (b-a)/Mx), >= 2       */
    int Nt;                 /* number of time steps, >= 1                                */
    const double* t;        /* host array of Nt+1 times, t[0] = 0 < t[1] < ... < t[Nt]   */
} mgrit_problem;

typedef struct {
    int m;                  /* coarsening factor, >= 2                                   */
    int max_levels;         /* levels including the finest, >= 2                         */
    int relax;              /* MGRIT_RELAX_F or MGRIT_RELAX_FCF                          */
    int coarse;             /* MGRIT_COARSE_*                                            */
    int precision;          /* MGRIT_PREC_*                                              */
    int max_iter;           /* MGRIT iterations, >= 1                                    */
    double tol_abs;         /* stop when the discrete L2 C-point residual norm < tol_abs */
    double tol_rel;         /* ... or < tol_rel x the norm of the first iteration (0: off)  */
    double cg_rtol;         /* CG stops when ||r||_2 <= cg_rtol ||b||_2                  */
    int cg_maxit;           /* CG iteration cap per solve                                */
    int precond;            /* MGRIT_PRECOND_*                                           */
    double cg_rtol_adapt;   /* > 0: inexact early iterations (mgrit_solve only): CG rtol  */
                            /* of iteration k = clamp(cg_rtol_adapt x ||r_k-1|| / ||r_0||, */
                            /* cg_rtol, 1e-4), ||r|| the level-0 residual norms; 0: off   */
    int warm_start;         /* 1: a relaxation that recomputes a point whose current value  */
                            /* is an iterate starts CG from that value; 0: always from the  */
                            /* propagated state (the converged result is the same)          */
    double divergence_factor; /* EDIVERGED when a norm exceeds this x the first (0: off) */
    int tile_policy;        /* MGRIT_TILE_*                                              */
    double cg_rtol_coarse;  /* > 0: CG rtol of the propagators on levels >= 1 (coarse     */
                            /* corrections only; the fixed point is set by level 0, so    */
                            /* this changes the MGRIT iteration count, not the solution); */
                            /* 0: cg_rtol                                                  */
    double inner_rtol;      /* mixed precision: floor of the inner FP32 tolerance (0: 1e-5) */
    int graphs;             /* 1: replay pairs of CG iterations as HIP graphs captured on   */
                            /* first use (needs a non-NULL stream; results are unchanged)   */
    int op;                 /* MGRIT_OP_*                                                */
    int coarse_relax;       /* relaxation on levels >= 1: MGRIT_RELAX_* (-1: as relax)   */
    int element;            /* MGRIT_ELEMENT_P1 (Section 2) or MGRIT_ELEMENT_Q1          */
} mgrit_options;

typedef struct {
    int iterations;             /* MGRIT iterations carried out                         */
    int converged;              /* 1 when the tolerance was met                         */
    int levels;                 /* levels in the hierarchy                              */
    long long phi_applications; /* propagator applications (one per slice)              */
    long long cg_iterations;    /* CG iterations summed over all slices                 */
    double residual_history[64];/* level-0 residual norm per iteration (first 64)       */
    long long refinements;      /* mixed precision: refinement steps summed over slices */
} mgrit_stats;

typedef struct mgrit_handle mgrit_handle;

/* Fill `opt` with defaults: m = 8, max_levels = 30, FCF, CN, FP64, max_iter = 100,
 * tol_abs = 1e-9, tol_rel = 0, cg_rtol = 1e-9 (the paper's tolerances, Section 3.2),
 * cg_maxit = 10000, precond = NONE, cg_rtol_adapt = 0, warm_start = 1,
 * divergence_factor = 0, tile_policy = AUTO, cg_rtol_coarse = 0, inner_rtol = 0,
 * graphs = 0, op = AUTO, coarse_relax = -1, element = P1. */
void mgrit_default_options(mgrit_options* opt);

/* Validate the problem, evaluate the Toeplitz generating sequences of Section 2
 * (entries of A_1^rho and A_2^rho, evaluated in 113-bit floating point and
 * rounded once to FP64) and the scales c_x, c_y, build the level hierarchy
 * t^(l+1) = t^(l)[::m] (Section 3.1) and allocate device memory.
 * `stream` is a hipStream_t or NULL.  Errors: EINVAL (beta or gamma outside
 * (1/2,1), K <= 0, a >= b or c >= d, Mx or My < 2, Nt < 1, t not strictly
 * increasing from 0, m < 2, max_levels < 2, unknown enum, OPT with odd m),
 * ENOMEM, EHIP. */
int mgrit_setup(const mgrit_problem* prob, const mgrit_options* opt, void* stream,
                mgrit_handle** out);

/* Solve the space-time system (eq. ode-03) by MGRIT V-cycles (Algorithm 3.1).
 * F: [Nt][n_y][n_x] load vectors F_1..F_Nt of eq. (chp-02-03) (NULL = zero load);
 * psi0: [n_y][n_x] nodal initial values U_0; U_init: optional [Nt+1][n_y][n_x]
 * initial iterate (NULL = zero; its slice 0 is ignored); U: [Nt+1][n_y][n_x]
 * output, U[0] = psi0.  Returns OK, ENOCONV or EDIVERGED (U written in all
 * three cases), or a negative error.  `st` may be NULL. */
int mgrit_solve(mgrit_handle* h, const double* F, const double* psi0, const double* U_init,
                double* U, int mem, mgrit_stats* st);

/* Several independent problems on one mesh solved together: probs[0..nprob)
 * share Mx, My and the domain and take the same options; each has its own
 * beta, gamma, K_x, K_y, time grid and N_t (all must give the same number of
 * levels; cg_rtol_adapt must be 0).  Every sweep of a level (each F- and
 * C-relaxation step, the C-point residual, each coarse step) gathers the
 * slices of all problems still iterating into one set of kernel launches.
 * Each problem stops on its own test (tolerances as in mgrit_solve) and leaves
 * the batches; every slice is computed as it would be alone, so a problem's
 * result equals its own mgrit_solve (bitwise, except that with FD_BF16 the
 * preconditioner chooses its small-batch kernel by the batch width, which
 * changes the rounding).  The handle owns a copy of all problems' loads and
 * states (the footprint grows by sum (2 N_t + 1) n_x n_y doubles).
 * Errors: EINVAL (as mgrit_setup, or meshes, domains or level counts that
 * differ), ENOMEM, EHIP. */
int mgrit_setup_group(const mgrit_problem* probs, int nprob, const mgrit_options* opt, void* stream,
                      mgrit_handle** out);

/* Solve every problem of a group handle.  F[p] (may be NULL, or F itself NULL:
 * zero loads), psi0[p] and U[p] as in mgrit_solve for problem p, all in the
 * memory space `mem`; st: nprob stats (may be NULL): iterations, converged and
 * residual_history per problem, phi_applications, cg_iterations and
 * refinements of the whole group.  Returns OK when all converged, EDIVERGED
 * when one diverged, else ENOCONV; every U[p] is written. */
int mgrit_solve_group(mgrit_handle* h, const double* const* F, const double* const* psi0, double* const* U,
                      int mem, mgrit_stats* st);

/* Exactly `iterations` MGRIT iterations (relaxation, C-point residual, coarse
 * solve, C-point correction) followed by a final F-relaxation, with no stop
 * test: the iterate the algorithm has after that many steps.  Arguments as in
 * mgrit_solve. */
int mgrit_iterate(mgrit_handle* h, const double* F, const double* psi0, const double* U_init,
                  int iterations, double* U, int mem, mgrit_stats* st);

/* Sequential time stepping U_n = Phi_n(U_{n-1}), n = 1..Nt (eq. chp-02-03), the
 * result MGRIT converges to.  Arguments as in mgrit_solve. */
int mgrit_sequential(mgrit_handle* h, const double* F, const double* psi0, double* U, int mem,
                     mgrit_stats* st);

/* Batched propagator of one level (eqs. equ-03-01, equ-03-02):
 *   level 0:  u_out[s] = [M + tau/2 A]^{-1} ([M - tau/2 A] u_in[s] + g[s])
 *             with tau = t[k] - t[k-1], k = step[s] (g = load F_k, may be NULL);
 *   level l:  u_out[s] = Psi^(l)_k u_in[s] + g[s] with the coarse propagator
 *             of the options and the step of level l (g may be NULL).
 * step: host array of nslices step indices, 1 <= k <= N_l.  u_in, g, u_out:
 * [nslices][n_y][n_x]; u_out may not overlap u_in.  Each slice is solved by
 * CG from the start vector u_in[s]. */
int mgrit_propagate(mgrit_handle* h, int level, const int* step, int nslices,
                    const double* u_in, const double* g, double* u_out, int mem);

/* Operator application (the matrix-vector product inside every CG iteration):
 *   out[s] = add[s] + sign * ( M_h v[s] + theta[s] A_h v[s] ),
 * theta: host array of nslices values, sign = +1 or -1, add may be NULL.
 * v, add, out: [nslices][n_y][n_x]; out may not overlap v. */
int mgrit_apply(mgrit_handle* h, int nslices, const double* theta, double sign,
                const double* v, const double* add, double* out, int mem);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operator application as mgrit_apply, with the same kernels and the same
 * results, that allocates nothing.  Its slice descriptors and the x-pass
 * workspace of the FFT operator live in a fixed per-GPU scratch array of
 * MGRIT_NOALLOC_SCRATCH_BYTES, held until the process ends; a call that
 * would need more (24 bytes per slice, rounded up to 256, plus 8 n_x n_y
 * bytes per slice with the FFT operator: 32 slices of 511 x 511, 128 of
 * 255 x 255) returns EINVAL before any work.  theta, v, add (may be NULL) and
 * out are DEVICE pointers (theta: nslices doubles); the work is enqueued on
 * the handle's stream and the call returns without waiting for it.  All calls
 * on one GPU share its scratch array: calls whose work overlaps on one GPU
 * (other streams, other threads, other handles) race and must be ordered by
 * the caller. */
#define MGRIT_NOALLOC_SCRATCH_BYTES (64u << 20)
int mgrit_apply_noalloc(mgrit_handle* h, int nslices, const double* theta, double sign,
                        const double* v, const double* add, double* out);

/* FP32 forms of the same operator, M_h + theta A_h of eq. (chp-02-03), as the
 * inner solves of mixed precision apply it (handles set up with MGRIT_PREC_MIXED
 * or MIXED_COARSE only; EINVAL otherwise).  The handle's operator kind and tile
 * policy choose the kernel: the Toeplitz products on the FP32 matrix cores
 * (DENSE, 64- or 32-node tiles) or by FP32 FFTs (FFT).  Sequences, spectra and
 * theta are rounded to FP32; dot products are accumulated in FP64.
 *   mgrit_apply_f32:    out[s] = M_h v[s] + theta[s] A_h v[s], v and out FP32;
 *   mgrit_rhs_f32:      b[s] = M_h u[s] + theta[s] A_h u[s] + f[s] (f may be NULL),
 *                       FP64 u and f rounded to FP32 as they are loaded, b FP32
 *                       (the right-hand side of a pass at a loose CG tolerance);
 *   mgrit_residual_f32: r[s] = b[s] - (M_h x[s] + theta[s] A_h x[s]), x FP64
 *                       rounded on load, b and r FP32 (its initial residual).
 * With MGRIT_PREC_MIXED_BF16, mgrit_apply_f32 applies the split-BF16 products.
 * The last two exist for the FFT operator only (EINVAL with DENSE).  theta: host
 * array of nslices values; arrays [nslices][n_y][n_x], all in the memory space
 * `mem`; outputs may not overlap inputs.  Returns after the stream has finished. */
int mgrit_apply_f32(mgrit_handle* h, int nslices, const double* theta, const float* v, float* out, int mem);
int mgrit_rhs_f32(mgrit_handle* h, int nslices, const double* theta, const double* u, const double* f,
                  float* b, int mem);
int mgrit_residual_f32(mgrit_handle* h, int nslices, const double* theta, const double* x, const float* b,
                       float* r, int mem);

/* Copy the FP64 generating sequences the device uses, already multiplied by
 * K c: seq_x = [t_x (n_x) | u_x (n_x) | w_x (n_x)], seq_y likewise with n_y,
 * where t[l] is the distance-l entry of A_1, u[l] the entry (k, k+l) and w[l]
 * the entry (k+l, k) of A_2 (w[0] repeats the diagonal); and the scalars
 * c_x, c_y.  Host buffers of 3 n_x and 3 n_y doubles.  With Q1 the x sequences
 * are K_x (4 h_y / 6) a_x (the factor of column j) and K_x (h_y / 6) a_x (columns
 * j +- 1), a_x the 1-D stiffness entries, likewise y, and c_x = c_y = 1. */
int mgrit_sequences(const mgrit_handle* h, double* seq_x, double* seq_y, double* cx, double* cy);

/* Host-only helper (no GPU needed): the generating sequences of A_1^rho and A_2^rho
 * (Section 2) for n interior nodes, each entry evaluated in IEEE binary128 and
 * rounded once to FP64.  t[l]: entry of A_1 at distance l; u[l]: entry (k, k+l)
 * of A_2; w[l]: entry (k+l, k) of A_2, l >= 1 (w[0] = u[0]).  Arrays of n doubles,
 * caller-owned; 1/2 < rho <= 1 is not checked here. */
void mgrit_toeplitz_sequences(double rho, int n, double* t, double* u, double* w);

/* Host-only helper: h_par^(1-2 rho) h_perp / (2 cos(rho pi) Gamma(5 - 2 rho)), the
 * scalar in front of the block stiffness matrix (c_x with h_par = h_x). */
double mgrit_stiffness_scale(double rho, double h_par, double h_perp);

/* Host-only helpers of the preconditioner (no GPU needed).  The spatial solves
 * may be preconditioned by the exact inverse of a Kronecker-structured
 * approximation of the step matrix,
 *   P = M_y (x) M_x + theta (M_y (x) K_x + K_y (x) M_x),
 * built from the 1-D lumped mass M = h I and a weighted 1-D fractional stiffness
 * K[i][j] = K_rho h^(1-2rho) / (2 cos(rho pi) Gamma(4-2rho)) g(|i-j|),
 * g(l) = |l-2|^p - 4|l-1|^p + 6|l|^p - 4|l+1|^p + |l+2|^p, p = 3 - 2 rho
 * (h_y K_x is the block stiffness A_x of Section 2 with its coupling across y
 * lumped onto the diagonal block; the solver passes 0.9 K_rho).
 * mgrit_fd_stiffness_entry returns K[i][i+l] (binary128 evaluation, rounded).
 * mgrit_fd_eigen solves K v = lambda M v, M = h I, for n nodes: V (n x n,
 * row-major, column i = eigenvector i, normalised so that V^T M V = I) and
 * lambda (n).  Returns 0, or a negative value when the eigen-iteration fails. */
double mgrit_fd_stiffness_entry(double rho, double h, double K, int l);
int mgrit_fd_eigen(double rho, int n, double h, double K, double* V, double* lambda);
/* The same with the consistent 1-D mass M = h/6 tridiag(1, 4, 1) (the Q1 pair):
 * K v = lambda M v, V^T M V = I. */
int mgrit_fd_eigen_consistent(double rho, int n, double h, double K, double* V, double* lambda);

/* Instrumentation.  While enabled, HIP events on the handle's stream bracket
 * every launch of the kernels of a CG iteration, per kernel class below
 * (enabling resets the counters; each pass ends with a stream synchronisation
 * to read the events, so instrumented solves run slower than plain ones).
 * mgrit_profile_read returns, for one class, the summed kernel time in ms, the
 * number of launches and the number of slice applications they performed (the
 * sum of CG iterations over slices).  Classes: the operator q = (M_h + theta
 * A_h) p in FP64 (64- or 32-node tiles; the FFT form counts as T64), in FP32
 * (likewise), and as split-BF16 products; the preconditioner (its four
 * products); the CG vector updates x += alpha p, r -= alpha q and the
 * direction updates p = z + beta p, in FP64 and in the FP32 inner solves. */
#define MGRIT_PROF_OP64_T64      0
#define MGRIT_PROF_OP64_T32      1
#define MGRIT_PROF_OP32_T64      2
#define MGRIT_PROF_OP32_T32      3
#define MGRIT_PROF_OP_BF16       4
#define MGRIT_PROF_PRECOND       5
#define MGRIT_PROF_UPDATE64      6
#define MGRIT_PROF_DIRECTION64   7
#define MGRIT_PROF_UPDATE32      8
#define MGRIT_PROF_DIRECTION32   9
#define MGRIT_PROF_CLASSES      10
int mgrit_profile_enable(mgrit_handle* h, int on);
int mgrit_profile_read(const mgrit_handle* h, int variant, double* apply_ms, long long* launches,
                       long long* slice_applies);

/* Device memory a handle for (prob, opt) allocates, plus staging of the
 * caller's arrays when mem = MGRIT_MEM_HOST (an upper estimate).  Only
 * the sizes of prob and opt are read. */
int mgrit_footprint(const mgrit_problem* prob, const mgrit_options* opt, int mem, size_t* bytes);
/* Device memory the handle owns now. */
int mgrit_device_bytes(const mgrit_handle* h, size_t* bytes);

/* Number of time points per level; writes up to `cap` values, returns the level count. */
int mgrit_levels(const mgrit_handle* h, int* n_per_level, int cap);

void mgrit_destroy(mgrit_handle* h);
const char* mgrit_last_error(void);

/* ---- Serving: many solves in flight on one GPU ----
 * A server admits submitted solves in arrival order while their footprint
 * (mgrit_footprint) fits the device budget and fewer than max_concurrent
 * run; each admitted solve gets its own handle and HIP stream (default
 * priority) on a worker thread, so the kernels of different solves overlap
 * on the device; memory is released as each solve finishes and the next
 * queued solves are admitted.  Every solve is computed exactly as alone
 * (all reductions are per slice in a fixed order), so its result does not
 * depend on the mix.  Inputs and U must stay valid until the solve is done;
 * with MGRIT_MEM_DEVICE they stay on the device throughout. */
typedef struct mgrit_server mgrit_server;

typedef struct {
    int rc;               /* return code of mgrit_solve (or of its setup)            */
    mgrit_stats stats;
    double submit_s;      /* seconds since server creation                           */
    double start_s;       /* admitted                                                */
    double finish_s;      /* result written                                          */
    size_t bytes;         /* footprint of the request alone                          */
    int group_size;       /* requests solved together in its group solve (1: alone)  */
} mgrit_request_info;

/* device_budget_bytes: memory the server may commit to solves at once;
 * max_concurrent >= 1.  Errors: EINVAL. */
int mgrit_server_create(size_t device_budget_bytes, int max_concurrent, mgrit_server** out);
/* Batching of requests: a worker that admits the oldest queued request also
 * takes up to max_members - 1 more queued requests with the same mesh, domain,
 * options and memory space (while the budget holds their footprints plus the
 * group's copies of their loads and states) and solves them as one group
 * (mgrit_setup_group): their propagator sweeps share kernel launches and each
 * result equals its solo solve (see mgrit_setup_group).  A group that cannot be
 * set up (different level counts) runs its requests one after another.
 * Default 1: every request alone.  Errors: EINVAL. */
int mgrit_server_set_group_limit(mgrit_server* s, int max_members);
/* Queue one solve (arguments as in mgrit_setup and mgrit_solve; the problem's
 * time grid is copied).  Returns EINVAL at once for invalid arguments or a
 * footprint above the whole budget.  *id identifies the request.  The solve
 * runs on the server's own stream, which waits for no other stream: device
 * inputs must be complete when this is called, and F, psi0 and U must stay
 * allocated until mgrit_server_wait (or poll) reports the request done. */
int mgrit_server_submit(mgrit_server* s, const mgrit_problem* prob, const mgrit_options* opt, const double* F,
                        const double* psi0, double* U, int mem, long long* id);
/* Block until request `id` has finished; fill *info (may be NULL). */
int mgrit_server_wait(mgrit_server* s, long long id, mgrit_request_info* info);
/* *done = 1 when request `id` has finished. */
int mgrit_server_poll(mgrit_server* s, long long id, int* done);
/* Wait for every request, stop the workers, free everything. */
void mgrit_server_destroy(mgrit_server* s);

#ifdef __cplusplus
}
#endif
#endif /* MGRIT_H */
