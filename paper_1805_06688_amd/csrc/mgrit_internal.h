// Internal interfaces between the host driver (mgrit_driver.cpp), the HIP
// kernels (kernels.hip) and the host set-up (toeplitz_setup.cpp).
#ifndef MGRIT_INTERNAL_H
#define MGRIT_INTERNAL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

// Output tiles of the operator and preconditioner kernels are TT x TT grid
// points (x rows, y columns) with TT = 64 (variant 0) or 32 (variant 1); the
// vector kernels work on chunks of 4096 consecutive elements.  Per-slice
// partial sums are stored per tile or chunk (at most pmax per slice) and are
// summed in index order, so every reduction has a fixed order.
#define MGRIT_TILE 64
// k-chunk of the Toeplitz contractions staged through LDS.
#define MGRIT_KC 32
#define MGRIT_CHUNK 4096

// One slice of a batched propagator call.  Indices refer to slices of the
// base arrays passed beside the descriptor array (stride n_x * n_y doubles).
typedef struct {
    int u;            // input state slice
    int x;            // output slice (the CG iterate)
    int f;            // load slice added to the right-hand side, -1 = none
    int g;            // slice added after the solve, -1 = none
    int x0;           // slice of the level's state holding the previous value of the
                      // target point (CG start vector when warm starts are on), -1 = none
    int prob;         // problem of the slice (tables at prob x the strides of Geom); 0 for one problem
    double theta_rhs; // right-hand side M u + theta_rhs A u (+ F)
    double theta_lhs; // system matrix M + theta_lhs A
} PropDesc;

// One slice of an operator application: out = add + sign (M v + theta A v).
typedef struct {
    int v;            // input slice
    int out;          // output slice
    int add;          // added slice, -1 = none
    int pad_;
    double theta;
} ApplyDesc;

// Geometry shared by every kernel.
typedef struct {
    int nx, ny;                 // interior nodes
    int tiles_x[2], tiles_y[2]; // ceil(n / TT) for TT = 64, 32
    int ntiles[2];              // tiles per slice for TT = 64, 32
    int nchunk;                 // vector-kernel chunks per slice
    int pmax;                   // partial sums stored per slice
    long long stride;           // doubles per slice = nx * ny
    int seq_off_x, seq_off_y;   // index of distance 0 in the padded sequence arrays
    double mass;                // h_x h_y / 12 (P1) or h_x h_y / 36 (Q1)
    int q1;                     // mass stencil: 0 the 7-point P1 stencil (6; 1 on the x, y and
                                // (+1,+1), (-1,-1) neighbours), 1 the 9-point Q1 one (16; 4; 1)
    int pad_;
    // Several problems of one mesh in one batch: each table holds one block per problem, problem p's
    // block p x stride elements after problem 0's (the pointers in Seqs, FftPlan, FdMats, FdMatsB)
    long long ps_seq;           // padded generating sequences (FP64 and FP32 copies alike)
    long long ps_spec;          // FFT kernel spectra (kx, ky and their FP32 copies)
    long long ps_fd;            // FP64 preconditioner matrices and eigenvalues
    long long ps_fdb;           // BF16 preconditioner matrices
    long long ps_fde;           // FP32 preconditioner eigenvalues
} Geom;

// Padded generating sequences on the device, already multiplied by K c:
// T1[d + off] = A_1 entry at distance |d|, A2[d + off] = A_2 entry (k, k+d)
// for d >= 0 and (k-d, k) for d < 0; zero for |d| >= n.
typedef struct {
    const double* T1x;
    const double* A2x;
    const double* T1y;
    const double* A2y;
} Seqs;

// FP32 roundings of the same sequences (inner solves of mixed precision).
typedef struct {
    const float* T1x;
    const float* A2x;
    const float* T1y;
    const float* A2y;
} Seqs32;

// Tables of the FFT operator (transform length L = 512 when 2 n - 1 <= 512 for
// both directions, else 1024, so n_x, n_y <= 512): tw[k] = exp(-2 pi i k / L)
// and, per direction, the spectra of the three circulant-embedded kernels
// (A_1, A_2, A_2^T, scaled by K c and divided by L) as 3 x L interleaved complex
// values; FP32 copies for mixed precision.  nbx, nby: workgroups per slice of
// the x and y line passes (ceil(n / 14)).
typedef struct {
    const double* tw;
    const double* kx;
    const double* ky;
    const float* tw32;
    const float* kx32;
    const float* ky32;
    int nbx, nby;
    int L;
} FftPlan;
#define MGRIT_FFT_LEN 1024
#define MGRIT_FFT_LINES 14

// Device matrices of the fast-diagonalisation preconditioner (row-major):
// Vx[k][i] = component k of eigenvector i (x), VxT its transpose, likewise y;
// lx, ly the generalised eigenvalues.
typedef struct {
    const double* Vx;
    const double* VxT;
    const double* Vy;
    const double* VyT;
    const double* lx;
    const double* ly;
} FdMats;

// BF16 copies for the reduced-precision preconditioner, zero-padded to
// npx = 64 tiles_x[0], npy = 64 tiles_y[0]: VxT[i][k] = Vx[k][i] and Vx[i][k]
// (ld npx) for the products over x; VyT[j][k] = Vy[k][j] and Vy[j][k] (ld npy)
// for the products over y; lx, ly padded with zeros.
typedef struct {
    const unsigned short* VxT;   // BF16 bit patterns
    const unsigned short* Vx;
    const unsigned short* VyT;
    const unsigned short* Vy;
    const float* lx;
    const float* ly;
} FdMatsB;

// Host set-up (toeplitz_setup.cpp).
void mgrit_toeplitz_sequences(double rho, int n, double* t, double* u, double* w);
double mgrit_stiffness_scale(double rho, double h_par, double h_perp);
// Fast-diagonalisation preconditioner set-up (fd_setup.cpp).
double mgrit_fd_stiffness_entry(double rho, double h, double K, int l);
int mgrit_fd_eigen(double rho, int n, double h, double K, double* V, double* lambda);
int mgrit_fd_eigen_consistent(double rho, int n, double h, double K, double* V, double* lambda);

// Kernel launchers (kernels.hip).  All return a hipError_t as int.  `tv`
// selects the operator/preconditioner tile edge (0: 64, 1: 32).  Partial-sum
// arrays hold pmax entries per slice; the tiled kernels write one per 32 x 32
// block (ntiles[1], whatever tv) and the vector kernels nchunk, and each
// consumer is told how many to sum.
// dot_mode: 0 none, 1 partial = sum v*out, 2 = sum out*out.
int launch_apply(const Geom* g, const Seqs* sq, int tv, const ApplyDesc* desc, int S, const double* vbase,
                 double* outbase, const double* addbase, double sign, int dot_mode, double* partial,
                 const int* active, void* stream);
// Right-hand side of a batched propagator: b[s] = M u + theta_rhs A u (+ F), partial of ||b||^2.
int launch_rhs(const Geom* g, const Seqs* sq, int tv, const PropDesc* desc, int S, const double* ubase,
               const double* fbase, double* bws, double* partial_bb, void* stream);
// CG start vector: x = x0base[x0] when warm and x0 >= 0, else x = u.
int launch_cg_init_x(const Geom* g, const PropDesc* desc, int S, const double* ubase, const double* x0base,
                     int warm, double* xbase, void* stream);
// r[s] = b[s] - (M x + theta_lhs A x), partial of ||r||^2.
int launch_init_residual(const Geom* g, const Seqs* sq, int tv, const PropDesc* desc, int S, const double* xbase,
                         const double* bws, double* rws, double* partial_rr, const int* mask, void* stream);
// q = B p for active slices, partial p.q.
int launch_cg_apply(const Geom* g, const Seqs* sq, int tv, const PropDesc* desc, int S, const double* pws,
                    double* qws, double* partial_pq, const int* active, void* stream);
// x = 0 when ||b|| = 0, p = z; active flags from ||r|| vs rtol ||b||, also stored into host_act,
// and the reset iteration counts into host_iters (pinned host memory, either may be NULL).
int launch_cg_start(const Geom* g, const PropDesc* desc, int S, const double* ubase, double* xbase,
                    const double* zws, double* pws, const double* partial_bb, int nbb, const double* partial_rr,
                    int nrr, double rtol2, double* bb, int* active, int* iters, int* host_act, int* host_iters,
                    void* stream);
// alpha = rho / p.q; x += alpha p, r -= alpha q; partial r.r (nchunk entries).
int launch_cg_update(const Geom* g, const PropDesc* desc, int S, double* xbase, double* rws, const double* pws,
                     const double* qws, const double* partial_rho, int nrho, const double* partial_pq, int npq,
                     double* partial_rr_new, const int* active, void* stream);
// p = z + (rho_new / rho) p; next active flags (from ||r||^2) and iteration counts.  The
// direction kernels also store the next flags into host_next (pinned host memory, may be
// NULL) and the iteration counts into host_iters (may be NULL), which the host reads without a
// copy once the iteration is complete.
int launch_cg_direction(const Geom* g, int S, const double* zws, double* pws, const double* partial_rho, int nrho,
                        const double* partial_rho_new, int nrho_new, const double* partial_rr_new, const double* bb,
                        double rtol2, int maxit, const int* active, int* active_next, int* iters, int* host_next,
                        int* host_iters, void* stream);
// z = P^{-1} r (four batched dense products), partial r.z; active may be NULL.
int launch_fd_apply(const Geom* g, const FdMats* fd, int tv, const PropDesc* desc, int S, const double* rws,
                    double* zws, double* t1, double* t2, double* partial_rz, const int* active, void* stream);
// Same with BF16 products and FP32 accumulation (64-tiles; t1, t2 hold S padded BF16 slices).
int launch_fdb_apply(const Geom* g, const FdMatsB* fd, const PropDesc* desc, int S, const double* rws, double* zws,
                     void* t1, void* t2, double* partial_rz, const int* active, void* stream);
// ---- mixed precision (inner FP32 solves of an iterative refinement; FP32 workspaces
// hold slice s at s * stride) ----
// Same preconditioner on FP32 r32 / z32; z32 is also copied to zcopy when given.
int launch_fdb_apply32(const Geom* g, const FdMatsB* fd, const PropDesc* desc, int S, const float* r32, float* z32,
                       float* zcopy, void* t1, void* t2, double* partial_rz, const int* active, const void* rimg,
                       void* stream);
// q32 = M p32 + theta_lhs A p32 (FP32 matrix cores) for active slices, partial p.q.
int launch_apply32(const Geom* g, const Seqs32* sq, int tv, const PropDesc* desc, int S, const float* p32,
                   float* q32, double* partial_pq, const int* active, void* stream);
// The same product with the Toeplitz products as split BF16 products on the matrix cores
// (a v = a_hi v_hi + a_hi v_lo + a_lo v_hi, FP32 accumulation; 64-tiles).
int launch_apply_bf16(const Geom* g, const Seqs32* sq, const PropDesc* desc, int S, const float* p32, float* q32,
                      double* partial_pq, const int* active, void* stream);
// Start of a refinement step from the FP64 residual (or, with rws == NULL, from an FP32
// residual already in r32, scaled in place): flags, scale ||r||, inner tolerance
// eta^2 = max(rtol^2 ||b||^2 / ||r||^2, eta_min2), r32 = r / ||r||, d32 = 0, and p32 = r32
// with partial r32.r32 when p32 != NULL; first: x = 0 where b = 0, counts reset.  The flags
// are also stored into host_act and the reset counts into host_iters (pinned host memory, either
// may be NULL).  trust_out[s] = 1 when the step's inner target is the pass tolerance itself (inner flag
// 2) or the slice was already settled; a slice with trust_in[s] = 1 (the previous step's trust_out) is
// settled and stays inactive (not read on the first step).
int launch_mx_begin(const Geom* g, const PropDesc* desc, int S, double* xbase, const double* rws,
                    const double* partial_bb, const double* partial_rr, int np, double rtol2, double eta_min2,
                    int first, double* bb, double* scale, double* eta2, int* oact, int* iact, int* iters, float* r32,
                    float* d32, float* p32, double* partial_rr32, int* host_act, int* host_iters,
                    const int* trust_in, int* trust_out, void* rimg, void* stream);
// alpha = rho / p.q; d32 += alpha p32, r32 -= alpha q32; partial r32.r32.
int launch_mx_update(const Geom* g, int S, float* d32, float* r32, const float* p32, const float* q32,
                     const double* partial_rho, int nrho, const double* partial_pq, int npq, double* partial_rr_new,
                     const int* active, void* rimg, void* stream);
// p32 = z32 + (rho_new / rho) p32; next flags from ||r32||^2 <= eta2[s] and the total count.
int launch_mx_direction(const Geom* g, int S, const float* z32, float* p32, const double* partial_rho, int nrho,
                        const double* partial_rho_new, int nrho_new, const double* partial_rr_new, const double* eta2,
                        int maxit, const int* active, int* active_next, int* iters, int* host_next, int* host_iters,
                        void* stream);
// x += scale[s] d32 where oact[s].
int launch_mx_refine(const Geom* g, const PropDesc* desc, int S, double* xbase, const float* d32,
                     const double* scale, const int* oact, const int* trust, int* need, void* stream);

// ---- operator by FFT (same results as the tiled kernels up to rounding; one
// partial per workgroup of the y pass, nby per slice; pbuf: S slices) ----
int launch_fft_apply(const Geom* g, const FftPlan* pl, const ApplyDesc* desc, int S, const double* vbase,
                     double* outbase, const double* addbase, double sign, int dot_mode, double* partial,
                     double* pbuf, void* stream);
int launch_fft_rhs(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* ubase,
                   const double* fbase, double* bws, double* partial_bb, double* pbuf, void* stream);
int launch_fft_init_residual(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* xbase,
                             const double* bws, double* rws, double* partial_rr, double* pbuf, const int* mask, void* stream);
int launch_fft_cg_apply(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* pws,
                        double* qws, double* partial_pq, const int* active, double* pbuf, void* stream);
int launch_fft_apply32(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const float* p32, float* q32,
                       double* partial_pq, const int* active, float* pbuf, void* stream);
// The right-hand side and the initial residual computed in FP32 from the FP64 U, F and X
// (rounded as they are loaded) into slot s of b32 and r32: b32 = M u + theta_rhs A u + f,
// partial ||b||^2; r32 = b32 - (M x + theta_lhs A x), partial ||r||^2.
int launch_fft_rhs32(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* ubase,
                     const double* fbase, float* b32, double* partial_bb, float* pbuf, void* stream);
int launch_fft_init_residual32(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* xbase,
                               const float* b32, float* r32, double* partial_rr, float* pbuf, void* stream);

// desc[s] = {v = s, out = s, add = has_add ? s : -1, theta = theta[s]} for s < S (theta on the device).
int launch_fill_apply_desc(int S, const double* theta, int has_add, ApplyDesc* desc, void* stream);
// x[s] += G[s] for slices with g >= 0.
int launch_add_g(const Geom* g, const PropDesc* desc, int S, double* xbase, const double* gbase, void* stream);
// y[yi[s]] += a * x[xi[s]]; when partial != NULL, partial of ||y||^2 after the update (nchunk entries).
int launch_axpy_slices(const Geom* g, int S, const int* yi, double* ybase, const int* xi, const double* xbase,
                       double a, double* partial, void* stream);
// Fill slices of an array with zero.
int launch_zero_slices(const Geom* g, int S, const int* idx, double* base, void* stream);

#ifdef __cplusplus
}
#endif
#endif
