// HIP kernels for gfx950 (CDNA4): the batched operator application of the
// space-time finite-element scheme and the vector kernels of batched CG.
//
// Operator (Section 2, block forms after eq. chp-02-03).  For a grid array U
// (n_x x n_y, x fastest) the stiffness A_h = K_x A_x + K_y A_y applied to U is
//   X = A1x U + (A2x U) shifted one column left + (A2x^T U) shifted one column right
//   Y = U A1y + rows of (U A2y^T) shifted one row up + rows of (U A2y) shifted one row down
// i.e. block row j of the block-tridiagonal A_x couples column j of U with
// columns j-1, j, j+1, and the permuted A_y couples row i with rows i-1, i, i+1.
// The six dense Toeplitz products are contractions over the full x (resp. y)
// extent: they run on the FP64 matrix cores (v_mfma_f64_16x16x4f64) with the
// three factors of one direction sharing a single LDS strip of U, and with the
// Toeplitz operands read from short windows of the generating sequences (a
// Toeplitz tile of 64 x 32 entries holds only 95 distinct values).  The
// 7-point mass stencil M_h, the scaling, the optional added vector and the
// per-tile dot product are applied in the epilogue, so one pass produces
//   out = add + sign (M_h v + theta A_h v).
//
// Work decomposition: one 256-thread workgroup per 64 x 64 output tile of one
// slice; the workgroup -> (slice, tile) map keeps every tile of a slice on one
// XCD (workgroups are dealt to the 8 XCDs round-robin), so the strips of a
// slice are fetched from HBM into one L2 only.
#include <hip/hip_runtime.h>

#include "mgrit_internal.h"

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int T = MGRIT_TILE;        // output tile edge
constexpr int KC = MGRIT_KC;         // contraction chunk
constexpr int NT = 256;              // threads per workgroup
constexpr int HALO = T + 2;          // tile plus one neighbour on each side
constexpr int SXS = KC + 2;          // LDS stride of the x-direction strip (per column)
constexpr int SYS = 80;              // LDS stride of the y-direction strip (per k row)
constexpr int WIN = KC + T;          // window of generating-sequence values per chunk
constexpr int XSTRIP = HALO * SXS;
constexpr int YSTRIP = KC * SYS;
constexpr int STAGE = (XSTRIP > YSTRIP ? XSTRIP : YSTRIP) + 3 * WIN;
constexpr int EPI = T * (T + 1);
constexpr int LDS_DOUBLES = STAGE > EPI ? STAGE : EPI;

__device__ __forceinline__ void decode_block(int ntiles, int S, int& s, int& tile) {
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int local = bid >> 3;
    s = (local / ntiles) * 8 + xcd;
    tile = local % ntiles;
    if (s >= S) s = -1;
}

inline int grid_blocks(int ntiles, int S) { return ntiles * ((S + 7) / 8) * 8; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the block in a fixed order (wave tree, then waves 0..3).
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ __forceinline__ double slice_sum(const double* partial, int s, int ntiles) {
    const double* p = partial + (long long)s * ntiles;
    double acc = 0.0;
    for (int i = 0; i < ntiles; ++i) acc += p[i];
    return acc;
}

// out = add + sign (M v + theta A v) on one 64 x 64 tile; returns the
// block-reduced dot product selected by dot_mode (valid in every thread).
__device__ void apply_tile(const Geom& g, const Seqs& sq, const double* __restrict__ v, double* __restrict__ out,
                           const double* __restrict__ add, double theta, double sign, int dot_mode, int tile,
                           double* lds, double* red, double* dot_out) {
    const int nx = g.nx, ny = g.ny;
    const int ti = tile % g.tiles_x, tj = tile / g.tiles_x;
    const int i0 = ti * T, j0 = tj * T;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int wi = wave & 1, wj = wave >> 1;

    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

    double* strip = lds;
    double* w0 = lds + (XSTRIP > YSTRIP ? XSTRIP : YSTRIP);
    double* w1 = w0 + WIN;
    double* w2 = w1 + WIN;

    // ---- x-direction: contraction over x with the A_x factors ----
    for (int k0 = 0; k0 < nx; k0 += KC) {
        for (int idx = tid; idx < HALO * KC; idx += NT) {
            const int jj = idx / KC, kk = idx - jj * KC;
            const int k = k0 + kk, j = j0 - 1 + jj;
            strip[jj * SXS + kk] = (k < nx && j >= 0 && j < ny) ? v[(long long)j * nx + k] : 0.0;
        }
        const int dbase = k0 - i0 - (T - 1);
        for (int q = tid; q < WIN; q += NT) {
            const int d = dbase + q;
            w0[q] = sq.T1x[g.seq_off_x + d];
            w1[q] = sq.A2x[g.seq_off_x + d];
            w2[q] = sq.A2x[g.seq_off_x - d];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int kk = ks + lk;
            double a0[2], a1[2], a2[2], b0[2], b1[2], b2[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const int il = wi * 32 + f * 16 + lr;
                const int q = kk - il + (T - 1);
                a0[f] = w0[q];
                a1[f] = w1[q];
                a2[f] = w2[q];
                const int jl = wj * 32 + f * 16 + lr;
                b0[f] = strip[(jl + 1) * SXS + kk];   // column j
                b1[f] = strip[(jl + 2) * SXS + kk];   // column j+1
                b2[f] = strip[jl * SXS + kk];         // column j-1
            }
#pragma unroll
            for (int fi = 0; fi < 2; ++fi)
#pragma unroll
                for (int fj = 0; fj < 2; ++fj) {
                    acc[fi][fj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[fi], b0[fj], acc[fi][fj], 0, 0, 0);
                    acc[fi][fj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[fi], b1[fj], acc[fi][fj], 0, 0, 0);
                    acc[fi][fj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[fi], b2[fj], acc[fi][fj], 0, 0, 0);
                }
        }
        __syncthreads();
    }

    // ---- y-direction: contraction over y with the A_y factors ----
    for (int k0 = 0; k0 < ny; k0 += KC) {
        for (int idx = tid; idx < KC * HALO; idx += NT) {
            const int kk = idx / HALO, ii = idx - kk * HALO;
            const int k = k0 + kk, i = i0 - 1 + ii;
            strip[kk * SYS + ii] = (k < ny && i >= 0 && i < nx) ? v[(long long)k * nx + i] : 0.0;
        }
        const int ebase = j0 - k0 - (KC - 1);
        for (int q = tid; q < WIN; q += NT) {
            const int e = ebase + q;
            w0[q] = sq.T1y[g.seq_off_y + e];
            w1[q] = sq.A2y[g.seq_off_y - e];   // A2y[k - j]: factor of row i+1
            w2[q] = sq.A2y[g.seq_off_y + e];   // A2y[j - k]: factor of row i-1
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int kk = ks + lk;
            double a0[2], a1[2], a2[2], b0[2], b1[2], b2[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const int il = wi * 32 + f * 16 + lr;
                a0[f] = strip[kk * SYS + il + 1];     // row i
                a1[f] = strip[kk * SYS + il + 2];     // row i+1
                a2[f] = strip[kk * SYS + il];         // row i-1
                const int jl = wj * 32 + f * 16 + lr;
                const int q = jl - kk + (KC - 1);
                b0[f] = w0[q];
                b1[f] = w1[q];
                b2[f] = w2[q];
            }
#pragma unroll
            for (int fi = 0; fi < 2; ++fi)
#pragma unroll
                for (int fj = 0; fj < 2; ++fj) {
                    acc[fi][fj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[fi], b0[fj], acc[fi][fj], 0, 0, 0);
                    acc[fi][fj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[fi], b1[fj], acc[fi][fj], 0, 0, 0);
                    acc[fi][fj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[fi], b2[fj], acc[fi][fj], 0, 0, 0);
                }
        }
        __syncthreads();
    }

    // ---- epilogue: stage A v through LDS, add the mass stencil ----
    double* epi = lds;
#pragma unroll
    for (int fi = 0; fi < 2; ++fi)
#pragma unroll
        for (int fj = 0; fj < 2; ++fj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wi * 32 + fi * 16 + lk + 4 * r;   // accumulator row = lane/16 + 4 r
                const int jl = wj * 32 + fj * 16 + lr;
                epi[jl * (T + 1) + il] = acc[fi][fj][r];
            }
    __syncthreads();

    double dot = 0.0;
    const double mass = g.mass;
    for (int idx = tid; idx < T * T; idx += NT) {
        const int jl = idx / T, il = idx - jl * T;
        const int i = i0 + il, j = j0 + jl;
        if (i >= nx || j >= ny) continue;
        const long long o = (long long)j * nx + i;
        const double c = v[o];
        const bool hl = i > 0, hr = i + 1 < nx, hd = j > 0, hu = j + 1 < ny;
        double m7 = 6.0 * c;
        m7 += hl ? v[o - 1] : 0.0;
        m7 += hr ? v[o + 1] : 0.0;
        m7 += hd ? v[o - nx] : 0.0;
        m7 += hu ? v[o + nx] : 0.0;
        m7 += (hr && hu) ? v[o + nx + 1] : 0.0;
        m7 += (hl && hd) ? v[o - nx - 1] : 0.0;
        double val = sign * (mass * m7 + theta * epi[jl * (T + 1) + il]);
        if (add) val += add[o];
        out[o] = val;
        if (dot_mode == 1) dot += c * val;
        else if (dot_mode == 2) dot += val * val;
    }
    if (dot_mode) *dot_out = block_sum(dot, red);
}

// ---- operator application over slices given by ApplyDesc ----
__global__ __launch_bounds__(NT) void k_apply(Geom g, Seqs sq, const ApplyDesc* __restrict__ desc, int S,
                                              const double* vbase, double* outbase, const double* addbase,
                                              double sign, int dot_mode, double* partial, const int* active) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0) return;
    if (active && !active[s]) return;
    __shared__ double lds[LDS_DOUBLES];
    __shared__ double red[4];
    const ApplyDesc d = desc[s];
    const double* addp = (addbase && d.add >= 0) ? addbase + d.add * g.stride : nullptr;
    double dot = 0.0;
    apply_tile(g, sq, vbase + d.v * g.stride, outbase + d.out * g.stride, addp, d.theta, sign, dot_mode, tile, lds,
               red, &dot);
    if (dot_mode && threadIdx.x == 0) partial[(long long)s * g.ntiles + tile] = dot;
}

// mode 0: right-hand side b = M u + theta_rhs A u (+F), partial ||b||^2
// mode 1: initial residual r = b - (M u + theta_lhs A u), partial ||r||^2
// mode 2: q = M p + theta_lhs A p (active slices), partial p.q
template <int MODE>
__global__ __launch_bounds__(NT) void k_prop_apply(Geom g, Seqs sq, const PropDesc* __restrict__ desc, int S,
                                                   const double* ubase, const double* fbase, const double* wsin,
                                                   double* wsout, double* partial, const int* active) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0) return;
    if (MODE == 2 && !active[s]) return;
    __shared__ double lds[LDS_DOUBLES];
    __shared__ double red[4];
    const PropDesc d = desc[s];
    const long long so = (long long)s * g.stride;
    double dot = 0.0;
    if (MODE == 0) {
        const double* f = (fbase && d.f >= 0) ? fbase + d.f * g.stride : nullptr;
        apply_tile(g, sq, ubase + d.u * g.stride, wsout + so, f, d.theta_rhs, 1.0, 2, tile, lds, red, &dot);
    } else if (MODE == 1) {
        apply_tile(g, sq, ubase + d.u * g.stride, wsout + so, wsin + so, d.theta_lhs, -1.0, 2, tile, lds, red, &dot);
    } else {
        apply_tile(g, sq, wsin + so, wsout + so, nullptr, d.theta_lhs, 1.0, 1, tile, lds, red, &dot);
    }
    if (threadIdx.x == 0) partial[(long long)s * g.ntiles + tile] = dot;
}

// Element range of chunk `tile` of a flattened slice.
__device__ __forceinline__ void chunk_range(const Geom& g, int tile, long long& lo, long long& hi) {
    lo = (long long)tile * (T * T);
    hi = lo + T * T;
    if (hi > g.stride) hi = g.stride;
}

__global__ __launch_bounds__(NT) void k_cg_start(Geom g, const PropDesc* __restrict__ desc, int S,
                                                 const double* ubase, double* xbase, const double* zws, double* pws,
                                                 const double* partial_bb, const double* partial_rr, double rtol2,
                                                 double* bb, int* active, int* iters) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0) return;
    const PropDesc d = desc[s];
    const double b2 = slice_sum(partial_bb, s, g.ntiles);
    const double r2 = slice_sum(partial_rr, s, g.ntiles);
    const double* u = ubase + d.u * g.stride;
    double* x = xbase + d.x * g.stride;
    const double* z = zws + (long long)s * g.stride;
    double* p = pws + (long long)s * g.stride;
    long long lo, hi;
    chunk_range(g, tile, lo, hi);
    const bool zero = !(b2 > 0.0);
    for (long long e = lo + threadIdx.x; e < hi; e += NT) {
        x[e] = zero ? 0.0 : u[e];
        p[e] = z[e];
    }
    if (tile == 0 && threadIdx.x == 0) {
        bb[s] = b2;
        active[s] = (!zero && r2 > rtol2 * b2) ? 1 : 0;
        iters[s] = 0;
    }
}

// alpha = rho / (p.q) with rho = r.z (z = r without preconditioner)
__global__ __launch_bounds__(NT) void k_cg_update(Geom g, const PropDesc* __restrict__ desc, int S, double* xbase,
                                                  double* rws, const double* pws, const double* qws,
                                                  const double* partial_rho, const double* partial_pq,
                                                  double* partial_rr_new, const int* active) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0 || !active[s]) return;
    __shared__ double red[4];
    const double rho = slice_sum(partial_rho, s, g.ntiles);
    const double pq = slice_sum(partial_pq, s, g.ntiles);
    const double alpha = rho / pq;
    double* x = xbase + desc[s].x * g.stride;
    const long long so = (long long)s * g.stride;
    double* r = rws + so;
    const double* p = pws + so;
    const double* q = qws + so;
    long long lo, hi;
    chunk_range(g, tile, lo, hi);
    double acc = 0.0;
    for (long long e = lo + threadIdx.x; e < hi; e += NT) {
        x[e] += alpha * p[e];
        const double rn = r[e] - alpha * q[e];
        r[e] = rn;
        acc += rn * rn;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial_rr_new[(long long)s * g.ntiles + tile] = acc;
}

// p = z + beta p, beta = rho_new / rho; convergence on ||r||^2 <= rtol^2 ||b||^2
__global__ __launch_bounds__(NT) void k_cg_direction(Geom g, int S, const double* zws, double* pws,
                                                     const double* partial_rho, const double* partial_rho_new,
                                                     const double* partial_rr_new, const double* bb, double rtol2,
                                                     int maxit, const int* active, int* active_next, int* iters) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0) return;
    if (!active[s]) {
        if (tile == 0 && threadIdx.x == 0) active_next[s] = 0;
        return;
    }
    const double rho = slice_sum(partial_rho, s, g.ntiles);
    const double rhon = slice_sum(partial_rho_new, s, g.ntiles);
    const double beta = rhon / rho;
    const long long so = (long long)s * g.stride;
    const double* z = zws + so;
    double* p = pws + so;
    long long lo, hi;
    chunk_range(g, tile, lo, hi);
    for (long long e = lo + threadIdx.x; e < hi; e += NT) p[e] = z[e] + beta * p[e];
    if (tile == 0 && threadIdx.x == 0) {
        const double rrn = slice_sum(partial_rr_new, s, g.ntiles);
        const int it = iters[s] + 1;
        iters[s] = it;
        active_next[s] = (rrn > rtol2 * bb[s] && it < maxit) ? 1 : 0;
    }
}

// ---- fast-diagonalisation preconditioner: batched dense FP64 products ----
// LEFT:  Y[s] = A X[s]   (contraction over x), A given transposed: AT[k][i] = A[i][k]
// RIGHT: Y[s] = X[s] B   (contraction over y), B[k][j] row-major
// EPI 0: store; 1: scale by 1 / (1 + theta_s (lx[i] + ly[j])); 2: store and partial dot with r
constexpr int GAS = 80;                        // LDS stride of [k][i] tiles
constexpr int GBS = KC + 2;                    // LDS stride of [j][k] tiles
constexpr int FD_LDS = (2 * KC * GAS > EPI) ? 2 * KC * GAS : EPI;
template <bool LEFT, int EPI>
__global__ __launch_bounds__(NT) void k_fd_gemm(Geom g, int S, const double* __restrict__ mat,
                                                const double* __restrict__ xin, double* __restrict__ yout,
                                                const PropDesc* __restrict__ desc, const double* __restrict__ lx,
                                                const double* __restrict__ ly, const double* __restrict__ rws,
                                                double* partial, const int* active) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0) return;
    if (active && !active[s]) return;
    __shared__ double lds[FD_LDS];
    __shared__ double red[4];
    const int nx = g.nx, ny = g.ny;
    const int ti = tile % g.tiles_x, tj = tile / g.tiles_x;
    const int i0 = ti * T, j0 = tj * T;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int wi = wave & 1, wj = wave >> 1;
    const long long so = (long long)s * g.stride;
    const double* X = xin + so;
    const int K = LEFT ? nx : ny;
    double* At = lds;                 // [k][i], stride GAS
    double* Bt = lds + KC * GAS;      // LEFT: [j][k] stride GBS; RIGHT: [k][j] stride GAS

    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < K; k0 += KC) {
        for (int idx = tid; idx < KC * T; idx += NT) {
            const int kk = idx / T, ii = idx - kk * T;
            const int k = k0 + kk;
            if (LEFT) {
                const int i = i0 + ii;        // A[i][k] = AT[k][i]
                At[kk * GAS + ii] = (k < nx && i < nx) ? mat[(long long)k * nx + i] : 0.0;
            } else {
                const int i = i0 + ii;        // A = X[i][k] = X[i + nx k]
                At[kk * GAS + ii] = (k < ny && i < nx) ? X[(long long)k * nx + i] : 0.0;
            }
        }
        for (int idx = tid; idx < KC * T; idx += NT) {
            if (LEFT) {                       // B = X[k][j] = X[k + nx j] -> [j][k]
                const int jj = idx / KC, kk = idx - jj * KC;
                const int k = k0 + kk, j = j0 + jj;
                Bt[jj * GBS + kk] = (k < nx && j < ny) ? X[(long long)j * nx + k] : 0.0;
            } else {                          // B = mat[k][j] -> [k][j]
                const int kk = idx / T, jj = idx - kk * T;
                const int k = k0 + kk, j = j0 + jj;
                Bt[kk * GAS + jj] = (k < ny && j < ny) ? mat[(long long)k * ny + j] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int kk = ks + lk;
            double a[2], b[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                a[f] = At[kk * GAS + wi * 32 + f * 16 + lr];
                const int jl = wj * 32 + f * 16 + lr;
                b[f] = LEFT ? Bt[jl * GBS + kk] : Bt[kk * GAS + jl];
            }
#pragma unroll
            for (int fi = 0; fi < 2; ++fi)
#pragma unroll
                for (int fj = 0; fj < 2; ++fj)
                    acc[fi][fj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[fi], b[fj], acc[fi][fj], 0, 0, 0);
        }
        __syncthreads();
    }
    double* epi = lds;
#pragma unroll
    for (int fi = 0; fi < 2; ++fi)
#pragma unroll
        for (int fj = 0; fj < 2; ++fj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wi * 32 + fi * 16 + lk + 4 * r;
                const int jl = wj * 32 + fj * 16 + lr;
                epi[jl * (T + 1) + il] = acc[fi][fj][r];
            }
    __syncthreads();
    double* Y = yout + so;
    const double theta = EPI == 1 ? desc[s].theta_lhs : 0.0;
    double dot = 0.0;
    for (int idx = tid; idx < T * T; idx += NT) {
        const int jl = idx / T, il = idx - jl * T;
        const int i = i0 + il, j = j0 + jl;
        if (i >= nx || j >= ny) continue;
        const long long o = (long long)j * nx + i;
        double v = epi[jl * (T + 1) + il];
        if (EPI == 1) v /= 1.0 + theta * (lx[i] + ly[j]);
        Y[o] = v;
        if (EPI == 2) dot += v * rws[so + o];
    }
    if (EPI == 2) {
        dot = block_sum(dot, red);
        if (threadIdx.x == 0) partial[(long long)s * g.ntiles + tile] = dot;
    }
}

__global__ __launch_bounds__(NT) void k_add_g(Geom g, const PropDesc* __restrict__ desc, int S, double* xbase,
                                              const double* gbase) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0) return;
    const PropDesc d = desc[s];
    if (d.g < 0) return;
    double* x = xbase + d.x * g.stride;
    const double* gg = gbase + d.g * g.stride;
    long long lo, hi;
    chunk_range(g, tile, lo, hi);
    for (long long e = lo + threadIdx.x; e < hi; e += NT) x[e] += gg[e];
}

__global__ __launch_bounds__(NT) void k_axpy_slices(Geom g, int S, const int* yi, double* ybase, const int* xi,
                                                    const double* xbase, double a, double* partial) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0) return;
    __shared__ double red[4];
    double* y = ybase + yi[s] * g.stride;
    const double* x = xbase + xi[s] * g.stride;
    long long lo, hi;
    chunk_range(g, tile, lo, hi);
    double acc = 0.0;
    for (long long e = lo + threadIdx.x; e < hi; e += NT) {
        const double v = y[e] + a * x[e];
        y[e] = v;
        acc += v * v;
    }
    if (partial) {
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) partial[(long long)s * g.ntiles + tile] = acc;
    }
}

__global__ __launch_bounds__(NT) void k_zero_slices(Geom g, int S, const int* idx, double* base) {
    int s, tile;
    decode_block(g.ntiles, S, s, tile);
    if (s < 0) return;
    double* y = base + idx[s] * g.stride;
    long long lo, hi;
    chunk_range(g, tile, lo, hi);
    for (long long e = lo + threadIdx.x; e < hi; e += NT) y[e] = 0.0;
}

}  // namespace

extern "C" {

int launch_apply(const Geom* g, const Seqs* sq, const ApplyDesc* desc, int S, const double* vbase,
                 double* outbase, const double* addbase, double sign, int dot_mode, double* partial,
                 const int* active, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_apply, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, *sq, desc, S,
                       vbase, outbase, addbase, sign, dot_mode, partial, active);
    return (int)hipGetLastError();
}

int launch_rhs(const Geom* g, const Seqs* sq, const PropDesc* desc, int S, const double* ubase,
               const double* fbase, double* bws, double* partial_bb, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_prop_apply<0>, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, *sq,
                       desc, S, ubase, fbase, (const double*)nullptr, bws, partial_bb, (const int*)nullptr);
    return (int)hipGetLastError();
}

int launch_init_residual(const Geom* g, const Seqs* sq, const PropDesc* desc, int S, const double* ubase,
                         const double* bws, double* rws, double* partial_rr, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_prop_apply<1>, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, *sq,
                       desc, S, ubase, (const double*)nullptr, bws, rws, partial_rr, (const int*)nullptr);
    return (int)hipGetLastError();
}

int launch_cg_start(const Geom* g, const PropDesc* desc, int S, const double* ubase, double* xbase,
                    const double* zws, double* pws, const double* partial_bb, const double* partial_rr,
                    double rtol2, double* bb, int* active, int* iters, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_cg_start, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, desc, S,
                       ubase, xbase, zws, pws, partial_bb, partial_rr, rtol2, bb, active, iters);
    return (int)hipGetLastError();
}

int launch_cg_apply(const Geom* g, const Seqs* sq, const PropDesc* desc, int S, const double* pws, double* qws,
                    double* partial_pq, const int* active, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_prop_apply<2>, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, *sq,
                       desc, S, (const double*)nullptr, (const double*)nullptr, pws, qws, partial_pq, active);
    return (int)hipGetLastError();
}

int launch_cg_update(const Geom* g, const PropDesc* desc, int S, double* xbase, double* rws, const double* pws,
                     const double* qws, const double* partial_rho, const double* partial_pq,
                     double* partial_rr_new, const int* active, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_cg_update, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, desc, S,
                       xbase, rws, pws, qws, partial_rho, partial_pq, partial_rr_new, active);
    return (int)hipGetLastError();
}

int launch_cg_direction(const Geom* g, int S, const double* zws, double* pws, const double* partial_rho,
                        const double* partial_rho_new, const double* partial_rr_new, const double* bb, double rtol2,
                        int maxit, const int* active, int* active_next, int* iters, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_cg_direction, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, S, zws,
                       pws, partial_rho, partial_rho_new, partial_rr_new, bb, rtol2, maxit, active, active_next,
                       iters);
    return (int)hipGetLastError();
}

int launch_fd_apply(const Geom* g, const FdMats* fd, const PropDesc* desc, int S, const double* rws, double* zws,
                    double* t1, double* t2, double* partial_rz, const int* active, void* stream) {
    if (S <= 0) return 0;
    const dim3 grid(grid_blocks(g->ntiles, S)), blk(NT);
    hipStream_t st = (hipStream_t)stream;
    // t1 = Vx^T r ; t2 = (t1 Vy) / (1 + theta (lx + ly)) ; t1 = Vx t2 ; z = t1 Vy^T (+ r.z)
    hipLaunchKernelGGL((k_fd_gemm<true, 0>), grid, blk, 0, st, *g, S, fd->Vx, rws, t1, desc, fd->lx, fd->ly,
                       (const double*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fd_gemm<false, 1>), grid, blk, 0, st, *g, S, fd->Vy, (const double*)t1, t2, desc, fd->lx,
                       fd->ly, (const double*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fd_gemm<true, 0>), grid, blk, 0, st, *g, S, fd->VxT, (const double*)t2, t1, desc, fd->lx,
                       fd->ly, (const double*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fd_gemm<false, 2>), grid, blk, 0, st, *g, S, fd->VyT, (const double*)t1, zws, desc, fd->lx,
                       fd->ly, rws, partial_rz, active);
    return (int)hipGetLastError();
}

int launch_add_g(const Geom* g, const PropDesc* desc, int S, double* xbase, const double* gbase, void* stream) {
    if (S <= 0 || !gbase) return 0;
    hipLaunchKernelGGL(k_add_g, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, desc, S,
                       xbase, gbase);
    return (int)hipGetLastError();
}

int launch_axpy_slices(const Geom* g, int S, const int* yi, double* ybase, const int* xi, const double* xbase,
                       double a, double* partial, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_axpy_slices, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, S, yi,
                       ybase, xi, xbase, a, partial);
    return (int)hipGetLastError();
}

int launch_zero_slices(const Geom* g, int S, const int* idx, double* base, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_zero_slices, dim3(grid_blocks(g->ntiles, S)), dim3(NT), 0, (hipStream_t)stream, *g, S, idx,
                       base);
    return (int)hipGetLastError();
}

}  // extern "C"
