// HIP kernels for gfx950 (CDNA4): the batched operator application of the
// space-time finite-element scheme, the fast-diagonalisation preconditioner
// and the vector kernels of batched (P)CG.
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
// Toeplitz tile of TT x 32 entries holds only TT + 31 distinct values).  The
// 7-point mass stencil M_h, the scaling, the optional added vector and the
// per-tile dot product are applied in the epilogue, so one pass produces
//   out = add + sign (M_h v + theta A_h v).
//
// Work decomposition: one 256-thread workgroup per TT x TT output tile of one
// slice (TT = 64 for large batches, 32 for small ones, where the larger tile
// would leave most compute units idle); the workgroup -> (slice, tile) map keeps
// every tile of a slice on one XCD (workgroups are dealt to the 8 XCDs
// round-robin), so the strips of a slice are fetched from HBM into one L2 only.
//
// MFMA f64 16x16x4 lane layout (gfx950): A[i][k] in lane i + 16 k, B[k][j] in
// lane j + 16 k, accumulator element r of lane l holds D[l/16 + 4 r][l % 16].
#include <hip/hip_runtime.h>

#include "mgrit_internal.h"

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Matrix-core step of the operator tiles per element type: FP64
// v_mfma_f64_16x16x4f64, or FP32 v_mfma_f32_16x16x4f32 for the inner solves
// of mixed precision.  Both take A[i][k] in lane i + 16 k and B[k][j] in lane
// j + 16 k; accumulator element r of lane l holds D[row(l/16, r)][l % 16] with
// row = l/16 + 4 r (FP64) or 4 (l/16) + r (FP32).
template <typename T>
struct MF;
template <>
struct MF<double> {
    typedef dbl4 V;
    typedef Seqs S;
    static __device__ __forceinline__ V mma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct MF<float> {
    typedef flt4 V;
    typedef Seqs32 S;
    static __device__ __forceinline__ V mma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

constexpr int KC = MGRIT_KC;         // contraction chunk
constexpr int NT = 256;              // threads per workgroup
constexpr int CH = 4096;             // elements per chunk of the vector kernels

template <int TT>
struct TC {
    static constexpr int FR = TT / 32;                 // fragments per wave per dimension
    static constexpr int WR = 16 * FR;                 // edge of the region one wave computes
    static constexpr int HALO = TT + 2;                // tile plus one neighbour on each side
    static constexpr int SXS = KC + 2;                 // LDS stride of the x strip (per column)
    static constexpr int SYS = TT == 64 ? 80 : 48;     // LDS stride of the y strip (per k row)
    static constexpr int WIN = KC + TT;                // generating-sequence window per chunk
    static constexpr int XSTRIP = HALO * SXS;
    static constexpr int YSTRIP = KC * SYS;
    static constexpr int STRIP = XSTRIP > YSTRIP ? XSTRIP : YSTRIP;
    static constexpr int STAGE = STRIP + 3 * WIN;
    static constexpr int EPI = TT * (TT + 1);
    static constexpr int LDS = STAGE > EPI ? STAGE : EPI;
    // preconditioner products: A tile [k][i] and B tile ([j][k] or [k][j])
    static constexpr int GAS = SYS;
    static constexpr int GBS = KC + 2;
    static constexpr int FD_LDS = (2 * KC * GAS > EPI) ? 2 * KC * GAS : EPI;
};

// Block -> (slice, tile).  Workgroups are dealt to the 8 XCDs round-robin;
// with 8 or more slices every tile of a slice goes to one XCD (its L2 holds
// the slice and the halos its tiles share), the grid padded to a multiple of
// 8 slices.  Fewer than 8 slices are spread over all XCDs instead.
__device__ __forceinline__ void decode_block(int ntiles, int S, int& s, int& tile) {
    const int bid = blockIdx.x;
    if (S < 8) {
        s = bid / ntiles;
        tile = bid - s * ntiles;
        return;
    }
    const int xcd = bid & 7;
    const int local = bid >> 3;
    s = (local / ntiles) * 8 + xcd;
    tile = local % ntiles;
    if (s >= S) s = -1;
}

inline int grid_blocks(int ntiles, int S) { return S < 8 ? ntiles * S : ntiles * ((S + 7) / 8) * 8; }

// The tables of problem p of a batch of several problems (Geom strides; p = 0 for one problem).
template <typename S>
__device__ __forceinline__ S seqs_of(const S& sq, const Geom& g, int p) {
    S r = sq;
    const long long o = (long long)__builtin_amdgcn_readfirstlane(p) * g.ps_seq;
    r.T1x += o;
    r.A2x += o;
    r.T1y += o;
    r.A2y += o;
    return r;
}

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

// Sums of a slice's partials (entries i < count of row s) by the whole block in a fixed order: thread t adds
// entries t, t + NT, ... in turn, then the wave tree and waves 0..3, so every block and batch that reduces a
// slice gets the same value.  Every thread of the block must call these (no divergent call sites); all get
// the sums.  red holds 8 doubles.
__device__ __forceinline__ void slice_sums(const double* pa, int na, const double* pb, int nb, int pmax, int s,
                                           double* red, double& a, double& b) {
    const int t = threadIdx.x;
    pa += (long long)s * pmax;
    pb += (long long)s * pmax;
    double va = 0.0, vb = 0.0;
    for (int i = t; i < na; i += NT) va += pa[i];
    for (int i = t; i < nb; i += NT) vb += pb[i];
    va = wave_sum(va);
    vb = wave_sum(vb);
    const int w = t >> 6;
    __syncthreads();
    if ((t & 63) == 0) {
        red[w] = va;
        red[4 + w] = vb;
    }
    __syncthreads();
    a = (red[0] + red[1]) + (red[2] + red[3]);
    b = (red[4] + red[5]) + (red[6] + red[7]);
}

__device__ __forceinline__ double slice_sum(const double* partial, int count, int pmax, int s, double* red) {
    const double* p = partial + (long long)s * pmax;
    double v = 0.0;
    for (int i = threadIdx.x; i < count; i += NT) v += p[i];
    return block_sum(v, red);
}

// Epilogue of an operator tile: epi[jl][il] (ld TT + 1) holds A v on the tile; writes
// out = add + sign (M v + theta A v) and, with dot_mode, the dot products of its 32 x 32 quadrants to
// dot_out[32-tile index] (per quadrant with the same thread -> element order for both tile sizes, so the
// sums do not depend on TT).
template <int TT, typename T>
__device__ __forceinline__ void tile_epilogue(const Geom& g, const T* __restrict__ v, T* __restrict__ out,
                                              const T* __restrict__ add, T theta, T sign, int dot_mode, int i0,
                                              int j0, const T* epi, double* red, double* dot_out) {
    const int nx = g.nx, ny = g.ny;
    const int tid = threadIdx.x;
    const T mass = (T)g.mass;
#pragma unroll
    for (int qd = 0; qd < (TT / 32) * (TT / 32); ++qd) {
        const int qx = qd % (TT / 32), qy = qd / (TT / 32);
        double dot = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int idx = tid + NT * k;
            const int jl = qy * 32 + idx / 32, il = qx * 32 + (idx & 31);
            const int i = i0 + il, j = j0 + jl;
            if (i >= nx || j >= ny) continue;
            const long long o = (long long)j * nx + i;
            const T c = v[o];
            const bool hl = i > 0, hr = i + 1 < nx, hd = j > 0, hu = j + 1 < ny;
            T m7;
            if (g.q1) {                   // bilinear: (4, 1, 1) in y times (4, 1, 1) in x
                m7 = T(16) * c;
                m7 += T(4) * ((hl ? v[o - 1] : T(0)) + (hr ? v[o + 1] : T(0)) + (hd ? v[o - nx] : T(0)) +
                              (hu ? v[o + nx] : T(0)));
                m7 += (hr && hu) ? v[o + nx + 1] : T(0);
                m7 += (hl && hd) ? v[o - nx - 1] : T(0);
                m7 += (hl && hu) ? v[o + nx - 1] : T(0);
                m7 += (hr && hd) ? v[o - nx + 1] : T(0);
            } else {
                m7 = T(6) * c;
                m7 += hl ? v[o - 1] : T(0);
                m7 += hr ? v[o + 1] : T(0);
                m7 += hd ? v[o - nx] : T(0);
                m7 += hu ? v[o + nx] : T(0);
                m7 += (hr && hu) ? v[o + nx + 1] : T(0);
                m7 += (hl && hd) ? v[o - nx - 1] : T(0);
            }
            T val = sign * (mass * m7 + theta * epi[jl * (TT + 1) + il]);
            if (add) val += add[o];
            out[o] = val;
            if (dot_mode == 1) dot += (double)c * (double)val;
            else if (dot_mode == 2) dot += (double)val * (double)val;
        }
        if (dot_mode) {
            dot = block_sum(dot, red);
            const int gx = i0 / 32 + qx, gy = j0 / 32 + qy;
            if (threadIdx.x == 0 && gx < g.tiles_x[1] && gy < g.tiles_y[1])
                dot_out[gx + g.tiles_x[1] * gy] = dot;
        }
    }
}

// out = add + sign (M v + theta A v) on one TT x TT tile; with dot_mode the
// dot products of its 32 x 32 quadrants go to dot_out[32-tile index].
template <int TT, typename T>
__device__ void apply_tile(const Geom& g, const typename MF<T>::S& sq, const T* __restrict__ v, T* __restrict__ out,
                           const T* __restrict__ add, double theta_d, double sign_d, int dot_mode, int tile, T* lds,
                           double* red, double* dot_out) {
    typedef typename MF<T>::V V;
    const T theta = (T)theta_d, sign = (T)sign_d;
    typedef TC<TT> C;
    constexpr int FR = C::FR;
    const int nx = g.nx, ny = g.ny;
    const int tv = TT == 64 ? 0 : 1;
    const int ti = tile % g.tiles_x[tv], tj = tile / g.tiles_x[tv];
    const int i0 = ti * TT, j0 = tj * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int wi = wave & 1, wj = wave >> 1;

    V acc[FR][FR];
#pragma unroll
    for (int a = 0; a < FR; ++a)
#pragma unroll
        for (int b = 0; b < FR; ++b) acc[a][b] = V{0, 0, 0, 0};

    T* strip = lds;
    T* w0 = lds + C::STRIP;
    T* w1 = w0 + C::WIN;
    T* w2 = w1 + C::WIN;

    // ---- x-direction: contraction over x with the A_x factors ----
    for (int k0 = 0; k0 < nx; k0 += KC) {
        for (int idx = tid; idx < C::HALO * KC; idx += NT) {
            const int jj = idx / KC, kk = idx - jj * KC;
            const int k = k0 + kk, j = j0 - 1 + jj;
            strip[jj * C::SXS + kk] = (k < nx && j >= 0 && j < ny) ? v[(long long)j * nx + k] : T(0);
        }
        const int dbase = k0 - i0 - (TT - 1);
        for (int q = tid; q < C::WIN; q += NT) {
            const int d = dbase + q;
            w0[q] = sq.T1x[g.seq_off_x + d];
            w1[q] = sq.A2x[g.seq_off_x + d];
            w2[q] = sq.A2x[g.seq_off_x - d];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int kk = ks + lk;
            T a0[FR], a1[FR], a2[FR], b0[FR], b1[FR], b2[FR];
#pragma unroll
            for (int f = 0; f < FR; ++f) {
                const int il = wi * C::WR + f * 16 + lr;
                const int q = kk - il + (TT - 1);
                a0[f] = w0[q];
                a1[f] = w1[q];
                a2[f] = w2[q];
                const int jl = wj * C::WR + f * 16 + lr;
                b0[f] = strip[(jl + 1) * C::SXS + kk];   // column j
                b1[f] = strip[(jl + 2) * C::SXS + kk];   // column j+1
                b2[f] = strip[jl * C::SXS + kk];         // column j-1
            }
#pragma unroll
            for (int fi = 0; fi < FR; ++fi)
#pragma unroll
                for (int fj = 0; fj < FR; ++fj) {
                    acc[fi][fj] = MF<T>::mma(a0[fi], b0[fj], acc[fi][fj]);
                    acc[fi][fj] = MF<T>::mma(a1[fi], b1[fj], acc[fi][fj]);
                    acc[fi][fj] = MF<T>::mma(a2[fi], b2[fj], acc[fi][fj]);
                }
        }
        __syncthreads();
    }

    // ---- y-direction: contraction over y with the A_y factors ----
    for (int k0 = 0; k0 < ny; k0 += KC) {
        for (int idx = tid; idx < KC * C::HALO; idx += NT) {
            const int kk = idx / C::HALO, ii = idx - kk * C::HALO;
            const int k = k0 + kk, i = i0 - 1 + ii;
            strip[kk * C::SYS + ii] = (k < ny && i >= 0 && i < nx) ? v[(long long)k * nx + i] : T(0);
        }
        const int ebase = j0 - k0 - (KC - 1);
        for (int q = tid; q < C::WIN; q += NT) {
            const int e = ebase + q;
            w0[q] = sq.T1y[g.seq_off_y + e];
            w1[q] = sq.A2y[g.seq_off_y - e];   // A2y[k - j]: factor of row i+1
            w2[q] = sq.A2y[g.seq_off_y + e];   // A2y[j - k]: factor of row i-1
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int kk = ks + lk;
            T a0[FR], a1[FR], a2[FR], b0[FR], b1[FR], b2[FR];
#pragma unroll
            for (int f = 0; f < FR; ++f) {
                const int il = wi * C::WR + f * 16 + lr;
                a0[f] = strip[kk * C::SYS + il + 1];     // row i
                a1[f] = strip[kk * C::SYS + il + 2];     // row i+1
                a2[f] = strip[kk * C::SYS + il];         // row i-1
                const int jl = wj * C::WR + f * 16 + lr;
                const int q = jl - kk + (KC - 1);
                b0[f] = w0[q];
                b1[f] = w1[q];
                b2[f] = w2[q];
            }
#pragma unroll
            for (int fi = 0; fi < FR; ++fi)
#pragma unroll
                for (int fj = 0; fj < FR; ++fj) {
                    acc[fi][fj] = MF<T>::mma(a0[fi], b0[fj], acc[fi][fj]);
                    acc[fi][fj] = MF<T>::mma(a1[fi], b1[fj], acc[fi][fj]);
                    acc[fi][fj] = MF<T>::mma(a2[fi], b2[fj], acc[fi][fj]);
                }
        }
        __syncthreads();
    }

    // ---- epilogue: stage A v through LDS, add the mass stencil ----
    T* epi = lds;
#pragma unroll
    for (int fi = 0; fi < FR; ++fi)
#pragma unroll
        for (int fj = 0; fj < FR; ++fj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wi * C::WR + fi * 16 + MF<T>::row(lk, r);
                const int jl = wj * C::WR + fj * 16 + lr;
                epi[jl * (TT + 1) + il] = acc[fi][fj][r];
            }
    __syncthreads();
    tile_epilogue<TT, T>(g, v, out, add, theta, sign, dot_mode, i0, j0, epi, red, dot_out);
}

// ---- operator application over slices given by ApplyDesc ----
template <int TT>
__global__ __launch_bounds__(NT) void k_apply(Geom g, Seqs sq, const ApplyDesc* __restrict__ desc, int S,
                                              const double* vbase, double* outbase, const double* addbase,
                                              double sign, int dot_mode, double* partial, const int* active) {
    const int tv = TT == 64 ? 0 : 1;
    int s, tile;
    decode_block(g.ntiles[tv], S, s, tile);
    if (s < 0) return;
    if (active && !active[s]) return;
    __shared__ double lds[TC<TT>::LDS];
    __shared__ double red[4];
    const ApplyDesc d = desc[s];
    const double* addp = (addbase && d.add >= 0) ? addbase + d.add * g.stride : nullptr;
    apply_tile<TT, double>(g, sq, vbase + d.v * g.stride, outbase + d.out * g.stride, addp, d.theta, sign, dot_mode, tile,
                   lds, red, dot_mode ? partial + (long long)s * g.pmax : nullptr);
}

// mode 0: right-hand side b = M u + theta_rhs A u (+F), partial ||b||^2
// mode 1: initial residual r = b - (M x + theta_lhs A x), partial ||r||^2 (ubase = x base; slices with
//         active[s] = 0 keep their r and partials when a mask is given)
// mode 2: q = M p + theta_lhs A p (active slices), partial p.q
template <int TT, int MODE>
__global__ __launch_bounds__(NT) void k_prop_apply(Geom g, Seqs sq0, const PropDesc* __restrict__ desc, int S,
                                                   const double* ubase, const double* fbase, const double* wsin,
                                                   double* wsout, double* partial, const int* active) {
    const int tv = TT == 64 ? 0 : 1;
    int s, tile;
    decode_block(g.ntiles[tv], S, s, tile);
    if (s < 0) return;
    if ((MODE == 1 || MODE == 2) && active && !active[s]) return;
    __shared__ double lds[TC<TT>::LDS];
    __shared__ double red[4];
    const PropDesc d = desc[s];
    const long long so = (long long)s * g.stride;
    double* part = partial + (long long)s * g.pmax;
    const Seqs sq = seqs_of(sq0, g, d.prob);
    if (MODE == 0) {
        const double* f = (fbase && d.f >= 0) ? fbase + d.f * g.stride : nullptr;
        apply_tile<TT, double>(g, sq, ubase + d.u * g.stride, wsout + so, f, d.theta_rhs, 1.0, 2, tile, lds, red, part);
    } else if (MODE == 1) {
        apply_tile<TT, double>(g, sq, ubase + d.x * g.stride, wsout + so, wsin + so, d.theta_lhs, -1.0, 2, tile, lds, red,
                       part);
    } else {
        apply_tile<TT, double>(g, sq, wsin + so, wsout + so, nullptr, d.theta_lhs, 1.0, 1, tile, lds, red, part);
    }
}

// Element range of chunk c of a flattened slice.
__device__ __forceinline__ void chunk_range(const Geom& g, int c, long long& lo, long long& hi) {
    lo = (long long)c * CH;
    hi = lo + CH;
    if (hi > g.stride) hi = g.stride;
}

// Elements per thread in a chunk.  The kernels below load all of a thread's
// elements (indices clamped into the chunk, so every load is in bounds) before
// they store any result: at small batches a chunk loop that waits for each
// element's loads in turn is bound by memory latency.  Positions k = 0, 1, ...
// of a thread are its elements lo + tid + k NT in the order a plain strided
// loop visits them, so sums over them keep that order.
constexpr int PT = CH / NT;
static_assert(CH % NT == 0, "chunk must be a multiple of the workgroup");

// ---- mixed precision: FP32 inner solves of an iterative refinement ----
// The outer loop keeps b, x and r = b - B x in FP64; each step solves
// B d = r / ||r|| by PCG in FP32 (operator on the FP32 matrix cores, vectors
// in FP32, every reduction accumulated in FP64) and sets x += ||r|| d.

// q32 = M p32 + theta_lhs A p32 on active slices, partial p.q.
template <int TT>
__global__ __launch_bounds__(NT) void k_apply32(Geom g, Seqs32 sq, const PropDesc* __restrict__ desc, int S,
                                                const float* pws, float* qws, double* partial, const int* active) {
    const int tv = TT == 64 ? 0 : 1;
    int s, tile;
    decode_block(g.ntiles[tv], S, s, tile);
    if (s < 0) return;
    if (active && !active[s]) return;
    __shared__ float lds[TC<TT>::LDS];
    __shared__ double red[4];
    const long long so = (long long)s * g.stride;
    const PropDesc d = desc[s];
    apply_tile<TT, float>(g, seqs_of(sq, g, d.prob), pws + so, qws + so, nullptr, d.theta_lhs, 1.0, 1, tile, lds,
                          red, partial + (long long)s * g.pmax);
}

// q32 = M p32 + theta_lhs A p32 with the Toeplitz products in BF16 on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Each FP32 operand x is split as
// x_hi = bf16(x), x_lo = bf16(x - x_hi), so |x - x_hi - x_lo| <= 2^-18 |x|, and every product
// a v is taken as a_hi v_hi + a_hi v_lo + a_lo v_hi: three BF16 products whose sum misses
// a v by at most 3 2^-18 |a| |v|.  64 x 64 output tiles as in apply_tile (same wave grid, same
// epilogue and partial sums); per 32-deep chunk of the contraction the workgroup stages the
// split strip of p (with its one-line halo) and the three split 64 x 32 Toeplitz tiles of one
// direction in LDS, rows 16-byte aligned, so every operand of the MFMA is one 16-byte read.
// MFMA 16x16x32 bf16 lane layout: A[i][k] and B^T[j][k] hold k = 8 (lane/16) + e, e = 0..7, of
// row i = lane % 16 (resp. column j); accumulator element r of lane l is D[4 (l/16) + r][l % 16].
namespace obf {
constexpr int TT = 64;
constexpr int KCH = 32;                       // contraction chunk: one MFMA depth
constexpr int LD = KCH + 8;                   // LDS row stride in BF16 elements (80 bytes)
constexpr int HALO = TT + 2;
constexpr int WIN = KCH + TT;                 // generating-sequence window per chunk
constexpr int STRIP = HALO * LD;              // one split part of the strip
constexpr int TILE = TT * LD;                 // one split part of one Toeplitz tile
constexpr int BYTES = (2 * STRIP + 6 * TILE) * 2 + 3 * WIN * 4;
constexpr int EPI_BYTES = TT * (TT + 1) * 4;
static_assert(EPI_BYTES <= BYTES, "epilogue staging must fit the operand staging");
}  // namespace obf

__device__ __forceinline__ unsigned int split_pair(float x0, float x1, unsigned int& lo) {
    const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
    const __bf16 l0 = (__bf16)(x0 - (float)h0), l1 = (__bf16)(x1 - (float)h1);
    lo = (unsigned int)__builtin_bit_cast(unsigned short, l0) |
         ((unsigned int)__builtin_bit_cast(unsigned short, l1) << 16);
    return (unsigned int)__builtin_bit_cast(unsigned short, h0) |
           ((unsigned int)__builtin_bit_cast(unsigned short, h1) << 16);
}

__global__ __launch_bounds__(NT) void k_apply_bf16(Geom g, Seqs32 sq0, const PropDesc* __restrict__ desc, int S,
                                                   const float* pws, float* qws, double* partial,
                                                   const int* active) {
    using namespace obf;
    int s, tile;
    decode_block(g.ntiles[0], S, s, tile);
    if (s < 0) return;
    if (active && !active[s]) return;
    const Seqs32 sq = seqs_of(sq0, g, desc[s].prob);
    __shared__ __attribute__((aligned(16))) unsigned char raw[BYTES];
    __shared__ double red[4];
    __bf16* Shi = (__bf16*)raw;                      // strip [row][k]
    __bf16* Slo = Shi + STRIP;
    __bf16* Thi = Slo + STRIP;                       // three Toeplitz tiles [row][k]
    __bf16* Tlo = Thi + 3 * TILE;
    float* w = (float*)(Tlo + 3 * TILE);             // three windows of WIN values
    const long long so = (long long)s * g.stride;
    const float* v = pws + so;
    const int nx = g.nx, ny = g.ny;
    const int ti = tile % g.tiles_x[0], tj = tile / g.tiles_x[0];
    const int i0 = ti * TT, j0 = tj * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int wi = wave & 1, wj = wave >> 1;

    flt4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};

    // Toeplitz tiles of one chunk: T_t[r][kk] = w_t[q(r, kk)], stored as split pairs along kk
    auto build_tiles = [&](bool xdir) {
        for (int idx = tid; idx < 3 * TT * (KCH / 2); idx += NT) {
            const int t = idx / (TT * (KCH / 2));
            const int rem = idx - t * (TT * (KCH / 2));
            const int r = rem / (KCH / 2), kk = 2 * (rem - r * (KCH / 2));
            // x: A[i][k] = w[k - i + TT - 1];  y: B^T[j][k] = w[j - k + KCH - 1]
            const int q0 = xdir ? kk - r + TT - 1 : r - kk + KCH - 1;
            const int q1 = xdir ? q0 + 1 : q0 - 1;
            unsigned int lo;
            const unsigned int hi = split_pair(w[t * WIN + q0], w[t * WIN + q1], lo);
            *(unsigned int*)&Thi[t * TILE + r * LD + kk] = hi;
            *(unsigned int*)&Tlo[t * TILE + r * LD + kk] = lo;
        }
    };
    // one chunk of products: acc += T_t (x: A operand) or strip rows (y: A operand) against the other
    auto multiply = [&](bool xdir) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            // strip row offset of factor t: x: columns j, j+1, j-1; y: rows i, i+1, i-1
            const int sh = t == 0 ? 1 : (t == 1 ? 2 : 0);
            bf8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const int il = wi * 32 + f * 16 + lr, jl = wj * 32 + f * 16 + lr;
                if (xdir) {
                    ah[f] = *(const bf8*)&Thi[t * TILE + il * LD + 8 * lg];
                    al[f] = *(const bf8*)&Tlo[t * TILE + il * LD + 8 * lg];
                    bh[f] = *(const bf8*)&Shi[(jl + sh) * LD + 8 * lg];
                    bl[f] = *(const bf8*)&Slo[(jl + sh) * LD + 8 * lg];
                } else {
                    ah[f] = *(const bf8*)&Shi[(il + sh) * LD + 8 * lg];
                    al[f] = *(const bf8*)&Slo[(il + sh) * LD + 8 * lg];
                    bh[f] = *(const bf8*)&Thi[t * TILE + jl * LD + 8 * lg];
                    bl[f] = *(const bf8*)&Tlo[t * TILE + jl * LD + 8 * lg];
                }
            }
#pragma unroll
            for (int fi = 0; fi < 2; ++fi)
#pragma unroll
                for (int fj = 0; fj < 2; ++fj) {
                    acc[fi][fj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[fi], bh[fj], acc[fi][fj], 0, 0, 0);
                    acc[fi][fj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[fi], bl[fj], acc[fi][fj], 0, 0, 0);
                    acc[fi][fj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[fi], bh[fj], acc[fi][fj], 0, 0, 0);
                }
        }
    };

    // ---- x-direction: X[i][j] = sum_k A1(k-i) v[j][k] + A2(k-i) v[j+1][k] + A2(i-k) v[j-1][k] ----
    for (int k0 = 0; k0 < nx; k0 += KCH) {
        for (int idx = tid; idx < HALO * (KCH / 2); idx += NT) {
            const int jj = idx / (KCH / 2), kk = 2 * (idx - jj * (KCH / 2));
            const int k = k0 + kk, j = j0 - 1 + jj;
            const bool row = j >= 0 && j < ny;
            const float x0 = (row && k < nx) ? v[(long long)j * nx + k] : 0.f;
            const float x1 = (row && k + 1 < nx) ? v[(long long)j * nx + k + 1] : 0.f;
            unsigned int lo;
            *(unsigned int*)&Shi[jj * LD + kk] = split_pair(x0, x1, lo);
            *(unsigned int*)&Slo[jj * LD + kk] = lo;
        }
        const int dbase = k0 - i0 - (TT - 1);
        for (int q = tid; q < WIN; q += NT) {
            const int d = dbase + q;
            w[q] = sq.T1x[g.seq_off_x + d];
            w[WIN + q] = sq.A2x[g.seq_off_x + d];
            w[2 * WIN + q] = sq.A2x[g.seq_off_x - d];
        }
        __syncthreads();
        build_tiles(true);
        __syncthreads();
        multiply(true);
        __syncthreads();
    }

    // ---- y-direction: Y[i][j] = sum_k v[k][i] A1(j-k) + v[k][i+1] A2(k-j) + v[k][i-1] A2(j-k) ----
    for (int k0 = 0; k0 < ny; k0 += KCH) {
        for (int idx = tid; idx < KCH * HALO; idx += NT) {
            const int kk = idx / HALO, ii = idx - kk * HALO;
            const int k = k0 + kk, i = i0 - 1 + ii;
            const float x = (k < ny && i >= 0 && i < nx) ? v[(long long)k * nx + i] : 0.f;
            const __bf16 hi = (__bf16)x;
            Shi[ii * LD + kk] = hi;
            Slo[ii * LD + kk] = (__bf16)(x - (float)hi);
        }
        const int ebase = j0 - k0 - (KCH - 1);
        for (int q = tid; q < WIN; q += NT) {
            const int e = ebase + q;
            w[q] = sq.T1y[g.seq_off_y + e];
            w[WIN + q] = sq.A2y[g.seq_off_y - e];
            w[2 * WIN + q] = sq.A2y[g.seq_off_y + e];
        }
        __syncthreads();
        build_tiles(false);
        __syncthreads();
        multiply(false);
        __syncthreads();
    }

    float* epi = (float*)raw;
#pragma unroll
    for (int fi = 0; fi < 2; ++fi)
#pragma unroll
        for (int fj = 0; fj < 2; ++fj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wi * 32 + fi * 16 + 4 * lg + r;
                const int jl = wj * 32 + fj * 16 + lr;
                epi[jl * (TT + 1) + il] = acc[fi][fj][r];
            }
    __syncthreads();
    tile_epilogue<TT, float>(g, v, qws + so, (const float*)nullptr, (float)desc[s].theta_lhs, 1.0f, 1, i0, j0, epi,
                             red, partial + (long long)s * g.pmax);
}

// The BF16 image of r32 that the first preconditioner product reads: slice s at s npx npy, row j at j npx
// (the zero-padded layout of the products' operands; the padding is zeroed once).  Element e = j n_x + k of
// the slice goes to row j, column k (j from a float quotient, corrected to the exact one).
__device__ __forceinline__ void put_rimg(const Geom& g, __bf16* __restrict__ rimg, long long sob, long long e,
                                         float v) {
    const int nx = g.nx;
    int j = (int)((float)e * (1.0f / (float)nx));
    int k = (int)e - j * nx;
    if (k < 0) {
        --j;
        k += nx;
    } else if (k >= nx) {
        ++j;
        k -= nx;
    }
    rimg[sob + (long long)j * (g.tiles_x[0] * 64) + k] = (__bf16)v;
}

// Start of a refinement step from the FP64 residual (np partials of ||b||^2
// and ||r||^2 per slice): outer flag ||r|| > rtol ||b||, scale ||r||, inner
// tolerance eta^2 = max(rtol^2 ||b||^2 / ||r||^2, eta_min^2), r32 = r / ||r||,
// d32 = 0 and, when p32 is given (no preconditioner), p32 = r32 with partial
// r32.r32.  On the first step x = 0 where b = 0 and the counts restart.  The
// inner flag is 2 instead of 1 when eta^2 >= 100 eta_min2.  RT = float: the
// residual was formed in FP32 in r32 itself (rws == r32), scaled in place.
template <typename RT>
__global__ __launch_bounds__(NT) void k_mx_begin(Geom g, const PropDesc* __restrict__ desc, int S, double* xbase,
                                                 const RT* rws, const double* partial_bb,
                                                 const double* partial_rr, int np, double rtol2, double eta_min2,
                                                 int first, double* bb, double* scale, double* eta2, int* oact,
                                                 int* iact, int* iters, float* r32, float* d32, float* p32,
                                                 double* partial_rr32, int* host_act, int* host_iters,
                                                 const int* trust_in, int* trust_out, __bf16* rimg) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    __shared__ double red[8];
    double b2, r2;
    slice_sums(partial_bb, np, partial_rr, np, g.pmax, s, red, b2, r2);
    const bool zero = !(b2 > 0.0);
    // a slice whose previous step was settled by its own inner test is done, whatever the other slices of
    // the batch need (so that each slice's result does not depend on the batch)
    const bool settled = !first && trust_in[s];
    const bool active = !settled && !zero && r2 > rtol2 * b2;
    const long long sob = (long long)s * (g.tiles_x[0] * 64) * (g.tiles_y[0] * 64);
    const long long so = (long long)s * g.stride;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    if (first && zero) {
        double* x = xbase + desc[s].x * g.stride;
        for (long long e = lo + threadIdx.x; e < hi; e += NT) x[e] = 0.0;
    }
    if (active) {
        const double inv = 1.0 / sqrt(r2);
        const RT* r = rws + so;
        double acc = 0.0;
        for (long long e = lo + threadIdx.x; e < hi; e += NT) {
            const float rv = (float)((double)r[e] * inv);
            r32[so + e] = rv;
            d32[so + e] = 0.0f;
            if (p32) p32[so + e] = rv;
            if (rimg) put_rimg(g, rimg, sob, e, rv);
            acc += (double)rv * (double)rv;
        }
        if (p32) {
            acc = block_sum(acc, red);
            if (threadIdx.x == 0) partial_rr32[(long long)s * g.pmax + c] = acc;
        }
    }
    if (c == 0 && threadIdx.x == 0) {
        bb[s] = b2;
        oact[s] = active ? 1 : 0;
        const double e2 = active ? fmax(rtol2 * b2 / r2, eta_min2) : 0.0;
        // 2: the inner target is the pass tolerance itself and at least 10 x the FP32 floor, so the
        // inner solve's own test settles the slice (see the refinement loop)
        const int flag = active ? (e2 >= 1e2 * eta_min2 ? 2 : 1) : 0;
        iact[s] = flag;
        trust_out[s] = (settled || flag == 2) ? 1 : 0;
        if (host_act) host_act[s] = flag;
        scale[s] = active ? sqrt(r2) : 0.0;
        eta2[s] = e2;
        if (first) {
            iters[s] = 0;
            if (host_iters) host_iters[s] = 0;
        }
    }
}

// 16-byte groups of chunk [lo, hi) of an FP32 workspace slice: with base = the chunk's first element in
// the array, the elements before the first 16-byte boundary (head) and after the last one (tail) are done
// one by one, the rest as float4 groups (GPT per thread: group tid + NT j).  The launchers require every
// array to start on a 16-byte boundary, so one split holds for all of a kernel's vectors.
constexpr int GPT = CH / (NT * 4);
static_assert(CH % (NT * 4) == 0, "chunk must hold whole float4 groups per thread");

struct Split16 {
    int head, ngr, tail0, len;
};

__device__ __forceinline__ Split16 split16(long long base, int len) {
    Split16 sp;
    sp.len = len;
    sp.head = (int)((4 - (base & 3)) & 3);
    if (sp.head > len) sp.head = len;
    sp.ngr = (len - sp.head) >> 2;
    sp.tail0 = sp.head + 4 * sp.ngr;
    return sp;
}

// alpha = rho / p.q; d32 += alpha p32, r32 -= alpha q32 on active slices; partial r32.r32 per chunk.
__global__ __launch_bounds__(NT) void k_mx_update(Geom g, int S, float* __restrict__ d32, float* __restrict__ r32,
                                                  const float* __restrict__ p32, const float* __restrict__ q32,
                                                  const double* partial_rho, int nrho, const double* partial_pq,
                                                  int npq, double* partial_rr_new, const int* active,
                                                  __bf16* __restrict__ rimg) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0 || !active[s]) return;
    __shared__ double red[8];
    const long long so = (long long)s * g.stride;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    const long long base = so + lo;
    const long long sob = (long long)s * (g.tiles_x[0] * 64) * (g.tiles_y[0] * 64);
    const Split16 sp = split16(base, (int)(hi - lo));
    const int tid = threadIdx.x;
    float4* D = (float4*)(d32 + base + sp.head);
    float4* R = (float4*)(r32 + base + sp.head);
    const float4* P = (const float4*)(p32 + base + sp.head);
    const float4* Q = (const float4*)(q32 + base + sp.head);
    float4 dv[GPT], rv[GPT], pv[GPT], qv[GPT];
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
        const int k = tid + NT * j;
        if (k < sp.ngr) {
            dv[j] = D[k];
            rv[j] = R[k];
            pv[j] = P[k];
            qv[j] = Q[k];
        }
    }
    // the one-by-one elements: thread t < head takes element t, thread t < len - tail0 element tail0 + t
    const bool hh = tid < sp.head, ht = tid < sp.len - sp.tail0;
    const long long eh = base + tid, et = base + sp.tail0 + tid;
    float dh = 0.f, rh = 0.f, ph = 0.f, qh = 0.f, dt = 0.f, rt = 0.f, pt = 0.f, qt = 0.f;
    if (hh) {
        dh = d32[eh];
        rh = r32[eh];
        ph = p32[eh];
        qh = q32[eh];
    }
    if (ht) {
        dt = d32[et];
        rt = r32[et];
        pt = p32[et];
        qt = q32[et];
    }
    double rho, pq;
    slice_sums(partial_rho, nrho, partial_pq, npq, g.pmax, s, red, rho, pq);
    const float alpha = (float)(rho / pq);
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
        const int k = tid + NT * j;
        if (k < sp.ngr) {
            float4 rn;
            rn.x = rv[j].x - alpha * qv[j].x;
            rn.y = rv[j].y - alpha * qv[j].y;
            rn.z = rv[j].z - alpha * qv[j].z;
            rn.w = rv[j].w - alpha * qv[j].w;
            float4 dn;
            dn.x = dv[j].x + alpha * pv[j].x;
            dn.y = dv[j].y + alpha * pv[j].y;
            dn.z = dv[j].z + alpha * pv[j].z;
            dn.w = dv[j].w + alpha * pv[j].w;
            D[k] = dn;
            R[k] = rn;
            if (rimg) {
                const long long e = lo + sp.head + 4LL * k;
                put_rimg(g, rimg, sob, e, rn.x);
                put_rimg(g, rimg, sob, e + 1, rn.y);
                put_rimg(g, rimg, sob, e + 2, rn.z);
                put_rimg(g, rimg, sob, e + 3, rn.w);
            }
            acc += (double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y + (double)rn.z * (double)rn.z +
                   (double)rn.w * (double)rn.w;
        }
    }
    if (hh) {
        const float rn = rh - alpha * qh;
        d32[eh] = dh + alpha * ph;
        r32[eh] = rn;
        if (rimg) put_rimg(g, rimg, sob, lo + tid, rn);
        acc += (double)rn * (double)rn;
    }
    if (ht) {
        const float rn = rt - alpha * qt;
        d32[et] = dt + alpha * pt;
        r32[et] = rn;
        if (rimg) put_rimg(g, rimg, sob, lo + sp.tail0 + tid, rn);
        acc += (double)rn * (double)rn;
    }
    acc = block_sum(acc, red);
    if (tid == 0) partial_rr_new[(long long)s * g.pmax + c] = acc;
}

// p32 = z32 + (rho_new / rho) p32 on active slices; next flags from ||r32||^2 <= eta2[s] and the count.
__global__ __launch_bounds__(NT) void k_mx_direction(Geom g, int S, const float* __restrict__ z32,
                                                     float* __restrict__ p32,
                                                     const double* partial_rho, int nrho,
                                                     const double* partial_rho_new, int nrho_new,
                                                     const double* partial_rr_new, const double* eta2, int maxit,
                                                     const int* active, int* active_next, int* iters,
                                                     int* host_next, int* host_iters) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    if (!active[s]) {
        if (c == 0 && threadIdx.x == 0) {
            active_next[s] = 0;
            if (host_next) host_next[s] = 0;
        }
        return;
    }
    __shared__ double red[8];
    const long long so = (long long)s * g.stride;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    const long long base = so + lo;
    const Split16 sp = split16(base, (int)(hi - lo));
    const int tid = threadIdx.x;
    const float4* Z = (const float4*)(z32 + base + sp.head);
    float4* P = (float4*)(p32 + base + sp.head);
    float4 zv[GPT], pv[GPT];
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
        const int k = tid + NT * j;
        if (k < sp.ngr) {
            zv[j] = Z[k];
            pv[j] = P[k];
        }
    }
    const bool hh = tid < sp.head, ht = tid < sp.len - sp.tail0;
    const long long eh = base + tid, et = base + sp.tail0 + tid;
    float zh = 0.f, ph = 0.f, zt = 0.f, pt = 0.f;
    if (hh) {
        zh = z32[eh];
        ph = p32[eh];
    }
    if (ht) {
        zt = z32[et];
        pt = p32[et];
    }
    double rhon, rho;
    slice_sums(partial_rho_new, nrho_new, partial_rho, nrho, g.pmax, s, red, rhon, rho);
    const float beta = (float)(rhon / rho);
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
        const int k = tid + NT * j;
        if (k < sp.ngr) {
            float4 pn;
            pn.x = zv[j].x + beta * pv[j].x;
            pn.y = zv[j].y + beta * pv[j].y;
            pn.z = zv[j].z + beta * pv[j].z;
            pn.w = zv[j].w + beta * pv[j].w;
            P[k] = pn;
        }
    }
    if (hh) p32[eh] = zh + beta * ph;
    if (ht) p32[et] = zt + beta * pt;
    if (c != 0) return;
    const double rrn = slice_sum(partial_rr_new, g.nchunk, g.pmax, s, red);
    if (tid == 0) {
        const int it = iters[s] + 1;
        iters[s] = it;
        if (host_iters) host_iters[s] = it;
        const int flag = (rrn > eta2[s] && it < maxit) ? 1 : 0;
        active_next[s] = flag;
        if (host_next) host_next[s] = flag;
    }
}

// x += ||r|| d32 on slices whose refinement step ran.
// need[s] = slices whose new iterate gets an FP64 check: active in this step and not settled by their own
// inner test (trust[s]); the others keep their residual (unchanged x, or not read again).
__global__ __launch_bounds__(NT) void k_mx_refine(Geom g, const PropDesc* __restrict__ desc, int S, double* xbase,
                                                  const float* d32, const double* scale, const int* oact,
                                                  const int* trust, int* need) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    if (c == 0 && threadIdx.x == 0) need[s] = (oact[s] && !trust[s]) ? 1 : 0;
    if (!oact[s]) return;
    double* x = xbase + desc[s].x * g.stride;
    const float* d = d32 + (long long)s * g.stride;
    const double a = scale[s];
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    const long long e0 = lo + threadIdx.x, last = hi - 1;
    double xv[PT];
    float dv[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const long long e = e0 + (long long)k * NT < last ? e0 + (long long)k * NT : last;
        xv[k] = x[e];
        dv[k] = d[e];
    }
#pragma unroll
    for (int k = 0; k < PT; ++k)
        if (e0 + (long long)k * NT <= last) x[e0 + (long long)k * NT] = xv[k] + a * (double)dv[k];
}

__global__ __launch_bounds__(NT) void k_cg_init_x(Geom g, const PropDesc* __restrict__ desc, int S,
                                                  const double* ubase, const double* x0base, int warm,
                                                  double* xbase) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    const PropDesc d = desc[s];
    const double* src = (warm && d.x0 >= 0) ? x0base + d.x0 * g.stride : ubase + d.u * g.stride;
    double* x = xbase + d.x * g.stride;
    if (src == x) return;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    for (long long e = lo + threadIdx.x; e < hi; e += NT) x[e] = src[e];
}


__global__ __launch_bounds__(NT) void k_cg_start(Geom g, const PropDesc* __restrict__ desc, int S,
                                                 double* xbase, const double* zws, double* pws,
                                                 const double* partial_bb, int nbb, const double* partial_rr, int nrr,
                                                 double rtol2, double* bb, int* active, int* iters,
                                                 int* host_act, int* host_iters) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    const PropDesc d = desc[s];
    __shared__ double red[8];
    double b2, r2;
    slice_sums(partial_bb, nbb, partial_rr, nrr, g.pmax, s, red, b2, r2);
    double* x = xbase + d.x * g.stride;
    const double* z = zws + (long long)s * g.stride;
    double* p = pws + (long long)s * g.stride;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    const bool zero = !(b2 > 0.0);
    for (long long e = lo + threadIdx.x; e < hi; e += NT) {
        if (zero) x[e] = 0.0;
        p[e] = z[e];
    }
    if (c == 0 && threadIdx.x == 0) {
        bb[s] = b2;
        const int flag = (!zero && r2 > rtol2 * b2) ? 1 : 0;
        active[s] = flag;
        if (host_act) host_act[s] = flag;
        iters[s] = 0;
        if (host_iters) host_iters[s] = 0;
    }
}

// alpha = rho / (p.q) with rho = r.z (z = r without preconditioner)
__global__ __launch_bounds__(NT) void k_cg_update(Geom g, const PropDesc* __restrict__ desc, int S, double* xbase,
                                                  double* rws, const double* pws, const double* qws,
                                                  const double* partial_rho, int nrho, const double* partial_pq,
                                                  int npq, double* partial_rr_new, const int* active) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0 || !active[s]) return;
    __shared__ double red[8];
    double rho, pq;
    slice_sums(partial_rho, nrho, partial_pq, npq, g.pmax, s, red, rho, pq);
    const double alpha = rho / pq;
    double* __restrict__ x = xbase + desc[s].x * g.stride;
    const long long so = (long long)s * g.stride;
    double* __restrict__ r = rws + so;
    const double* __restrict__ p = pws + so;
    const double* __restrict__ q = qws + so;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    const long long e0 = lo + threadIdx.x, last = hi - 1;
    double acc = 0.0;
#pragma unroll
    for (int k0 = 0; k0 < PT; k0 += PT / 2) {                     // two halves: 64 FP64 values in flight
        double xv[PT / 2], rv[PT / 2], pv[PT / 2], qv[PT / 2];
#pragma unroll
        for (int k = 0; k < PT / 2; ++k) {
            const long long e1 = e0 + (long long)(k0 + k) * NT, e = e1 < last ? e1 : last;
            xv[k] = x[e];
            rv[k] = r[e];
            pv[k] = p[e];
            qv[k] = q[e];
        }
#pragma unroll
        for (int k = 0; k < PT / 2; ++k) {
            const long long e = e0 + (long long)(k0 + k) * NT;
            const double rn = rv[k] - alpha * qv[k];
            if (e <= last) {
                x[e] = xv[k] + alpha * pv[k];
                r[e] = rn;
                acc += rn * rn;
            }
        }
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial_rr_new[(long long)s * g.pmax + c] = acc;
}

// p = z + beta p, beta = rho_new / rho; convergence on ||r||^2 <= rtol^2 ||b||^2
__global__ __launch_bounds__(NT) void k_cg_direction(Geom g, int S, const double* zws, double* pws,
                                                     const double* partial_rho, int nrho,
                                                     const double* partial_rho_new, int nrho_new,
                                                     const double* partial_rr_new, const double* bb, double rtol2,
                                                     int maxit, const int* active, int* active_next, int* iters,
                                                     int* host_next, int* host_iters) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    if (!active[s]) {
        if (c == 0 && threadIdx.x == 0) {
            active_next[s] = 0;
            if (host_next) host_next[s] = 0;
        }
        return;
    }
    __shared__ double red[8];
    const long long so = (long long)s * g.stride;
    const double* __restrict__ z = zws + so;
    double* __restrict__ p = pws + so;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    const long long e0 = lo + threadIdx.x, last = hi - 1;
    double zv[PT], pv[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const long long e = e0 + (long long)k * NT < last ? e0 + (long long)k * NT : last;
        zv[k] = z[e];
        pv[k] = p[e];
    }
    double rho, rhon;
    slice_sums(partial_rho, nrho, partial_rho_new, nrho_new, g.pmax, s, red, rho, rhon);
    const double beta = rhon / rho;
#pragma unroll
    for (int k = 0; k < PT; ++k)
        if (e0 + (long long)k * NT <= last) p[e0 + (long long)k * NT] = zv[k] + beta * pv[k];
    if (c != 0) return;
    const double rrn = slice_sum(partial_rr_new, g.nchunk, g.pmax, s, red);
    if (threadIdx.x == 0) {
        const int it = iters[s] + 1;
        iters[s] = it;
        if (host_iters) host_iters[s] = it;
        const int flag = (rrn > rtol2 * bb[s] && it < maxit) ? 1 : 0;
        active_next[s] = flag;
        if (host_next) host_next[s] = flag;
    }
}

// ---- fast-diagonalisation preconditioner: batched dense FP64 products ----
// LEFT:  Y[s] = A X[s]   (contraction over x), A given transposed: AT[k][i] = A[i][k]
// RIGHT: Y[s] = X[s] B   (contraction over y), B[k][j] row-major
// EPI 0: store; 1: scale by 1 / (1 + theta_s (lx[i] + ly[j])); 2: store and partial dot with r
template <int TT, bool LEFT, int EPI>
__global__ __launch_bounds__(NT) void k_fd_gemm(Geom g, int S, const double* __restrict__ mat,
                                                const double* __restrict__ xin, double* __restrict__ yout,
                                                const PropDesc* __restrict__ desc, const double* __restrict__ lx,
                                                const double* __restrict__ ly, const double* __restrict__ rws,
                                                double* partial, const int* active) {
    typedef TC<TT> C;
    constexpr int FR = C::FR;
    const int tv = TT == 64 ? 0 : 1;
    int s, tile;
    decode_block(g.ntiles[tv], S, s, tile);
    if (s < 0) return;
    if (active && !active[s]) return;
    {
        const long long o = (long long)__builtin_amdgcn_readfirstlane(desc[s].prob) * g.ps_fd;
        mat += o;
        lx += o;
        ly += o;
    }
    __shared__ double lds[C::FD_LDS];
    __shared__ double red[4];
    const int nx = g.nx, ny = g.ny;
    const int ti = tile % g.tiles_x[tv], tj = tile / g.tiles_x[tv];
    const int i0 = ti * TT, j0 = tj * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int wi = wave & 1, wj = wave >> 1;
    const long long so = (long long)s * g.stride;
    const double* X = xin + so;
    const int K = LEFT ? nx : ny;
    double* At = lds;                     // [k][i], stride GAS
    double* Bt = lds + KC * C::GAS;       // LEFT: [j][k] stride GBS; RIGHT: [k][j] stride GAS

    dbl4 acc[FR][FR];
#pragma unroll
    for (int a = 0; a < FR; ++a)
#pragma unroll
        for (int b = 0; b < FR; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < K; k0 += KC) {
        for (int idx = tid; idx < KC * TT; idx += NT) {
            const int kk = idx / TT, ii = idx - kk * TT;
            const int k = k0 + kk, i = i0 + ii;
            if (LEFT) At[kk * C::GAS + ii] = (k < nx && i < nx) ? mat[(long long)k * nx + i] : 0.0;
            else At[kk * C::GAS + ii] = (k < ny && i < nx) ? X[(long long)k * nx + i] : 0.0;
        }
        for (int idx = tid; idx < KC * TT; idx += NT) {
            if (LEFT) {                       // B = X[k][j] = X[k + nx j] -> [j][k]
                const int jj = idx / KC, kk = idx - jj * KC;
                const int k = k0 + kk, j = j0 + jj;
                Bt[jj * C::GBS + kk] = (k < nx && j < ny) ? X[(long long)j * nx + k] : 0.0;
            } else {                          // B = mat[k][j] -> [k][j]
                const int kk = idx / TT, jj = idx - kk * TT;
                const int k = k0 + kk, j = j0 + jj;
                Bt[kk * C::GAS + jj] = (k < ny && j < ny) ? mat[(long long)k * ny + j] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int kk = ks + lk;
            double a[FR], b[FR];
#pragma unroll
            for (int f = 0; f < FR; ++f) {
                a[f] = At[kk * C::GAS + wi * C::WR + f * 16 + lr];
                const int jl = wj * C::WR + f * 16 + lr;
                b[f] = LEFT ? Bt[jl * C::GBS + kk] : Bt[kk * C::GAS + jl];
            }
#pragma unroll
            for (int fi = 0; fi < FR; ++fi)
#pragma unroll
                for (int fj = 0; fj < FR; ++fj)
                    acc[fi][fj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[fi], b[fj], acc[fi][fj], 0, 0, 0);
        }
        __syncthreads();
    }
    double* epi = lds;
#pragma unroll
    for (int fi = 0; fi < FR; ++fi)
#pragma unroll
        for (int fj = 0; fj < FR; ++fj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wi * C::WR + fi * 16 + lk + 4 * r;
                const int jl = wj * C::WR + fj * 16 + lr;
                epi[jl * (TT + 1) + il] = acc[fi][fj][r];
            }
    __syncthreads();
    double* Y = yout + so;
    const double theta = EPI == 1 ? desc[s].theta_lhs : 0.0;
#pragma unroll
    for (int qd = 0; qd < (TT / 32) * (TT / 32); ++qd) {     // per 32 x 32 quadrant, as in apply_tile
        const int qx = qd % (TT / 32), qy = qd / (TT / 32);
        double dot = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int idx = tid + NT * k;
            const int jl = qy * 32 + idx / 32, il = qx * 32 + (idx & 31);
            const int i = i0 + il, j = j0 + jl;
            if (i >= nx || j >= ny) continue;
            const long long o = (long long)j * nx + i;
            double v = epi[jl * (TT + 1) + il];
            if (EPI == 1) v /= 1.0 + theta * (lx[i] + ly[j]);
            Y[o] = v;
            if (EPI == 2) dot += v * rws[so + o];
        }
        if (EPI == 2) {
            dot = block_sum(dot, red);
            const int gx = i0 / 32 + qx, gy = j0 / 32 + qy;
            if (threadIdx.x == 0 && gx < g.tiles_x[1] && gy < g.tiles_y[1])
                partial[(long long)s * g.pmax + gx + g.tiles_x[1] * gy] = dot;
        }
    }
}

// ---- fast-diagonalisation preconditioner in BF16 (FP32 accumulation) ----
// v_mfma_f32_16x16x32_bf16 lane layout (gfx950): A[i][k] and B^T[j][k] hold 8
// consecutive k (k = 8 (lane/16) + e) of row i = lane % 16 (resp. column j);
// accumulator element r of lane l holds D[4 (l/16) + r][l % 16].
// Operands are zero-padded to npx x npy (multiples of 64) so the products need
// no bounds checks except on the FP64 input r and the FP64 output z.
// LEFT:  Y[s] = A X[s], A[i][k] row-major (ld npx)        RIGHT: Y[s] = X[s] B, B^T[j][k] row-major (ld npy),
//        X given transposed (X^T[i][k], ld npy)
// IN 0: X = r [ny][nx] (RT = FP64, or FP32 in the inner solves of mixed precision);  IN 1: X = BF16 padded
// EPI 0: Y BF16 padded, transposed ([i][j], ld npy); 1: scaled by 1 / (1 + theta (lx + ly)), BF16 padded
//        ([j][i], ld npx); 2: Y = z [ny][nx] (RT) + r.z,
//        also copied to ycopy when given
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));
constexpr int BK = 64;            // k-chunk of the BF16 products
constexpr int BLD = BK + 8;       // LDS row stride in BF16 elements ([row][k] tiles)

union Pack8 {
    uint4 u;
    __bf16 h[8];
};

// The BF16 intermediates between the products are stored transposed ([i][j],
// y fastest) after a product over x, so that the next product, over y, reads
// its operand rows directly instead of transposing them through LDS.
// The last product gets a register budget of 8 workgroups per compute unit (64 registers), so that
// 128 slices of 16 tiles are resident at once (the others would spill at that budget).
template <bool LEFT, int IN, int EPI, typename RT>
__global__ __launch_bounds__(NT, EPI == 2 ? 8 : 1) void k_fdb_gemm(Geom g, int S, const __bf16* __restrict__ mat,
                                                 const void* __restrict__ xin, void* __restrict__ yout,
                                                 const PropDesc* __restrict__ desc, const float* __restrict__ lx,
                                                 const float* __restrict__ ly, const RT* __restrict__ rws,
                                                 RT* __restrict__ ycopy, double* partial, const int* active) {
    int s, tile;
    decode_block(g.ntiles[0], S, s, tile);
    if (s < 0) return;
    if (active && !active[s]) return;
    {
        const int pr = __builtin_amdgcn_readfirstlane(desc[s].prob);     // uniform: scalar offsets
        mat += (long long)pr * g.ps_fdb;
        lx += (long long)pr * g.ps_fde;
        ly += (long long)pr * g.ps_fde;
    }
    __shared__ __attribute__((aligned(16))) unsigned char raw[2 * 64 * BLD * 2 > 64 * 65 * 4 ? 2 * 64 * BLD * 2
                                                                                              : 64 * 65 * 4];
    __shared__ double red[4];
    __bf16* As = (__bf16*)raw;                 // [i][k]
    __bf16* Bs = As + 64 * BLD;                // [j][k]
    const int nx = g.nx, ny = g.ny;
    const int npx = g.tiles_x[0] * 64, npy = g.tiles_y[0] * 64;
    const int ti = tile % g.tiles_x[0], tj = tile / g.tiles_x[0];
    const int i0 = ti * 64, j0 = tj * 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int wi = wave & 1, wj = wave >> 1;
    const long long sob = (long long)s * npx * npy;          // BF16 padded slice offset
    const long long so = (long long)s * g.stride;            // slice offset of r and z
    const int K = LEFT ? npx : npy;

    flt4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};

    // Operands of chunk k0 + BK are loaded into registers while chunk k0 is multiplied
    // (each thread: two 16-byte pieces of the A tile; two of the B tile, or 16 values of r).
    const __bf16* Xb = (const __bf16*)xin + sob;
    uint4 ra0, ra1, rb0, rb1;
    float rr[LEFT && IN == 0 ? 16 : 1];
#define FDB_LOAD(K0)                                                                                          \
    {                                                                                                       \
        const int r0 = tid >> 3, r1 = (tid + NT) >> 3, kv = tid & 7;                                        \
        ra0 = LEFT ? *(const uint4*)&mat[(long long)(i0 + r0) * npx + (K0) + 8 * kv]                        \
                   : *(const uint4*)&Xb[(long long)(i0 + r0) * npy + (K0) + 8 * kv];                        \
        ra1 = LEFT ? *(const uint4*)&mat[(long long)(i0 + r1) * npx + (K0) + 8 * kv]                        \
                   : *(const uint4*)&Xb[(long long)(i0 + r1) * npy + (K0) + 8 * kv];                        \
        if (!(LEFT && IN == 0)) {                                                                           \
            rb0 = LEFT ? *(const uint4*)&Xb[(long long)(j0 + r0) * npx + (K0) + 8 * kv]                     \
                       : *(const uint4*)&mat[(long long)(j0 + r0) * npy + (K0) + 8 * kv];                   \
            rb1 = LEFT ? *(const uint4*)&Xb[(long long)(j0 + r1) * npx + (K0) + 8 * kv]                     \
                       : *(const uint4*)&mat[(long long)(j0 + r1) * npy + (K0) + 8 * kv];                   \
        } else {                                                                                            \
            const RT* X = rws + so;                                                                         \
            _Pragma("unroll") for (int q = 0; q < (LEFT && IN == 0 ? 16 : 1); ++q) {                        \
                const int idx = tid + NT * q, jj = idx >> 6, kk = idx & 63;                                 \
                const int k = (K0) + kk, j = j0 + jj;                                                       \
                rr[q] = (k < nx && j < ny) ? (float)X[(long long)j * nx + k] : 0.0f;                        \
            }                                                                                               \
        }                                                                                                   \
    }
    FDB_LOAD(0)
    for (int k0 = 0; k0 < K; k0 += BK) {
        {
            const int r0 = tid >> 3, r1 = (tid + NT) >> 3, kv = tid & 7;
            *(uint4*)&As[r0 * BLD + 8 * kv] = ra0;
            *(uint4*)&As[r1 * BLD + 8 * kv] = ra1;
            if (!(LEFT && IN == 0)) {
                *(uint4*)&Bs[r0 * BLD + 8 * kv] = rb0;
                *(uint4*)&Bs[r1 * BLD + 8 * kv] = rb1;
            } else {
#pragma unroll
                for (int q = 0; q < (LEFT && IN == 0 ? 16 : 1); ++q) {
                    const int idx = tid + NT * q, jj = idx >> 6, kk = idx & 63;
                    Bs[jj * BLD + kk] = (__bf16)rr[q];
                }
            }
        }
        __syncthreads();
        if (k0 + BK < K) FDB_LOAD(k0 + BK)
#pragma unroll
        for (int ks = 0; ks < BK; ks += 32) {
            bf8 a[2], b[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                a[f] = *(const bf8*)&As[(wi * 32 + f * 16 + lr) * BLD + ks + 8 * lg];
                b[f] = *(const bf8*)&Bs[(wj * 32 + f * 16 + lr) * BLD + ks + 8 * lg];
            }
#pragma unroll
            for (int fi = 0; fi < 2; ++fi)
#pragma unroll
                for (int fj = 0; fj < 2; ++fj)
                    acc[fi][fj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fi], b[fj], acc[fi][fj], 0, 0, 0);
        }
        __syncthreads();
    }
#undef FDB_LOAD
    float* epi = (float*)raw;
#pragma unroll
    for (int fi = 0; fi < 2; ++fi)
#pragma unroll
        for (int fj = 0; fj < 2; ++fj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wi * 32 + fi * 16 + 4 * lg + r;
                const int jl = wj * 32 + fj * 16 + lr;
                epi[jl * 65 + il] = acc[fi][fj][r];
            }
    __syncthreads();
    if (EPI == 0) {                                           // transposed BF16 output [i][j], y fastest
        for (int idx = tid; idx < 64 * 64; idx += NT) {
            const int il = idx >> 6, jl = idx & 63;
            ((__bf16*)yout)[sob + (long long)(i0 + il) * npy + j0 + jl] = (__bf16)epi[jl * 65 + il];
        }
        return;
    }
    // the scale 1 / (1 + theta (lx + ly)) (lx, ly >= 0) in FP32 by the hardware reciprocal: its error
    // is far below the BF16 rounding of the product it scales
    const float theta = EPI == 1 ? (float)desc[s].theta_lhs : 0.0f;
    double dot[4] = {0.0, 0.0, 0.0, 0.0};                     // per 32 x 32 quadrant, as in apply_tile
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
        const int qx = qd & 1, qy = qd >> 1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int idx = tid + NT * k;
            const int jl = qy * 32 + idx / 32, il = qx * 32 + (idx & 31);
            const int i = i0 + il, j = j0 + jl;
            float v = epi[jl * 65 + il];
            if (EPI == 1) v *= __builtin_amdgcn_rcpf(1.0f + theta * (lx[i] + ly[j]));
            if (EPI == 2) {
                if (i < nx && j < ny) {
                    const long long o = (long long)j * nx + i;
                    ((RT*)yout)[so + o] = (RT)v;
                    if (ycopy) ycopy[so + o] = (RT)v;
                    dot[qd] += (double)v * (double)rws[so + o];
                }
            } else {
                ((__bf16*)yout)[sob + (long long)j * npx + i] = (__bf16)v;
            }
        }
    }
    if (EPI == 2) {
        // the four quadrant sums reduced together: wave sums, then waves 0..3 in the order of block_sum
        __shared__ double red4[4][4];
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) dot[qd] = wave_sum(dot[qd]);
        if ((tid & 63) == 0) {
#pragma unroll
            for (int qd = 0; qd < 4; ++qd) red4[tid >> 6][qd] = dot[qd];
        }
        __syncthreads();
        if (tid < 4) {
            const int qd = tid, gx = i0 / 32 + (qd & 1), gy = j0 / 32 + (qd >> 1);
            if (gx < g.tiles_x[1] && gy < g.tiles_y[1])
                partial[(long long)s * g.pmax + gx + g.tiles_x[1] * gy] =
                    (red4[0][qd] + red4[1][qd]) + (red4[2][qd] + red4[3][qd]);
        }
    }
}

// The same products for small batches (npx, npy <= 256): 32 x 32 output tiles covering the padded
// extent, all of K loaded at once, the contraction split over the four waves (k-chunks of 32 dealt
// round-robin) and summed through LDS in wave order; epilogues as in k_fdb_gemm, with one r.z partial per
// 32 x 32 tile at the index k_fdb_gemm gives that quadrant.
constexpr int SLD = 256 + 8;        // LDS row stride (BF16) of the [row][k] tiles

template <bool LEFT, int IN, int EPI, typename RT>
__global__ __launch_bounds__(NT) void k_fdb_gemm32(Geom g, int S, const __bf16* __restrict__ mat,
                                                   const void* __restrict__ xin, void* __restrict__ yout,
                                                   const PropDesc* __restrict__ desc, const float* __restrict__ lx,
                                                   const float* __restrict__ ly, const RT* __restrict__ rws,
                                                   RT* __restrict__ ycopy, double* partial, const int* active) {
    const int npx = g.tiles_x[0] * 64, npy = g.tiles_y[0] * 64;
    const int tx = npx / 32, ty = npy / 32;
    int s, tile;
    decode_block(tx * ty, S, s, tile);
    if (s < 0) return;
    if (active && !active[s]) return;
    {
        const int pr = __builtin_amdgcn_readfirstlane(desc[s].prob);     // uniform: scalar offsets
        mat += (long long)pr * g.ps_fdb;
        lx += (long long)pr * g.ps_fde;
        ly += (long long)pr * g.ps_fde;
    }
    __shared__ __attribute__((aligned(16))) unsigned char raw[2 * 32 * SLD * 2 > 4 * 32 * 33 * 4 ? 2 * 32 * SLD * 2
                                                                                                 : 4 * 32 * 33 * 4];
    __shared__ double red[4];
    __bf16* As = (__bf16*)raw;                 // [i][k]
    __bf16* Bs = As + 32 * SLD;                // [j][k]
    const int nx = g.nx, ny = g.ny;
    const int i0 = (tile % tx) * 32, j0 = (tile / tx) * 32;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const long long sob = (long long)s * npx * npy;
    const long long so = (long long)s * g.stride;
    const int K = LEFT ? npx : npy;
    const int kv8 = K >> 3;
    const __bf16* Xb = (const __bf16*)xin + sob;
    for (int idx = tid; idx < 32 * kv8; idx += NT) {             // A rows i, B rows j (16-byte pieces)
        const int row = idx / kv8, kv = idx - row * kv8;
        *(uint4*)&As[row * SLD + 8 * kv] = LEFT ? *(const uint4*)&mat[(long long)(i0 + row) * npx + 8 * kv]
                                                : *(const uint4*)&Xb[(long long)(i0 + row) * npy + 8 * kv];
        if (!(LEFT && IN == 0))
            *(uint4*)&Bs[row * SLD + 8 * kv] = LEFT ? *(const uint4*)&Xb[(long long)(j0 + row) * npx + 8 * kv]
                                                    : *(const uint4*)&mat[(long long)(j0 + row) * npy + 8 * kv];
    }
    if (LEFT && IN == 0) {                                         // rows j0 + wave + 4q of r, lanes along k
        const RT* X = rws + so;
        for (int k = lane; k < K; k += 64) {
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + wave + 4 * q;
                v[q] = (k < nx && j < ny) ? (float)X[(long long)j * nx + k] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) Bs[(wave + 4 * q) * SLD + k] = (__bf16)v[q];
        }
    }
    __syncthreads();
    flt4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 32 * wave; ks < K; ks += 128) {                // this wave's k-chunks: wave, wave + 4, ...
        bf8 a[2], b[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            a[f] = *(const bf8*)&As[(f * 16 + lr) * SLD + ks + 8 * lg];
            b[f] = *(const bf8*)&Bs[(f * 16 + lr) * SLD + ks + 8 * lg];
        }
#pragma unroll
        for (int fi = 0; fi < 2; ++fi)
#pragma unroll
            for (int fj = 0; fj < 2; ++fj)
                acc[fi][fj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fi], b[fj], acc[fi][fj], 0, 0, 0);
    }
    __syncthreads();
    float* part = (float*)raw;                                     // [wave][j][i], stride 33
#pragma unroll
    for (int fi = 0; fi < 2; ++fi)
#pragma unroll
        for (int fj = 0; fj < 2; ++fj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                part[wave * 32 * 33 + (fj * 16 + lr) * 33 + fi * 16 + 4 * lg + r] = acc[fi][fj][r];
    __syncthreads();
    // the scale 1 / (1 + theta (lx + ly)) (lx, ly >= 0) in FP32 by the hardware reciprocal: its error
    // is far below the BF16 rounding of the product it scales
    const float theta = EPI == 1 ? (float)desc[s].theta_lhs : 0.0f;
    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int idx = tid + NT * k;
        const int jl = idx >> 5, il = idx & 31;
        const int i = i0 + il, j = j0 + jl;
        const int o32 = jl * 33 + il;
        float v = ((part[o32] + part[32 * 33 + o32]) + part[2 * 32 * 33 + o32]) + part[3 * 32 * 33 + o32];
        if (EPI == 0) {
            ((__bf16*)yout)[sob + (long long)i * npy + j] = (__bf16)v;      // transposed, as in k_fdb_gemm
        } else if (EPI == 1) {
            v *= __builtin_amdgcn_rcpf(1.0f + theta * (lx[i] + ly[j]));
            ((__bf16*)yout)[sob + (long long)j * npx + i] = (__bf16)v;
        } else if (i < nx && j < ny) {
            const long long o = (long long)j * nx + i;
            ((RT*)yout)[so + o] = (RT)v;
            if (ycopy) ycopy[so + o] = (RT)v;
            dot += (double)v * (double)rws[so + o];
        }
    }
    if (EPI == 2) {
        dot = block_sum(dot, red);
        const int gx = i0 / 32, gy = j0 / 32;
        if (tid == 0 && gx < g.tiles_x[1] && gy < g.tiles_y[1]) partial[(long long)s * g.pmax + gx + g.tiles_x[1] * gy] = dot;
    }
}

__global__ __launch_bounds__(NT) void k_fill_apply_desc(int S, const double* __restrict__ theta, int has_add,
                                                      ApplyDesc* __restrict__ desc) {
    const int s = blockIdx.x * NT + threadIdx.x;
    if (s >= S) return;
    ApplyDesc d;
    d.v = s;
    d.out = s;
    d.add = has_add ? s : -1;
    d.pad_ = 0;
    d.theta = theta[s];
    desc[s] = d;
}

__global__ __launch_bounds__(NT) void k_add_g(Geom g, const PropDesc* __restrict__ desc, int S, double* xbase,
                                              const double* gbase) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    const PropDesc d = desc[s];
    if (d.g < 0) return;
    double* x = xbase + d.x * g.stride;
    const double* gg = gbase + d.g * g.stride;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    for (long long e = lo + threadIdx.x; e < hi; e += NT) x[e] += gg[e];
}

__global__ __launch_bounds__(NT) void k_axpy_slices(Geom g, int S, const int* yi, double* ybase, const int* xi,
                                                    const double* xbase, double a, double* partial) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    __shared__ double red[4];
    double* y = ybase + yi[s] * g.stride;
    const double* x = xbase + xi[s] * g.stride;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    double acc = 0.0;
    for (long long e = lo + threadIdx.x; e < hi; e += NT) {
        const double v = y[e] + a * x[e];
        y[e] = v;
        acc += v * v;
    }
    if (partial) {
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) partial[(long long)s * g.pmax + c] = acc;
    }
}

__global__ __launch_bounds__(NT) void k_zero_slices(Geom g, int S, const int* idx, double* base) {
    int s, c;
    decode_block(g.nchunk, S, s, c);
    if (s < 0) return;
    double* y = base + idx[s] * g.stride;
    long long lo, hi;
    chunk_range(g, c, lo, hi);
    for (long long e = lo + threadIdx.x; e < hi; e += NT) y[e] = 0.0;
}

// ---- the operator by FFT: Toeplitz products as circulant convolutions ----
// A Toeplitz product along a grid line is a linear convolution with a kernel
// of 2n - 1 taps; embedded in a circulant of length FL >= 2n - 1 it becomes a
// product of spectra.  The pass over x (line j = the n_x nodes of row j) forms
//   X_j = c1 * v_j + c2 * v_{j+1} + c3 * v_{j-1}
// with c1, c2, c3 the kernels of A_1, A_2 and A_2^T; the pass over y does the
// same along columns with the y kernels.  Two real lines travel as one
// complex transform (real and imaginary part), and two output lines are
// packed the same way for the inverse transform.  Transforms are Stockham
// FFTs of L = 512 points (three radix-8 passes) or 1024 points (radix 16, 8,
// 8), one wavefront per transform, L / 64 points per lane.  The slice's theta scales the kernel
// spectra of the x pass, where the 7-point mass stencil enters as three more (3-tap) kernels, so
// the x pass writes M v + theta X to a workspace; the y pass adds theta Y (theta applied to its
// output) and applies the rest of the epilogue (sign, added vector, dot-product partial) as the
// tiled kernels do.
constexpr int FJ = 14;               // output lines per workgroup
constexpr int FNT = 512;             // threads per workgroup: 8 waves, one input pair each
template <int L>
struct FftLen {
    static constexpr int NP = L / 64;                     // points per lane
    static constexpr int PAD = L + L / (L == 1024 ? 16 : 8);   // padded LDS length of one transform
    static constexpr int FE = (L / 2 * FJ + FNT - 1) / FNT;   // epilogue elements per thread (n <= L / 2)
};

template <typename T>
struct cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
    return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
    return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cmi(cpx<T> a) {   // a * (-i)
    return {a.y, -a.x};
}
// LDS index of entry k of a transform: one pad entry per 8 (512 points) or 16 (1024 points) entries, so that
// the first pass's stores (lane l writes entries 8 l + r, resp. 16 l + r) hit distinct banks in every group of
// 16 lanes (strides of 9 and 17 entries), and runs of consecutive entries stay conflict-free.
template <int L>
__device__ __forceinline__ int fpidx(int k) { return L == 1024 ? k + (k >> 4) : k + (k >> 3); }

// Forward DFT of 8 points in registers (two radix-2 splittings in frequency).
template <typename T>
__device__ __forceinline__ void dft8(cpx<T>* a) {
    const T h = (T)0.70710678118654752440;
    const cpx<T> b0 = cadd(a[0], a[4]), b1 = cadd(a[1], a[5]), b2 = cadd(a[2], a[6]), b3 = cadd(a[3], a[7]);
    const cpx<T> b4 = csub(a[0], a[4]), d5 = csub(a[1], a[5]), d6 = csub(a[2], a[6]), d7 = csub(a[3], a[7]);
    const cpx<T> b5 = {h * (d5.x + d5.y), h * (d5.y - d5.x)};     // * exp(-i pi / 4)
    const cpx<T> b6 = cmi(d6);                                    // * exp(-i pi / 2)
    const cpx<T> b7 = {h * (d7.y - d7.x), -h * (d7.x + d7.y)};    // * exp(-3 i pi / 4)
    const cpx<T> c0 = cadd(b0, b2), c2 = csub(b0, b2), c1 = cadd(b1, b3), c3 = cmi(csub(b1, b3));
    const cpx<T> c4 = cadd(b4, b6), c6 = csub(b4, b6), c5 = cadd(b5, b7), c7 = cmi(csub(b5, b7));
    a[0] = cadd(c0, c1);
    a[4] = csub(c0, c1);
    a[2] = cadd(c2, c3);
    a[6] = csub(c2, c3);
    a[1] = cadd(c4, c5);
    a[5] = csub(c4, c5);
    a[3] = cadd(c6, c7);
    a[7] = csub(c6, c7);
}

// a[r] *= w^r, r = 1..7
template <typename T>
__device__ __forceinline__ void twiddle8(cpx<T>* a, cpx<T> w) {
    cpx<T> wr = w;
#pragma unroll
    for (int r = 1; r < 8; ++r) {
        a[r] = cmul(a[r], wr);
        if (r < 7) wr = cmul(wr, w);
    }
}

// Forward FFT of FL points with a[r] = x[lane + 64 r] on entry and
// a[r] = X[lane + 64 r] on return; buf is this wave's FPAD-entry LDS region
// (only this wave touches it), tw[k] = exp(-2 pi i k / FL).
template <typename T>
__device__ __forceinline__ void fft512(cpx<T>* a, cpx<T>* buf, const cpx<T>* __restrict__ tw, int lane) {
    dft8(a);                                              // sub-transforms of length 1 -> 8
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[fpidx<512>(8 * lane + r)] = a[r];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = buf[fpidx<512>(lane + 64 * r)];
    twiddle8(a, tw[(lane & 7) * 8]);                      // 8 -> 64
    dft8(a);
    const int d1 = (lane >> 3) * 64 + (lane & 7);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[fpidx<512>(d1 + 8 * r)] = a[r];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = buf[fpidx<512>(lane + 64 * r)];
    twiddle8(a, tw[lane]);                                // 64 -> 512
    dft8(a);
    __builtin_amdgcn_wave_barrier();
}

// Forward DFT of 16 points: a[n] +- a[n + 8] (the odd half times exp(-2 pi i n / 16)),
// then two DFTs of 8; even outputs from the first, odd from the second.
template <typename T>
__device__ __forceinline__ void dft16(cpx<T>* a) {
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, h = (T)0.70710678118654752440;
    const cpx<T> w[8] = {{T(1), T(0)}, {c1, -s1}, {h, -h}, {s1, -c1}, {T(0), T(-1)}, {-s1, -c1}, {-h, -h}, {-c1, -s1}};
    cpx<T> b[8], c[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        b[n] = cadd(a[n], a[n + 8]);
        c[n] = cmul(csub(a[n], a[n + 8]), w[n]);
    }
    dft8(b);
    dft8(c);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[2 * k] = b[k];
        a[2 * k + 1] = c[k];
    }
}

// Forward FFT of 1024 points, a[m] = x[lane + 64 m] on entry and X[lane + 64 m] on return
// (m < 16): a radix-16 pass, then two radix-8 passes of two butterflies per lane
// (butterflies j = lane and lane + 64).
template <typename T>
__device__ __forceinline__ void fft1024(cpx<T>* a, cpx<T>* buf, const cpx<T>* __restrict__ tw, int lane) {
    dft16(a);                                             // length 1 -> 16
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[fpidx<1024>(16 * lane + r)] = a[r];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int half = 0; half < 2; ++half) {                // 16 -> 128
        const int j = lane + 64 * half;
        cpx<T>* v = a + 8 * half;
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = buf[fpidx<1024>(j + 128 * r)];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int j = lane + 64 * half;
        cpx<T>* v = a + 8 * half;
        twiddle8(v, tw[(j & 15) * 8]);
        dft8(v);
        const int d = (j >> 4) * 128 + (j & 15);
#pragma unroll
        for (int r = 0; r < 8; ++r) buf[fpidx<1024>(d + 16 * r)] = v[r];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int half = 0; half < 2; ++half) {                // 128 -> 1024
        const int j = lane + 64 * half;
        cpx<T>* v = a + 8 * half;
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = buf[fpidx<1024>(j + 128 * r)];
        twiddle8(v, tw[j]);
        dft8(v);
    }
    // butterfly `half` holds X[lane + 64 half + 128 r] in a[8 half + r]: interleave to a[m], m = 2 r + half
    cpx<T> t[16];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        t[2 * r] = a[r];
        t[2 * r + 1] = a[8 + r];
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) a[m] = t[m];
    __builtin_amdgcn_wave_barrier();
}

template <typename T, int L>
__device__ __forceinline__ void fft(cpx<T>* a, cpx<T>* buf, const cpx<T>* __restrict__ tw, int lane) {
    if constexpr (L == 512) fft512(a, buf, tw, lane);
    else fft1024(a, buf, tw, lane);
}

// Sum over a 512-thread block in a fixed order.
__device__ __forceinline__ double block_sum8(double v, double* red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red[0] + red[1]) + (red[2] + red[3])) + ((red[4] + red[5]) + (red[6] + red[7]));
}

// Slice operands of one operator use (MODE as in k_prop_apply: 0 right-hand
// side, 1 initial residual, 2 CG product; 3 the ApplyDesc form of k_apply).  TV and TA
// are the element types of v and of the added vector (FP64 operands of an FP32 pass
// are rounded as they are loaded); wsin holds TA elements in mode 1, TV in mode 2.
template <typename T, typename TV, typename TA, int MODE>
__device__ __forceinline__ void fft_operands(const Geom& g, const void* desc, int s, const TV* vbase,
                                             const void* wsin, const TA* addbase, T* outbase, const TV*& v,
                                             const TA*& add, T*& out, double& theta, int& prob) {
    const long long so = (long long)s * g.stride;
    if (MODE == 3) {
        const ApplyDesc d = ((const ApplyDesc*)desc)[s];
        v = vbase + d.v * g.stride;
        add = (addbase && d.add >= 0) ? addbase + d.add * g.stride : nullptr;
        out = outbase + d.out * g.stride;
        theta = d.theta;
        prob = 0;
        return;
    }
    const PropDesc d = ((const PropDesc*)desc)[s];
    prob = d.prob;
    if (MODE == 0) {
        v = vbase + d.u * g.stride;
        add = (addbase && d.f >= 0) ? addbase + d.f * g.stride : nullptr;
        theta = d.theta_rhs;
    } else if (MODE == 1) {
        v = vbase + d.x * g.stride;
        add = (const TA*)wsin + so;
        theta = d.theta_lhs;
    } else {
        v = (const TV*)wsin + so;
        add = nullptr;
        theta = d.theta_lhs;
    }
    out = outbase + so;
}

// One line pass of the FFT operator.  DIR 0: lines along x, writes
// pbuf = M v + theta X.  DIR 1: lines along y; out = add + sign (pbuf + theta Y)
// and, with dot_mode, the block's partial of v.out (1) or out.out (2).
// The FP32 CG product (MODE 2: no added vector) takes v.out from the spectra: a zero-padded
// real line v and the real output y = sum_k W_k exp(2 pi i j k / L) of its pass give
// sum_j v_j y_j = sum_k Re(conj(V_k) W_k), V the forward transform of v.  The x pass
// writes sign v.pbuf at partial entry nby + blk, the y pass sign theta v.Y at entry blk,
// so the product's nbx + nby partials sum to v.out and no pass reads v twice.  The FP64
// product, whose CG runs to tolerances near its rounding level, sums v.out from the values
// written (nby partials).
template <typename T, typename TV, typename TA, int DIR, int MODE, int L>
__device__ __forceinline__ void fft_line(const Geom& g, const FftPlan& pl, const void* __restrict__ desc, int S,
                                         const TV* vbase, const void* wsin, const TA* addbase, T* outbase, T* pbuf,
                                         double sign_d, int dot_mode, double* partial, const int* active) {
    const int nb = DIR == 0 ? pl.nbx : pl.nby;
    int s, blk;
    decode_block(nb, S, s, blk);
    if (s < 0) return;
    if ((MODE == 1 || MODE == 2) && active && !active[s]) return;
    constexpr int NP = FftLen<L>::NP, FPAD = FftLen<L>::PAD, FL = L;
    __shared__ __attribute__((aligned(16))) cpx<T> lds[8 * FPAD];
    __shared__ double red[8];
    const TV* v;
    const TA* add;
    T* out;
    double theta_d;
    int prob;
    fft_operands<T, TV, TA, MODE>(g, desc, s, vbase, wsin, addbase, outbase, v, add, out, theta_d, prob);
    const T theta = (T)theta_d;
    const T sign = (T)sign_d;
    constexpr int FE = FftLen<L>::FE;
    T* P = pbuf + (long long)s * g.stride;
    const int nx = g.nx, ny = g.ny;
    const int n = DIR == 0 ? nx : ny;        // line length
    const int nl = DIR == 0 ? ny : nx;       // number of lines
    const int l0 = blk * FJ;                 // first output line
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const cpx<T>* tw = (const cpx<T>*)(sizeof(T) == 8 ? (const void*)pl.tw : (const void*)pl.tw32);
    const long long kof = (long long)__builtin_amdgcn_readfirstlane(prob) * g.ps_spec;
    const cpx<T>* K = (const cpx<T>*)(sizeof(T) == 8 ? (const void*)((DIR == 0 ? pl.kx : pl.ky) + kof)
                                                      : (const void*)((DIR == 0 ? pl.kx32 : pl.ky32) + kof));
    cpx<T>* buf = lds + wave * FPAD;
    // FP32, 512 points: the kernel spectra and twiddles (4 x 512 values) are staged in LDS; their
    // loads are issued together with those of the lines, so the combination step waits for nothing
    constexpr bool KST = sizeof(T) == 4 && L == 512;
    __shared__ __attribute__((aligned(16))) cpx<T> kst[KST ? 4 * L : 1];
    cpx<T> kreg[KST ? 4 : 1];
    if constexpr (KST) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + FNT * q;
            kreg[q] = idx < 3 * L ? K[idx] : tw[idx - 3 * L];
        }
    }

    // ---- load the input pair of this wave: lines la = l0 - 1 + 2 wave and la + 1 ----
    const int la = l0 - 1 + 2 * wave, lb = la + 1;
    cpx<T> a[NP];
    if (DIR == 0) {
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            const int pos = lane + 64 * r;
            a[r].x = (la >= 0 && la < nl && pos < n) ? (T)v[(long long)la * nx + pos] : T(0);
            a[r].y = (lb >= 0 && lb < nl && pos < n) ? (T)v[(long long)lb * nx + pos] : T(0);
        }
        if constexpr (KST) {
#pragma unroll
            for (int q = 0; q < 4; ++q) kst[tid + FNT * q] = kreg[q];
            __syncthreads();
            K = kst;
            tw = kst + 3 * L;
        }
    } else {
        // columns l0 - 1 .. l0 + 14 of every row, staged through LDS (row segments are contiguous);
        // all of a thread's loads are issued before the first store
        T* stg = (T*)lds;
        constexpr int SG = L / 2 * 16 / FNT;                    // staged values per thread (ny <= L / 2)
        T sv[SG];
#pragma unroll
        for (int q = 0; q < SG; ++q) {
            const int idx = tid + FNT * q, pos = idx >> 4, col = l0 - 1 + (idx & 15);
            sv[q] = (pos < ny && col >= 0 && col < nx) ? (T)v[(long long)pos * nx + col] : T(0);
        }
#pragma unroll
        for (int q = 0; q < SG; ++q) {
            const int idx = tid + FNT * q, pos = idx >> 4;
            if (pos < ny) stg[pos * 17 + (idx & 15)] = sv[q];
        }
        if constexpr (KST) {
#pragma unroll
            for (int q = 0; q < 4; ++q) kst[tid + FNT * q] = kreg[q];
            K = kst;
            tw = kst + 3 * L;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            const int pos = lane + 64 * r;
            a[r].x = pos < n ? stg[pos * 17 + 2 * wave] : T(0);
            a[r].y = pos < n ? stg[pos * 17 + 2 * wave + 1] : T(0);
        }
        __syncthreads();
    }
    fft<T, L>(a, buf, tw, lane);
#pragma unroll
    for (int r = 0; r < NP; ++r) buf[fpidx<L>(lane + 64 * r)] = a[r];
    __syncthreads();

    // ---- spectra of the output pair (lines oa = l0 + 2 wave, ob = oa + 1) ----
    const int oa = l0 + 2 * wave, ob = oa + 1;
    const bool work = wave < 7 && oa < nl;
    const bool sdot_on = MODE == 2 && dot_mode == 1 && sizeof(T) == 4;
    double sdot = 0.0;                       // this lane's terms of sum_k Re(conj(V_k) W_k), both lines
    if (work) {
        const cpx<T>* Z1 = buf;              // lines oa - 1, oa
        const cpx<T>* Z2 = buf + FPAD;       // lines oa + 1, oa + 2
        const T half = (T)0.5;
        const T mlen = (T)(g.mass / FL);     // spectra carry the 1 / FL of the inverse
        // the mass stencil as three more kernels of the x pass, a0 + a1 cos on line j and b0 + b1 cos -+ i bs sin
        // on lines j +- 1: P1: 6 v + v(i-1) + v(i+1) on line j, v(i) + v(i+1) on line j+1, v(i) + v(i-1) on
        // line j-1 (6, 2; 1, 1, 1); bilinear: 4 (4 v + v(i-1) + v(i+1)) on line j, 4 v + v(i-1) + v(i+1) on
        // j +- 1 (16, 8; 4, 2, 0)
        const T ma0 = mlen * (g.q1 ? T(16) : T(6)), ma1 = mlen * (g.q1 ? T(8) : T(2));
        const T mb0 = mlen * (g.q1 ? T(4) : T(1)), mb1 = mlen * (g.q1 ? T(2) : T(1)), mbs = g.q1 ? T(0) : mlen;
        // The lines are real, the kernel of A_1 is symmetric (real spectrum; its rounding residue in the
        // imaginary part is dropped) and the spectrum of A_2^T is the conjugate of A_2's, so the combined
        // spectra at L - k are the conjugates of those at k.  Each lane combines its rows r < NP / 2 (k < L / 2)
        // and passes the value at L - k to the lane that holds it: lane 64 - lane, row NP - 1 - r (lane 0
        // keeps it: row NP - r).  Lane 0 also combines row NP / 2 itself (k = L / 2).
        constexpr int NH = NP / 2;
        const int src = (64 - lane) & 63;
        // packed output at k (own) and at L - k (mirror) of row r
        // (wgt: how often the lane's k stands in the sum over k = 0 .. L - 1: 1 at 0 and L / 2, 2 for the
        // pairs k, L - k, 0 for a row another lane has counted)
        auto combine = [&](int r, cpx<T>& own, cpx<T>& mirror, int wgt) {
            const int k = lane + 64 * r, kk = (FL - k) & (FL - 1);
            const cpx<T> z1 = Z1[fpidx<L>(k)], z1c = Z1[fpidx<L>(kk)], z2 = Z2[fpidx<L>(k)], z2c = Z2[fpidx<L>(kk)];
            // unpack: first line (z + conj z(-k)) / 2, second line (z - conj z(-k)) / (2 i)
            const cpx<T> vm = {half * (z1.x + z1c.x), half * (z1.y - z1c.y)};
            const cpx<T> v0 = {half * (z1.y + z1c.y), half * (z1c.x - z1.x)};
            const cpx<T> vp = {half * (z2.x + z2c.x), half * (z2.y - z2c.y)};
            const cpx<T> vq = {half * (z2.y + z2c.y), half * (z2c.x - z2.x)};
            T c1 = K[k].x;
            cpx<T> c2 = K[FL + k];
            if (DIR == 0) {                  // (the y pass applies theta to its output instead)
                const cpx<T> w = tw[k];
                c1 = theta * c1 + (ma0 + ma1 * w.x);
                c2 = {theta * c2.x + (mb0 + mb1 * w.x), theta * c2.y - mbs * w.y};
            }
            // xa = c1 v0 + c2 vp + conj(c2) vm,  xb = c1 vp + c2 vq + conj(c2) v0
            const cpx<T> sa = cadd(vp, vm), da = csub(vp, vm), sb = cadd(vq, v0), db = csub(vq, v0);
            const cpx<T> xa = {c1 * v0.x + c2.x * sa.x - c2.y * da.y, c1 * v0.y + c2.x * sa.y + c2.y * da.x};
            const cpx<T> xb = {c1 * vp.x + c2.x * sb.x - c2.y * db.y, c1 * vp.y + c2.x * sb.y + c2.y * db.x};
            // W = xa + i xb; the inverse transform is conj(FFT(conj W)); at L - k, conj W = xa - i xb
            if (sdot_on) sdot += (double)wgt * (double)((v0.x * xa.x + v0.y * xa.y) + (vp.x * xb.x + vp.y * xb.y));
            own = {xa.x - xb.y, -(xa.y + xb.x)};
            mirror = {xa.x + xb.y, xa.y - xb.x};
        };
#pragma unroll
        for (int r = 0; r < NH; ++r) {
            cpx<T> m;
            combine(r, a[r], m, (r == 0 && lane == 0) ? 1 : 2);
            const cpx<T> got = {__shfl(m.x, src, 64), __shfl(m.y, src, 64)};
            if (lane != 0) a[NP - 1 - r] = got;
            if (r > 0 && lane == 0) a[NP - r] = m;
        }
        cpx<T> mid, unused;
        combine(NH, mid, unused, lane == 0 ? 1 : 0);
        if (lane == 0) a[NH] = mid;
    }
    if (sdot_on) {                           // per-wave sums, read after the barrier below
        sdot = wave_sum(sdot);
        if (lane == 0) red[wave] = sdot;
    }
    __syncthreads();
    if (work) fft<T, L>(a, buf, tw, lane);      // a[r] = conj of the packed output at lane + 64 r
    // the block's spectral sum (nothing writes red after the barrier above on this path)
    auto sdot_blk = [&]() { return ((red[0] + red[1]) + (red[2] + red[3])) + ((red[4] + red[5]) + (red[6] + red[7])); };

    if (DIR == 0) {
        if (work) {
#pragma unroll
            for (int r = 0; r < NP; ++r) {
                const int pos = lane + 64 * r;
                if (pos < n) {
                    P[(long long)oa * nx + pos] = a[r].x;
                    if (ob < nl) P[(long long)ob * nx + pos] = -a[r].y;
                }
            }
        }
        if (sdot_on && tid == 0) partial[(long long)s * g.pmax + pl.nby + blk] = sign_d * sdot_blk();
        return;
    }
    // ---- y pass: stage Y as [row][column] and apply the epilogue with theta ----
    __syncthreads();
    T* stg = (T*)lds;
    if (work) {
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            const int pos = lane + 64 * r;
            if (pos < n) {
                stg[pos * 15 + 2 * wave] = a[r].x;
                stg[pos * 15 + 2 * wave + 1] = -a[r].y;
            }
        }
    }
    __syncthreads();
    // epilogue in groups of FG elements per thread: the loads of a group are issued before its stores
    constexpr int FG = FE <= 8 ? FE : 8;
    double dot = 0.0;
#pragma unroll 1
    for (int e0 = 0; e0 < FE; e0 += FG) {
        T pv[FG], av[FG], cv[FG];
#pragma unroll
        for (int q = 0; q < FG; ++q) {
            const int idx = tid + FNT * (e0 + q);
            const int j = idx / FJ, c = idx - j * FJ, i = l0 + c;
            const bool in = e0 + q < FE && j < ny && i < nx;
            const long long o = (long long)j * nx + i;
            pv[q] = in ? P[o] : T(0);
            av[q] = (in && add) ? (T)add[o] : T(0);
            cv[q] = (in && dot_mode == 1 && !sdot_on) ? (T)v[o] : T(0);
        }
#pragma unroll
        for (int q = 0; q < FG; ++q) {
            const int idx = tid + FNT * (e0 + q);
            const int j = idx / FJ, c = idx - j * FJ, i = l0 + c;
            if (e0 + q >= FE || j >= ny || i >= nx) continue;
            const T val = sign * (pv[q] + theta * stg[j * 15 + c]) + av[q];
            out[(long long)j * nx + i] = val;
            if (dot_mode == 1 && !sdot_on) dot += (double)cv[q] * (double)val;
            else if (dot_mode == 2) dot += (double)val * (double)val;
        }
    }
    if (sdot_on) {
        if (tid == 0) partial[(long long)s * g.pmax + blk] = sign_d * (double)theta * sdot_blk();
    } else if (dot_mode) {
        dot = block_sum8(dot, red);
        if (tid == 0) partial[(long long)s * g.pmax + blk] = dot;
    }
}

template <typename T, int DIR, int MODE, int L>
__global__ __launch_bounds__(FNT) void k_fft_line(Geom g, FftPlan pl, const void* __restrict__ desc, int S,
                                                  const T* vbase, const T* wsin, const T* addbase, T* outbase,
                                                  T* pbuf, double sign_d, int dot_mode, double* partial,
                                                  const int* active) {
    fft_line<T, T, T, DIR, MODE, L>(g, pl, desc, S, vbase, wsin, addbase, outbase, pbuf, sign_d, dot_mode, partial,
                                    active);
}

// the FP32 instance with a register budget of three (L = 512) or two workgroups per compute unit
template <int DIR, int MODE, int L, typename TV, typename TA>
__global__ __launch_bounds__(FNT, L == 512 ? 6 : 4) void k_fft_line32(Geom g, FftPlan pl, const void* __restrict__ desc,
                                                                      int S, const TV* vbase, const void* wsin,
                                                                      const TA* addbase, float* outbase,
                                                                      float* pbuf, double sign_d, int dot_mode,
                                                                      double* partial, const int* active) {
    fft_line<float, TV, TA, DIR, MODE, L>(g, pl, desc, S, vbase, wsin, addbase, outbase, pbuf, sign_d, dot_mode,
                                          partial, active);
}

template <typename T, int MODE, int L, typename TV, typename TA>
void fft_op_len(const Geom* g, const FftPlan* pl, const void* desc, int S, const TV* vbase, const void* wsin,
                const TA* addbase, T* outbase, T* pbuf, double sign, int dot_mode, double* partial,
                const int* active, hipStream_t st) {
    if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((k_fft_line32<0, MODE, L, TV, TA>), dim3(grid_blocks(pl->nbx, S)), dim3(FNT), 0, st, *g,
                           *pl, desc, S, vbase, wsin, addbase, outbase, pbuf, sign, dot_mode, partial, active);
        hipLaunchKernelGGL((k_fft_line32<1, MODE, L, TV, TA>), dim3(grid_blocks(pl->nby, S)), dim3(FNT), 0, st, *g,
                           *pl, desc, S, vbase, wsin, addbase, outbase, pbuf, sign, dot_mode, partial, active);
    } else {
        hipLaunchKernelGGL((k_fft_line<T, 0, MODE, L>), dim3(grid_blocks(pl->nbx, S)), dim3(FNT), 0, st, *g, *pl,
                           desc, S, vbase, (const T*)wsin, addbase, outbase, pbuf, sign, dot_mode, partial, active);
        hipLaunchKernelGGL((k_fft_line<T, 1, MODE, L>), dim3(grid_blocks(pl->nby, S)), dim3(FNT), 0, st, *g, *pl,
                           desc, S, vbase, (const T*)wsin, addbase, outbase, pbuf, sign, dot_mode, partial, active);
    }
}

// vbase and addbase hold TV and TA elements (both T unless given).
template <typename T, int MODE, typename TV = T, typename TA = T>
void fft_op(const Geom* g, const FftPlan* pl, const void* desc, int S, const void* vbase, const void* wsin,
            const void* addbase, T* outbase, T* pbuf, double sign, int dot_mode, double* partial, const int* active,
            hipStream_t st) {
    const TV* v = (const TV*)vbase;
    const TA* a = (const TA*)addbase;
    if (pl->L == 512)
        fft_op_len<T, MODE, 512, TV, TA>(g, pl, desc, S, v, wsin, a, outbase, pbuf, sign, dot_mode, partial, active,
                                         st);
    else
        fft_op_len<T, MODE, 1024, TV, TA>(g, pl, desc, S, v, wsin, a, outbase, pbuf, sign, dot_mode, partial,
                                          active, st);
}

template <int TT>
void fd_chain(const Geom* g, const FdMats* fd, const PropDesc* desc, int S, const double* rws, double* zws,
              double* t1, double* t2, double* partial_rz, const int* active, hipStream_t st) {
    const dim3 grid(grid_blocks(g->ntiles[TT == 64 ? 0 : 1], S)), blk(NT);
    // t1 = Vx^T r ; t2 = (t1 Vy) / (1 + theta (lx + ly)) ; t1 = Vx t2 ; z = t1 Vy^T (+ r.z)
    hipLaunchKernelGGL((k_fd_gemm<TT, true, 0>), grid, blk, 0, st, *g, S, fd->Vx, rws, t1, desc, fd->lx, fd->ly,
                       (const double*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fd_gemm<TT, false, 1>), grid, blk, 0, st, *g, S, fd->Vy, (const double*)t1, t2, desc,
                       fd->lx, fd->ly, (const double*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fd_gemm<TT, true, 0>), grid, blk, 0, st, *g, S, fd->VxT, (const double*)t2, t1, desc,
                       fd->lx, fd->ly, (const double*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fd_gemm<TT, false, 2>), grid, blk, 0, st, *g, S, fd->VyT, (const double*)t1, zws, desc,
                       fd->lx, fd->ly, rws, partial_rz, active);
}

template <int MODE>
void prop_apply(const Geom* g, const Seqs* sq, int tv, const PropDesc* desc, int S, const double* ubase,
                const double* fbase, const double* wsin, double* wsout, double* partial, const int* active,
                hipStream_t st) {
    if (tv == 0)
        hipLaunchKernelGGL((k_prop_apply<64, MODE>), dim3(grid_blocks(g->ntiles[0], S)), dim3(NT), 0, st, *g, *sq,
                           desc, S, ubase, fbase, wsin, wsout, partial, active);
    else
        hipLaunchKernelGGL((k_prop_apply<32, MODE>), dim3(grid_blocks(g->ntiles[1], S)), dim3(NT), 0, st, *g, *sq,
                           desc, S, ubase, fbase, wsin, wsout, partial, active);
}

}  // namespace

extern "C" {

int launch_apply(const Geom* g, const Seqs* sq, int tv, const ApplyDesc* desc, int S, const double* vbase,
                 double* outbase, const double* addbase, double sign, int dot_mode, double* partial,
                 const int* active, void* stream) {
    if (S <= 0) return 0;
    if (tv == 0)
        hipLaunchKernelGGL(k_apply<64>, dim3(grid_blocks(g->ntiles[0], S)), dim3(NT), 0, (hipStream_t)stream, *g, *sq,
                           desc, S, vbase, outbase, addbase, sign, dot_mode, partial, active);
    else
        hipLaunchKernelGGL(k_apply<32>, dim3(grid_blocks(g->ntiles[1], S)), dim3(NT), 0, (hipStream_t)stream, *g, *sq,
                           desc, S, vbase, outbase, addbase, sign, dot_mode, partial, active);
    return (int)hipGetLastError();
}

int launch_rhs(const Geom* g, const Seqs* sq, int tv, const PropDesc* desc, int S, const double* ubase,
               const double* fbase, double* bws, double* partial_bb, void* stream) {
    if (S <= 0) return 0;
    prop_apply<0>(g, sq, tv, desc, S, ubase, fbase, nullptr, bws, partial_bb, nullptr, (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_cg_init_x(const Geom* g, const PropDesc* desc, int S, const double* ubase, const double* x0base,
                     int warm, double* xbase, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_cg_init_x, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, desc, S,
                       ubase, x0base, warm, xbase);
    return (int)hipGetLastError();
}

int launch_init_residual(const Geom* g, const Seqs* sq, int tv, const PropDesc* desc, int S, const double* xbase,
                         const double* bws, double* rws, double* partial_rr, const int* mask, void* stream) {
    if (S <= 0) return 0;
    prop_apply<1>(g, sq, tv, desc, S, xbase, nullptr, bws, rws, partial_rr, mask, (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_cg_apply(const Geom* g, const Seqs* sq, int tv, const PropDesc* desc, int S, const double* pws,
                    double* qws, double* partial_pq, const int* active, void* stream) {
    if (S <= 0) return 0;
    prop_apply<2>(g, sq, tv, desc, S, nullptr, nullptr, pws, qws, partial_pq, active, (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_cg_start(const Geom* g, const PropDesc* desc, int S, const double* ubase, double* xbase,
                    const double* zws, double* pws, const double* partial_bb, int nbb, const double* partial_rr,
                    int nrr, double rtol2, double* bb, int* active, int* iters, int* host_act, int* host_iters,
                    void* stream) {
    if (S <= 0) return 0;
    (void)ubase;
    hipLaunchKernelGGL(k_cg_start, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, desc, S,
                       xbase, zws, pws, partial_bb, nbb, partial_rr, nrr, rtol2, bb, active, iters, host_act,
                       host_iters);
    return (int)hipGetLastError();
}

int launch_cg_update(const Geom* g, const PropDesc* desc, int S, double* xbase, double* rws, const double* pws,
                     const double* qws, const double* partial_rho, int nrho, const double* partial_pq, int npq,
                     double* partial_rr_new, const int* active, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_cg_update, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, desc, S,
                       xbase, rws, pws, qws, partial_rho, nrho, partial_pq, npq, partial_rr_new, active);
    return (int)hipGetLastError();
}

int launch_cg_direction(const Geom* g, int S, const double* zws, double* pws, const double* partial_rho, int nrho,
                        const double* partial_rho_new, int nrho_new, const double* partial_rr_new, const double* bb,
                        double rtol2, int maxit, const int* active, int* active_next, int* iters, int* host_next,
                        int* host_iters, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_cg_direction, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, S, zws,
                       pws, partial_rho, nrho, partial_rho_new, nrho_new, partial_rr_new, bb, rtol2, maxit, active,
                       active_next, iters, host_next, host_iters);
    return (int)hipGetLastError();
}

int launch_fd_apply(const Geom* g, const FdMats* fd, int tv, const PropDesc* desc, int S, const double* rws,
                    double* zws, double* t1, double* t2, double* partial_rz, const int* active, void* stream) {
    if (S <= 0) return 0;
    if (tv == 0) fd_chain<64>(g, fd, desc, S, rws, zws, t1, t2, partial_rz, active, (hipStream_t)stream);
    else fd_chain<32>(g, fd, desc, S, rws, zws, t1, t2, partial_rz, active, (hipStream_t)stream);
    return (int)hipGetLastError();
}


}  // extern "C"

namespace {

// t1 = Vx^T r ; t2 = (t1 Vy) / (1 + theta (lx + ly)) ; t1 = Vx t2 ; z = t1 Vy^T (+ r.z)
template <typename RT>
void fdb_chain(const Geom* g, const FdMatsB* fd, const PropDesc* desc, int S, const RT* rws, RT* zws, RT* zcopy,
               void* t1, void* t2, double* partial_rz, const int* active, const void* rimg, hipStream_t st) {
    const int npx = g->tiles_x[0] * 64, npy = g->tiles_y[0] * 64;
    if (npx <= 256 && npy <= 256 && S * g->ntiles[0] < 256) {      // batches that leave compute units idle
        const dim3 grid(grid_blocks((npx / 32) * (npy / 32), S)), blk(NT);
        const __bf16* VxT = (const __bf16*)fd->VxT;
        const __bf16* Vx = (const __bf16*)fd->Vx;
        const __bf16* VyT = (const __bf16*)fd->VyT;
        const __bf16* Vy = (const __bf16*)fd->Vy;
        if (rimg)               // the first product from the BF16 image of r (same values as rounding r here)
            hipLaunchKernelGGL((k_fdb_gemm32<true, 1, 0, RT>), grid, blk, 0, st, *g, S, VxT, rimg, t1, desc, fd->lx,
                               fd->ly, rws, (RT*)nullptr, (double*)nullptr, active);
        else
            hipLaunchKernelGGL((k_fdb_gemm32<true, 0, 0, RT>), grid, blk, 0, st, *g, S, VxT, (const void*)nullptr,
                               t1, desc, fd->lx, fd->ly, rws, (RT*)nullptr, (double*)nullptr, active);
        hipLaunchKernelGGL((k_fdb_gemm32<false, 1, 1, RT>), grid, blk, 0, st, *g, S, VyT, (const void*)t1, t2,
                           desc, fd->lx, fd->ly, rws, (RT*)nullptr, (double*)nullptr, active);
        hipLaunchKernelGGL((k_fdb_gemm32<true, 1, 0, RT>), grid, blk, 0, st, *g, S, Vx, (const void*)t2, t1,
                           desc, fd->lx, fd->ly, rws, (RT*)nullptr, (double*)nullptr, active);
        hipLaunchKernelGGL((k_fdb_gemm32<false, 1, 2, RT>), grid, blk, 0, st, *g, S, Vy, (const void*)t1,
                           (void*)zws, desc, fd->lx, fd->ly, rws, zcopy, partial_rz, active);
        return;
    }
    const dim3 grid(grid_blocks(g->ntiles[0], S)), blk(NT);
    const __bf16* VxT = (const __bf16*)fd->VxT;
    const __bf16* Vx = (const __bf16*)fd->Vx;
    const __bf16* VyT = (const __bf16*)fd->VyT;
    const __bf16* Vy = (const __bf16*)fd->Vy;
    if (rimg)
        hipLaunchKernelGGL((k_fdb_gemm<true, 1, 0, RT>), grid, blk, 0, st, *g, S, VxT, rimg, t1, desc, fd->lx, fd->ly,
                           rws, (RT*)nullptr, (double*)nullptr, active);
    else
        hipLaunchKernelGGL((k_fdb_gemm<true, 0, 0, RT>), grid, blk, 0, st, *g, S, VxT, (const void*)nullptr, t1,
                           desc, fd->lx, fd->ly, rws, (RT*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fdb_gemm<false, 1, 1, RT>), grid, blk, 0, st, *g, S, VyT, (const void*)t1, t2, desc,
                       fd->lx, fd->ly, rws, (RT*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fdb_gemm<true, 1, 0, RT>), grid, blk, 0, st, *g, S, Vx, (const void*)t2, t1, desc,
                       fd->lx, fd->ly, rws, (RT*)nullptr, (double*)nullptr, active);
    hipLaunchKernelGGL((k_fdb_gemm<false, 1, 2, RT>), grid, blk, 0, st, *g, S, Vy, (const void*)t1, (void*)zws,
                       desc, fd->lx, fd->ly, rws, zcopy, partial_rz, active);
}

}  // namespace

extern "C" {

int launch_fdb_apply(const Geom* g, const FdMatsB* fd, const PropDesc* desc, int S, const double* rws, double* zws,
                     void* t1, void* t2, double* partial_rz, const int* active, void* stream) {
    if (S <= 0) return 0;
    fdb_chain<double>(g, fd, desc, S, rws, zws, nullptr, t1, t2, partial_rz, active, nullptr, (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_fdb_apply32(const Geom* g, const FdMatsB* fd, const PropDesc* desc, int S, const float* r32, float* z32,
                       float* zcopy, void* t1, void* t2, double* partial_rz, const int* active, const void* rimg,
                       void* stream) {
    if (S <= 0) return 0;
    fdb_chain<float>(g, fd, desc, S, r32, z32, zcopy, t1, t2, partial_rz, active, rimg, (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_apply32(const Geom* g, const Seqs32* sq, int tv, const PropDesc* desc, int S, const float* p32,
                   float* q32, double* partial_pq, const int* active, void* stream) {
    if (S <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    if (tv == 0)
        hipLaunchKernelGGL(k_apply32<64>, dim3(grid_blocks(g->ntiles[0], S)), dim3(NT), 0, st, *g, *sq, desc, S, p32,
                           q32, partial_pq, active);
    else
        hipLaunchKernelGGL(k_apply32<32>, dim3(grid_blocks(g->ntiles[1], S)), dim3(NT), 0, st, *g, *sq, desc, S, p32,
                           q32, partial_pq, active);
    return (int)hipGetLastError();
}

int launch_apply_bf16(const Geom* g, const Seqs32* sq, const PropDesc* desc, int S, const float* p32, float* q32,
                      double* partial_pq, const int* active, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_apply_bf16, dim3(grid_blocks(g->ntiles[0], S)), dim3(NT), 0, (hipStream_t)stream, *g, *sq,
                       desc, S, p32, q32, partial_pq, active);
    return (int)hipGetLastError();
}

int launch_mx_begin(const Geom* g, const PropDesc* desc, int S, double* xbase, const double* rws,
                    const double* partial_bb, const double* partial_rr, int np, double rtol2, double eta_min2,
                    int first, double* bb, double* scale, double* eta2, int* oact, int* iact, int* iters, float* r32,
                    float* d32, float* p32, double* partial_rr32, int* host_act, int* host_iters,
                    const int* trust_in, int* trust_out, void* rimg, void* stream) {
    if (S <= 0) return 0;
    const dim3 grid(grid_blocks(g->nchunk, S)), blk(NT);
    if (rws)
        hipLaunchKernelGGL(k_mx_begin<double>, grid, blk, 0, (hipStream_t)stream, *g, desc, S, xbase, rws,
                           partial_bb, partial_rr, np, rtol2, eta_min2, first, bb, scale, eta2, oact, iact, iters, r32,
                           d32, p32, partial_rr32, host_act, host_iters, trust_in, trust_out, (__bf16*)rimg);
    else
        hipLaunchKernelGGL(k_mx_begin<float>, grid, blk, 0, (hipStream_t)stream, *g, desc, S, xbase,
                           (const float*)r32, partial_bb, partial_rr, np, rtol2, eta_min2, first, bb, scale, eta2,
                           oact, iact, iters, r32, d32, p32, partial_rr32, host_act, host_iters, trust_in, trust_out,
                           (__bf16*)rimg);
    return (int)hipGetLastError();
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int launch_mx_update(const Geom* g, int S, float* d32, float* r32, const float* p32, const float* q32,
                     const double* partial_rho, int nrho, const double* partial_pq, int npq, double* partial_rr_new,
                     const int* active, void* rimg, void* stream) {
    if (S <= 0) return 0;
    if (!aligned16(d32) || !aligned16(r32) || !aligned16(p32) || !aligned16(q32)) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mx_update, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, S, d32,
                       r32, p32, q32, partial_rho, nrho, partial_pq, npq, partial_rr_new, active, (__bf16*)rimg);
    return (int)hipGetLastError();
}

int launch_mx_direction(const Geom* g, int S, const float* z32, float* p32, const double* partial_rho, int nrho,
                        const double* partial_rho_new, int nrho_new, const double* partial_rr_new, const double* eta2,
                        int maxit, const int* active, int* active_next, int* iters, int* host_next,
                        int* host_iters, void* stream) {
    if (S <= 0) return 0;
    if (!aligned16(z32) || !aligned16(p32)) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mx_direction, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, S,
                       z32, p32, partial_rho, nrho, partial_rho_new, nrho_new, partial_rr_new, eta2, maxit, active,
                       active_next, iters, host_next, host_iters);
    return (int)hipGetLastError();
}

int launch_mx_refine(const Geom* g, const PropDesc* desc, int S, double* xbase, const float* d32,
                     const double* scale, const int* oact, const int* trust, int* need, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_mx_refine, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, desc, S,
                       xbase, d32, scale, oact, trust, need);
    return (int)hipGetLastError();
}

int launch_fill_apply_desc(int S, const double* theta, int has_add, ApplyDesc* desc, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_fill_apply_desc, dim3((S + NT - 1) / NT), dim3(NT), 0, (hipStream_t)stream, S, theta,
                       has_add, desc);
    return (int)hipGetLastError();
}

int launch_add_g(const Geom* g, const PropDesc* desc, int S, double* xbase, const double* gbase, void* stream) {
    if (S <= 0 || !gbase) return 0;
    hipLaunchKernelGGL(k_add_g, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, desc, S, xbase,
                       gbase);
    return (int)hipGetLastError();
}

int launch_axpy_slices(const Geom* g, int S, const int* yi, double* ybase, const int* xi, const double* xbase,
                       double a, double* partial, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_axpy_slices, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, S, yi,
                       ybase, xi, xbase, a, partial);
    return (int)hipGetLastError();
}

// ---- operator by FFT (see k_fft_line); pbuf: S slices of workspace ----
int launch_fft_apply(const Geom* g, const FftPlan* pl, const ApplyDesc* desc, int S, const double* vbase,
                     double* outbase, const double* addbase, double sign, int dot_mode, double* partial,
                     double* pbuf, void* stream) {
    if (S <= 0) return 0;
    fft_op<double, 3>(g, pl, desc, S, vbase, nullptr, addbase, outbase, pbuf, sign, dot_mode, partial, nullptr,
                      (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_fft_rhs(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* ubase,
                   const double* fbase, double* bws, double* partial_bb, double* pbuf, void* stream) {
    if (S <= 0) return 0;
    fft_op<double, 0>(g, pl, desc, S, ubase, nullptr, fbase, bws, pbuf, 1.0, 2, partial_bb, nullptr,
                      (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_fft_init_residual(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* xbase,
                             const double* bws, double* rws, double* partial_rr, double* pbuf, const int* mask,
                             void* stream) {
    if (S <= 0) return 0;
    fft_op<double, 1>(g, pl, desc, S, xbase, bws, nullptr, rws, pbuf, -1.0, 2, partial_rr, mask,
                      (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_fft_cg_apply(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* pws,
                        double* qws, double* partial_pq, const int* active, double* pbuf, void* stream) {
    if (S <= 0) return 0;
    fft_op<double, 2>(g, pl, desc, S, nullptr, pws, nullptr, qws, pbuf, 1.0, 1, partial_pq, active,
                      (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_fft_rhs32(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* ubase,
                     const double* fbase, float* b32, double* partial_bb, float* pbuf, void* stream) {
    if (S <= 0) return 0;
    fft_op<float, 0, double, double>(g, pl, desc, S, ubase, nullptr, fbase, b32, pbuf, 1.0, 2, partial_bb, nullptr,
                                     (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_fft_init_residual32(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const double* xbase,
                               const float* b32, float* r32, double* partial_rr, float* pbuf, void* stream) {
    if (S <= 0) return 0;
    fft_op<float, 1, double, float>(g, pl, desc, S, xbase, b32, nullptr, r32, pbuf, -1.0, 2, partial_rr, nullptr,
                                    (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_fft_apply32(const Geom* g, const FftPlan* pl, const PropDesc* desc, int S, const float* p32, float* q32,
                       double* partial_pq, const int* active, float* pbuf, void* stream) {
    if (S <= 0) return 0;
    fft_op<float, 2>(g, pl, desc, S, nullptr, p32, nullptr, q32, pbuf, 1.0, 1, partial_pq, active,
                     (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_zero_slices(const Geom* g, int S, const int* idx, double* base, void* stream) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL(k_zero_slices, dim3(grid_blocks(g->nchunk, S)), dim3(NT), 0, (hipStream_t)stream, *g, S, idx,
                       base);
    return (int)hipGetLastError();
}

}  // extern "C"
