// Host driver of the MGRIT solver: the C ABI declared in include/mgrit.h.
//
// Algorithm 3.1 (MGRIT V-cycle) over the space-time system (eq. ode-03):
// every relaxation sweep, C-point residual and coarsest solve is a *batch* of
// independent propagator applications, one per coarse interval, handed to the
// batched CG solver in one set of kernel launches (slices stacked along the
// grid of workgroups).  Readings of the paper implemented here:
//   * levels l = 0..L-1, level L-1 solved by sequential stepping; coarsening
//     stops when the next level would hold fewer than two intervals;
//   * C-points are the multiples of m; trailing F-points are F-relaxed only;
//   * linear correction scheme with the injected residual in solution space,
//     r_k = Phi_km(U_km-1) - U_km, zero start on coarse levels (step 3);
//   * Remark 3.1: C-point-only correction on level 0; injection plus
//     F-relaxation (the ideal interpolation) on coarser levels;
//   * stop test after the level-0 relaxation on the discrete L2 norm
//     sqrt(h_x h_y sum_k ||r_k||^2) (Section 3.2's "discrete L2 sense");
//   * CG (Section 3.2) stops on ||r||_2 <= rtol ||b||_2 and starts from the
//     propagated state; a zero right-hand side gives the zero vector.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/mgrit.h"
#include "mgrit_internal.h"

// Scratch memory of mgrit_apply_noalloc (callers that cannot allocate device memory): the slice
// descriptors and the x-pass workspace of the FFT operator live in this fixed array instead of memory
// the call would allocate.  Each GPU holds its own copy until the process ends.  In host code the
// name only stands in for the symbol: its device address is looked up once per device at set-up
// (scratch_address) and only that address is ever passed to a kernel.
static __device__ __align__(256) unsigned char scratch[MGRIT_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (hipError_t)(expr);                                                            \
        if (e_ != hipSuccess) return fail(MGRIT_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define CHK(expr)                   \
    do {                            \
        int rc_ = (expr);           \
        if (rc_ != 0) return rc_;   \
    } while (0)

// A batch of propagator applications: one or two passes (two for the
// two-half-step coarse propagator), descriptors resident on the device.
struct Pass {
    int S = 0;
    std::vector<PropDesc> h;
    PropDesc* d = nullptr;
    mutable int last_iters = 0;   // CG iterations the slowest slice needed last time (launch schedule)
    mutable int last_inner[4] = {0, 0, 0, 0};   // the same for the inner solves of mixed precision, per step
};

struct Batch {
    Pass pass[2];
    int npass = 0;
    int S() const { return pass[0].S; }
};

struct IndexPair {           // y[yi[s]] (+)= a x[xi[s]]
    int S = 0;
    int* yi = nullptr;
    int* xi = nullptr;
};

// One problem of a handle: its statement, time grid and level hierarchy, and where its slices sit in
// the state arrays the handle's batches index.  A handle set up by mgrit_setup has one member; one set
// up by mgrit_setup_group has several on one mesh, whose sweeps share the batches of every level.
struct Member {
    mgrit_problem prob{};
    std::vector<double> t;
    std::vector<int> N;                       // intervals per level
    std::vector<std::vector<int>> fine;       // level-0 index of each point, per level
    std::vector<std::vector<double>> tau;     // tau[l][k], k = 1..N[l]
    std::vector<long long> off;               // first slice of the member in each level's state
    long long f_off = 0;                      // first load slice of the member in the level-0 loads
    std::vector<double> seq_x, seq_y;         // host generating sequences, scaled (as the device uses them)
};

// A level of the hierarchy over all members: batches gather the slices of the members that are still
// iterating, in member order.
struct Level {
    int N = 0;                       // intervals (the most of any member)
    long long ns = 0;                // slices of the level's state, all members
    double* U = nullptr;             // [ns] slices (levels >= 1; level 0 uses U0)
    double* G = nullptr;             // [ns] slices (levels >= 1)
    std::vector<Batch> frelax;       // F-relaxation, one batch per F sub-step
    Batch crelax;                    // C-relaxation
    Batch resid;                     // residual propagation into the next level's G
    std::vector<Batch> step_list;    // per-step batches (coarsest level / sequential stepping)
    IndexPair correct;               // U[km] += E[k]
    IndexPair subtract;              // Gnext[k] -= U[km]
    std::vector<int> sub_count;      // subtract pairs of each batched member (per-member norms)
    int* all_idx = nullptr;          // 0..ns-1 (zeroing)
    int* first_idx = nullptr;        // first slice of every member (E_0 = 0, G_0 = 0)
    int nfirst = 0;
};

}  // namespace

struct mgrit_handle {
    mgrit_problem prob;                      // the first member's (mesh and domain are common)
    mgrit_options opt;
    std::vector<double> t;                   // the first member's time grid
    std::vector<Member> mem;                 // the problems (one unless set up as a group)
    std::vector<char> batched;               // members whose slices the current batches hold
    std::vector<void*> batch_allocs;         // device descriptors of the current batches
    double* gU = nullptr;                    // groups: level-0 state and loads of all members
    double* gF = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;                          // device current at set-up
    void* scratch = nullptr;                 // device address of that device's scratch array
    Geom geom;
    Seqs seqs;
    double* d_seq = nullptr;                 // T1x | A2x | T1y | A2y
    float* d_seq32 = nullptr;                // FP32 copy (mixed precision)
    Seqs32 seqs32{};
    // operator by FFT: tables, the x-pass workspaces, partials per slice
    bool use_fft = false;
    FftPlan plan{};
    double* pfft = nullptr;
    float* pfft32 = nullptr;
    int nop = 0;                             // operator partials per slice
    int nop_pq = 0;                          // p.q partials of the FP32 CG product (both FFT passes write them)
    std::vector<double> host_seq_x, host_seq_y;
    double cx = 0, cy = 0;
    std::vector<Level> lv;
    int Smax = 0;
    // CG workspace
    double *b = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *tmp = nullptr;
    double *z = nullptr, *t1 = nullptr, *t2 = nullptr;      // preconditioner workspace
    void *tb1 = nullptr, *tb2 = nullptr;                    // BF16 preconditioner workspace
    void* rimg = nullptr;                    // mixed precision: BF16 image of r32 (zero-padded npx x npy slices)
    FdMats fd;
    FdMatsB fdb;
    double *pbb = nullptr, *prr[2] = {nullptr, nullptr}, *ppq = nullptr, *pnorm = nullptr;
    double* prz[2] = {nullptr, nullptr};
    double* bb = nullptr;
    // mixed precision: FP32 inner workspace, per-slice scale, inner tolerance
    // and outer flags, partials of the FP64 outer residual
    float *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
    double *mx_scale = nullptr, *mx_eta2 = nullptr, *pout = nullptr;
    int* mx_oact = nullptr;
    int* mx_need = nullptr;                  // slices whose iterate gets an FP64 residual after a step
    int* mx_trust = nullptr;                 // 2 x Smax: settled slices of a refinement step (parity buffers)
    long long refine_count = 0;             // refinement steps summed over slices
    int* act[2] = {nullptr, nullptr};
    int* iters = nullptr;
    int* h_flags = nullptr;                  // pinned, 2 x Smax: act[0], act[1] as the direction kernels set them
    int* d_flags = nullptr;                  // the device address of h_flags
    int* h_start = nullptr;                  // pinned, Smax: the flags at the start of a solve or step
    int* d_start = nullptr;                  // the device address of h_start
    hipEvent_t flag_ev[2] = {};
    int* h_iters = nullptr;                  // pinned: iteration counts as the start and direction kernels set them
    int* d_iters = nullptr;                  // the device address of h_iters
    int* h_iters_step = nullptr;             // 4 x Smax: iteration counts after each refinement step
    double* h_norm = nullptr;                // pinned
    long long phi_count = 0, cg_count = 0;
    std::vector<void*> allocations;
    size_t dev_bytes = 0;           // device memory owned by the handle
    double cur_rtol = 0.0;          // CG tolerance of the current MGRIT iteration
    int cur_level = 0;              // level of the passes being run
    std::map<int, int> tile_of;     // tile variant chosen per batch width (autotuned)
    std::map<int, int> tile_of32;   // the same for the FP32 inner operator
    // captured pairs of CG iterations, keyed by every argument of their launches
    struct GraphKey {
        const void* d;
        const void* x;
        int S, tv, nrho, nrho_next, maxit, parity, kind;
        double rtol2;
        bool operator<(const GraphKey& o) const {
            return std::tie(d, x, S, tv, nrho, nrho_next, maxit, parity, kind, rtol2) <
                   std::tie(o.d, o.x, o.S, o.tv, o.nrho, o.nrho_next, o.maxit, o.parity, o.kind, o.rtol2);
        }
    };
    std::map<GraphKey, hipGraphExec_t> graphs;
    hipEvent_t tune_ev[5] = {};
    // instrumentation of the CG operator kernel
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_tv;                 // tile variant of each recorded event pair
    size_t prof_used = 0;
    double prof_ms[MGRIT_PROF_CLASSES] = {};                  // per kernel class (MGRIT_PROF_*)
    long long prof_launches[MGRIT_PROF_CLASSES] = {}, prof_slices[MGRIT_PROF_CLASSES] = {};
    // caller arrays of the current solve (level 0)
    double* U0 = nullptr;
    const double* F0 = nullptr;
};

namespace {

// Device address of the scratch array on device `dev` (the current device), looked up once per device.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(MGRIT_EINVAL, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MGRIT_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

// A failed allocation is ENOMEM; the runtime's last-error state is cleared so that the next kernel launch
// check does not report it again.
int alloc_failed(hipError_t e, size_t bytes) {
    (void)hipGetLastError();
    return fail(MGRIT_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
}

int dmalloc(mgrit_handle* h, void** p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return alloc_failed(e, bytes);
    h->allocations.push_back(*p);
    h->dev_bytes += bytes;
    return 0;
}

template <class T>
int dalloc(mgrit_handle* h, T** p, size_t count) {
    return dmalloc(h, (void**)p, count * sizeof(T));
}

// Device memory of the current batches (descriptors, index pairs): freed when the batches are rebuilt.
int batch_alloc(mgrit_handle* h, void** p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return alloc_failed(e, bytes);
    h->batch_allocs.push_back(*p);
    return 0;
}

int upload_pass(mgrit_handle* h, Pass& ps) {
    ps.S = (int)ps.h.size();
    if (ps.S == 0) return 0;
    CHK(batch_alloc(h, (void**)&ps.d, ps.h.size() * sizeof(PropDesc)));
    HIPCHK(hipMemcpy(ps.d, ps.h.data(), ps.h.size() * sizeof(PropDesc), hipMemcpyHostToDevice));
    return 0;
}

int upload_pairs(mgrit_handle* h, IndexPair& ip, const std::vector<int>& y, const std::vector<int>& x) {
    ip.S = (int)y.size();
    if (ip.S == 0) return 0;
    CHK(batch_alloc(h, (void**)&ip.yi, y.size() * sizeof(int)));
    CHK(batch_alloc(h, (void**)&ip.xi, x.size() * sizeof(int)));
    HIPCHK(hipMemcpy(ip.yi, y.data(), y.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ip.xi, x.data(), x.size() * sizeof(int), hipMemcpyHostToDevice));
    return 0;
}

// Descriptor of one application of member p's level-l propagator from point k-1 to k, reading slice `u`
// and writing slice `x` of the level's state (indices include the member's offset); x0 is the slice that
// holds the previous value of point k (-1: none).  The loads (level 0) and affine terms (levels >= 1) are
// the member's own.  One or two passes.
void make_step(const mgrit_handle* h, int p, int l, int k, int u, int x, int tmp_slot, Batch& b, int x0 = -1) {
    const Member& M = h->mem[p];
    const double tau = M.tau[l][k];
    PropDesc d;
    d.u = u;
    d.x = x;
    d.f = -1;
    d.g = -1;
    d.x0 = x0;
    d.prob = p;
    if (l == 0) {
        d.f = (int)(M.f_off + k - 1);  // load F_k
        d.theta_rhs = -0.5 * tau;
        d.theta_lhs = 0.5 * tau;
        b.pass[0].h.push_back(d);
        b.npass = 1;
        return;
    }
    d.g = (int)(M.off[l] + k);          // affine term G^(l)_k
    if (h->opt.coarse == MGRIT_COARSE_BE) {
        d.theta_rhs = 0.0;
        d.theta_lhs = tau;
        b.pass[0].h.push_back(d);
        b.npass = 1;
    } else if (h->opt.coarse == MGRIT_COARSE_CN2 || h->opt.coarse == MGRIT_COARSE_OPT) {
        double s1 = 0.5 * tau, s2 = 0.5 * tau;   // two half steps
        if (h->opt.coarse == MGRIT_COARSE_OPT) {
            // Match the product of the level-0 Crank-Nicolson factors inside
            // this coarse step at small and at large tau~ sigma.
            const int i0 = M.fine[l][k - 1], i1 = M.fine[l][k];
            double inv = 0.0;
            for (int n = i0 + 1; n <= i1; ++n) inv += 1.0 / (M.t[n] - M.t[n - 1]);
            const double c = 4.0 * tau * inv;
            const double dd = std::sqrt(c * c / 16.0 - c);
            const double a1 = c / 4.0 + dd, a2 = c / 4.0 - dd;
            s1 = 2.0 * tau / a1;   // short step first
            s2 = 2.0 * tau / a2;
        }
        PropDesc d1 = d, d2 = d;
        d1.x = tmp_slot;
        d1.g = -1;
        d1.x0 = -1;
        d1.theta_rhs = -0.5 * s1;
        d1.theta_lhs = 0.5 * s1;
        d2.u = tmp_slot;
        d2.theta_rhs = -0.5 * s2;
        d2.theta_lhs = 0.5 * s2;
        b.pass[0].h.push_back(d1);
        b.pass[1].h.push_back(d2);
        b.npass = 2;
    } else {
        d.theta_rhs = -0.5 * tau;
        d.theta_lhs = 0.5 * tau;
        b.pass[0].h.push_back(d);
        b.npass = 1;
    }
}

int upload_batch(mgrit_handle* h, Batch& b) {
    for (int i = 0; i < b.npass; ++i) CHK(upload_pass(h, b.pass[i]));
    return 0;
}

// Level hierarchy of one member (Section 3.1): t^(l+1) = t^(l)[::m] while the coarse grid keeps at
// least two intervals, at most max_levels levels.
void member_levels(const mgrit_handle* h, Member& M) {
    const int m = h->opt.m;
    M.N.assign(1, M.prob.Nt);
    M.fine.assign(1, std::vector<int>(M.prob.Nt + 1));
    for (int i = 0; i <= M.prob.Nt; ++i) M.fine[0][i] = i;
    while ((int)M.N.size() < h->opt.max_levels) {
        const int Nc = M.N.back() / m;
        if (Nc < 2) break;
        std::vector<int> f(Nc + 1);
        for (int k = 0; k <= Nc; ++k) f[k] = M.fine.back()[k * m];
        M.N.push_back(Nc);
        M.fine.push_back(f);
    }
    M.tau.assign(M.N.size(), std::vector<double>());
    for (size_t l = 0; l < M.N.size(); ++l) {
        M.tau[l].assign(M.N[l] + 1, 0.0);
        for (int k = 1; k <= M.N[l]; ++k) M.tau[l][k] = M.t[M.fine[l][k]] - M.t[M.fine[l][k - 1]];
    }
}

// (Re)build every level's batches over the members marked in h->batched, in member order: the slices
// of all of them go into one set of launches per relaxation step, residual and coarse step.  *smax: the
// largest batch.
int build_batches(mgrit_handle* h, int* smax_out = nullptr) {
    if (!h->batch_allocs.empty()) {
        HIPCHK(hipStreamSynchronize(h->stream));         // nothing queued still reads the old batches
        for (void* q : h->batch_allocs) (void)hipFree(q);
        h->batch_allocs.clear();
    }
    const int m = h->opt.m;
    const int nl = (int)h->lv.size();
    const int P = (int)h->mem.size();
    int smax = 1;
    for (int l = 0; l < nl; ++l) {
        Level& L = h->lv[l];
        L.frelax.clear();
        L.crelax = Batch();
        L.resid = Batch();
        L.step_list.clear();
        L.correct = IndexPair();
        L.subtract = IndexPair();
        L.sub_count.clear();
        const bool coarsest = (l == nl - 1);
        if (!coarsest) {
            L.frelax.assign(m - 1, Batch());
            for (int j = 1; j < m; ++j) {
                Batch& b = L.frelax[j - 1];
                int slot = 0;
                for (int p = 0; p < P; ++p) {
                    if (!h->batched[p]) continue;
                    const Member& M = h->mem[p];
                    const int o = (int)M.off[l];
                    for (int c = 0; c + j <= M.N[l]; c += m)
                        make_step(h, p, l, c + j, o + c + j - 1, o + c + j, slot++, b, o + c + j);
                }
                smax = std::max(smax, (int)b.pass[0].h.size());
            }
            int slot = 0, slot2 = 0;
            std::vector<int> y, x, y2, x2;
            for (int p = 0; p < P; ++p) {
                if (!h->batched[p]) continue;
                const Member& M = h->mem[p];
                const int o = (int)M.off[l], oc = (int)M.off[l + 1], Nc = M.N[l + 1];
                for (int k = 1; k <= Nc; ++k) make_step(h, p, l, k * m, o + k * m - 1, o + k * m, slot++, L.crelax, o + k * m);
                for (int k = 1; k <= Nc; ++k) make_step(h, p, l, k * m, o + k * m - 1, oc + k, slot2++, L.resid, o + k * m);
                for (int k = 0; k <= Nc; ++k) {
                    y.push_back(o + k * m);
                    x.push_back(oc + k);
                }
                for (int k = 1; k <= Nc; ++k) {
                    y2.push_back(oc + k);
                    x2.push_back(o + k * m);
                }
                L.sub_count.push_back(Nc);
            }
            smax = std::max(smax, slot);
            CHK(upload_pairs(h, L.correct, y, x));
            CHK(upload_pairs(h, L.subtract, y2, x2));
            for (Batch& b : L.frelax) CHK(upload_batch(h, b));
            CHK(upload_batch(h, L.crelax));
            CHK(upload_batch(h, L.resid));
        }
        // single-step batches: for the coarsest level (E_k = Phi(E_k-1)) and for sequential stepping on
        // level 0: step k of every member that has it
        if (coarsest || l == 0) {
            int kmax = 0;
            for (int p = 0; p < P; ++p)
                if (h->batched[p]) kmax = std::max(kmax, h->mem[p].N[l]);
            L.step_list.assign(kmax, Batch());
            for (int k = 1; k <= kmax; ++k) {
                int slot = 0;
                for (int p = 0; p < P; ++p) {
                    if (!h->batched[p] || h->mem[p].N[l] < k) continue;
                    const int o = (int)h->mem[p].off[l];
                    make_step(h, p, l, k, o + k - 1, o + k, slot++, L.step_list[k - 1]);
                }
                smax = std::max(smax, slot);
            }
            // one device array for all single-step descriptors (pass by pass)
            const int np = kmax ? L.step_list[0].npass : 0;
            for (int pi = 0; pi < np; ++pi) {
                std::vector<PropDesc> all;
                std::vector<size_t> first;
                for (Batch& b : L.step_list) {
                    first.push_back(all.size());
                    all.insert(all.end(), b.pass[pi].h.begin(), b.pass[pi].h.end());
                }
                PropDesc* d = nullptr;
                CHK(batch_alloc(h, (void**)&d, all.size() * sizeof(PropDesc)));
                HIPCHK(hipMemcpy(d, all.data(), all.size() * sizeof(PropDesc), hipMemcpyHostToDevice));
                for (size_t k = 0; k < L.step_list.size(); ++k) {
                    L.step_list[k].pass[pi].S = (int)L.step_list[k].pass[pi].h.size();
                    L.step_list[k].pass[pi].d = d + first[k];
                }
            }
        }
    }
    if (smax_out) *smax_out = smax;
    return 0;
}

// Levels over all members: slice offsets, the level state arrays (levels >= 1) and the zeroing index
// lists; then the batches with every member.
int build_levels(mgrit_handle* h) {
    const int P = (int)h->mem.size();
    for (Member& M : h->mem) member_levels(h, M);
    const int nl = (int)h->mem[0].N.size();
    if (nl < 2)
        return fail(MGRIT_EINVAL, "time grid too short for one coarsening (Nt=%d, m=%d)", h->mem[0].prob.Nt, h->opt.m);
    for (int p = 1; p < P; ++p)
        if ((int)h->mem[p].N.size() != nl)
            return fail(MGRIT_EINVAL, "the problems of a group need the same number of levels (problem %d: %d, not %d)",
                        p, (int)h->mem[p].N.size(), nl);
    h->lv.assign(nl, Level());
    long long f = 0;
    for (int p = 0; p < P; ++p) {
        h->mem[p].f_off = f;
        f += h->mem[p].prob.Nt;
    }
    for (int l = 0; l < nl; ++l) {
        Level& L = h->lv[l];
        long long o = 0;
        std::vector<int> first;
        for (int p = 0; p < P; ++p) {
            Member& M = h->mem[p];
            M.off.resize(nl);
            M.off[l] = o;
            first.push_back((int)o);
            o += M.N[l] + 1;
            L.N = std::max(L.N, M.N[l]);
        }
        L.ns = o;
        if (o >= (1LL << 31)) return fail(MGRIT_EINVAL, "too many slices in one level (%lld)", o);
        std::vector<int> all(o);
        for (long long i = 0; i < o; ++i) all[i] = (int)i;
        CHK(dalloc(h, &L.all_idx, all.size()));
        HIPCHK(hipMemcpy(L.all_idx, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice));
        L.nfirst = P;
        CHK(dalloc(h, &L.first_idx, first.size()));
        HIPCHK(hipMemcpy(L.first_idx, first.data(), first.size() * sizeof(int), hipMemcpyHostToDevice));
        if (l > 0) {
            CHK(dalloc(h, &L.U, (size_t)o * h->geom.stride));
            CHK(dalloc(h, &L.G, (size_t)o * h->geom.stride));
        }
    }
    h->batched.assign(P, 1);
    return build_batches(h, &h->Smax);
}

// Host generating sequences of one member, scaled as the device uses them (see mgrit_sequences).
void member_sequences(const mgrit_handle* h, Member& M, double* cx, double* cy) {
    const mgrit_problem& p = M.prob;
    const int nx = p.Mx - 1, ny = p.My - 1;
    const double hx = (p.b - p.a) / p.Mx, hy = (p.d - p.c) / p.My;
    M.seq_x.assign(3 * (size_t)nx, 0.0);
    M.seq_y.assign(3 * (size_t)ny, 0.0);
    if (h->opt.element == MGRIT_ELEMENT_Q1) {
        // K_x M_y (x) A_x: column j of the grid array gets (4 h_y / 6) A_x v_j + (h_y / 6) A_x (v_j+1 + v_j-1),
        // the three factors of the x contraction; likewise for y with h_x
        *cx = *cy = 1.0;
        for (int l = 0; l < nx; ++l) {
            const double a = p.Kx * mgrit_fd_stiffness_entry(p.beta, hx, 1.0, l);
            M.seq_x[l] = 4.0 * hy / 6.0 * a;
            M.seq_x[nx + l] = M.seq_x[2 * nx + l] = hy / 6.0 * a;
        }
        for (int l = 0; l < ny; ++l) {
            const double a = p.Ky * mgrit_fd_stiffness_entry(p.gamma, hy, 1.0, l);
            M.seq_y[l] = 4.0 * hx / 6.0 * a;
            M.seq_y[ny + l] = M.seq_y[2 * ny + l] = hx / 6.0 * a;
        }
        return;
    }
    *cx = mgrit_stiffness_scale(p.beta, hx, hy);
    *cy = mgrit_stiffness_scale(p.gamma, hy, hx);
    mgrit_toeplitz_sequences(p.beta, nx, &M.seq_x[0], &M.seq_x[nx], &M.seq_x[2 * nx]);
    mgrit_toeplitz_sequences(p.gamma, ny, &M.seq_y[0], &M.seq_y[ny], &M.seq_y[2 * ny]);
    const double sx = p.Kx * *cx, sy = p.Ky * *cy;
    for (double& v : M.seq_x) v *= sx;
    for (double& v : M.seq_y) v *= sy;
}

// Padded generating sequences on the device: one block [T1x | A2x | T1y | A2y] per member.
int build_sequences(mgrit_handle* h) {
    const int nx = h->geom.nx, ny = h->geom.ny;
    const int P = (int)h->mem.size();
    for (int p = 0; p < P; ++p) {
        double cx, cy;
        member_sequences(h, h->mem[p], &cx, &cy);
        if (p == 0) {
            h->cx = cx;
            h->cy = cy;
            h->host_seq_x = h->mem[0].seq_x;
            h->host_seq_y = h->mem[0].seq_y;
        }
    }
    Geom& g = h->geom;
    const int offx = g.seq_off_x, offy = g.seq_off_y;
    const size_t lx = 2 * (size_t)offx + 1, ly = 2 * (size_t)offy + 1;
    const size_t blk = 2 * lx + 2 * ly;
    g.ps_seq = (long long)blk;
    std::vector<double> buf(blk * P, 0.0);
    for (int p = 0; p < P; ++p) {
        double* T1x = &buf[blk * p];
        double* A2x = T1x + lx;
        double* T1y = A2x + lx;
        double* A2y = T1y + ly;
        const double* tx = &h->mem[p].seq_x[0];
        const double* ux = &h->mem[p].seq_x[nx];
        const double* wx = &h->mem[p].seq_x[2 * nx];
        for (int d = -(nx - 1); d <= nx - 1; ++d) {
            T1x[offx + d] = tx[std::abs(d)];
            A2x[offx + d] = d >= 0 ? ux[d] : wx[-d];
        }
        const double* ty = &h->mem[p].seq_y[0];
        const double* uy = &h->mem[p].seq_y[ny];
        const double* wy = &h->mem[p].seq_y[2 * ny];
        for (int d = -(ny - 1); d <= ny - 1; ++d) {
            T1y[offy + d] = ty[std::abs(d)];
            A2y[offy + d] = d >= 0 ? uy[d] : wy[-d];
        }
    }
    CHK(dalloc(h, &h->d_seq, buf.size()));
    HIPCHK(hipMemcpy(h->d_seq, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice));
    h->seqs.T1x = h->d_seq;
    h->seqs.A2x = h->d_seq + lx;
    h->seqs.T1y = h->d_seq + 2 * lx;
    h->seqs.A2y = h->d_seq + 2 * lx + ly;
    if (h->opt.precision != MGRIT_PREC_FP64) {
        std::vector<float> b32(buf.begin(), buf.end());
        CHK(dalloc(h, &h->d_seq32, b32.size()));
        HIPCHK(hipMemcpy(h->d_seq32, b32.data(), b32.size() * sizeof(float), hipMemcpyHostToDevice));
        h->seqs32.T1x = h->d_seq32;
        h->seqs32.A2x = h->d_seq32 + lx;
        h->seqs32.T1y = h->d_seq32 + 2 * lx;
        h->seqs32.A2y = h->d_seq32 + 2 * lx + ly;
    }
    return 0;
}

// Tables of the FFT operator.  Kernels of one direction (sequences t, u, w of
// length n, scaled): c1(m) = t(|m|) for A_1; c2(m) = A2(-m) for A_2 (applied
// to the next line) and c3(m) = A2(m) for A_2^T (the previous line), with
// A2(d) = u(d) for d >= 0 and w(-d) for d < 0, so that the product along a
// line is sum_k c(i - k) v(k).  Each kernel is embedded in a circulant of
// length L (c(m) at m mod L, |m| < n) and transformed by a direct DFT in
// extended precision; the spectra are divided by L for the inverse.
int build_fft_plan(mgrit_handle* h) {
    const Geom& g = h->geom;
    const int L = (2 * std::max(g.nx, g.ny) - 1 <= 512) ? 512 : 1024;
    h->plan.L = L;
    std::vector<long double> cs(L), sn(L);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < L; ++k) {
        cs[k] = cosl(2.0L * pi * k / L);
        sn[k] = -sinl(2.0L * pi * k / L);
    }
    std::vector<double> tw(2 * L);
    for (int k = 0; k < L; ++k) {
        tw[2 * k] = (double)cs[k];
        tw[2 * k + 1] = (double)sn[k];
    }
    auto spectra = [&](const std::vector<double>& seq, int n, std::vector<double>& out) {
        const double* t = &seq[0];
        const double* u = &seq[n];
        const double* w = &seq[2 * n];
        auto A2 = [&](int d) { return d >= 0 ? u[d] : w[-d]; };
        out.assign(3 * 2 * (size_t)L, 0.0);
        for (int c = 0; c < 3; ++c) {
            std::vector<long double> e(L, 0.0L);
            for (int m = -(n - 1); m <= n - 1; ++m) {
                const double val = c == 0 ? t[std::abs(m)] : (c == 1 ? A2(-m) : A2(m));
                e[(m + L) % L] = val;
            }
            for (int k = 0; k < L; ++k) {
                long double re = 0.0L, im = 0.0L;
                for (int m = 0; m < L; ++m) {
                    if (e[m] == 0.0L) continue;
                    const int q = (int)(((long long)m * k) % L);
                    re += e[m] * cs[q];
                    im += e[m] * sn[q];
                }
                out[(size_t)2 * (c * L + k)] = (double)(re / L);
                out[(size_t)2 * (c * L + k) + 1] = (double)(im / L);
            }
        }
    };
    // [tw | kx, ky of member 0 | kx, ky of member 1 | ...]
    std::vector<double> all(tw);
    const size_t kn = 3 * 2 * (size_t)L;
    for (const Member& M : h->mem) {
        std::vector<double> kx, ky;
        spectra(M.seq_x, g.nx, kx);
        spectra(M.seq_y, g.ny, ky);
        all.insert(all.end(), kx.begin(), kx.end());
        all.insert(all.end(), ky.begin(), ky.end());
    }
    h->geom.ps_spec = (long long)(2 * kn);
    double* d = nullptr;
    CHK(dalloc(h, &d, all.size()));
    HIPCHK(hipMemcpy(d, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice));
    h->plan.tw = d;
    h->plan.kx = d + tw.size();
    h->plan.ky = d + tw.size() + kn;
    if (h->opt.precision != MGRIT_PREC_FP64) {
        std::vector<float> f(all.begin(), all.end());
        float* d32 = nullptr;
        CHK(dalloc(h, &d32, f.size()));
        HIPCHK(hipMemcpy(d32, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
        h->plan.tw32 = d32;
        h->plan.kx32 = d32 + tw.size();
        h->plan.ky32 = d32 + tw.size() + kn;
    }
    h->plan.nbx = (g.ny + MGRIT_FFT_LINES - 1) / MGRIT_FFT_LINES;
    h->plan.nby = (g.nx + MGRIT_FFT_LINES - 1) / MGRIT_FFT_LINES;
    return 0;
}

// FP64 -> BF16 bit pattern, round to nearest even (finite inputs).
unsigned short to_bf16(double v) {
    const float f = (float)v;
    unsigned int u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// Eigen-decompositions of the 1-D (K, M) pairs of the preconditioner.  The
// stiffness is weighted by FD_STIFFNESS_WEIGHT: the lumped mass exceeds M_h on
// the highest modes (up to 3x), and a slightly lighter stiffness balances the
// two ends of the preconditioned spectrum (fewest PCG iterations over orders
// 0.55..0.95 and theta from 5e-4 to 0.25 at 255 x 255).
constexpr double FD_STIFFNESS_WEIGHT = 0.9;

// Mixed-precision passes whose CG tolerance is at least this run wholly in FP32
// (right-hand side, initial residual, one refinement step).
constexpr double COARSE_FP32_RTOL = 1e-4;

int build_fd(mgrit_handle* h) {
    const int nx = h->geom.nx, ny = h->geom.ny;
    const int P = (int)h->mem.size();
    const bool bf16 = h->opt.precond == MGRIT_PRECOND_FD_BF16;
    const int npx = h->geom.tiles_x[0] * 64, npy = h->geom.tiles_y[0] * 64;
    // per member: FP64 [Vx | VxT | Vy | VyT | lx | ly]; BF16 [VxT | Vx | VyT | Vy] (padded); FP32 [lx | ly] (padded)
    const size_t b64 = 2 * (size_t)nx * nx + 2 * (size_t)ny * ny + nx + ny;
    const size_t b16 = 2 * (size_t)npx * npx + 2 * (size_t)npy * npy;
    const size_t bf = (size_t)npx + npy;
    h->geom.ps_fd = (long long)b64;
    h->geom.ps_fdb = bf16 ? (long long)b16 : 0;
    h->geom.ps_fde = bf16 ? (long long)bf : 0;
    std::vector<double> all64(b64 * P);
    std::vector<unsigned short> all16(bf16 ? b16 * P : 0, 0);
    std::vector<float> allf(bf16 ? bf * P : 0, 0.f);
    // P1: lumped mass and a lightened stiffness (an approximation of the step matrix); Q1: the consistent
    // 1-D mass and the unweighted stiffness, whose Kronecker form is the step matrix itself
    const bool q1 = h->opt.element == MGRIT_ELEMENT_Q1;
    auto eig = q1 ? mgrit_fd_eigen_consistent : mgrit_fd_eigen;
    const double wgt = q1 ? 1.0 : FD_STIFFNESS_WEIGHT;
    for (int m = 0; m < P; ++m) {
        const mgrit_problem& p = h->mem[m].prob;
        const double hx = (p.b - p.a) / p.Mx, hy = (p.d - p.c) / p.My;
        std::vector<double> Vx((size_t)nx * nx), lx(nx), Vy((size_t)ny * ny), ly(ny);
        if (eig(p.beta, nx, hx, wgt * p.Kx, Vx.data(), lx.data()) != 0 ||
            eig(p.gamma, ny, hy, wgt * p.Ky, Vy.data(), ly.data()) != 0)
            return fail(MGRIT_EINVAL, "eigen-decomposition of the preconditioner failed");
        double* B = &all64[b64 * m];
        double* VxT = B + (size_t)nx * nx;
        double* VyB = VxT + (size_t)nx * nx;
        double* VyT = VyB + (size_t)ny * ny;
        std::copy(Vx.begin(), Vx.end(), B);
        std::copy(Vy.begin(), Vy.end(), VyB);
        for (int i = 0; i < nx; ++i)
            for (int k = 0; k < nx; ++k) VxT[(size_t)i * nx + k] = Vx[(size_t)k * nx + i];
        for (int i = 0; i < ny; ++i)
            for (int k = 0; k < ny; ++k) VyT[(size_t)i * ny + k] = Vy[(size_t)k * ny + i];
        std::copy(lx.begin(), lx.end(), VyT + (size_t)ny * ny);
        std::copy(ly.begin(), ly.end(), VyT + (size_t)ny * ny + nx);
        if (!bf16) continue;
        // zero-padded BF16 copies: A operands of the products over x are row-major
        // [i][k] (VxT for Vx^T X, Vx for Vx X); B^T operands of the products over y
        // are row-major [j][k] (VyT for X Vy, Vy for X Vy^T)
        unsigned short* bx1 = &all16[b16 * m];
        unsigned short* bx2 = bx1 + (size_t)npx * npx;
        unsigned short* by1 = bx2 + (size_t)npx * npx;
        unsigned short* by2 = by1 + (size_t)npy * npy;
        for (int i = 0; i < nx; ++i)
            for (int k = 0; k < nx; ++k) {
                bx1[(size_t)i * npx + k] = to_bf16(Vx[(size_t)k * nx + i]);    // (Vx^T)[i][k]
                bx2[(size_t)i * npx + k] = to_bf16(Vx[(size_t)i * nx + k]);    // Vx[i][k]
            }
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < ny; ++k) {
                by1[(size_t)j * npy + k] = to_bf16(Vy[(size_t)k * ny + j]);    // B = Vy: B^T[j][k] = Vy[k][j]
                by2[(size_t)j * npy + k] = to_bf16(Vy[(size_t)j * ny + k]);    // B = Vy^T: B^T[j][k] = Vy[j][k]
            }
        float* lf = &allf[bf * m];
        for (int i = 0; i < nx; ++i) lf[i] = (float)lx[i];
        for (int j = 0; j < ny; ++j) lf[npx + j] = (float)ly[j];
    }
    double* d = nullptr;
    CHK(dalloc(h, &d, all64.size()));
    HIPCHK(hipMemcpy(d, all64.data(), all64.size() * sizeof(double), hipMemcpyHostToDevice));
    h->fd.Vx = d;
    h->fd.VxT = d + (size_t)nx * nx;
    h->fd.Vy = d + 2 * (size_t)nx * nx;
    h->fd.VyT = h->fd.Vy + (size_t)ny * ny;
    h->fd.lx = h->fd.VyT + (size_t)ny * ny;
    h->fd.ly = h->fd.lx + nx;
    if (!bf16) return 0;
    unsigned short* b = nullptr;
    CHK(dalloc(h, &b, all16.size()));
    HIPCHK(hipMemcpy(b, all16.data(), all16.size() * 2, hipMemcpyHostToDevice));
    h->fdb.VxT = b;
    h->fdb.Vx = b + (size_t)npx * npx;
    h->fdb.VyT = b + 2 * (size_t)npx * npx;
    h->fdb.Vy = h->fdb.VyT + (size_t)npy * npy;
    float* f = nullptr;
    CHK(dalloc(h, &f, allf.size()));
    HIPCHK(hipMemcpy(f, allf.data(), allf.size() * sizeof(float), hipMemcpyHostToDevice));
    h->fdb.lx = f;
    h->fdb.ly = f + npx;
    return 0;
}

int alloc_workspace(mgrit_handle* h, int S) {
    const size_t st = (size_t)h->geom.stride;
    const size_t nt = (size_t)h->geom.pmax;
    CHK(dalloc(h, &h->b, S * st));
    CHK(dalloc(h, &h->r, S * st));
    CHK(dalloc(h, &h->p, S * st));
    CHK(dalloc(h, &h->q, S * st));
    if (h->opt.coarse == MGRIT_COARSE_CN2 || h->opt.coarse == MGRIT_COARSE_OPT) CHK(dalloc(h, &h->tmp, S * st));
    if (h->opt.precond != MGRIT_PRECOND_NONE) {
        CHK(dalloc(h, &h->z, S * st));
        CHK(dalloc(h, &h->prz[0], S * nt));
        CHK(dalloc(h, &h->prz[1], S * nt));
    }
    if (h->opt.precond == MGRIT_PRECOND_FD) {
        CHK(dalloc(h, &h->t1, S * st));
        CHK(dalloc(h, &h->t2, S * st));
    }
    if (h->opt.precond == MGRIT_PRECOND_FD_BF16) {
        const size_t pb = (size_t)h->geom.tiles_x[0] * 64 * h->geom.tiles_y[0] * 64 * sizeof(unsigned short);
        CHK(dmalloc(h, &h->tb1, S * pb));
        CHK(dmalloc(h, &h->tb2, S * pb));
    }
    CHK(dalloc(h, &h->pbb, S * nt));
    CHK(dalloc(h, &h->prr[0], S * nt));
    CHK(dalloc(h, &h->prr[1], S * nt));
    CHK(dalloc(h, &h->ppq, S * nt));
    CHK(dalloc(h, &h->pnorm, S * nt));
    CHK(dalloc(h, &h->bb, S));
    CHK(dalloc(h, &h->act[0], S));
    CHK(dalloc(h, &h->act[1], S));
    CHK(dalloc(h, &h->iters, S));
    if (h->use_fft) {
        CHK(dalloc(h, &h->pfft, S * st));
        if (h->opt.precision != MGRIT_PREC_FP64) CHK(dalloc(h, &h->pfft32, S * st));
    }
    if (h->opt.precision != MGRIT_PREC_FP64) {
        CHK(dalloc(h, &h->r32, S * st));
        CHK(dalloc(h, &h->z32, S * st));
        CHK(dalloc(h, &h->p32, S * st));
        CHK(dalloc(h, &h->q32, S * st));
        CHK(dalloc(h, &h->d32, S * st));
        CHK(dalloc(h, &h->mx_scale, S));
        CHK(dalloc(h, &h->mx_eta2, S));
        CHK(dalloc(h, &h->mx_oact, S));
        CHK(dalloc(h, &h->mx_need, S));
        CHK(dalloc(h, &h->mx_trust, 2 * (size_t)S));
        if (h->opt.precond == MGRIT_PRECOND_FD_BF16) {
            // written where r32 is (only inside n_x x n_y): the padding stays zero
            const size_t pb = (size_t)h->geom.tiles_x[0] * 64 * h->geom.tiles_y[0] * 64 * sizeof(unsigned short);
            CHK(dmalloc(h, &h->rimg, S * pb));
            HIPCHK(hipMemset(h->rimg, 0, S * pb));
        }
        CHK(dalloc(h, &h->pout, S * nt));
        if (!h->prz[0]) {
            CHK(dalloc(h, &h->prz[0], S * nt));
            CHK(dalloc(h, &h->prz[1], S * nt));
        }
    }
    HIPCHK(hipHostMalloc((void**)&h->h_flags, 2 * S * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void**)&h->d_flags, h->h_flags, 0));
    for (int i = 0; i < 2 * S; ++i) h->h_flags[i] = 0;
    HIPCHK(hipHostMalloc((void**)&h->h_start, S * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void**)&h->d_start, h->h_start, 0));
    for (int i = 0; i < S; ++i) h->h_start[i] = 0;
    for (hipEvent_t& e : h->flag_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipHostMalloc((void**)&h->h_iters, S * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void**)&h->d_iters, h->h_iters, 0));
    for (int i = 0; i < S; ++i) h->h_iters[i] = 0;
    HIPCHK(hipHostMalloc((void**)&h->h_iters_step, 4 * (size_t)S * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&h->h_norm, S * nt * sizeof(double), hipHostMallocDefault));
    return 0;
}

// Instrumentation marks: an event recorded on the stream before each instrumented launch, tagged with
// the launch's kernel class; the time from one mark to the next is that launch's (class -1 closes a
// sequence of launches without starting a new one).
int prof_record(mgrit_handle* h, int cls) {
    if (h->prof_used == h->prof_ev.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        h->prof_ev.push_back(e);
        h->prof_tv.push_back(0);
    }
    h->prof_tv[h->prof_used] = cls;
    HIPCHK(hipEventRecord(h->prof_ev[h->prof_used++], h->stream));
    return 0;
}

// Accumulate the recorded marks (the stream has been synchronised).
int prof_drain(mgrit_handle* h) {
    for (size_t i = 0; i + 1 < h->prof_used; ++i) {
        const int cls = h->prof_tv[i];
        if (cls < 0) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->prof_ev[i], h->prof_ev[i + 1]));
        h->prof_ms[cls] += ms;
        h->prof_launches[cls] += 1;
    }
    h->prof_used = 0;
    return 0;
}

// Operator launches: the tiled matrix-core kernels or the two FFT passes.
int op_rhs(mgrit_handle* h, int tv, const Pass& ps, const double* ubase, const double* fbase) {
    if (h->use_fft)
        return launch_fft_rhs(&h->geom, &h->plan, ps.d, ps.S, ubase, fbase, h->b, h->pbb, h->pfft, h->stream);
    return launch_rhs(&h->geom, &h->seqs, tv, ps.d, ps.S, ubase, fbase, h->b, h->pbb, h->stream);
}

// (mask: the slices to recompute, the others keep r and their partials; null: all)
int op_resid(mgrit_handle* h, int tv, const Pass& ps, const double* xbase, double* partial,
             const int* mask = nullptr) {
    if (h->use_fft)
        return launch_fft_init_residual(&h->geom, &h->plan, ps.d, ps.S, xbase, h->b, h->r, partial, h->pfft, mask,
                                        h->stream);
    return launch_init_residual(&h->geom, &h->seqs, tv, ps.d, ps.S, xbase, h->b, h->r, partial, mask, h->stream);
}

int op_cg(mgrit_handle* h, int tv, const Pass& ps, const double* pin, double* qout, const int* act) {
    if (h->use_fft)
        return launch_fft_cg_apply(&h->geom, &h->plan, ps.d, ps.S, pin, qout, h->ppq, act, h->pfft, h->stream);
    return launch_cg_apply(&h->geom, &h->seqs, tv, ps.d, ps.S, pin, qout, h->ppq, act, h->stream);
}

int op_cg32(mgrit_handle* h, int tv, const Pass& ps, const float* pin, float* qout, const int* act) {
    if (h->opt.precision == MGRIT_PREC_MIXED_BF16)
        return launch_apply_bf16(&h->geom, &h->seqs32, ps.d, ps.S, pin, qout, h->ppq, act, h->stream);
    if (h->use_fft)
        return launch_fft_apply32(&h->geom, &h->plan, ps.d, ps.S, pin, qout, h->ppq, act, h->pfft32, h->stream);
    return launch_apply32(&h->geom, &h->seqs32, tv, ps.d, ps.S, pin, qout, h->ppq, act, h->stream);
}

// Operator tile edge for a batch of S slices (0: 64, 1: 32).  RULE: 64 when
// the batch fills the chip with such tiles.  AUTO: the first pass of each
// batch width times the CG operator kernel in both variants on the pass's
// right-hand sides (it writes q and its partials, recomputed before use) and
// keeps the faster; without a pass to time on, the rule.  The FP32 operator
// of mixed precision is timed on its own, on the scaled residuals.  The iterates do not depend on the choice: every tiled
// kernel sums its dot products per 32 x 32 block in one fixed order.
int tile_variant(mgrit_handle* h, const Pass* ps, int S, int* tv, bool fp32 = false) {
    const int rule = (long long)S * h->geom.ntiles[0] >= 512 ? 0 : 1;
    if (h->use_fft) {                                   // the FFT passes have no tiles
        *tv = 0;
        return 0;
    }
    switch (h->opt.tile_policy) {
        case MGRIT_TILE_64: *tv = 0; return 0;
        case MGRIT_TILE_32: *tv = 1; return 0;
        case MGRIT_TILE_RULE: *tv = rule; return 0;
        default: break;
    }
    std::map<int, int>& cache = fp32 ? h->tile_of32 : h->tile_of;
    auto it = cache.find(S);
    if (it != cache.end()) {
        *tv = it->second;
        return 0;
    }
    if (!ps) {                                          // nothing to time on: the rule
        *tv = rule;
        return 0;
    }
    if (!h->tune_ev[0])
        for (hipEvent_t& e : h->tune_ev) HIPCHK(hipEventCreate(&e));
    const Geom* g = &h->geom;
    const int order[4] = {0, 1, 0, 1};                  // alternate to average out clocks
    HIPCHK(hipEventRecord(h->tune_ev[0], h->stream));
    for (int k = 0; k < 4; ++k) {
        if (fp32)
            HIPCHK(launch_apply32(g, &h->seqs32, order[k], ps->d, S, h->r32, h->q32, h->ppq, nullptr,
                                  (void*)h->stream));
        else
            HIPCHK(launch_cg_apply(g, &h->seqs, order[k], ps->d, S, h->b, h->q, h->ppq, nullptr, (void*)h->stream));
        HIPCHK(hipEventRecord(h->tune_ev[k + 1], h->stream));
    }
    HIPCHK(hipEventSynchronize(h->tune_ev[4]));
    float ms[2] = {0.f, 0.f};
    for (int k = 0; k < 4; ++k) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, h->tune_ev[k], h->tune_ev[k + 1]));
        ms[order[k]] += t;
    }
    *tv = ms[0] <= ms[1] ? 0 : 1;
    cache[S] = *tv;
    return 0;
}

// Launches n CG iterations starting at flag parity cur.  With graphs on, pairs
// of iterations (which leave the parity unchanged) are captured once per set
// of launch arguments and replayed as one HIP graph; a single iteration and
// the first one of a solve without preconditioner (its rho partials differ)
// are launched directly.
int launch_iterations(mgrit_handle* h, mgrit_handle::GraphKey key, int n, int& cur, int& nrho,
                      const std::function<int(int, int)>& iter) {
    const bool graphs = h->opt.graphs && h->stream && !h->prof_on;
    while (n > 0) {
        if (graphs && n >= 2 && nrho == key.nrho_next) {
            key.parity = cur;
            key.nrho = nrho;
            auto it = h->graphs.find(key);
            if (it == h->graphs.end()) {
                hipGraph_t graph = nullptr;
                HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
                int rc = iter(cur, nrho);
                if (!rc) rc = iter(cur ^ 1, nrho);
                const hipError_t e = hipStreamEndCapture(h->stream, &graph);
                if (rc) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return rc;
                }
                if (e != hipSuccess) return fail(MGRIT_EHIP, "graph capture failed: %s", hipGetErrorString(e));
                hipGraphExec_t exec = nullptr;
                const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e2 != hipSuccess) return fail(MGRIT_EHIP, "graph instantiation failed: %s", hipGetErrorString(e2));
                it = h->graphs.emplace(key, exec).first;
            }
            HIPCHK(hipGraphLaunch(it->second, h->stream));
            n -= 2;
        } else {
            CHK(iter(cur, nrho));
            cur ^= 1;
            nrho = key.nrho_next;
            n -= 1;
        }
    }
    return 0;
}

// Runs CG iterations in chunks (n_first, then one at a time) until no slice
// is active or maxit iterations were launched.  The host reads the flags of
// one chunk while the next is already queued, so the GPU does not wait for
// the check; the one iteration queued after the last slice converged finds
// every slice inactive and does nothing.  sync_first: wait for the flags at
// the start before queueing anything (when all slices are likely converged).
// *n_active0: active slices at the start.  The flags at the start are the
// ones the start kernel (k_cg_start, k_mx_begin) also stored into h_start,
// which nothing else writes during the solve; later checks read the pinned
// mirror the direction kernels write, h_flags[parity], which the single
// queued iteration does not touch (it writes the other parity).
int run_checked(mgrit_handle* h, int S, int n_first, int maxit, bool sync_first, int& cur, int& it,
                int* n_active0, const std::function<int(int)>& launch_chunk, int* n_ones0 = nullptr) {
    const int* src[2] = {nullptr, nullptr};
    auto queue_flags = [&](int k, bool start) -> int {
        src[k] = start ? h->h_start : h->h_flags + (size_t)cur * h->Smax;
        HIPCHK(hipEventRecord(h->flag_ev[k], h->stream));
        return 0;
    };
    auto count = [&](int k) -> int {
        const int* f = src[k];
        int nact = 0, ones = 0;
        for (int s = 0; s < S; ++s) {
            nact += f[s] != 0;
            ones += f[s] == 1;
        }
        if (n_ones0) {                       // flags at the start only
            *n_ones0 = ones;
            n_ones0 = nullptr;
        }
        return nact;
    };
    CHK(queue_flags(0, true));
    if (sync_first) {
        HIPCHK(hipEventSynchronize(h->flag_ev[0]));
        const int nact = count(0);
        if (n_active0) *n_active0 = nact;
        n_active0 = nullptr;
        if (nact == 0) return 0;
    }
    int k = 0, n = std::min(n_first, maxit - it);
    while (true) {
        const bool launched = n > 0;
        if (launched) {
            CHK(launch_chunk(n));
            it += n;
            CHK(queue_flags(k ^ 1, false));
        }
        HIPCHK(hipEventSynchronize(h->flag_ev[k]));
        const int nact = count(k);
        if (n_active0) *n_active0 = nact;
        n_active0 = nullptr;
        if (nact == 0 || !launched) break;
        k ^= 1;
        n = std::min(1, maxit - it);
    }
    return 0;
}

int run_pass_mixed(mgrit_handle* h, const Pass& ps, const double* ubase, double* xbase, const double* fbase,
                   const double* gbase, const double* x0base, int warm);

// Batched CG solve of one pass (S <= Smax slices).
int run_pass(mgrit_handle* h, const Pass& ps, const double* ubase, double* xbase, const double* fbase,
             const double* gbase, const double* x0base = nullptr, int warm = 0) {
    const int S = ps.S;
    if (S == 0) return 0;
    if (S > h->Smax) return fail(MGRIT_EINVAL, "batch of %d slices exceeds workspace (%d)", S, h->Smax);
    if (h->opt.precision == MGRIT_PREC_MIXED || h->opt.precision == MGRIT_PREC_MIXED_BF16 ||
        (h->opt.precision == MGRIT_PREC_MIXED_COARSE && h->cur_level > 0))
        return run_pass_mixed(h, ps, ubase, xbase, fbase, gbase, x0base, warm);
    const Geom* g = &h->geom;
    void* st = (void*)h->stream;
    double rtol = h->cur_rtol > 0.0 ? h->cur_rtol : h->opt.cg_rtol;
    if (h->cur_level > 0 && h->opt.cg_rtol_coarse > 0.0) rtol = h->opt.cg_rtol_coarse;
    const double rtol2 = rtol * rtol;
    const int pk = h->opt.precond;
    const bool pc = pk != MGRIT_PRECOND_NONE;
    int tv = 0;
    CHK(tile_variant(h, nullptr, S, &tv));
    // Tiled kernels leave one partial sum per 32 x 32 block whatever their tile
    // size, so the reductions (and the iterates) do not depend on tv.
    const int nop = h->nop, npc = g->ntiles[1], nc = g->nchunk;   // partials: operator, preconditioner, vectors
    auto precondition = [&](double* prz_out, const int* act) -> int {
        if (pk == MGRIT_PRECOND_FD)
            return launch_fd_apply(g, &h->fd, tv, ps.d, S, h->r, h->z, h->t1, h->t2, prz_out, act, st);
        return launch_fdb_apply(g, &h->fdb, ps.d, S, h->r, h->z, h->tb1, h->tb2, prz_out, act, st);
    };
    HIPCHK(op_rhs(h, tv, ps, ubase, fbase));
    CHK(tile_variant(h, &ps, S, &tv));
    HIPCHK(launch_cg_init_x(g, ps.d, S, ubase, x0base, (x0base && warm && h->opt.warm_start) ? 1 : 0, xbase, st));
    HIPCHK(op_resid(h, tv, ps, xbase, h->prr[0]));
    const bool prof = h->prof_on;
    if (pc) {
        if (prof) CHK(prof_record(h, MGRIT_PROF_PRECOND));
        HIPCHK(precondition(h->prz[0], nullptr));
        if (prof) CHK(prof_record(h, -1));
    }
    double* zws = pc ? h->z : h->r;
    double** prho = pc ? h->prz : h->prr;        // rho = r.z (r.r without preconditioner)
    HIPCHK(launch_cg_start(g, ps.d, S, ubase, xbase, zws, h->p, h->pbb, nop, h->prr[0], nop, rtol2, h->bb, h->act[0],
                           h->iters, h->d_start, h->d_iters, st));
    int cur = 0;
    int it = 0;
    int nrho = pc ? npc : nop;                               // entries of the current rho partials
    const int nrho_next = pc ? npc : nc;
    const int maxit = h->opt.cg_maxit;
    // The first chunk covers what this pass needed last time, later chunks are
    // short, so few launches find every slice converged.
    const int first = ps.last_iters > 0 ? ps.last_iters : (pc ? 8 : 16);
    auto iter = [&](int c0, int nr) -> int {
        const int nxt = c0 ^ 1;
        if (prof) CHK(prof_record(h, tv));
        HIPCHK(op_cg(h, tv, ps, h->p, h->q, h->act[c0]));
        if (prof) CHK(prof_record(h, MGRIT_PROF_UPDATE64));
        HIPCHK(launch_cg_update(g, ps.d, S, xbase, h->r, h->p, h->q, prho[c0], nr, h->ppq, nop, h->prr[nxt],
                                h->act[c0], st));
        if (prof && pc) CHK(prof_record(h, MGRIT_PROF_PRECOND));
        if (pc) HIPCHK(precondition(h->prz[nxt], h->act[c0]));
        if (prof) CHK(prof_record(h, MGRIT_PROF_DIRECTION64));
        HIPCHK(launch_cg_direction(g, S, zws, h->p, prho[c0], nr, prho[nxt], nrho_next, h->prr[nxt], h->bb, rtol2,
                                   maxit, h->act[c0], h->act[nxt], h->iters, h->d_flags + (size_t)nxt * h->Smax,
                                   h->d_iters, st));
        if (prof) CHK(prof_record(h, -1));
        return 0;
    };
    auto chunk = [&](int n) -> int {
        return launch_iterations(h, {ps.d, xbase, S, tv, nrho, nrho_next, maxit, 0, 0, rtol2}, n, cur, nrho, iter);
    };
    CHK(run_checked(h, S, first, maxit, false, cur, it, nullptr, chunk));
    // the counts are final once run_checked has seen every slice inactive (or maxit): the direction
    // kernels that set them have completed, later (queued) iterations leave inactive slices alone
    HIPCHK(launch_add_g(g, ps.d, S, xbase, gbase, st));
    if (h->prof_on) {
        HIPCHK(hipStreamSynchronize(h->stream));
        CHK(prof_drain(h));
    }
    long long its = 0;
    int most = 0;
    for (int s = 0; s < S; ++s) {
        its += h->h_iters[s];
        most = std::max(most, h->h_iters[s]);
    }
    ps.last_iters = most;
    h->cg_count += its;
    if (h->prof_on) {
        h->prof_slices[tv] += its;
        h->prof_slices[MGRIT_PROF_UPDATE64] += its;
        h->prof_slices[MGRIT_PROF_DIRECTION64] += its;
        // the preconditioner also starts the pass, on every slice
        if (pc) h->prof_slices[MGRIT_PROF_PRECOND] += its + S;
    }
    h->phi_count += S;
    return 0;
}

// The same solve by iterative refinement: b, x and the residual r = b - B x
// in FP64; each step solves B d = r / ||r|| by PCG in FP32 (FP32 matrix-core
// operator, BF16 preconditioner products, FP64 reductions) to the relative
// tolerance max(rtol ||b|| / ||r||, inner_rtol) and sets x += ||r|| d, until
// the FP64 residual meets ||r|| <= rtol ||b|| (the test of the FP64 solve).
int run_pass_mixed(mgrit_handle* h, const Pass& ps, const double* ubase, double* xbase, const double* fbase,
                   const double* gbase, const double* x0base, int warm) {
    const int S = ps.S;
    const Geom* g = &h->geom;
    void* st = (void*)h->stream;
    double rtol = h->cur_rtol > 0.0 ? h->cur_rtol : h->opt.cg_rtol;
    if (h->cur_level > 0 && h->opt.cg_rtol_coarse > 0.0) rtol = h->opt.cg_rtol_coarse;
    const double rtol2 = rtol * rtol;
    const double eta = h->opt.inner_rtol > 0.0 ? h->opt.inner_rtol : 1e-5;
    const bool pc = h->opt.precond == MGRIT_PRECOND_FD_BF16;
    const int nop = h->nop, npc = g->ntiles[1], nc = g->nchunk;
    // p.q partials of the inner operator: one per 32 x 32 block from the tiled kernels (dense FP32, split
    // BF16), one per workgroup of either pass from the FFT passes
    const int nop32 = (h->use_fft && h->opt.precision != MGRIT_PREC_MIXED_BF16) ? h->nop_pq : g->ntiles[1];
    const int maxit = h->opt.cg_maxit;
    const bool prof = h->prof_on;
    int tv = 0, tv32 = -1, op32_class = MGRIT_PROF_OP32_T64;
    // Loose passes (coarse levels) form the right-hand side and the initial residual in FP32 as
    // well: their rounding (~1e-7 of ||b||) is far below the tolerance, and one refinement step,
    // whose inner target is then the pass tolerance itself, settles the pass.
    const bool all32 = h->use_fft && rtol >= COARSE_FP32_RTOL;
    if (all32) {
        HIPCHK(launch_cg_init_x(g, ps.d, S, ubase, x0base, (x0base && warm && h->opt.warm_start) ? 1 : 0, xbase,
                                st));
        HIPCHK(launch_fft_rhs32(g, &h->plan, ps.d, S, ubase, fbase, h->z32, h->pbb, h->pfft32, h->stream));
        HIPCHK(launch_fft_init_residual32(g, &h->plan, ps.d, S, xbase, h->z32, h->r32, h->pout, h->pfft32,
                                          h->stream));
    } else {
        CHK(tile_variant(h, nullptr, S, &tv));
        HIPCHK(op_rhs(h, tv, ps, ubase, fbase));
        CHK(tile_variant(h, &ps, S, &tv));
        HIPCHK(launch_cg_init_x(g, ps.d, S, ubase, x0base, (x0base && warm && h->opt.warm_start) ? 1 : 0, xbase,
                                st));
        HIPCHK(op_resid(h, tv, ps, xbase, h->pout));
    }
    float* zws = pc ? h->z32 : h->r32;
    double** prho = pc ? h->prz : h->prr;        // rho = r.z (r.r without preconditioner)
    int steps = 0, nrec = 0;
    for (int outer = 0; outer < 32; ++outer) {
        HIPCHK(launch_mx_begin(g, ps.d, S, xbase, all32 ? nullptr : h->r, h->pbb, h->pout, nop, rtol2, eta * eta,
                               outer == 0 ? 1 : 0, h->bb, h->mx_scale, h->mx_eta2, h->mx_oact, h->act[0], h->iters,
                               h->r32, h->d32, pc ? nullptr : h->p32, h->prr[0], h->d_start, h->d_iters,
                               h->mx_trust + (size_t)(outer & 1) * h->Smax,
                               h->mx_trust + (size_t)((outer + 1) & 1) * h->Smax, h->rimg, st));
        if (tv32 < 0) {
            if (h->opt.precision == MGRIT_PREC_MIXED_BF16) tv32 = 0;     // one tile size
            else CHK(tile_variant(h, &ps, S, &tv32, true));
            op32_class = h->opt.precision == MGRIT_PREC_MIXED_BF16 ? MGRIT_PROF_OP_BF16 : MGRIT_PROF_OP32_T64 + tv32;
        }
        if (pc) {
            if (prof) CHK(prof_record(h, MGRIT_PROF_PRECOND));
            HIPCHK(launch_fdb_apply32(g, &h->fdb, ps.d, S, h->r32, h->z32, h->p32, h->tb1, h->tb2, h->prz[0],
                                      h->act[0], h->rimg, st));
            if (prof) CHK(prof_record(h, -1));
        }
        int cur = 0, it = 0, nact = 0;
        int nrho = pc ? npc : nc;
        const int nrho_next = pc ? npc : nc;
        auto iter = [&](int c0, int nr) -> int {
            const int nxt = c0 ^ 1;
            if (prof) CHK(prof_record(h, op32_class));
            HIPCHK(op_cg32(h, tv32, ps, h->p32, h->q32, h->act[c0]));
            if (prof) CHK(prof_record(h, MGRIT_PROF_UPDATE32));
            HIPCHK(launch_mx_update(g, S, h->d32, h->r32, h->p32, h->q32, prho[c0], nr, h->ppq, nop32, h->prr[nxt],
                                    h->act[c0], h->rimg, st));
            if (prof && pc) CHK(prof_record(h, MGRIT_PROF_PRECOND));
            if (pc)
                HIPCHK(launch_fdb_apply32(g, &h->fdb, ps.d, S, h->r32, h->z32, nullptr, h->tb1, h->tb2, h->prz[nxt],
                                          h->act[c0], h->rimg, st));
            if (prof) CHK(prof_record(h, MGRIT_PROF_DIRECTION32));
            HIPCHK(launch_mx_direction(g, S, zws, h->p32, prho[c0], nr, prho[nxt], nrho_next, h->prr[nxt],
                                       h->mx_eta2, maxit, h->act[c0], h->act[nxt], h->iters,
                                       h->d_flags + (size_t)nxt * h->Smax, h->d_iters, st));
            if (prof) CHK(prof_record(h, -1));
            return 0;
        };
        auto chunk = [&](int n) -> int {
            return launch_iterations(h, {ps.d, nullptr, S, tv32, nrho, nrho_next, maxit, 0, 1, 0.0}, n, cur, nrho,
                                     iter);
        };
        // the flags at the start are the outer ones: none active ends the refinement.  The first
        // chunk is what the slowest slice of this step needed last time (then one iteration at a
        // time, one queued ahead of each flag check).
        const int li = ps.last_inner[std::min(outer, 3)];
        const int first = li > 0 ? li : 6;
        int untrusted = 0;
        CHK(run_checked(h, S, first, maxit, outer > 0, cur, it, &nact, chunk, &untrusted));
        if (nact == 0) break;
        steps += nact;
        if (outer < 4) {                     // counts after this step (final: see run_pass)
            std::memcpy(h->h_iters_step + (size_t)outer * h->Smax, h->h_iters, S * sizeof(int));
            nrec = outer + 1;
        }
        int* trust_next = h->mx_trust + (size_t)((outer + 1) & 1) * h->Smax;
        HIPCHK(launch_mx_refine(g, ps.d, S, xbase, h->d32, h->mx_scale, h->mx_oact, trust_next, h->mx_need, st));
        // An inner solve whose target was the pass tolerance itself and at least 10 x the FP32 floor
        // (inner flag 2) settles its slice by its own test: the FP32 residual it reached agrees with the
        // FP64 one to FP32 rounding (about 1e-6 of the step's starting residual, 1 % of the smallest such
        // target), so such slices get no FP64 check (k_mx_begin keeps them inactive); when every slice
        // of the step is one of them the pass ends here.  Steps that ran to the floor (the first ones at
        // tight tolerances) are checked in FP64.
        if (untrusted == 0 || all32) break;
        HIPCHK(op_resid(h, tv, ps, xbase, h->pout, h->mx_need));
    }
    HIPCHK(launch_add_g(g, ps.d, S, xbase, gbase, st));
    if (h->prof_on) {
        HIPCHK(hipStreamSynchronize(h->stream));
        CHK(prof_drain(h));
    }
    long long its = 0;
    for (int s = 0; s < S; ++s) its += h->h_iters[s];
    for (int k = 0; k < nrec; ++k) {         // iterations the slowest slice needed in step k
        const int* c = h->h_iters_step + (size_t)k * h->Smax;
        const int* p = k > 0 ? c - h->Smax : nullptr;
        int most = 0;
        for (int s = 0; s < S; ++s) most = std::max(most, c[s] - (p ? p[s] : 0));
        ps.last_inner[k] = most;
    }
    h->cg_count += its;
    h->refine_count += steps;
    if (h->prof_on && tv32 >= 0) {
        h->prof_slices[op32_class] += its;
        h->prof_slices[MGRIT_PROF_UPDATE32] += its;
        h->prof_slices[MGRIT_PROF_DIRECTION32] += its;
        // the preconditioner also starts each refinement step of its active slices
        if (pc) h->prof_slices[MGRIT_PROF_PRECOND] += its + steps;
    }
    h->phi_count += S;
    return 0;
}

// Bases of the level-l arrays.
struct Bases {
    double* U;
    const double* F;
    const double* G;
};

Bases bases(mgrit_handle* h, int l) {
    if (l == 0) return Bases{h->U0, h->F0, nullptr};
    return Bases{h->lv[l].U, nullptr, h->lv[l].G};
}

// Run a batch on level l with output array `xout` (the level's U unless given).
// warm: the level's state holds meaningful previous values of the target
// points, used as CG start vectors (descriptors with x0 >= 0).
int run_batch(mgrit_handle* h, int l, const Batch& b, double* xout = nullptr, int warm = 0) {
    h->cur_level = l;
    Bases B = bases(h, l);
    double* X = xout ? xout : B.U;
    if (b.npass == 1) return run_pass(h, b.pass[0], B.U, X, B.F, B.G, B.U, warm);
    CHK(run_pass(h, b.pass[0], B.U, h->tmp, B.F, nullptr));
    return run_pass(h, b.pass[1], h->tmp, X, B.F, B.G, B.U, warm);
}

int f_relax(mgrit_handle* h, int l, int warm) {
    for (const Batch& b : h->lv[l].frelax) CHK(run_batch(h, l, b, nullptr, warm));
    return 0;
}

// warm: the level's state already holds an iterate (not the zero start).
int relax(mgrit_handle* h, int l, int warm) {
    CHK(f_relax(h, l, warm));
    const int kind = (l > 0 && h->opt.coarse_relax >= 0) ? h->opt.coarse_relax : h->opt.relax;
    if (kind == MGRIT_RELAX_FCF) {
        CHK(run_batch(h, l, h->lv[l].crelax, nullptr, warm));
        CHK(f_relax(h, l, 1));
    }
    return 0;
}

// G^(l+1)_k = Phi^(l)_km(U_km-1) - U_km; optionally the squared norm of the residual of every batched
// member (in member order).
int residual(mgrit_handle* h, int l, std::vector<double>* norm2) {
    Level& L = h->lv[l];
    Level& C = h->lv[l + 1];
    CHK(run_batch(h, l, L.resid, C.G, 1));
    const Geom* g = &h->geom;
    Bases B = bases(h, l);
    HIPCHK(launch_zero_slices(g, C.nfirst, C.first_idx, C.G, (void*)h->stream));       // G_0 = 0
    HIPCHK(launch_axpy_slices(g, L.subtract.S, L.subtract.yi, C.G, L.subtract.xi, B.U, -1.0,
                              norm2 ? h->pnorm : nullptr, (void*)h->stream));
    if (norm2) {
        const size_t n = (size_t)L.subtract.S * g->pmax;
        HIPCHK(hipMemcpyAsync(h->h_norm, h->pnorm, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        norm2->clear();
        int s = 0;
        for (int cnt : L.sub_count) {
            double acc = 0.0;
            for (int e = 0; e < cnt; ++e, ++s)
                for (int c = 0; c < g->nchunk; ++c) acc += h->h_norm[(size_t)s * g->pmax + c];
            norm2->push_back(acc);
        }
    }
    return 0;
}

int coarsest_solve(mgrit_handle* h, int l) {
    Level& L = h->lv[l];
    HIPCHK(launch_zero_slices(&h->geom, L.nfirst, L.first_idx, L.U, (void*)h->stream));   // E_0 = G_0 = 0
    for (const Batch& b : L.step_list) CHK(run_batch(h, l, b));
    return 0;
}

int cycle(mgrit_handle* h, int l) {
    Level& L = h->lv[l];
    if (l == (int)h->lv.size() - 1) return coarsest_solve(h, l);
    CHK(relax(h, l, 0));
    CHK(residual(h, l, nullptr));
    Level& C = h->lv[l + 1];
    HIPCHK(launch_zero_slices(&h->geom, (int)C.ns, C.all_idx, C.U, (void*)h->stream));
    CHK(cycle(h, l + 1));
    HIPCHK(launch_axpy_slices(&h->geom, L.correct.S, L.correct.yi, L.U, L.correct.xi, C.U, 1.0, nullptr,
                              (void*)h->stream));
    return f_relax(h, l, 1);
}

// One level-0 correction after the residual has been restricted.
int coarse_correct0(mgrit_handle* h) {
    Level& L = h->lv[0];
    Level& C = h->lv[1];
    HIPCHK(launch_zero_slices(&h->geom, (int)C.ns, C.all_idx, C.U, (void*)h->stream));
    CHK(cycle(h, 1));
    HIPCHK(launch_axpy_slices(&h->geom, L.correct.S, L.correct.yi, h->U0, L.correct.xi, C.U, 1.0, nullptr,
                              (void*)h->stream));
    return 0;
}

// Device staging of the caller's arrays for one call.
struct Staging {
    mgrit_handle* h;
    std::vector<void*> owned;
    ~Staging() {
        for (void* p : owned) (void)hipFree(p);
    }
    int in(const double* src, size_t count, int mem, const double** out) {
        if (!src) {
            *out = nullptr;
            return 0;
        }
        if (mem == MGRIT_MEM_DEVICE) {
            *out = src;
            return 0;
        }
        void* d = nullptr;
        hipError_t e = hipMalloc(&d, count * sizeof(double));
        if (e != hipSuccess) return alloc_failed(e, count * sizeof(double));
        owned.push_back(d);
        HIPCHK(hipMemcpyAsync(d, src, count * sizeof(double), hipMemcpyHostToDevice, h->stream));
        *out = (const double*)d;
        return 0;
    }
    int outbuf(double* dst, size_t count, int mem, double** out) {
        if (mem == MGRIT_MEM_DEVICE) {
            *out = dst;
            return 0;
        }
        void* d = nullptr;
        hipError_t e = hipMalloc(&d, count * sizeof(double));
        if (e != hipSuccess) return alloc_failed(e, count * sizeof(double));
        owned.push_back(d);
        *out = (double*)d;
        return 0;
    }
};

int check_mem(int mem) {
    if (mem != MGRIT_MEM_HOST && mem != MGRIT_MEM_DEVICE) return fail(MGRIT_EINVAL, "mem must be HOST or DEVICE");
    return 0;
}

void fill_stats(mgrit_handle* h, mgrit_stats* st, int iters, int conv, const std::vector<double>& hist) {
    if (!st) return;
    st->iterations = iters;
    st->converged = conv;
    st->levels = (int)h->lv.size();
    st->phi_applications = h->phi_count;
    st->cg_iterations = h->cg_count;
    st->refinements = h->refine_count;
    for (int i = 0; i < 64; ++i) st->residual_history[i] = i < (int)hist.size() ? hist[i] : 0.0;
}

// Common entry of solve / iterate: stage inputs, initialise U.
int begin_solve(mgrit_handle* h, Staging& sg, const double* F, const double* psi0, const double* U_init, double* U,
                int mem, double** dU) {
    CHK(check_mem(mem));
    if (!psi0 || !U) return fail(MGRIT_EINVAL, "psi0 and U must not be NULL");
    const size_t st = (size_t)h->geom.stride;
    const size_t nt1 = (size_t)h->prob.Nt + 1;
    const double *dF, *dpsi, *dinit;
    CHK(sg.in(F, (size_t)h->prob.Nt * st, mem, &dF));
    CHK(sg.in(psi0, st, mem, &dpsi));
    CHK(sg.in(U_init, nt1 * st, mem, &dinit));
    CHK(sg.outbuf(U, nt1 * st, mem, dU));
    if (dinit) {
        if (dinit != *dU)
            HIPCHK(hipMemcpyAsync(*dU + st, dinit + st, (nt1 - 1) * st * sizeof(double), hipMemcpyDeviceToDevice,
                                  h->stream));
    } else {
        HIPCHK(hipMemsetAsync(*dU + st, 0, (nt1 - 1) * st * sizeof(double), h->stream));
    }
    HIPCHK(hipMemcpyAsync(*dU, dpsi, st * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    h->U0 = *dU;
    h->F0 = dF;
    h->cur_rtol = 0.0;
    h->phi_count = 0;
    h->refine_count = 0;
    h->cg_count = 0;
    return 0;
}

int end_solve(mgrit_handle* h, double* U, const double* dU, int mem) {
    if (mem == MGRIT_MEM_HOST) {
        const size_t n = ((size_t)h->prob.Nt + 1) * h->geom.stride;
        HIPCHK(hipMemcpyAsync(U, dU, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    h->U0 = nullptr;
    h->F0 = nullptr;
    return 0;
}

}  // namespace

extern "C" {

void mgrit_default_options(mgrit_options* o) {
    if (!o) return;
    o->m = 8;
    o->max_levels = 30;
    o->relax = MGRIT_RELAX_FCF;
    o->coarse = MGRIT_COARSE_CN;
    o->precision = MGRIT_PREC_FP64;
    o->max_iter = 100;
    o->tol_abs = 1e-9;
    o->tol_rel = 0.0;
    o->cg_rtol = 1e-9;
    o->cg_maxit = 10000;
    o->precond = MGRIT_PRECOND_NONE;
    o->cg_rtol_adapt = 0.0;
    o->warm_start = 1;
    o->divergence_factor = 0.0;
    o->tile_policy = MGRIT_TILE_AUTO;
    o->cg_rtol_coarse = 0.0;
    o->inner_rtol = 0.0;
    o->graphs = 0;
    o->op = MGRIT_OP_AUTO;
    o->coarse_relax = -1;
    o->element = MGRIT_ELEMENT_P1;
}

const char* mgrit_last_error(void) { return g_err; }

}  // extern "C"

namespace {

// Set-up of one problem (group = false) or of several problems on one mesh (group = true).
int setup_impl(const mgrit_problem* probs, int nprob, const mgrit_options* opt, void* stream, mgrit_handle** out,
               bool group) {
    if (!probs || !opt || !out || nprob < 1) return fail(MGRIT_EINVAL, "NULL argument or no problem");
    *out = nullptr;
    for (int q = 0; q < nprob; ++q) {
        const mgrit_problem& p = probs[q];
        if (!(p.beta > 0.5 && p.beta < 1.0) || !(p.gamma > 0.5 && p.gamma < 1.0))
            return fail(MGRIT_EINVAL, "orders must satisfy 1/2 < beta, gamma < 1");
        if (!(p.Kx > 0.0) || !(p.Ky > 0.0)) return fail(MGRIT_EINVAL, "K_x, K_y must be positive");
        if (!(p.a < p.b) || !(p.c < p.d)) return fail(MGRIT_EINVAL, "domain must satisfy a < b, c < d");
        if (p.Mx < 2 || p.My < 2) return fail(MGRIT_EINVAL, "Mx, My must be >= 2");
        if (p.Nt < 1 || !p.t) return fail(MGRIT_EINVAL, "Nt >= 1 and a time grid are required");
        if (p.t[0] != 0.0) return fail(MGRIT_EINVAL, "t[0] must be 0");
        for (int i = 1; i <= p.Nt; ++i)
            if (!(p.t[i] > p.t[i - 1])) return fail(MGRIT_EINVAL, "time grid must increase strictly (index %d)", i);
        if (p.Mx != probs[0].Mx || p.My != probs[0].My || p.a != probs[0].a || p.b != probs[0].b ||
            p.c != probs[0].c || p.d != probs[0].d)
            return fail(MGRIT_EINVAL, "the problems of a group need one mesh and domain (problem %d differs)", q);
    }
    if (group && opt->cg_rtol_adapt > 0.0)
        return fail(MGRIT_EINVAL, "a group takes no adaptive CG tolerance (cg_rtol_adapt = 0)");
    const mgrit_problem& p = probs[0];
    const mgrit_options& o = *opt;
    if (o.m < 2) return fail(MGRIT_EINVAL, "m must be >= 2");
    if (o.max_levels < 2) return fail(MGRIT_EINVAL, "max_levels must be >= 2");
    if (o.relax != MGRIT_RELAX_F && o.relax != MGRIT_RELAX_FCF) return fail(MGRIT_EINVAL, "unknown relaxation");
    if (o.coarse < MGRIT_COARSE_CN || o.coarse > MGRIT_COARSE_OPT)
        return fail(MGRIT_EINVAL, "unknown coarse propagator");
    if (o.coarse == MGRIT_COARSE_OPT && (o.m % 2))
        return fail(MGRIT_EINVAL, "the OPT coarse propagator needs an even coarsening factor");
    if (o.precision < MGRIT_PREC_FP64 || o.precision > MGRIT_PREC_MIXED_BF16)
        return fail(MGRIT_EINVAL, "unknown precision");
    if (o.precision != MGRIT_PREC_FP64 && o.precond == MGRIT_PRECOND_FD)
        return fail(MGRIT_EINVAL, "mixed precision takes precond NONE or FD_BF16");
    if (!(o.inner_rtol >= 0.0 && o.inner_rtol < 1.0)) return fail(MGRIT_EINVAL, "bad inner_rtol");
    if (o.graphs != 0 && o.graphs != 1) return fail(MGRIT_EINVAL, "graphs must be 0 or 1");
    if (o.op < MGRIT_OP_AUTO || o.op > MGRIT_OP_FFT) return fail(MGRIT_EINVAL, "unknown operator kind");
    if (o.coarse_relax != -1 && o.coarse_relax != MGRIT_RELAX_F && o.coarse_relax != MGRIT_RELAX_FCF)
        return fail(MGRIT_EINVAL, "unknown coarse relaxation");
    if (o.element != MGRIT_ELEMENT_P1 && o.element != MGRIT_ELEMENT_Q1) return fail(MGRIT_EINVAL, "unknown element");
    if (o.precond < MGRIT_PRECOND_NONE || o.precond > MGRIT_PRECOND_FD_BF16)
        return fail(MGRIT_EINVAL, "unknown preconditioner");
    if (!(o.cg_rtol_coarse >= 0.0 && o.cg_rtol_coarse < 1.0)) return fail(MGRIT_EINVAL, "bad cg_rtol_coarse");
    if (o.tile_policy < MGRIT_TILE_AUTO || o.tile_policy > MGRIT_TILE_32)
        return fail(MGRIT_EINVAL, "unknown tile policy");
    if (o.max_iter < 1 || o.cg_maxit < 1 || !(o.cg_rtol > 0.0) || !(o.tol_abs >= 0.0) || !(o.tol_rel >= 0.0) ||
        !(o.cg_rtol_adapt >= 0.0) || (o.warm_start != 0 && o.warm_start != 1))
        return fail(MGRIT_EINVAL, "bad iteration limits or tolerances");
    const long long nx = p.Mx - 1, ny = p.My - 1;
    if (nx * ny > (1LL << 30)) return fail(MGRIT_EINVAL, "grid too large");

    mgrit_handle* h = new (std::nothrow) mgrit_handle();
    if (!h) return fail(MGRIT_ENOMEM, "host allocation failed");
    h->opt = o;
    h->mem.resize(nprob);
    for (int q = 0; q < nprob; ++q) {
        Member& M = h->mem[q];
        M.prob = probs[q];
        M.t.assign(probs[q].t, probs[q].t + probs[q].Nt + 1);
        M.prob.t = M.t.data();
    }
    h->t = h->mem[0].t;
    h->prob = h->mem[0].prob;
    h->prob.t = h->t.data();
    h->stream = (hipStream_t)stream;
    Geom& g = h->geom;
    g.nx = (int)nx;
    g.ny = (int)ny;
    for (int v = 0; v < 2; ++v) {
        const int TT = v == 0 ? 64 : 32;
        g.tiles_x[v] = (g.nx + TT - 1) / TT;
        g.tiles_y[v] = (g.ny + TT - 1) / TT;
        g.ntiles[v] = g.tiles_x[v] * g.tiles_y[v];
    }
    g.stride = nx * ny;
    g.nchunk = (int)((g.stride + MGRIT_CHUNK - 1) / MGRIT_CHUNK);
    g.pmax = std::max(g.ntiles[1], g.nchunk);
    const bool fft_fits = 2 * nx - 1 <= MGRIT_FFT_LEN && 2 * ny - 1 <= MGRIT_FFT_LEN;
    if (o.op == MGRIT_OP_FFT && !fft_fits) {
        delete h;
        return fail(MGRIT_EINVAL, "the FFT operator takes n_x, n_y <= %d", (MGRIT_FFT_LEN + 1) / 2);
    }
    {   // the device current at set-up, and its scratch array (once per device)
        const hipError_t e = hipGetDevice(&h->device);
        int rc0 = e == hipSuccess ? 0 : fail(MGRIT_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
        if (!rc0) rc0 = scratch_address(h->device, &h->scratch);
        if (rc0) {
            delete h;
            return rc0;
        }
    }
    h->use_fft = o.op == MGRIT_OP_FFT || (o.op == MGRIT_OP_AUTO && fft_fits);
    const int fft_nby = (int)((nx + MGRIT_FFT_LINES - 1) / MGRIT_FFT_LINES);    // y-pass workgroups
    const int fft_nbx = (int)((ny + MGRIT_FFT_LINES - 1) / MGRIT_FFT_LINES);    // x-pass workgroups
    if (h->use_fft) g.pmax = std::max(g.pmax, fft_nby + fft_nbx);
    h->nop = h->use_fft ? fft_nby : g.ntiles[1];
    h->nop_pq = h->use_fft ? fft_nby + fft_nbx : g.ntiles[1];
    g.seq_off_x = g.tiles_x[0] * 64 + 64 + MGRIT_KC;
    g.seq_off_y = g.tiles_y[0] * 64 + 64 + MGRIT_KC;
    g.q1 = o.element == MGRIT_ELEMENT_Q1 ? 1 : 0;
    g.pad_ = 0;
    g.mass = ((p.b - p.a) / p.Mx) * ((p.d - p.c) / p.My) / (g.q1 ? 36.0 : 12.0);
    int rc = build_sequences(h);
    if (!rc && h->use_fft) rc = build_fft_plan(h);
    if (!rc && o.precond != MGRIT_PRECOND_NONE) rc = build_fd(h);
    if (!rc) rc = build_levels(h);
    if (!rc) rc = alloc_workspace(h, h->Smax);
    if (!rc && group) {
        long long nf = 0;
        for (const Member& M : h->mem) nf += M.prob.Nt;
        rc = dalloc(h, &h->gU, (size_t)h->lv[0].ns * h->geom.stride);
        if (!rc) rc = dalloc(h, &h->gF, (size_t)nf * h->geom.stride);
    }
    if (rc) {
        mgrit_destroy(h);
        return rc;
    }
    *out = h;
    return MGRIT_OK;
}

}  // namespace

extern "C" {

int mgrit_setup(const mgrit_problem* prob, const mgrit_options* opt, void* stream, mgrit_handle** out) {
    return setup_impl(prob, 1, opt, stream, out, false);
}

int mgrit_setup_group(const mgrit_problem* probs, int nprob, const mgrit_options* opt, void* stream,
                      mgrit_handle** out) {
    return setup_impl(probs, nprob, opt, stream, out, true);
}

int mgrit_solve_group(mgrit_handle* h, const double* const* F, const double* const* psi0, double* const* U, int mem,
                      mgrit_stats* st) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    if (!h->gU) return fail(MGRIT_EINVAL, "the handle was not set up by mgrit_setup_group");
    CHK(check_mem(mem));
    const int P = (int)h->mem.size();
    if (!psi0 || !U) return fail(MGRIT_EINVAL, "psi0 and U must not be NULL");
    for (int p = 0; p < P; ++p)
        if (!psi0[p] || !U[p]) return fail(MGRIT_EINVAL, "psi0[%d] and U[%d] must not be NULL", p, p);
    const size_t st1 = (size_t)h->geom.stride;
    const hipMemcpyKind in = mem == MGRIT_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int p = 0; p < P; ++p) {       // the members' loads and initial values into the group's arrays
        const Member& M = h->mem[p];
        double* f = h->gF + (size_t)M.f_off * st1;
        if (F && F[p]) HIPCHK(hipMemcpyAsync(f, F[p], (size_t)M.prob.Nt * st1 * sizeof(double), in, h->stream));
        else HIPCHK(hipMemsetAsync(f, 0, (size_t)M.prob.Nt * st1 * sizeof(double), h->stream));
        double* u = h->gU + (size_t)M.off[0] * st1;
        HIPCHK(hipMemcpyAsync(u, psi0[p], st1 * sizeof(double), in, h->stream));
        HIPCHK(hipMemsetAsync(u + st1, 0, (size_t)M.prob.Nt * st1 * sizeof(double), h->stream));
    }
    h->U0 = h->gU;
    h->F0 = h->gF;
    h->cur_rtol = 0.0;
    h->phi_count = h->cg_count = h->refine_count = 0;
    const double hxy = ((h->prob.b - h->prob.a) / h->prob.Mx) * ((h->prob.d - h->prob.c) / h->prob.My);
    std::vector<std::vector<double>> hist(P);
    std::vector<int> its(P, 0), conv(P, 0), div(P, 0);
    bool all = true;
    for (char b : h->batched) all = all && b;
    if (!all) {
        h->batched.assign(P, 1);
        CHK(build_batches(h));
    }
    // MGRIT iterations of every member still iterating, their sweeps in shared batches; a member leaves
    // the batches when its own stop test (or divergence guard) ends its solve, as it would alone
    int it = 0;
    while (it < h->opt.max_iter) {
        CHK(relax(h, 0, it > 0 ? 1 : 0));
        std::vector<double> n2;
        CHK(residual(h, 0, &n2));
        bool changed = false;
        int k = 0;
        for (int p = 0; p < P; ++p) {
            if (!h->batched[p]) continue;
            const double norm = std::sqrt(hxy * n2[k++]);
            hist[p].push_back(norm);
            if (norm < h->opt.tol_abs || norm < h->opt.tol_rel * hist[p][0]) conv[p] = 1;
            else if (h->opt.divergence_factor > 0.0 && norm > h->opt.divergence_factor * hist[p][0]) div[p] = 1;
            else ++its[p];
            if (conv[p] || div[p]) {
                h->batched[p] = 0;
                changed = true;
            }
        }
        ++it;
        int left = 0;
        for (char b : h->batched) left += b;
        if (left == 0) break;
        if (changed) CHK(build_batches(h));
        CHK(coarse_correct0(h));
    }
    // members without convergence end with an F-relaxation (Remark 3.1)
    std::vector<char> fin(P, 0);
    bool any = false;
    for (int p = 0; p < P; ++p) {
        fin[p] = !conv[p];
        any = any || fin[p];
    }
    if (any) {
        if (h->batched != fin) {
            h->batched = fin;
            CHK(build_batches(h));
        }
        CHK(f_relax(h, 0, 1));
    }
    const hipMemcpyKind outk = mem == MGRIT_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int p = 0; p < P; ++p) {
        const Member& M = h->mem[p];
        HIPCHK(hipMemcpyAsync(U[p], h->gU + (size_t)M.off[0] * st1, ((size_t)M.prob.Nt + 1) * st1 * sizeof(double),
                              outk, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    h->U0 = nullptr;
    h->F0 = nullptr;
    int rc = MGRIT_OK;
    for (int p = 0; p < P; ++p) {
        if (st) fill_stats(h, &st[p], its[p], conv[p], hist[p]);
        if (div[p]) rc = MGRIT_EDIVERGED;
        else if (!conv[p] && rc == MGRIT_OK) rc = MGRIT_ENOCONV;
    }
    if (rc == MGRIT_EDIVERGED) return fail(rc, "a residual norm grew beyond the divergence guard");
    if (rc == MGRIT_ENOCONV) return fail(rc, "no convergence in %d iterations", h->opt.max_iter);
    return MGRIT_OK;
}

}  // extern "C"

extern "C" {

void mgrit_destroy(mgrit_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (void* p : h->allocations) (void)hipFree(p);
    for (void* p : h->batch_allocs) (void)hipFree(p);
    for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->tune_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    if (h->h_flags) (void)hipHostFree(h->h_flags);
    if (h->h_start) (void)hipHostFree(h->h_start);
    for (hipEvent_t e : h->flag_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->h_iters) (void)hipHostFree(h->h_iters);
    if (h->h_iters_step) (void)hipHostFree(h->h_iters_step);
    if (h->h_norm) (void)hipHostFree(h->h_norm);
    delete h;
}

int mgrit_solve(mgrit_handle* h, const double* F, const double* psi0, const double* U_init, double* U, int mem,
                mgrit_stats* st) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    Staging sg{h};
    double* dU = nullptr;
    CHK(begin_solve(h, sg, F, psi0, U_init, U, mem, &dU));
    const double hxy = ((h->prob.b - h->prob.a) / h->prob.Mx) * ((h->prob.d - h->prob.c) / h->prob.My);
    std::vector<double> hist;
    int it = 0, conv = 0, diverged = 0;
    while (it < h->opt.max_iter) {
        if (h->opt.cg_rtol_adapt > 0.0) {
            const double rho = hist.empty() ? 1.0 : hist.back() / hist[0];
            h->cur_rtol = std::min(1e-4, std::max(h->opt.cg_rtol, h->opt.cg_rtol_adapt * rho));
        }
        CHK(relax(h, 0, it > 0 ? 1 : 0));
        std::vector<double> n2;
        CHK(residual(h, 0, &n2));
        const double norm = std::sqrt(hxy * n2[0]);
        hist.push_back(norm);
        if (norm < h->opt.tol_abs || norm < h->opt.tol_rel * hist[0]) {
            conv = 1;
            break;
        }
        if (h->opt.divergence_factor > 0.0 && norm > h->opt.divergence_factor * hist[0]) {
            diverged = 1;
            break;
        }
        ++it;
        CHK(coarse_correct0(h));
    }
    if (!conv) {
        h->cur_rtol = 0.0;
        CHK(f_relax(h, 0, 1));
    }
    h->cur_rtol = 0.0;
    CHK(end_solve(h, U, dU, mem));
    fill_stats(h, st, it, conv, hist);
    if (diverged) return fail(MGRIT_EDIVERGED, "residual norm grew beyond the divergence guard");
    if (!conv) return fail(MGRIT_ENOCONV, "no convergence in %d iterations", h->opt.max_iter);
    return MGRIT_OK;
}

int mgrit_iterate(mgrit_handle* h, const double* F, const double* psi0, const double* U_init, int iterations,
                  double* U, int mem, mgrit_stats* st) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    if (iterations < 0) return fail(MGRIT_EINVAL, "iterations must be >= 0");
    Staging sg{h};
    double* dU = nullptr;
    CHK(begin_solve(h, sg, F, psi0, U_init, U, mem, &dU));
    std::vector<double> hist;
    for (int i = 0; i < iterations; ++i) {
        CHK(relax(h, 0, i > 0 ? 1 : 0));
        CHK(residual(h, 0, nullptr));
        CHK(coarse_correct0(h));
    }
    CHK(f_relax(h, 0, iterations > 0 ? 1 : 0));
    CHK(end_solve(h, U, dU, mem));
    fill_stats(h, st, iterations, 0, hist);
    return MGRIT_OK;
}

int mgrit_sequential(mgrit_handle* h, const double* F, const double* psi0, double* U, int mem, mgrit_stats* st) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    Staging sg{h};
    double* dU = nullptr;
    CHK(begin_solve(h, sg, F, psi0, nullptr, U, mem, &dU));
    for (int k = 1; k <= h->prob.Nt; ++k) CHK(run_batch(h, 0, h->lv[0].step_list[k - 1]));
    CHK(end_solve(h, U, dU, mem));
    std::vector<double> hist;
    fill_stats(h, st, 0, 1, hist);
    return MGRIT_OK;
}

int mgrit_propagate(mgrit_handle* h, int level, const int* step, int nslices, const double* u_in, const double* g,
                    double* u_out, int mem) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    CHK(check_mem(mem));
    if (level < 0 || level >= (int)h->lv.size()) return fail(MGRIT_EINVAL, "level out of range");
    if (nslices < 0 || (nslices > 0 && (!step || !u_in || !u_out))) return fail(MGRIT_EINVAL, "bad slices");
    if (nslices == 0) return MGRIT_OK;
    for (int s = 0; s < nslices; ++s)
        if (step[s] < 1 || step[s] > h->mem[0].N[level])
            return fail(MGRIT_EINVAL, "step index %d out of range", step[s]);
    const size_t st = (size_t)h->geom.stride;
    Staging sg{h};
    const double *du, *dg;
    double* dout;
    CHK(sg.in(u_in, nslices * st, mem, &du));
    CHK(sg.in(g, nslices * st, mem, &dg));
    CHK(sg.outbuf(u_out, nslices * st, mem, &dout));
    h->cur_level = level;
    for (int s0 = 0; s0 < nslices; s0 += h->Smax) {
        const int S = std::min(h->Smax, nslices - s0);
        Batch b;
        for (int s = 0; s < S; ++s) {
            Batch one;
            make_step(h, 0, level, step[s0 + s], s, s, s, one);
            for (int pi = 0; pi < one.npass; ++pi) {
                PropDesc d = one.pass[pi].h[0];
                if (level == 0) d.f = dg ? s : -1;
                else if (pi == one.npass - 1) d.g = dg ? s : -1;
                b.pass[pi].h.push_back(d);
            }
            b.npass = one.npass;
        }
        Staging descs{h};
        for (int pi = 0; pi < b.npass; ++pi) {
            Pass& ps = b.pass[pi];
            ps.S = S;
            void* d = nullptr;
            hipError_t e = hipMalloc(&d, S * sizeof(PropDesc));
            if (e != hipSuccess) return alloc_failed(e, S * sizeof(PropDesc));
            descs.owned.push_back(d);
            ps.d = (PropDesc*)d;
            HIPCHK(hipMemcpyAsync(ps.d, ps.h.data(), S * sizeof(PropDesc), hipMemcpyHostToDevice, h->stream));
        }
        const double* ub = du + s0 * st;
        double* ob = dout + s0 * st;
        const double* gb = dg ? dg + s0 * st : nullptr;
        if (b.npass == 1) {
            CHK(run_pass(h, b.pass[0], ub, ob, level == 0 ? gb : nullptr, level == 0 ? nullptr : gb));
        } else {
            CHK(run_pass(h, b.pass[0], ub, h->tmp, nullptr, nullptr));
            CHK(run_pass(h, b.pass[1], h->tmp, ob, nullptr, gb));
        }
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    if (mem == MGRIT_MEM_HOST)
        HIPCHK(hipMemcpyAsync(u_out, dout, nslices * st * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return MGRIT_OK;
}

int mgrit_apply(mgrit_handle* h, int nslices, const double* theta, double sign, const double* v, const double* add,
                double* out, int mem) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    CHK(check_mem(mem));
    if (nslices < 0 || (nslices > 0 && (!theta || !v || !out))) return fail(MGRIT_EINVAL, "bad slices");
    if (sign != 1.0 && sign != -1.0) return fail(MGRIT_EINVAL, "sign must be +1 or -1");
    if (nslices == 0) return MGRIT_OK;
    const size_t st = (size_t)h->geom.stride;
    Staging sg{h};
    const double *dv, *da;
    double* dout;
    CHK(sg.in(v, nslices * st, mem, &dv));
    CHK(sg.in(add, nslices * st, mem, &da));
    CHK(sg.outbuf(out, nslices * st, mem, &dout));
    std::vector<ApplyDesc> hd(nslices);
    for (int s = 0; s < nslices; ++s) {
        hd[s].v = s;
        hd[s].out = s;
        hd[s].add = da ? s : -1;
        hd[s].pad_ = 0;
        hd[s].theta = theta[s];
    }
    void* dd = nullptr;
    hipError_t e = hipMalloc(&dd, nslices * sizeof(ApplyDesc));
    if (e != hipSuccess) return alloc_failed(e, nslices * sizeof(ApplyDesc));
    sg.owned.push_back(dd);
    HIPCHK(hipMemcpyAsync(dd, hd.data(), nslices * sizeof(ApplyDesc), hipMemcpyHostToDevice, h->stream));
    int tv = 0;
    CHK(tile_variant(h, nullptr, nslices, &tv));
    if (h->use_fft) {
        for (int s0 = 0; s0 < nslices; s0 += h->Smax)        // the x-pass workspace holds Smax slices
            HIPCHK(launch_fft_apply(&h->geom, &h->plan, (const ApplyDesc*)dd + s0, std::min(h->Smax, nslices - s0),
                                    dv, dout, da, sign, 0, nullptr, h->pfft, (void*)h->stream));
    } else {
        HIPCHK(launch_apply(&h->geom, &h->seqs, tv, (const ApplyDesc*)dd, nslices, dv, dout, da, sign, 0, nullptr,
                            nullptr, (void*)h->stream));
    }
    if (mem == MGRIT_MEM_HOST)
        HIPCHK(hipMemcpyAsync(out, dout, nslices * st * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return MGRIT_OK;
}

}  // extern "C"

namespace {

// FP32 operator forms of the inner solves of mixed precision.  kind 0: out32 = M v32 + theta A v32 (the
// inner CG operator); kind 1: out32 = M u + theta A u + add (FP64 u and add rounded on load: the
// right-hand side of a loose pass); kind 2: out32 = add32 - (M u + theta A u) (FP64 u, FP32 add: the
// initial residual of a loose pass).
int apply_f32(mgrit_handle* h, int kind, int nslices, const double* theta, const void* v, const void* add,
              float* out, int mem) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    CHK(check_mem(mem));
    if (h->opt.precision == MGRIT_PREC_FP64)
        return fail(MGRIT_EINVAL, "the FP32 operator tables exist only in handles set up for mixed precision");
    if (kind > 0 && !h->use_fft)
        return fail(MGRIT_EINVAL, "FP32 right-hand sides and residuals are formed by the FFT operator only");
    if (nslices < 0 || (nslices > 0 && (!theta || !v || !out))) return fail(MGRIT_EINVAL, "bad slices");
    if (kind == 2 && nslices > 0 && !add) return fail(MGRIT_EINVAL, "the residual needs its right-hand side");
    if (nslices == 0) return MGRIT_OK;
    const size_t st = (size_t)h->geom.stride;
    const size_t wv = kind == 0 ? 4 : 8, wa = kind == 1 ? 8 : 4;
    std::vector<void*> owned;
    struct Free {
        std::vector<void*>& o;
        ~Free() {
            for (void* p : o) (void)hipFree(p);
        }
    } fr{owned};
    auto stage = [&](const void* src, size_t bytes, bool copy, void** dst) -> int {
        if (mem == MGRIT_MEM_DEVICE || !src) {
            *dst = (void*)src;
            return 0;
        }
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return alloc_failed(e, bytes);
        owned.push_back(*dst);
        if (copy) HIPCHK(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, h->stream));
        return 0;
    };
    void *dv = nullptr, *da = nullptr, *dout = nullptr;
    CHK(stage(v, nslices * st * wv, true, &dv));
    CHK(stage(add, nslices * st * wa, true, &da));
    CHK(stage(out, nslices * st * 4, false, &dout));
    const int chunk = h->Smax;              // the operator workspaces and partials hold Smax slices
    void* ddesc = nullptr;
    hipError_t e = hipMalloc(&ddesc, std::min(chunk, nslices) * sizeof(PropDesc));
    if (e != hipSuccess) return alloc_failed(e, std::min(chunk, nslices) * sizeof(PropDesc));
    owned.push_back(ddesc);
    std::vector<PropDesc> hd;
    const Geom* g = &h->geom;
    for (int s0 = 0; s0 < nslices; s0 += chunk) {
        const int S = std::min(chunk, nslices - s0);
        hd.assign(S, PropDesc());
        for (int s = 0; s < S; ++s) {
            hd[s].u = s;
            hd[s].x = s;
            hd[s].f = (kind == 1 && da) ? s : -1;
            hd[s].g = -1;
            hd[s].x0 = -1;
            hd[s].theta_rhs = theta[s0 + s];
            hd[s].theta_lhs = theta[s0 + s];
        }
        HIPCHK(hipMemcpyAsync(ddesc, hd.data(), S * sizeof(PropDesc), hipMemcpyHostToDevice, h->stream));
        const PropDesc* d = (const PropDesc*)ddesc;
        const char* vb = (const char*)dv + s0 * st * wv;
        const char* ab = da ? (const char*)da + s0 * st * wa : nullptr;
        float* ob = (float*)dout + s0 * st;
        if (kind == 0) {
            int tv = 0;
            CHK(tile_variant(h, nullptr, S, &tv));
            if (h->opt.precision == MGRIT_PREC_MIXED_BF16)
                HIPCHK(launch_apply_bf16(g, &h->seqs32, d, S, (const float*)vb, ob, h->ppq, nullptr, h->stream));
            else if (h->use_fft)
                HIPCHK(launch_fft_apply32(g, &h->plan, d, S, (const float*)vb, ob, h->ppq, nullptr, h->pfft32,
                                          h->stream));
            else
                HIPCHK(launch_apply32(g, &h->seqs32, tv, d, S, (const float*)vb, ob, h->ppq, nullptr, h->stream));
        } else if (kind == 1) {
            HIPCHK(launch_fft_rhs32(g, &h->plan, d, S, (const double*)vb, (const double*)ab, ob, h->pbb, h->pfft32,
                                    h->stream));
        } else {
            HIPCHK(launch_fft_init_residual32(g, &h->plan, d, S, (const double*)vb, (const float*)ab, ob, h->pout,
                                              h->pfft32, h->stream));
        }
    }
    if (mem == MGRIT_MEM_HOST)
        HIPCHK(hipMemcpyAsync(out, dout, nslices * st * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return MGRIT_OK;
}

}  // namespace

extern "C" {

int mgrit_apply_noalloc(mgrit_handle* h, int nslices, const double* theta, double sign, const double* v,
                        const double* add, double* out) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    if (nslices < 0 || (nslices > 0 && (!theta || !v || !out))) return fail(MGRIT_EINVAL, "bad slices");
    if (sign != 1.0 && sign != -1.0) return fail(MGRIT_EINVAL, "sign must be +1 or -1");
    if (nslices == 0) return MGRIT_OK;
    const size_t desc_bytes = ((size_t)nslices * sizeof(ApplyDesc) + 255) / 256 * 256;
    const size_t ws_bytes = h->use_fft ? (size_t)nslices * h->geom.stride * sizeof(double) : 0;
    if (desc_bytes + ws_bytes > (size_t)MGRIT_NOALLOC_SCRATCH_BYTES)
        return fail(MGRIT_EINVAL, "%d slices need %zu bytes of scratch, more than its %zu bytes", nslices,
                    desc_bytes + ws_bytes, (size_t)MGRIT_NOALLOC_SCRATCH_BYTES);
    ApplyDesc* d = (ApplyDesc*)h->scratch;
    double* pbuf = (double*)((char*)h->scratch + desc_bytes);
    HIPCHK(launch_fill_apply_desc(nslices, theta, add ? 1 : 0, d, h->stream));
    if (h->use_fft) {
        HIPCHK(launch_fft_apply(&h->geom, &h->plan, d, nslices, v, out, add, sign, 0, nullptr, pbuf, h->stream));
    } else {
        int tv = 0;
        CHK(tile_variant(h, nullptr, nslices, &tv));
        HIPCHK(launch_apply(&h->geom, &h->seqs, tv, d, nslices, v, out, add, sign, 0, nullptr, nullptr, h->stream));
    }
    return MGRIT_OK;
}

int mgrit_apply_f32(mgrit_handle* h, int nslices, const double* theta, const float* v, float* out, int mem) {
    return apply_f32(h, 0, nslices, theta, v, nullptr, out, mem);
}

int mgrit_rhs_f32(mgrit_handle* h, int nslices, const double* theta, const double* u, const double* f, float* b,
                  int mem) {
    return apply_f32(h, 1, nslices, theta, u, f, b, mem);
}

int mgrit_residual_f32(mgrit_handle* h, int nslices, const double* theta, const double* x, const float* b, float* r,
                       int mem) {
    return apply_f32(h, 2, nslices, theta, x, b, r, mem);
}

int mgrit_sequences(const mgrit_handle* h, double* seq_x, double* seq_y, double* cx, double* cy) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    if (seq_x) std::memcpy(seq_x, h->host_seq_x.data(), h->host_seq_x.size() * sizeof(double));
    if (seq_y) std::memcpy(seq_y, h->host_seq_y.data(), h->host_seq_y.size() * sizeof(double));
    if (cx) *cx = h->cx;
    if (cy) *cy = h->cy;
    return MGRIT_OK;
}

int mgrit_profile_enable(mgrit_handle* h, int on) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    HIPCHK(hipStreamSynchronize(h->stream));
    h->prof_on = on != 0;
    h->prof_used = 0;
    for (int v = 0; v < MGRIT_PROF_CLASSES; ++v) {
        h->prof_ms[v] = 0.0;
        h->prof_launches[v] = 0;
        h->prof_slices[v] = 0;
    }
    return MGRIT_OK;
}

int mgrit_profile_read(const mgrit_handle* h, int variant, double* apply_ms, long long* launches,
                       long long* slice_applies) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    if (variant < 0 || variant >= MGRIT_PROF_CLASSES)
        return fail(MGRIT_EINVAL, "kernel class must be 0..%d", MGRIT_PROF_CLASSES - 1);
    if (apply_ms) *apply_ms = h->prof_ms[variant];
    if (launches) *launches = h->prof_launches[variant];
    if (slice_applies) *slice_applies = h->prof_slices[variant];
    return MGRIT_OK;
}

int mgrit_device_bytes(const mgrit_handle* h, size_t* bytes) {
    if (!h || !bytes) return fail(MGRIT_EINVAL, "NULL argument");
    *bytes = h->dev_bytes;
    return MGRIT_OK;
}

int mgrit_footprint(const mgrit_problem* p, const mgrit_options* o, int mem, size_t* bytes) {
    if (!p || !o || !bytes) return fail(MGRIT_EINVAL, "NULL argument");
    if (p->Mx < 2 || p->My < 2 || p->Nt < 1 || o->m < 2 || o->max_levels < 2)
        return fail(MGRIT_EINVAL, "bad sizes");
    const double nx = p->Mx - 1, ny = p->My - 1, st = nx * ny;
    const double tx0 = std::ceil(nx / 64), ty0 = std::ceil(ny / 64);
    const double npx = tx0 * 64, npy = ty0 * 64;
    const double nt1 = std::ceil(nx / 32) * std::ceil(ny / 32), nch = std::ceil(st / MGRIT_CHUNK);
    const double pmax = std::max(nt1, nch);
    std::vector<int> N(1, p->Nt);
    while ((int)N.size() < o->max_levels && N.back() / o->m >= 2) N.push_back(N.back() / o->m);
    double smax = 1, d = 0;                                  // d: doubles
    double desc = 0;                                         // descriptor and index bytes
    const bool two = o->coarse == MGRIT_COARSE_CN2 || o->coarse == MGRIT_COARSE_OPT;
    for (size_t l = 0; l < N.size(); ++l) {
        if (l > 0) d += 2.0 * (N[l] + 1) * st;
        desc += 4.0 * (N[l] + 1) + 48.0 * (two ? 2 : 1) * (3.0 * N[l] + 4);
        if (l + 1 < N.size()) smax = std::max(smax, std::max((double)((N[l] - 1) / o->m + 1), (double)N[l + 1]));
    }
    const bool pc = o->precond != MGRIT_PRECOND_NONE;
    d += 2 * (2 * (npx + 96) + 1) + 2 * (2 * (npy + 96) + 1);                       // sequences
    d += smax * st * (4 + (two ? 1 : 0) + (pc ? 1 : 0) + (o->precond == MGRIT_PRECOND_FD ? 2 : 0));
    d += smax * pmax * (5 + (pc ? 2 : 0)) + smax * 3;
    double b = 0;
    if (pc) d += 2 * nx * nx + 2 * ny * ny + nx + ny;
    if (o->precond == MGRIT_PRECOND_FD_BF16) b += 4 * npx * npx + 4 * npy * npy + 4 * (npx + npy) + 4 * smax * npx * npy;
    if (o->precond == MGRIT_PRECOND_FD_BF16 && o->precision != MGRIT_PREC_FP64) b += 2 * smax * npx * npy;  // r image
    if (mem == MGRIT_MEM_HOST) d += (2.0 * p->Nt + 2) * st;
    const bool fft = o->op == MGRIT_OP_FFT ||
                     (o->op == MGRIT_OP_AUTO && 2 * nx - 1 <= MGRIT_FFT_LEN && 2 * ny - 1 <= MGRIT_FFT_LEN);
    if (fft) {
        d += smax * st + 14.0 * MGRIT_FFT_LEN +                                       // x-pass ws, tables
             smax * (std::ceil(nx / MGRIT_FFT_LINES) + std::ceil(ny / MGRIT_FFT_LINES)) * 7;   // partials
        if (o->precision != MGRIT_PREC_FP64) b += 4.0 * smax * st + 4.0 * 14 * MGRIT_FFT_LEN;
    }
    if (o->precision != MGRIT_PREC_FP64) {
        b += 4.0 * (2 * (npx + 96) + 1) * 2 + 4.0 * (2 * (npy + 96) + 1) * 2;          // FP32 sequences
        b += 4.0 * 5 * smax * st + 32.0 * smax;                                        // FP32 workspace, flags
        d += smax * pmax * (pc ? 1 : 3);                                                // partials
    }
    const double total = 8 * d + b + desc + smax * 12;
    *bytes = (size_t)(total * 1.02) + (size_t)64 * 4096;
    return MGRIT_OK;
}

int mgrit_levels(const mgrit_handle* h, int* n_per_level, int cap) {
    if (!h) return fail(MGRIT_EINVAL, "NULL handle");
    const int L = (int)h->lv.size();
    for (int l = 0; l < L && l < cap; ++l) n_per_level[l] = h->mem[0].N[l] + 1;
    return L;
}

}  // extern "C"
