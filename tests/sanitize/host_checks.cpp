// Host-side checks of libmgrit built with AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed):
// the binary128 Toeplitz sequences and the eigen-decompositions of the preconditioner set-up, argument
// validation of every entry point that fails before touching the device, the footprint estimate and
// the server's validation.  Exits non-zero on a failed check; the sanitizers abort on their findings.
#include <cmath>
#include <cstdio>
#include <vector>

#include "mgrit.h"

static int failures = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            std::printf("check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                               \
        }                                                             \
    } while (0)

int main() {
    // sequences: A_2 sub- and super-diagonal entries of distance l + 1 and l agree (w_m = u_{m+1})
    for (int n : {1, 2, 3, 17, 300}) {
        std::vector<double> t(n), u(n), w(n);
        mgrit_toeplitz_sequences(0.7, n, t.data(), u.data(), w.data());
        for (int l = 1; l + 1 < n; ++l) CHECK(std::fabs(w[l] - u[l + 1]) <= 1e-12 * std::fabs(u[l + 1]) + 1e-300);
        CHECK(std::isfinite(t[0]) && t[0] != 0.0 && std::isfinite(u[0]));
    }
    // K v = lambda M v with M = h I: V^T (h I) V = I and residuals small
    for (int n : {1, 5, 64, 129}) {
        const double h = 1.0 / (n + 1), K = 1.3;
        std::vector<double> V((size_t)n * n), lam(n);
        CHECK(mgrit_fd_eigen(0.65, n, h, K, V.data(), lam.data()) == 0);
        double orth = 0.0, res = 0.0, scale = 0.0;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += V[(size_t)k * n + i] * h * V[(size_t)k * n + j];
                orth = std::fmax(orth, std::fabs(s - (i == j ? 1.0 : 0.0)));
            }
            for (int r = 0; r < n; ++r) {
                double kv = 0.0;
                for (int k = 0; k < n; ++k) kv += mgrit_fd_stiffness_entry(0.65, h, K, std::abs(r - k)) * V[(size_t)k * n + i];
                res = std::fmax(res, std::fabs(kv - lam[i] * h * V[(size_t)r * n + i]));
                scale = std::fmax(scale, std::fabs(lam[i] * h * V[(size_t)r * n + i]));
            }
        }
        CHECK(orth <= 1e-10);
        CHECK(res <= 1e-9 * scale);
    }
    // validation before any device work
    std::vector<double> t(65);
    for (int i = 0; i <= 64; ++i) t[i] = i / 64.0;
    const mgrit_problem good{0.7, 0.8, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, 40, 30, 64, t.data()};
    mgrit_options o;
    mgrit_default_options(&o);
    mgrit_handle* h = nullptr;
    auto setup_rc = [&](mgrit_problem p, mgrit_options q) { return mgrit_setup(&p, &q, nullptr, &h); };
    mgrit_problem p = good;
    p.beta = 0.5;
    CHECK(setup_rc(p, o) == MGRIT_EINVAL && h == nullptr);
    p = good;
    p.Ky = 0.0;
    CHECK(setup_rc(p, o) == MGRIT_EINVAL);
    p = good;
    p.c = 2.0;
    CHECK(setup_rc(p, o) == MGRIT_EINVAL);
    p = good;
    p.Mx = 1;
    CHECK(setup_rc(p, o) == MGRIT_EINVAL);
    std::vector<double> tb(t);
    tb[10] = tb[9];
    p = good;
    p.t = tb.data();
    CHECK(setup_rc(p, o) == MGRIT_EINVAL);
    mgrit_options q = o;
    q.m = 1;
    CHECK(setup_rc(good, q) == MGRIT_EINVAL);
    q = o;
    q.coarse = MGRIT_COARSE_OPT;
    q.m = 3;
    CHECK(setup_rc(good, q) == MGRIT_EINVAL);
    q = o;
    q.precision = 9;
    CHECK(setup_rc(good, q) == MGRIT_EINVAL);
    q = o;
    q.precision = MGRIT_PREC_MIXED_BF16;
    q.precond = MGRIT_PRECOND_FD;
    CHECK(setup_rc(good, q) == MGRIT_EINVAL);
    CHECK(mgrit_last_error()[0] != '\0');
    CHECK(mgrit_setup(nullptr, &o, nullptr, &h) == MGRIT_EINVAL);
    CHECK(mgrit_solve(nullptr, nullptr, nullptr, nullptr, nullptr, MGRIT_MEM_DEVICE, nullptr) == MGRIT_EINVAL);
    CHECK(mgrit_apply_noalloc(nullptr, 1, nullptr, 1.0, nullptr, nullptr, nullptr) == MGRIT_EINVAL);
    CHECK(mgrit_apply_f32(nullptr, 1, nullptr, nullptr, nullptr, MGRIT_MEM_HOST) == MGRIT_EINVAL);
    // footprint grows with the problem
    size_t b1 = 0, b2 = 0;
    CHECK(mgrit_footprint(&good, &o, MGRIT_MEM_DEVICE, &b1) == MGRIT_OK);
    p = good;
    p.Mx = 80;
    CHECK(mgrit_footprint(&p, &o, MGRIT_MEM_HOST, &b2) == MGRIT_OK);
    CHECK(b2 > b1 && b1 > 0);
    // server: creation, rejected submissions, destruction with nothing queued
    mgrit_server* s = nullptr;
    CHECK(mgrit_server_create(0, 2, &s) == MGRIT_EINVAL);
    CHECK(mgrit_server_create(1 << 16, 2, &s) == MGRIT_OK && s);
    long long id = 0;
    double dummy[4] = {0, 0, 0, 0};
    CHECK(mgrit_server_submit(s, &good, &o, dummy, dummy, dummy, MGRIT_MEM_DEVICE, &id) == MGRIT_EINVAL);  // too big
    CHECK(mgrit_server_submit(s, &good, &o, dummy, nullptr, dummy, MGRIT_MEM_DEVICE, &id) == MGRIT_EINVAL);
    CHECK(mgrit_server_wait(s, 12345, nullptr) == MGRIT_EINVAL);
    mgrit_server_destroy(s);
    std::printf("host checks: %d failures\n", failures);
    return failures ? 1 : 0;
}
