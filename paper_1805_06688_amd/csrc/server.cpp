// Serving: admission of many MGRIT solves by device-memory footprint, each on
// its own stream and worker thread so that their kernels overlap on the GPU
// (continuous batching at the level of solves: a queued solve starts as soon
// as memory and a slot are free, while the others keep running).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/mgrit.h"

namespace {

struct Request {
    long long id = 0;
    mgrit_problem prob{};
    std::vector<double> t;
    mgrit_options opt{};
    const double* F = nullptr;
    const double* psi0 = nullptr;
    double* U = nullptr;
    int mem = MGRIT_MEM_DEVICE;
    mgrit_request_info info{};
    bool done = false;
};

// Requests that may share one group solve: the same mesh, domain, options and memory space.
bool same_group(const Request* a, const Request* b) {
    const mgrit_problem &p = a->prob, &q = b->prob;
    return p.Mx == q.Mx && p.My == q.My && p.a == q.a && p.b == q.b && p.c == q.c && p.d == q.d &&
           a->mem == b->mem && std::memcmp(&a->opt, &b->opt, sizeof(mgrit_options)) == 0;
}

// Device memory a group solve of these requests holds: their own footprints plus the group's copy of
// their loads and states.
size_t group_bytes(const std::vector<Request*>& rs) {
    size_t b = 0;
    for (const Request* r : rs) {
        const size_t n = (size_t)(r->prob.Mx - 1) * (r->prob.My - 1);
        b += r->info.bytes + (2 * (size_t)r->prob.Nt + 1) * n * sizeof(double);
    }
    return b;
}

}  // namespace

struct mgrit_server {
    size_t budget = 0;
    int max_concurrent = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request*> queue;
    std::map<long long, std::unique_ptr<Request>> all;
    size_t in_use = 0;
    int running = 0;
    bool stop = false;
    long long next_id = 1;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0;
    int group_limit = 1;                  // requests one worker may take into one group solve

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Run one group of admitted requests: alone (one request) as mgrit_solve, else as one group solve whose
// sweeps share launches; a group that cannot be set up (level counts differ) runs its requests one by one.
void run_requests(mgrit_server* s, std::vector<Request*>& rs) {
    hipStream_t st = nullptr;
    int rc = (hipStreamCreate(&st) == hipSuccess) ? MGRIT_OK : MGRIT_EHIP;
    std::vector<int> rcs(rs.size(), rc);
    bool grouped = false;
    if (rc == MGRIT_OK && rs.size() > 1) {
        std::vector<mgrit_problem> probs;
        for (Request* r : rs) probs.push_back(r->prob);
        mgrit_handle* h = nullptr;
        if (mgrit_setup_group(probs.data(), (int)probs.size(), &rs[0]->opt, (void*)st, &h) == MGRIT_OK) {
            std::vector<const double*> F, P;
            std::vector<double*> U;
            std::vector<mgrit_stats> stats(rs.size());
            for (Request* r : rs) {
                F.push_back(r->F);
                P.push_back(r->psi0);
                U.push_back(r->U);
            }
            const int grc = mgrit_solve_group(h, F.data(), P.data(), U.data(), rs[0]->mem, stats.data());
            for (size_t i = 0; i < rs.size(); ++i) {
                rs[i]->info.stats = stats[i];
                const mgrit_stats& q = stats[i];
                const bool grew = rs[i]->opt.divergence_factor > 0.0 && q.iterations + 1 <= 64 &&
                                  q.residual_history[q.iterations] > rs[i]->opt.divergence_factor * q.residual_history[0];
                rcs[i] = grc < 0 ? grc : (q.converged ? MGRIT_OK : (grew ? MGRIT_EDIVERGED : MGRIT_ENOCONV));
            }
            mgrit_destroy(h);
            grouped = true;
        }
    }
    if (rc == MGRIT_OK && !grouped) {
        for (size_t i = 0; i < rs.size(); ++i) {
            Request* r = rs[i];
            mgrit_handle* h = nullptr;
            int q = mgrit_setup(&r->prob, &r->opt, (void*)st, &h);
            if (q == MGRIT_OK) q = mgrit_solve(h, r->F, r->psi0, nullptr, r->U, r->mem, &r->info.stats);
            if (h) mgrit_destroy(h);
            rcs[i] = q;
        }
    }
    if (st) (void)hipStreamDestroy(st);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const double now = s->now();
        for (size_t i = 0; i < rs.size(); ++i) {
            rs[i]->info.rc = rcs[i];
            rs[i]->info.finish_s = now;
            rs[i]->info.group_size = (int)rs.size();
            rs[i]->done = true;
        }
        s->in_use -= rs.size() > 1 ? group_bytes(rs) : rs[0]->info.bytes;
        s->running -= 1;
    }
    s->cv.notify_all();
}

void worker_loop(mgrit_server* s) {
    (void)hipSetDevice(0);
    while (true) {
        std::vector<Request*> rs;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] {
                if (s->stop && s->queue.empty()) return true;
                if (s->queue.empty() || s->running >= s->max_concurrent) return false;
                return s->in_use + s->queue.front()->info.bytes <= s->budget;
            });
            if (s->queue.empty()) return;      // stopping
            // the oldest request, and queued ones that can share its group solve while memory allows
            rs.push_back(s->queue.front());
            s->queue.pop_front();
            for (auto it = s->queue.begin(); it != s->queue.end() && (int)rs.size() < s->group_limit;) {
                std::vector<Request*> trial(rs);
                trial.push_back(*it);
                if (same_group(rs[0], *it) && s->in_use + group_bytes(trial) <= s->budget) {
                    rs.push_back(*it);
                    it = s->queue.erase(it);
                } else {
                    ++it;
                }
            }
            s->in_use += rs.size() > 1 ? group_bytes(rs) : rs[0]->info.bytes;
            s->running += 1;
            const double now = s->now();
            for (Request* r : rs) r->info.start_s = now;
        }
        run_requests(s, rs);
    }
}

}  // namespace

extern "C" {

int mgrit_server_create(size_t device_budget_bytes, int max_concurrent, mgrit_server** out) {
    if (!out || max_concurrent < 1 || device_budget_bytes == 0) return MGRIT_EINVAL;
    mgrit_server* s = new (std::nothrow) mgrit_server();
    if (!s) return MGRIT_ENOMEM;
    s->budget = device_budget_bytes;
    s->max_concurrent = max_concurrent;
    s->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < max_concurrent; ++i) s->workers.emplace_back(worker_loop, s);
    *out = s;
    return MGRIT_OK;
}

int mgrit_server_set_group_limit(mgrit_server* s, int max_members) {
    if (!s || max_members < 1) return MGRIT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->group_limit = max_members;
    return MGRIT_OK;
}

int mgrit_server_submit(mgrit_server* s, const mgrit_problem* prob, const mgrit_options* opt, const double* F,
                        const double* psi0, double* U, int mem, long long* id) {
    if (!s || !prob || !opt || !psi0 || !U || !id || !prob->t || prob->Nt < 1) return MGRIT_EINVAL;
    if (mem != MGRIT_MEM_HOST && mem != MGRIT_MEM_DEVICE) return MGRIT_EINVAL;
    size_t bytes = 0;
    int rc = mgrit_footprint(prob, opt, mem, &bytes);
    if (rc != MGRIT_OK) return rc;
    if (bytes > s->budget) return MGRIT_EINVAL;
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return MGRIT_ENOMEM;
    r->prob = *prob;
    r->t.assign(prob->t, prob->t + prob->Nt + 1);
    r->prob.t = r->t.data();
    r->opt = *opt;
    r->F = F;
    r->psi0 = psi0;
    r->U = U;
    r->mem = mem;
    r->info.bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return MGRIT_EINVAL;
        r->id = s->next_id++;
        r->info.submit_s = s->now();
        *id = r->id;
        s->queue.push_back(r.get());
        s->all[r->id] = std::move(r);
    }
    s->cv.notify_all();
    return MGRIT_OK;
}

int mgrit_server_wait(mgrit_server* s, long long id, mgrit_request_info* info) {
    if (!s) return MGRIT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return MGRIT_EINVAL;
    Request* r = it->second.get();
    s->cv.wait(lk, [&] { return r->done; });
    if (info) *info = r->info;
    return MGRIT_OK;
}

int mgrit_server_poll(mgrit_server* s, long long id, int* done) {
    if (!s || !done) return MGRIT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return MGRIT_EINVAL;
    *done = it->second->done ? 1 : 0;
    return MGRIT_OK;
}

void mgrit_server_destroy(mgrit_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (std::thread& t : s->workers) t.join();
    delete s;
}

}  // extern "C"
