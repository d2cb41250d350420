// Serving: admission of many MGRIT solves by device-memory footprint, each on
// its own stream and worker thread so that their kernels overlap on the GPU
// (continuous batching at the level of solves: a queued solve starts as soon
// as memory and a slot are free, while the others keep running).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
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

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void worker_loop(mgrit_server* s) {
    (void)hipSetDevice(0);
    while (true) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] {
                if (s->stop && s->queue.empty()) return true;
                if (s->queue.empty() || s->running >= s->max_concurrent) return false;
                return s->in_use + s->queue.front()->info.bytes <= s->budget;
            });
            if (s->queue.empty()) return;      // stopping
            r = s->queue.front();
            s->queue.pop_front();
            s->in_use += r->info.bytes;
            s->running += 1;
            r->info.start_s = s->now();
        }
        hipStream_t st = nullptr;
        int rc = (hipStreamCreate(&st) == hipSuccess) ? MGRIT_OK : MGRIT_EHIP;
        mgrit_handle* h = nullptr;
        if (rc == MGRIT_OK) rc = mgrit_setup(&r->prob, &r->opt, (void*)st, &h);
        if (rc == MGRIT_OK) rc = mgrit_solve(h, r->F, r->psi0, nullptr, r->U, r->mem, &r->info.stats);
        if (h) mgrit_destroy(h);
        if (st) (void)hipStreamDestroy(st);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            r->info.rc = rc;
            r->info.finish_s = s->now();
            r->done = true;
            s->in_use -= r->info.bytes;
            s->running -= 1;
        }
        s->cv.notify_all();
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
