// Serving engine for Smith-form requests: a request queue, worker threads
// that each own a context (hence their own HIP streams, so admitted requests
// run concurrently on the device), and admission by estimated HBM footprint.
//
// Admission: a free worker takes the oldest request whose footprint fits in
// the remaining budget (first-in first-out with backfill).  A request that has
// waited longer than the aging bound blocks backfill until it is admitted, so
// a large request cannot starve.  A request larger than the whole budget runs
// when nothing else is running.  Each request's status is its own: a singular
// or failing request does not affect the others.
#include "internal.hpp"

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <thread>
#include <vector>

namespace {

double mono_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    std::vector<int64_t> A;
    int64_t n = 0;
    uint64_t seed = 0;
    size_t footprint = 0;
    double t_submit = 0, t_start = 0, t_end = 0;
    int status = RNS_EPENDING;
    int worker = -1;
    bool done = false;
    rns_smith_result *res = nullptr;
};

}  // namespace

struct rns_server {
    int device = 0;
    size_t budget = 0;
    size_t in_use = 0;
    size_t high_water = 0;
    double aging_s = 2.0;
    double t0 = 0;
    int running = 0;
    int max_running = 0;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::vector<rns_ctx *> ctxs;
    std::vector<std::thread> threads;
    std::deque<Request *> queue;
    std::map<uint64_t, std::unique_ptr<Request>> all;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;

    Request *take_locked() {
        for (size_t i = 0; i < queue.size(); ++i) {
            Request *r = queue[i];
            const bool fits = in_use + r->footprint <= budget || (running == 0 && i == 0);
            if (fits) {
                queue.erase(queue.begin() + (long)i);
                return r;
            }
            // The head blocks backfill once it has waited past the aging bound.
            if (i == 0 && mono_s() - r->t_submit > aging_s) return nullptr;
        }
        return nullptr;
    }

    void worker(int w) {
        rns_ctx *ctx = ctxs[w];
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            Request *r = nullptr;
            cv_work.wait(lk, [&] { return stop || (r = take_locked()) != nullptr; });
            if (!r) return;                      // stop requested and nothing admitted
            in_use += r->footprint;
            high_water = std::max(high_water, in_use);
            ++running;
            max_running = std::max(max_running, running);
            r->t_start = mono_s() - t0;
            r->worker = w;
            lk.unlock();
            rns_smith_result *res = nullptr;
            const int st = smith_form(ctx, r->A.data(), r->n, r->seed, &res);
            lk.lock();
            r->status = st;
            r->res = res;
            r->t_end = mono_s() - t0;
            r->done = true;
            r->A.clear();
            r->A.shrink_to_fit();
            in_use -= r->footprint;
            --running;
            cv_done.notify_all();
            cv_work.notify_all();               // memory was freed: others may fit now
        }
    }
};

extern "C" int rns_server_footprint(int64_t n, size_t *bytes) {
    if (n < 0 || !bytes) return RNS_EINVAL;
    // Device memory of one smith_form call with up to 16 reconstruction primes
    // and about 20 check primes: the Gauss-Jordan planes (128 n^2), s A^-1 in
    // 8 words (64 n^2), the check planes and product workspace (~400 n^2), the
    // input and local-elimination buffers (16 n^2), plus fixed tables.
    *bytes = (size_t)n * (size_t)n * 640 + ((size_t)64 << 20);
    return RNS_OK;
}

extern "C" int rns_server_create(int device, int workers, size_t hbm_budget, rns_server **out) {
    if (!out || workers < 1 || workers > 64) return RNS_EINVAL;
    *out = nullptr;
    rns_server *s = new (std::nothrow) rns_server;
    if (!s) return RNS_ENOMEM;
    s->device = device;
    s->t0 = mono_s();
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipSetDevice(device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return RNS_EDEVICE;
        }
        hbm_budget = fr - fr / 8;               // keep one eighth in reserve
    }
    s->budget = hbm_budget;
    for (int w = 0; w < workers; ++w) {
        rns_ctx *c = nullptr;
        const int st = rns_ctx_create(&c, device, nullptr, 24, 0);
        if (st != RNS_OK) {
            for (auto *x : s->ctxs) rns_ctx_destroy(x);
            delete s;
            return st;
        }
        s->ctxs.push_back(c);
    }
    for (int w = 0; w < workers; ++w) s->threads.emplace_back([s, w] { s->worker(w); });
    *out = s;
    return RNS_OK;
}

extern "C" int rns_server_set_aging(rns_server *s, double seconds) {
    if (!s || seconds < 0) return RNS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    s->aging_s = seconds;
    return RNS_OK;
}

extern "C" int rns_server_submit(rns_server *s, const int64_t *A_host, int64_t n, uint64_t seed,
                                 uint64_t *ticket) {
    if (!s || !ticket || n < 0 || (n > 0 && !A_host)) return RNS_EINVAL;
    auto r = std::unique_ptr<Request>(new (std::nothrow) Request);
    if (!r) return RNS_ENOMEM;
    r->A.assign(A_host, A_host + n * n);
    r->n = n;
    r->seed = seed;
    rns_server_footprint(n, &r->footprint);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return RNS_EINVAL;
    r->ticket = s->next_ticket++;
    r->t_submit = mono_s();
    Request *raw = r.get();
    *ticket = r->ticket;
    s->all[r->ticket] = std::move(r);
    s->queue.push_back(raw);
    s->cv_work.notify_one();
    return RNS_OK;
}

extern "C" int rns_server_wait(rns_server *s, uint64_t ticket, double timeout_s,
                               rns_smith_result **out, rns_request_info *info) {
    if (!s || !out) return RNS_EINVAL;
    *out = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return RNS_EINVAL;
    Request *r = it->second.get();
    const bool ok = timeout_s < 0
                        ? (s->cv_done.wait(lk, [&] { return r->done; }), true)
                        : s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                              [&] { return r->done; });
    if (!ok) return RNS_EPENDING;
    if (info) {
        info->status = r->status;
        info->t_submit = r->t_submit - s->t0;
        info->t_start = r->t_start;
        info->t_end = r->t_end;
        info->footprint = r->footprint;
        info->worker = r->worker;
    }
    *out = r->res;                   // ownership passes to the caller
    const int st = r->status;
    s->all.erase(it);
    return st;
}

extern "C" int rns_server_stats(rns_server *s, rns_server_counters *st) {
    if (!s || !st) return RNS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    st->budget = s->budget;
    st->in_use = s->in_use;
    st->high_water = s->high_water;
    st->running = s->running;
    st->max_running = s->max_running;
    st->queued = (int)s->queue.size();
    return RNS_OK;
}

extern "C" void rns_server_destroy(rns_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->threads) t.join();
    for (auto &kv : s->all)
        if (kv.second->res) rns_smith_free(kv.second->res);
    for (auto *c : s->ctxs) rns_ctx_destroy(c);
    delete s;
}
