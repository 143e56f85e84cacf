// Drives the serving loop from several host threads at once (test
// infrastructure only): submitters, waiters that wait on tickets while new
// ones are being submitted, a canceller, a status poller, two waiters on the
// same ticket, and a shutdown with requests still queued. Exits non-zero if
// a ticket is lost or resolved twice.
#include <atomic>
#include <cstdio>
#include <mutex>
#include <thread>
#include <vector>

#include "sic_serve.h"

int main() {
    sic_server_options o;
    sic_server_options_default(&o);
    o.slots = 4;
    const int64_t n = 64, m = 16;
    std::vector<double> X((size_t)n * m, 0.5);
    sic_problem p{};
    p.X = X.data();
    p.n = n;
    p.m = m;
    p.tol = 1e-6;
    p.lambda = 0.1;
    sic_server* srv = nullptr;
    o.hbm_budget = 3 * sic_server_footprint(nullptr, &p);   // null server: 0, set below
    if (sic_server_create(&srv, &o) != SIC_OK) return 2;
    const size_t fp = sic_server_footprint(srv, &p);
    std::printf("footprint %zu\n", fp);
    sic_server_destroy(srv);
    o.hbm_budget = 3 * fp;   // at most three requests admitted together
    if (sic_server_create(&srv, &o) != SIC_OK) return 2;

    const int per_thread = 60, submitters = 3;
    std::mutex mu;
    std::vector<uint64_t> tickets;
    std::atomic<int> resolved{0}, cancelled{0}, bad{0};
    std::atomic<bool> submitting{true};
    std::vector<std::thread> th;
    for (int s = 0; s < submitters; ++s)
        th.emplace_back([&, s]() {
            for (int k = 0; k < per_thread; ++k) {
                sic_problem q = p;
                double path[3] = {0.3, 0.2, 0.1};
                if (k % 7 == 3) {
                    q.lambda_path = path;
                    q.n_lambda = 3;
                }
                if (k % 11 == 5) q.tol = 1.0;   // the stub fails these
                uint64_t t = 0;
                if (sic_server_submit(srv, &q, &t) != SIC_OK) {
                    bad++;
                    continue;
                }
                std::lock_guard<std::mutex> lk(mu);
                tickets.push_back(t);
            }
            (void)s;
        });
    auto take = [&]() -> uint64_t {
        std::lock_guard<std::mutex> lk(mu);
        if (tickets.empty()) return 0;
        uint64_t t = tickets.back();
        tickets.pop_back();
        return t;
    };
    for (int w = 0; w < 3; ++w)
        th.emplace_back([&]() {
            for (;;) {
                uint64_t t = take();
                if (!t) {
                    if (!submitting.load()) return;
                    std::this_thread::yield();
                    continue;
                }
                sic_csr A[3] = {};
                sic_info info[3] = {};
                sic_request_times tm{};
                const int st = sic_server_wait(srv, t, -1.0, A, info, &tm);
                if (st == SIC_ECANCELED)
                    cancelled++;
                else if (st != SIC_OK && st != SIC_ENOTPD)
                    bad++;
                for (auto& a : A) sic_csr_free(&a);
                resolved++;
            }
        });
    th.emplace_back([&]() {   // canceller: tries the newest queued tickets
        for (int k = 0; k < 200; ++k) {
            uint64_t t = 0;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (!tickets.empty()) t = tickets.front();
            }
            if (t) (void)sic_server_cancel(srv, t);
            std::this_thread::yield();
        }
    });
    th.emplace_back([&]() {   // status poller
        for (int k = 0; k < 2000; ++k) {
            int q = 0, r = 0, d = 0;
            size_t held = 0;
            sic_server_status(srv, &q, &r, &d, &held);
            std::this_thread::yield();
        }
    });
    for (int s = 0; s < submitters; ++s) th[s].join();
    submitting = false;
    for (size_t k = submitters; k < th.size(); ++k) th[k].join();
    // two waiters on one ticket: exactly one claims it
    uint64_t t = 0;
    if (sic_server_submit(srv, &p, &t) != SIC_OK) return 3;
    std::atomic<int> ok{0}, einval{0};
    std::thread w1([&]() { (sic_server_wait(srv, t, -1.0, nullptr, nullptr, nullptr) == SIC_OK ? ok : einval)++; });
    std::thread w2([&]() { (sic_server_wait(srv, t, -1.0, nullptr, nullptr, nullptr) == SIC_OK ? ok : einval)++; });
    w1.join();
    w2.join();
    // shutdown with work still queued
    for (int k = 0; k < 20; ++k) {
        uint64_t u = 0;
        (void)sic_server_submit(srv, &p, &u);
    }
    sic_server_destroy(srv);
    const int expect = submitters * per_thread;
    std::printf("resolved %d of %d (cancelled %d), bad %d, double-wait ok %d einval %d\n",
                resolved.load(), expect, cancelled.load(), bad.load(), ok.load(), einval.load());
    return (resolved.load() == expect && bad.load() == 0 && ok.load() == 1 && einval.load() == 1) ? 0 : 1;
}
