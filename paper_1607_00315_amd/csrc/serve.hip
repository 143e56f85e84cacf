// Serving loop (sic_serve.h): a FIFO of estimation problems admitted by
// device-memory footprint into a fixed set of slots. Each slot is one solver
// context (its own non-blocking streams and workspace) driven by one host
// worker thread, so the block updates of the admitted problems run
// concurrently on the device while every worker waits only on its own stream.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "sic_serve.h"
#include "solver.h"

namespace {

using clk = std::chrono::steady_clock;

enum ReqState { QUEUED, RUNNING, DONE };

struct Request {
    uint64_t id = 0;
    sic_problem prob{};
    std::vector<double> path;                       // copy of lambda_path
    std::vector<int64_t> a0_rowptr;                 // copy of A0
    std::vector<int32_t> a0_col;
    std::vector<double> a0_val;
    sic_csr a0{};
    size_t footprint = 0;
    ReqState state = QUEUED;
    int status = SIC_OK;
    std::string error;
    std::vector<sic_csr> A;
    std::vector<sic_info> info;
    sic_request_times times{};
};

struct Slot {
    sic::Context ctx;
    std::unique_ptr<sic::Problem> P;
    std::shared_ptr<Request> running;
    size_t cap = 0;   // bytes this slot may hold while its request runs
    std::thread th;
};

}  // namespace

struct sic_server {
    sic_server_options opt{};
    int device = 0;
    size_t budget = 0;
    int block = 256;
    clk::time_point t0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::mutex mu;
    std::condition_variable cv_work;   // queue or memory changed
    std::condition_variable cv_done;   // a request finished
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
    uint64_t next_id = 1;
    int n_running = 0;
    bool stopping = false;

    double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }

    // bytes held or promised by every slot but `self` (lock held); *idle_held
    // receives the part that idle slots hold as reusable workspace
    size_t committed_others(const Slot* self, size_t* idle_held) const {
        size_t c = 0, idle = 0;
        for (const auto& s : slots) {
            if (s.get() == self) continue;
            const size_t held = s->ctx.acct->bytes.load();
            c += s->running ? std::max(held, s->cap) : held;
            if (!s->running) idle += held;
        }
        *idle_held = idle;
        return c;
    }

    enum Decision { WAIT, ADMIT, ADMIT_AFTER_RELEASE, SHRINK };
    // What the idle slot S does about the head of the queue (lock held).
    Decision decide(const Slot* S) const {
        if (queue.empty()) return WAIT;
        const size_t need = queue.front()->footprint;
        size_t idle = 0;
        const size_t others = committed_others(S, &idle);
        const size_t held = S->ctx.acct->bytes.load();
        if (others + held + need <= budget) return ADMIT;
        if (others + need <= budget) return ADMIT_AFTER_RELEASE;
        // it would fit if the idle slots gave back their workspace: give ours
        if (held > 0 && others - idle + need <= budget) return SHRINK;
        return WAIT;
    }

    void worker(Slot* S, int index);
};

namespace {

thread_local std::string t_last_error;

size_t footprint_of(int64_t n, int64_t m, int x_dtype, int block, int n_lambda) {
    (void)n_lambda;
    const double dn = (double)n, dm = (double)m, b = (double)std::min<int64_t>(block, n);
    const double esz = x_dtype == SIC_X_F64 ? 0.0 : (x_dtype == SIC_X_F32 ? 4.0 : 2.0);
    double bytes = 16.0 * dn * dm + esz * dn * dm;   // X, X^T (float64), staged input
    bytes += 2.0 * (8.0 * (dn + 1) + 12.0 * dn * dn);   // A and its rebuild, up to dense
    bytes += 8.0 * 4.0 * dn * b;                        // S_J, W_I, A_J, new values
    bytes += 8.0 * 5.0 * dn * dn;                       // CG vectors and W_N on all columns
    bytes += 8.0 * dn * dn;                             // W on the neighbourhood (dense)
    const double hc = std::min(dn * b, 4096.0);
    bytes += 8.0 * hc * hc;                             // coordinate Hessian
    bytes += 60.0 * dn * b;                             // free lists and coordinates
    bytes += 8.0 * 40.0 * b * b + 64.0 * dn + (16 << 20);   // line search, flags, slack
    if (sic::warm_store_fits(n)) bytes += 16.0 * dn * dn + dn;   // warm-start store, cached S
    return (size_t)bytes;
}

int map_exceptions(const std::function<int()>& f, std::string& err) {
    try {
        return f();
    } catch (const sic::SicError& e) {
        err = e.what();
        return e.code;
    } catch (const sic::HipError& e) {
        err = e.what();
        return SIC_EHIP;
    } catch (const std::bad_alloc&) {
        err = "host allocation failed";
        return SIC_ENOMEM;
    } catch (const std::exception& e) {
        err = e.what();
        return SIC_EINTERNAL;
    }
}

}  // namespace

void sic_server::worker(Slot* S, int index) {
    (void)hipSetDevice(device);
    sic::AccountScope scope(S->ctx.acct);
    sic::set_blocking_waits(true);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        Decision d = WAIT;
        cv_work.wait(lk, [&]() {
            if (stopping) return true;
            d = decide(S);
            return d != WAIT;
        });
        if (!stopping && d == SHRINK) {
            lk.unlock();
            std::string e2;
            map_exceptions([&]() {
                S->P.reset();
                sic::release_workspace(S->ctx);
                return SIC_OK;
            }, e2);
            lk.lock();
            cv_work.notify_all();
            continue;
        }
        const bool release = d == ADMIT_AFTER_RELEASE;
        if (stopping) break;
        std::shared_ptr<Request> r = queue.front();
        queue.pop_front();
        r->state = RUNNING;
        r->times.admitted = now();
        r->times.slot = index;
        S->running = r;
        const size_t held = release ? 0 : S->ctx.acct->bytes.load();
        S->cap = held + r->footprint;
        ++n_running;
        lk.unlock();

        std::string err;
        const int nl = sic::request_results(r->prob);
        r->A.assign(nl, sic_csr{});
        r->info.assign(nl, sic_info{});
        const int st = map_exceptions([&]() {
            if (release) {
                S->P.reset();
                sic::release_workspace(S->ctx);
            }
            if (!S->P) S->P = std::make_unique<sic::Problem>();
            S->ctx.acct->budget = S->cap;
            return sic::solve_request(S->ctx, *S->P, r->prob, r->A.data(), r->info.data());
        }, err);
        if (st != SIC_OK)
            for (auto& in : r->info)
                if (in.status == SIC_OK) in.status = st;
        if (st != SIC_OK && st != SIC_ENOCONV) {
            // a failed request leaves no partial results and no workspace behind
            for (auto& a : r->A) sic_csr_free(&a);
            std::string e2;
            map_exceptions([&]() {
                S->P.reset();
                sic::release_workspace(S->ctx);
                return SIC_OK;
            }, e2);
        }

        lk.lock();
        r->status = st;
        r->error = err;
        r->times.finished = now();
        r->state = DONE;
        S->running.reset();
        S->cap = 0;
        --n_running;
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

extern "C" {

void sic_server_options_default(sic_server_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->slots = 4;
    sic_options_default(&o->solver);
}

int sic_request_results(const sic_problem* p) { return p ? sic::request_results(*p) : 0; }

int sic_server_create(sic_server** out, const sic_server_options* opt) {
    if (!out) return SIC_EINVAL;
    *out = nullptr;
    sic_server_options o;
    sic_server_options_default(&o);
    if (opt) o = *opt;
    if (o.slots == 0) o.slots = 4;
    if (o.slots < 1 || o.slots > 64) return SIC_EINVAL;
    std::string err;
    auto srv = std::make_unique<sic_server>();
    const int st = map_exceptions([&]() {
        SIC_HIP(hipSetDevice(o.device));
        size_t free_b = 0, total_b = 0;
        SIC_HIP(hipMemGetInfo(&free_b, &total_b));
        srv->opt = o;
        srv->device = o.device;
        srv->budget = o.hbm_budget ? o.hbm_budget : (size_t)(0.8 * (double)free_b);
        srv->block = o.solver.block > 0 ? o.solver.block : 256;
        srv->t0 = clk::now();
        sic_options so = o.solver;
        so.device = o.device;
        so.stream = nullptr;
        so.trace = nullptr;
        so.trace_cap = 0;
        so.hbm_budget = 0;
        for (int k = 0; k < o.slots; ++k) {
            auto S = std::make_unique<Slot>();
            sic::context_init(S->ctx, so);
            srv->slots.push_back(std::move(S));
        }
        for (int k = 0; k < o.slots; ++k) {
            Slot* S = srv->slots[k].get();
            S->th = std::thread([s = srv.get(), S, k]() { s->worker(S, k); });
        }
        return SIC_OK;
    }, err);
    if (st != SIC_OK) {
        t_last_error = err;
        sic_server_destroy(srv.release());
        return st;
    }
    *out = srv.release();
    return SIC_OK;
}

size_t sic_server_footprint(const sic_server* srv, const sic_problem* p) {
    if (!srv || !p || p->n < 1 || p->m < 1) return 0;
    return footprint_of(p->n, p->m, p->x_dtype, srv->block, p->n_lambda);
}

int sic_server_submit(sic_server* srv, const sic_problem* p, uint64_t* ticket) {
    if (!srv || !p || !ticket || !p->X || p->n < 1 || p->m < 1 || !(p->tol > 0.0) ||
        (p->n_lambda > 0 && !p->lambda_path) || p->n_lambda < 0)
        return SIC_EINVAL;
    auto r = std::make_shared<Request>();
    r->prob = *p;
    if (p->n_lambda > 0) {
        r->path.assign(p->lambda_path, p->lambda_path + p->n_lambda);
        r->prob.lambda_path = r->path.data();
    }
    if (p->A0) {
        const sic_csr& a = *p->A0;
        if (a.n != p->n || a.nnz < 0 || !a.rowptr || (a.nnz > 0 && (!a.col || !a.val)))
            return SIC_EINVAL;
        r->a0_rowptr.assign(a.rowptr, a.rowptr + a.n + 1);
        r->a0_col.assign(a.col, a.col + a.nnz);
        r->a0_val.assign(a.val, a.val + a.nnz);
        r->a0 = sic_csr{a.n, a.nnz, r->a0_rowptr.data(), r->a0_col.data(), r->a0_val.data()};
        r->prob.A0 = &r->a0;
    }
    r->footprint = footprint_of(p->n, p->m, p->x_dtype, srv->block, p->n_lambda);
    if (r->footprint > srv->budget) {
        t_last_error = "problem footprint exceeds the server's device-memory budget";
        return SIC_ENOMEM;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return SIC_ECANCELED;
    r->id = srv->next_id++;
    r->times.submitted = srv->now();
    r->times.footprint = r->footprint;
    r->times.slot = -1;
    srv->reqs[r->id] = r;
    srv->queue.push_back(r);
    *ticket = r->id;
    srv->cv_work.notify_all();
    return SIC_OK;
}

int sic_server_wait(sic_server* srv, uint64_t ticket, double timeout_s, sic_csr* A_out,
                    sic_info* info, sic_request_times* times) {
    if (!srv) return SIC_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    std::shared_ptr<Request> r;
    {
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) return SIC_EINVAL;
        r = it->second;   // no iterator is kept across the wait: submits may rehash
    }
    auto done = [&]() { return r->state == DONE; };
    if (timeout_s < 0) {
        srv->cv_done.wait(lk, done);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        return 1;
    }
    // retire the ticket by key; a second waiter on the same ticket finds it
    // already claimed
    if (srv->reqs.erase(ticket) == 0) return SIC_EINVAL;
    lk.unlock();
    for (size_t k = 0; k < r->A.size(); ++k) {
        if (A_out)
            A_out[k] = r->A[k];
        else
            sic_csr_free(&r->A[k]);
    }
    if (info)
        for (size_t k = 0; k < r->info.size(); ++k) info[k] = r->info[k];
    if (times) *times = r->times;
    r->A.clear();
    if (r->status != SIC_OK) t_last_error = r->error;
    return r->status;
}

int sic_server_cancel(sic_server* srv, uint64_t ticket) {
    if (!srv) return SIC_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second->state != QUEUED) return SIC_EINVAL;
    std::shared_ptr<Request> r = it->second;
    for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q)
        if (*q == r) {
            srv->queue.erase(q);
            break;
        }
    r->state = DONE;
    r->status = SIC_ECANCELED;
    r->error = "cancelled before admission";
    r->times.finished = srv->now();
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
    return SIC_OK;
}

void sic_server_status(const sic_server* srv, int* queued, int* running, int* done,
                       size_t* held_bytes) {
    if (!srv) return;
    sic_server* s = const_cast<sic_server*>(srv);
    std::lock_guard<std::mutex> lk(s->mu);
    int d = 0;
    for (const auto& kv : s->reqs) d += kv.second->state == DONE;
    size_t held = 0;
    for (const auto& sl : s->slots) held += sl->ctx.acct->bytes.load();
    if (queued) *queued = (int)s->queue.size();
    if (running) *running = s->n_running;
    if (done) *done = d;
    if (held_bytes) *held_bytes = held;
}

void sic_server_destroy(sic_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        for (auto& r : srv->queue) {
            r->state = DONE;
            r->status = SIC_ECANCELED;
        }
        srv->queue.clear();
        srv->cv_work.notify_all();
        srv->cv_done.notify_all();
    }
    for (auto& S : srv->slots)
        if (S->th.joinable()) S->th.join();
    for (auto& kv : srv->reqs)
        for (auto& a : kv.second->A) sic_csr_free(&a);
    srv->reqs.clear();
    for (auto& S : srv->slots) {
        (void)hipSetDevice(srv->device);
        S->P.reset();
        sic::context_release(S->ctx);
    }
    delete srv;
}

}  // extern "C"
