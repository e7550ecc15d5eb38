// Serving loop: snapshots of different sizes arrive over time (as in an MD
// trajectory driven through the method's calculator interface, Sec. 4) and
// are run on one GPU with continuous admission.
//
// A scheduler thread owns a fixed set of slots.  Each slot is a library
// context with its own HIP stream and device state (cell list, u scratch, B
// cache, energy window, DOS partials, outputs), so the kernels of requests in
// different slots overlap on the device.  Requests are admitted strictly in
// arrival order (no overtaking, hence no starvation) whenever a slot is free
// and the device memory held by all slots plus what the request would add to
// the chosen slot (summed buffer by buffer) stays within the budget; idle
// slots give their cached buffers back first when the budget is tight.
// mala_server_reserve sizes every slot once for the largest expected request,
// after which requests within it allocate nothing.  Each request runs exactly
// the single-snapshot path with its own fixed work partition, so its result
// does not depend on what else is in flight.  Kernel launches and result
// copies run outside the scheduler's lock; results come back through pinned
// memory with asynchronous copies (the kernels' capacity flags included).
//
// The executor is an interface: the GPU executor below, or a host-only mock
// (a timer per request) that exercises the same scheduler without a device.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mala.h"
#include "mala_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    std::vector<double> pos;
    int32_t n_atoms = 0;
    mala_cell_grid cg{};
    double rcut = 0;
    int32_t twojmax = 0;
    mala_egrid eg{};
    double T = 0, ne = 0;
    double* dos_out = nullptr;       // host [eg.n]
    double* density_out = nullptr;   // host [N] or NULL
    size_t need = 0;                 // device bytes in an empty slot
    mala::PredictPlan plan{};
    int64_t n_pts = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    mala_result res{};
    mala_status status = MALA_OK;
    std::string err;
    int state = 0;                   // 0 queued, 1 running, 2 done
};

struct Executor {
    virtual ~Executor() {}
    virtual int slots() const = 0;
    virtual size_t slot_bytes(int s) = 0;                        // device bytes the slot holds
    virtual size_t growth(int s, const Request& r) = 0;          // bytes the slot would add for r
    virtual void trim(int s) = 0;
    virtual mala_status reserve(const mala::PredictPlan& p, int64_t max_pts) = 0;
    virtual uint64_t allocs() = 0;                               // allocations made so far
    virtual mala_status launch(int s, Request& r) = 0;
    virtual bool done(int s) = 0;
    virtual mala_status finish(int s, Request& r) = 0;
};

// ------------------------------------------------------------------ GPU
// Makes `dev` current for a scope and restores the caller's device.
struct DevScope {
    int prev = -1;
    explicit DevScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DevScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct GpuSlot {
    mala_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    double* dos = nullptr;       // device [256]
    double* dens = nullptr;      // device, cap_dens
    size_t cap_dens = 0;
    void* res = nullptr;         // device mala_result
    double* h_dos = nullptr;     // pinned
    double* h_dens = nullptr;    // pinned, cap_dens
    mala_result* h_res = nullptr;
    int* h_err = nullptr;        // pinned copy of the context's capacity flags
};

struct GpuExecutor : Executor {
    int device;
    mala_weights* w = nullptr;
    std::vector<GpuSlot> s;
    uint64_t own_allocs = 0;
    GpuExecutor(int dev, int n) : device(dev), s(n) {}
    ~GpuExecutor() override {
        DevScope d(device);
        for (auto& x : s) {
            if (x.stream) (void)hipStreamSynchronize(x.stream);
            if (x.ctx) mala_destroy(x.ctx);
            if (x.ev) (void)hipEventDestroy(x.ev);
            if (x.dos) (void)hipFree(x.dos);
            if (x.dens) (void)hipFree(x.dens);
            if (x.res) (void)hipFree(x.res);
            if (x.h_dos) (void)hipHostFree(x.h_dos);
            if (x.h_dens) (void)hipHostFree(x.h_dens);
            if (x.h_res) (void)hipHostFree(x.h_res);
            if (x.h_err) (void)hipHostFree(x.h_err);
            if (x.stream) (void)hipStreamDestroy(x.stream);
        }
        if (w) mala_weights_free(w);
    }
    mala_status init(const void* blob, size_t bytes, int32_t precision) {
        DevScope d(device);
        for (auto& x : s) {
            if (hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking) != hipSuccess) return MALA_E_HIP;
            if (hipEventCreateWithFlags(&x.ev, hipEventDisableTiming) != hipSuccess) return MALA_E_HIP;
            mala_status st = mala_create(device, x.stream, &x.ctx);
            if (st) return st;
            if (hipMalloc(&x.dos, sizeof(double) * 256) != hipSuccess) return MALA_E_OOM;
            if (hipMalloc(&x.res, sizeof(mala_result)) != hipSuccess) return MALA_E_OOM;
            if (hipHostMalloc(&x.h_dos, sizeof(double) * 256, hipHostMallocDefault) != hipSuccess) return MALA_E_OOM;
            if (hipHostMalloc(&x.h_res, sizeof(mala_result), hipHostMallocDefault) != hipSuccess) return MALA_E_OOM;
            if (hipHostMalloc(&x.h_err, sizeof(int), hipHostMallocDefault) != hipSuccess) return MALA_E_OOM;
        }
        return mala_weights_load(s[0].ctx, blob, bytes, precision, &w);
    }
    int slots() const override { return (int)s.size(); }
    size_t slot_bytes(int i) override { return mala::ctx_device_bytes(s[i].ctx) + s[i].cap_dens * sizeof(double); }
    size_t growth(int i, const Request& r) override {
        size_t g = mala::plan_growth_bytes(s[i].ctx, r.plan);
        if (r.density_out && s[i].cap_dens < (size_t)r.n_pts) g += (r.n_pts - s[i].cap_dens) * sizeof(double);
        return g;
    }
    void trim(int i) override {
        (void)hipSetDevice(device);
        mala::ctx_trim(s[i].ctx);
        if (s[i].dens) (void)hipFree(s[i].dens);
        if (s[i].h_dens) (void)hipHostFree(s[i].h_dens);
        s[i].dens = nullptr;
        s[i].h_dens = nullptr;
        s[i].cap_dens = 0;
    }
    mala_status grow_density(GpuSlot& x, size_t n) {
        if (x.cap_dens >= n) return MALA_OK;
        if (x.dens) (void)hipFree(x.dens);
        if (x.h_dens) (void)hipHostFree(x.h_dens);
        x.dens = nullptr;
        x.h_dens = nullptr;
        x.cap_dens = 0;
        own_allocs += 2;
        if (hipMalloc(&x.dens, sizeof(double) * n) != hipSuccess) return MALA_E_OOM;
        if (hipHostMalloc(&x.h_dens, sizeof(double) * n, hipHostMallocDefault) != hipSuccess) return MALA_E_OOM;
        x.cap_dens = n;
        return MALA_OK;
    }
    mala_status reserve(const mala::PredictPlan& p, int64_t max_pts) override {
        DevScope d(device);
        for (auto& x : s) {
            mala_status st = mala::ctx_reserve(x.ctx, p);
            if (st) return st;
            if ((st = grow_density(x, (size_t)max_pts))) return st;
        }
        return MALA_OK;
    }
    uint64_t allocs() override {
        uint64_t n = own_allocs;
        for (auto& x : s) n += mala::ctx_alloc_count(x.ctx);
        return n;
    }
    mala_status launch(int i, Request& r) override {
        (void)hipSetDevice(device);
        GpuSlot& x = s[i];
        if (r.density_out) {
            mala_status st = grow_density(x, (size_t)r.n_pts);
            if (st) return st;
        }
        mala_status st = mala_predict(x.ctx, w, r.pos.data(), r.n_atoms, &r.cg, r.rcut, r.twojmax, &r.eg, r.T, r.ne,
                                      x.dos, r.density_out ? x.dens : nullptr, static_cast<mala_result*>(x.res),
                                      nullptr);
        if (st) return st;
        int* err = mala::ctx_error_flags(x.ctx);
        if (hipMemcpyAsync(x.h_dos, x.dos, sizeof(double) * r.eg.n, hipMemcpyDeviceToHost, x.stream) != hipSuccess ||
            hipMemcpyAsync(x.h_res, x.res, sizeof(mala_result), hipMemcpyDeviceToHost, x.stream) != hipSuccess ||
            hipMemcpyAsync(x.h_err, err, sizeof(int), hipMemcpyDeviceToHost, x.stream) != hipSuccess ||
            hipMemsetAsync(err, 0, sizeof(int), x.stream) != hipSuccess)
            return MALA_E_HIP;
        if (r.density_out &&
            hipMemcpyAsync(x.h_dens, x.dens, sizeof(double) * r.n_pts, hipMemcpyDeviceToHost, x.stream) != hipSuccess)
            return MALA_E_HIP;
        return hipEventRecord(x.ev, x.stream) == hipSuccess ? MALA_OK : MALA_E_HIP;
    }
    bool done(int i) override { return hipEventQuery(s[i].ev) != hipErrorNotReady; }
    mala_status finish(int i, Request& r) override {
        GpuSlot& x = s[i];
        if (hipEventSynchronize(x.ev) != hipSuccess) return MALA_E_HIP;
        memcpy(r.dos_out, x.h_dos, sizeof(double) * r.eg.n);
        if (r.density_out) memcpy(r.density_out, x.h_dens, sizeof(double) * r.n_pts);
        r.res = *x.h_res;
        const int flags = *x.h_err;
        if (flags & mala::kErrCand) {
            r.err = "more than 1024 atom images near one 64-point tile";
            return MALA_E_CAPACITY;
        }
        if (flags & mala::kErrNbr) {
            r.err = "more than 128 neighbours within rcut of a grid point";
            return MALA_E_CAPACITY;
        }
        return MALA_OK;
    }
};

// ------------------------------------------------------------------ mock
struct MockExecutor : Executor {
    struct S {
        size_t bytes = 0;
        double until = 0;
        bool busy = false;
    };
    std::vector<S> s;
    double ns_per_point;
    Clock::time_point t0;
    uint64_t n_allocs = 0;
    MockExecutor(int n, double ns, Clock::time_point t) : s(n), ns_per_point(ns), t0(t) {}
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    int slots() const override { return (int)s.size(); }
    size_t slot_bytes(int i) override { return s[i].bytes; }
    size_t growth(int i, const Request& r) override { return r.need > s[i].bytes ? r.need - s[i].bytes : 0; }
    void trim(int i) override { s[i].bytes = 0; }
    mala_status reserve(const mala::PredictPlan&, int64_t) override { return MALA_OK; }
    uint64_t allocs() override { return n_allocs; }
    mala_status launch(int i, Request& r) override {
        if (s[i].bytes < r.need) {
            s[i].bytes = r.need;
            ++n_allocs;
        }
        s[i].until = now() + 1e-9 * ns_per_point * (double)r.n_pts;
        s[i].busy = true;
        return MALA_OK;
    }
    bool done(int i) override { return now() >= s[i].until; }
    mala_status finish(int i, Request& r) override {
        s[i].busy = false;
        for (int e = 0; e < r.eg.n; ++e) r.dos_out[e] = (double)r.ticket;
        if (r.density_out)
            for (int64_t p = 0; p < r.n_pts; ++p) r.density_out[p] = (double)r.ticket;
        r.res.e_fermi = (double)r.n_pts;
        r.res.status = 0;
        return MALA_OK;
    }
};

// Device bytes a request needs in an empty slot: every buffer of its plan at
// the size it is grown to, plus the slot's density output.
size_t footprint(const Request& r) {
    const mala::PredictPlan& p = r.plan;
    auto g = [](size_t n, size_t elem) { return n ? (n + n / 8 + 64) * elem : 0; };
    size_t b = g(p.pos, 8) + 3 * g(p.cells, 4) + g(p.atoms, 4) + 2 * g(p.atoms, 32) + g(p.u, 8) + g(p.B, 4) +
               g(p.partials, 8) + g(p.fermi_w, 8) + g(p.est_partials, 8) + g(p.window, 4) + g(p.prefix, 8);
    if (r.density_out) b += (size_t)r.n_pts * sizeof(double);
    return b;
}

}  // namespace

struct mala_server {
    std::unique_ptr<Executor> ex;
    size_t budget = 0;
    int device = 0;
    Clock::time_point t0 = Clock::now();
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::map<uint64_t, std::unique_ptr<Request>> all;
    std::vector<Request*> running;       // per slot: admitted and not yet finished
    std::vector<size_t> bytes;           // per slot device bytes (updated by the scheduler thread)
    uint64_t allocs = 0;                 // allocations made by the slots (updated by the scheduler thread)
    size_t reserved_bytes = 0;           // per slot, after mala_server_reserve
    int64_t inflight_cap = 0;            // grid points in flight above which no request joins (0: none)
    uint64_t next_ticket = 1;
    bool stop = false;
    size_t peak_bytes = 0;
    std::thread th;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    size_t held() const {
        size_t h = 0;
        for (size_t b : bytes) h += b;
        return h;
    }

    // Scheduler thread only: the executor's slot state is touched by no other
    // thread, so launches and result copies run without the lock; the lock
    // covers the queue, the request states and the per-slot records.
    void loop(bool gpu) {
        if (gpu) (void)hipSetDevice(device);
        std::vector<std::pair<int, Request*>> fin, go;
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            // completions: detected under the lock, copied out without it
            fin.clear();
            for (int i = 0; i < ex->slots(); ++i)
                if (running[i] && running[i]->state == 1 && ex->done(i)) fin.push_back({i, running[i]});
            if (!fin.empty()) {
                lk.unlock();
                for (auto& f : fin) {
                    mala_status st = ex->finish(f.first, *f.second);
                    if (st && !f.second->status) {
                        f.second->status = st;
                        if (f.second->err.empty()) f.second->err = mala_last_error();
                    }
                }
                lk.lock();
                for (auto& f : fin) {
                    f.second->t_done = now();
                    f.second->state = 2;
                    running[f.first] = nullptr;
                }
                cv_done.notify_all();
            }
            // admissions, strictly in arrival order; the slot that grows least
            // (then the one holding most) takes the next request
            go.clear();
            size_t pending = 0;
            while (!queue.empty()) {
                Request* r = queue.front();
                int slot = -1;
                size_t g_slot = 0;
                for (int i = 0; i < ex->slots(); ++i) {
                    if (running[i]) continue;
                    const size_t g = ex->growth(i, *r);
                    if (slot < 0 || g < g_slot || (g == g_slot && bytes[i] > bytes[slot])) {
                        slot = i;
                        g_slot = g;
                    }
                }
                if (slot < 0) break;
                if (inflight_cap > 0) {                  // a request joins running work only below the cap
                    int64_t pts = 0;
                    bool any = false;
                    for (auto* q : running)
                        if (q) {
                            pts += q->n_pts;
                            any = true;
                        }
                    if (any && pts + r->n_pts > inflight_cap) break;
                }
                if (held() + pending + g_slot > budget) {
                    for (int i = 0; i < ex->slots(); ++i)
                        if (!running[i] && i != slot) {
                            ex->trim(i);
                            bytes[i] = ex->slot_bytes(i);
                        }
                    g_slot = ex->growth(slot, *r);
                    if (held() + pending + g_slot > budget) {
                        ex->trim(slot);
                        bytes[slot] = ex->slot_bytes(slot);
                        g_slot = ex->growth(slot, *r);
                    }
                    if (held() + pending + g_slot > budget) break;      // wait for running work to finish
                }
                queue.pop_front();
                r->t_start = now();
                r->state = 1;
                running[slot] = r;
                pending += g_slot;
                go.push_back({slot, r});
            }
            if (!go.empty()) {
                lk.unlock();
                for (auto& q : go) {
                    mala_status st = ex->launch(q.first, *q.second);
                    if (st) {
                        q.second->status = st;
                        q.second->err = mala_last_error();
                    }
                }
                const uint64_t na = ex->allocs();
                lk.lock();
                allocs = na;
                for (auto& q : go) {
                    bytes[q.first] = ex->slot_bytes(q.first);
                    if (q.second->status) {          // launch failed: done with its error
                        q.second->t_done = now();
                        q.second->state = 2;
                        running[q.first] = nullptr;
                    }
                }
                if (held() > peak_bytes) peak_bytes = held();
                cv_done.notify_all();
                continue;                            // look for completions again before sleeping
            }
            bool busy = false;
            for (auto* r : running) busy = busy || r;
            cv_work.wait_for(lk, busy ? std::chrono::microseconds(50) : std::chrono::milliseconds(5));
        }
    }
};

namespace {
thread_local std::string g_serr;
mala_status sfail(mala_status st, const char* m) {
    g_serr = m;
    return st;
}
}  // namespace

extern "C" {

mala_status mala_server_create(int32_t device, const void* blob, size_t bytes, int32_t precision, size_t hbm_budget,
                               int32_t max_inflight, mala_server** out) {
    if (!out || !blob || max_inflight < 1 || max_inflight > 64) return MALA_E_INVALID_ARG;
    *out = nullptr;
    auto* sv = new mala_server();
    auto* g = new GpuExecutor(device, max_inflight);
    sv->ex.reset(g);
    sv->device = device;
    sv->budget = hbm_budget;
    mala_status st = g->init(blob, bytes, precision);
    if (st) {
        delete sv;
        return st;
    }
    sv->running.assign(max_inflight, nullptr);
    sv->bytes.assign(max_inflight, 0);
    for (int i = 0; i < max_inflight; ++i) sv->bytes[i] = sv->ex->slot_bytes(i);
    sv->allocs = sv->ex->allocs();
    sv->th = std::thread([sv] { sv->loop(true); });
    *out = sv;
    return MALA_OK;
}

mala_status mala_server_create_mock(int32_t slots, size_t hbm_budget, double ns_per_point, mala_server** out) {
    if (!out || slots < 1 || slots > 64 || !(ns_per_point >= 0)) return MALA_E_INVALID_ARG;
    auto* sv = new mala_server();
    sv->ex.reset(new MockExecutor(slots, ns_per_point, sv->t0));
    sv->budget = hbm_budget;
    sv->running.assign(slots, nullptr);
    sv->bytes.assign(slots, 0);
    sv->th = std::thread([sv] { sv->loop(false); });
    *out = sv;
    return MALA_OK;
}

mala_status mala_server_destroy(mala_server* sv) {
    if (!sv) return MALA_OK;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        // let running work drain, drop queued requests
        sv->queue.clear();
        sv->cv_done.wait(lk, [&] {
            for (auto* r : sv->running)
                if (r) return false;
            return true;
        });
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    sv->th.join();
    delete sv;
    return MALA_OK;
}

mala_status mala_server_submit(mala_server* sv, const mala_request* q, uint64_t* ticket) {
    if (!sv || !q || !ticket) return MALA_E_INVALID_ARG;
    if (q->n_atoms < 0 || (q->n_atoms > 0 && !q->positions) || !q->dos_out) return MALA_E_INVALID_ARG;
    auto r = std::make_unique<Request>();
    r->pos.assign(q->positions, q->positions + 3 * (size_t)q->n_atoms);
    r->n_atoms = q->n_atoms;
    r->cg = q->cell_grid;
    r->rcut = q->rcut;
    r->twojmax = q->twojmax;
    r->eg = q->egrid;
    r->T = q->T_kelvin;
    r->ne = q->n_electrons;
    r->dos_out = q->dos_out;
    r->density_out = q->density_out;
    r->n_pts = (int64_t)q->cell_grid.N[0] * q->cell_grid.N[1] * q->cell_grid.N[2];
    if (q->cell_grid.N[0] < 1 || q->cell_grid.N[1] < 1 || q->cell_grid.N[2] < 1 || r->twojmax < 2 || r->twojmax > mala::kMaxTwojmax || (r->twojmax & 1) ||
        r->eg.n < 2 || r->eg.n > mala::kMlpMaxOut || !(r->eg.de > 0) || !(r->T > 0))
        return MALA_E_INVALID_ARG;
    if (!(r->rcut > 0) || r->n_atoms > (1 << 24)) return MALA_E_INVALID_ARG;
    r->plan = mala::plan_predict(&r->cg, r->n_atoms, r->rcut, r->twojmax, &r->eg, r->T, r->density_out != nullptr, 0,
                                 false);
    r->need = footprint(*r);
    if (r->need > sv->budget) return MALA_E_OOM;
    std::lock_guard<std::mutex> lk(sv->mu);
    r->ticket = sv->next_ticket++;
    r->t_submit = sv->now();
    *ticket = r->ticket;
    sv->queue.push_back(r.get());
    sv->all[r->ticket] = std::move(r);
    sv->cv_work.notify_all();
    return MALA_OK;
}

static mala_status take(mala_server* sv, uint64_t ticket, mala_result* res, double* times) {
    auto it = sv->all.find(ticket);
    Request* r = it->second.get();
    if (res) *res = r->res;
    if (times) {
        times[0] = r->t_submit;
        times[1] = r->t_start;
        times[2] = r->t_done;
    }
    mala_status st = r->status;
    if (st) g_serr = r->err;
    sv->all.erase(it);
    return st;
}

mala_status mala_server_poll(mala_server* sv, uint64_t ticket, mala_result* res, double* times) {
    if (!sv) return MALA_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return MALA_E_INVALID_ARG;
    if (it->second->state != 2) return MALA_E_BUSY;
    return take(sv, ticket, res, times);
}

mala_status mala_server_wait(mala_server* sv, uint64_t ticket, double timeout_s, mala_result* res, double* times) {
    if (!sv) return MALA_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return MALA_E_INVALID_ARG;
    Request* r = it->second.get();
    const bool ok = sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return r->state == 2; });
    if (!ok) return MALA_E_BUSY;
    return take(sv, ticket, res, times);
}

mala_status mala_server_reserve(mala_server* sv, const mala_request* reqs, int32_t n) {
    if (!sv || !reqs || n < 1) return sfail(MALA_E_INVALID_ARG, "reserve: no requests");
    std::unique_lock<std::mutex> lk(sv->mu);
    for (auto* r : sv->running)
        if (r) return sfail(MALA_E_BUSY, "reserve: requests are running");
    if (!sv->queue.empty()) return sfail(MALA_E_BUSY, "reserve: requests are queued");
    mala::PredictPlan p{};
    int64_t max_pts = 0;
    for (int32_t k = 0; k < n; ++k) {
        const mala_request& q = reqs[k];
        const int64_t np = (int64_t)q.cell_grid.N[0] * q.cell_grid.N[1] * q.cell_grid.N[2];
        if (q.cell_grid.N[0] < 1 || q.cell_grid.N[1] < 1 || q.cell_grid.N[2] < 1 || q.n_atoms < 0 || q.twojmax < 2 || q.twojmax > mala::kMaxTwojmax || (q.twojmax & 1) ||
            q.egrid.n < 2 || q.egrid.n > mala::kMlpMaxOut || !(q.egrid.de > 0) || !(q.T_kelvin > 0) || !(q.rcut > 0))
            return sfail(MALA_E_INVALID_ARG, "reserve: invalid request");
        const mala::PredictPlan pk = mala::plan_predict(&q.cell_grid, q.n_atoms, q.rcut, q.twojmax, &q.egrid,
                                                        q.T_kelvin, q.density_out != nullptr, 0, false);
        p = k ? mala::plan_max(p, pk) : pk;
        if (q.density_out && np > max_pts) max_pts = np;
    }
    Request probe;
    probe.plan = p;
    probe.n_pts = max_pts;
    probe.density_out = max_pts ? reinterpret_cast<double*>(&probe) : nullptr;
    const size_t per_slot = footprint(probe);
    if (per_slot * (size_t)sv->ex->slots() > sv->budget)
        return sfail(MALA_E_OOM, "reserve: the slots would exceed the HBM budget");
    // the scheduler is idle (nothing queued or running) and admits nothing
    // while the lock is held, so the slots can be sized from this thread
    mala_status st = sv->ex->reserve(p, max_pts);
    for (int i = 0; i < sv->ex->slots(); ++i) sv->bytes[i] = sv->ex->slot_bytes(i);
    sv->allocs = sv->ex->allocs();
    if (sv->held() > sv->peak_bytes) sv->peak_bytes = sv->held();
    if (st) return sfail(st, mala_last_error());
    sv->reserved_bytes = per_slot;
    return MALA_OK;
}

mala_status mala_server_set_inflight_points(mala_server* sv, int64_t max_points) {
    if (!sv || max_points < 0) return sfail(MALA_E_INVALID_ARG, "inflight points must be >= 0");
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->inflight_cap = max_points;
    sv->cv_work.notify_all();
    return MALA_OK;
}

mala_status mala_server_stats(mala_server* sv, double* stats) {
    if (!sv || !stats) return MALA_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    int run = 0;
    for (auto* r : sv->running) run += r != nullptr;
    stats[0] = (double)sv->queue.size();
    stats[1] = (double)run;
    stats[2] = (double)sv->held();
    stats[3] = (double)sv->peak_bytes;
    stats[4] = (double)sv->budget;
    stats[5] = (double)sv->allocs;
    stats[6] = (double)sv->reserved_bytes;
    return MALA_OK;
}

const char* mala_server_last_error(void) { return g_serr.c_str(); }

}  // extern "C"
