// Serving loop: snapshots of different sizes arrive over time (as in an MD
// trajectory driven through the method's calculator interface, Sec. 4) and
// are run on one GPU with continuous admission.
//
// A scheduler thread owns a fixed set of slots.  Each slot is a library
// context with its own HIP stream and device state (cell list, u scratch, B
// cache, energy window, DOS partials, outputs), so the kernels of requests in
// different slots overlap on the device.  Requests are admitted strictly in
// arrival order (no overtaking, hence no starvation) whenever a slot is free
// and the device memory held by all slots plus what the request needs stays
// within the budget; idle slots give their cached buffers back first when the
// budget is tight.  Each request runs exactly the single-snapshot path with
// its own fixed work partition, so its result does not depend on what else is
// in flight.
//
// The executor is an interface: the GPU executor above, or a host-only mock
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
    size_t need = 0;                 // device bytes
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
    virtual size_t slot_bytes(int s) = 0;
    virtual void trim(int s) = 0;
    virtual mala_status launch(int s, Request& r) = 0;
    virtual bool done(int s) = 0;
    virtual mala_status finish(int s, Request& r) = 0;
};

// ------------------------------------------------------------------ GPU
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
};

struct GpuExecutor : Executor {
    int device;
    mala_weights* w = nullptr;
    std::vector<GpuSlot> s;
    GpuExecutor(int dev, int n) : device(dev), s(n) {}
    ~GpuExecutor() override {
        (void)hipSetDevice(device);
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
            if (x.stream) (void)hipStreamDestroy(x.stream);
        }
        if (w) mala_weights_free(w);
    }
    mala_status init(const void* blob, size_t bytes, int32_t precision) {
        (void)hipSetDevice(device);
        for (auto& x : s) {
            if (hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking) != hipSuccess) return MALA_E_HIP;
            if (hipEventCreateWithFlags(&x.ev, hipEventDisableTiming) != hipSuccess) return MALA_E_HIP;
            mala_status st = mala_create(device, x.stream, &x.ctx);
            if (st) return st;
            if (hipMalloc(&x.dos, sizeof(double) * 256) != hipSuccess) return MALA_E_OOM;
            if (hipMalloc(&x.res, sizeof(mala_result)) != hipSuccess) return MALA_E_OOM;
            if (hipHostMalloc(&x.h_dos, sizeof(double) * 256, hipHostMallocDefault) != hipSuccess) return MALA_E_OOM;
            if (hipHostMalloc(&x.h_res, sizeof(mala_result), hipHostMallocDefault) != hipSuccess) return MALA_E_OOM;
        }
        return mala_weights_load(s[0].ctx, blob, bytes, precision, &w);
    }
    int slots() const override { return (int)s.size(); }
    size_t slot_bytes(int i) override { return mala::ctx_device_bytes(s[i].ctx) + s[i].cap_dens * sizeof(double); }
    void trim(int i) override {
        (void)hipSetDevice(device);
        mala::ctx_trim(s[i].ctx);
        if (s[i].dens) (void)hipFree(s[i].dens);
        if (s[i].h_dens) (void)hipHostFree(s[i].h_dens);
        s[i].dens = nullptr;
        s[i].h_dens = nullptr;
        s[i].cap_dens = 0;
    }
    mala_status launch(int i, Request& r) override {
        (void)hipSetDevice(device);
        GpuSlot& x = s[i];
        if (r.density_out && x.cap_dens < (size_t)r.n_pts) {
            if (x.dens) (void)hipFree(x.dens);
            if (x.h_dens) (void)hipHostFree(x.h_dens);
            x.dens = nullptr;
            x.h_dens = nullptr;
            x.cap_dens = 0;
            if (hipMalloc(&x.dens, sizeof(double) * r.n_pts) != hipSuccess) return MALA_E_OOM;
            if (hipHostMalloc(&x.h_dens, sizeof(double) * r.n_pts, hipHostMallocDefault) != hipSuccess)
                return MALA_E_OOM;
            x.cap_dens = r.n_pts;
        }
        mala_status st = mala_predict(x.ctx, w, r.pos.data(), r.n_atoms, &r.cg, r.rcut, r.twojmax, &r.eg, r.T, r.ne,
                                      x.dos, r.density_out ? x.dens : nullptr, static_cast<mala_result*>(x.res),
                                      nullptr);
        if (st) return st;
        if (hipMemcpyAsync(x.h_dos, x.dos, sizeof(double) * r.eg.n, hipMemcpyDeviceToHost, x.stream) != hipSuccess ||
            hipMemcpyAsync(x.h_res, x.res, sizeof(mala_result), hipMemcpyDeviceToHost, x.stream) != hipSuccess)
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
        return mala_check_device_errors(x.ctx);
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
    MockExecutor(int n, double ns, Clock::time_point t) : s(n), ns_per_point(ns), t0(t) {}
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    int slots() const override { return (int)s.size(); }
    size_t slot_bytes(int i) override { return s[i].bytes; }
    void trim(int i) override { s[i].bytes = 0; }
    mala_status launch(int i, Request& r) override {
        if (s[i].bytes < r.need) s[i].bytes = r.need;
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

// Device bytes mala_predict holds for one request (matches its allocations).
size_t footprint(const Request& r) {
    using namespace mala;
    const int64_t N = r.n_pts;
    const size_t nb = (size_t)n_triples(r.twojmax);
    const int64_t chunk = N < (1 << 19) ? N : (1 << 19);
    const size_t tiles = (size_t)((chunk + kTile - 1) / kTile);
    const double kT = kBoltzmannEv * r.T;
    size_t wmax = (size_t)std::min(r.eg.n, (int)ceil(2.0 * (40.0 * kT + 0.3) / r.eg.de) + 3);
    size_t b = 0;
    b += (size_t)N * nb * 4;                           // B cache
    b += tiles * n_half(r.twojmax) * kTile * 8;        // u scratch
    b += (size_t)kMlpBlocks * kMlpMaxOut * 8 * 2;      // DOS partials
    if (r.density_out) b += (size_t)N * (wmax * 4 + 8 + 8);   // window, prefix, density
    b += (size_t)r.n_atoms * 80 + (1 << 20);           // positions, cells, small records
    return b + b / 8;                                  // growth slack of the buffers
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
    std::vector<Request*> running;
    uint64_t next_ticket = 1;
    bool stop = false;
    size_t peak_bytes = 0;
    std::thread th;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    size_t held() {
        size_t h = 0;
        for (int i = 0; i < ex->slots(); ++i) h += ex->slot_bytes(i);
        return h;
    }

    void loop(bool gpu) {
        if (gpu) (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            // completions
            for (int i = 0; i < ex->slots(); ++i) {
                Request* r = running[i];
                if (r && ex->done(i)) {
                    mala_status st = ex->finish(i, *r);
                    if (st && !r->status) {
                        r->status = st;
                        r->err = mala_last_error();
                    }
                    r->t_done = now();
                    r->state = 2;
                    running[i] = nullptr;
                    cv_done.notify_all();
                }
            }
            // admissions, strictly in arrival order
            while (!queue.empty()) {
                Request* r = queue.front();
                int slot = -1;
                for (int i = 0; i < ex->slots(); ++i)
                    if (!running[i] && (slot < 0 || ex->slot_bytes(i) > ex->slot_bytes(slot))) slot = i;
                if (slot < 0) break;
                auto grow = [&]() {
                    const size_t cur = ex->slot_bytes(slot);
                    return r->need > cur ? r->need - cur : 0;
                };
                if (held() + grow() > budget) {
                    for (int i = 0; i < ex->slots(); ++i)
                        if (!running[i] && i != slot) ex->trim(i);
                    if (held() + grow() > budget) ex->trim(slot);
                    if (held() + grow() > budget) break;      // wait for running work to finish
                }
                queue.pop_front();
                r->t_start = now();
                r->state = 1;
                mala_status st = ex->launch(slot, *r);
                const size_t h = held() > r->need ? held() : r->need;
                if (h > peak_bytes) peak_bytes = h;
                if (st) {
                    r->status = st;
                    r->err = mala_last_error();
                    r->t_done = now();
                    r->state = 2;
                    cv_done.notify_all();
                    continue;
                }
                running[slot] = r;
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
    if (r->n_pts <= 0 || r->twojmax < 2 || r->twojmax > mala::kMaxTwojmax || (r->twojmax & 1) ||
        r->eg.n < 2 || r->eg.n > mala::kMlpMaxOut || !(r->eg.de > 0) || !(r->T > 0))
        return MALA_E_INVALID_ARG;
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
    return MALA_OK;
}

const char* mala_server_last_error(void) { return g_serr.c_str(); }

}  // extern "C"
