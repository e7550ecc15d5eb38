// C ABI of the gfx950 grid-inference library: argument checks, scratch
// management, weight packing and launch sequencing.  All arithmetic of the
// path runs in the HIP kernels of this directory.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include <stddef.h>

#include "mala.h"
#include "ace.h"
#include "mala_internal.h"

using namespace mala;

// the kernels write mala_result through their own record type
static_assert(sizeof(mala_result) == sizeof(ResultRec), "result record layout");
static_assert(offsetof(mala_result, status) == offsetof(ResultRec, status), "result record layout");
static_assert(offsetof(mala_result, entropy) == offsetof(ResultRec, entropy), "result record layout");
static_assert(offsetof(mala_result, e_entropy) == offsetof(ResultRec, e_entropy), "result record layout");

namespace {

thread_local std::string g_err;

mala_status fail(mala_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? MALA_E_OOM : MALA_E_HIP,             \
                        std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;   // elements
};

// Elements a buffer is grown to when it must hold n (slack against regrowth).
inline size_t grown_size(size_t n) { return n + n / 8 + 64; }

template <typename T>
hipError_t ensure(uint64_t& n_allocs, DevBuf<T>& b, size_t n) {
    if (n <= b.cap) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);    // synchronising: no kernel still uses it
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = grown_size(n);
    ++n_allocs;
    hipError_t e = hipMalloc(&b.p, want * sizeof(T));
    if (e != hipSuccess) return e;
    b.cap = want;
    return hipSuccess;
}

template <typename T>
void release(DevBuf<T>& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

struct TjTables {
    bool ready = false;
    float* cg = nullptr;
    int* cg_off = nullptr;
    int* waves = nullptr;
    int zb_waves = 0;
    bool adj_ready = false;      // descriptor adjoint: coupled-pair CG blocks, wave unit plan
    float* cgy = nullptr;
    int* cgy_off = nullptr;
    int* yunits = nullptr;
};

constexpr int kChunk = 1 << 19;          // grid points per descriptor chunk
// grid points per descriptor chunk of the fused path: more points per
// k_ui / k_zb launch shrink the share of each launch's tail, where the last
// blocks finish alone (2^19 -> 2^20 -> 2^21: 0.5% and 0.3% of a slab
// snapshot; 4.5 GB of u scratch per context at twojmax 10)
constexpr int kPredictChunk = 1 << 21;
constexpr double kWindowMargin = 0.3;     // eV around the E_F estimate kept in the stored LDOS window

struct Ace4Tables {
    bool ready = false;
    int n4 = 0, max_slots = 0, n_phases = 0;
    int* l_units = nullptr;           // unit and descriptor offsets per phase
    int4* units = nullptr;
    float* coef = nullptr;
    int* l_descs = nullptr;
    int4* descs = nullptr;
};

struct AceTables {
    bool ready = false;
    int n3 = 0, n_groups = 0;
    int* groups = nullptr;            // point-major plan
    int* groups_dm = nullptr;         // descriptor-major order
    int n_groups_dm = 0;
    float* coef = nullptr;
};

}  // namespace

struct mala_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuf<double> pos;
    double* pos_stage = nullptr;         // pinned staging for positions
    size_t pos_stage_cap = 0;
    hipEvent_t stage_ev = nullptr;
    DevBuf<int> cell_count, cell_start, cell_fill, atom_cell;
    DevBuf<double4> atoms_tmp, atoms_sorted;
    DevBuf<float2> u;
    DevBuf<float2> yadj;                 // dL/du of the descriptor adjoint, laid out like u
    DevBuf<float2> aceA;                 // projected grid ACE basis of one chunk [tile][60][64]
    DevBuf<float> ace4S;                 // rank-4 descriptor planes of one point-major chunk
    DevBuf<float> Bbuf;
    DevBuf<double> partials, est_partials;
    DevBuf<double> fermi_w;
    DevBuf<float> window;
    DevBuf<double> prefix;
    WindowRec* win = nullptr;
    int density_mode = 0;              // 0: stored energy window (recompute if not covered), 1: recompute
    int* err = nullptr;
    double* li_coef = nullptr;
    uint64_t n_allocs = 0;               // device/pinned allocations made by this context
    TjTables tj[kMaxTwojmax + 1];
    AceTables ace[kAceMaxN + 1][kAceMaxL + 1];
    Ace4Tables ace4[kAce4MaxN + 1][kAce4MaxL + 1];
    // stage timing
    bool prof_on = false;
    struct Rec {
        int stage;
        hipEvent_t a, b;
        int64_t pts;
    };
    std::vector<Rec> prof_pending;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[MALA_N_STAGES] = {};
    int64_t prof_n[MALA_N_STAGES] = {}, prof_pts[MALA_N_STAGES] = {};
};

struct mala_weights {
    int device = 0;
    MlpArgs args{};
    std::vector<void*> allocs;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

hipEvent_t pool_event(mala_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch `fn` as one stage; with timing on, bracket it with events.
template <typename F>
hipError_t staged(mala_ctx* c, int stage, int64_t pts, F&& fn) {
    if (!c->prof_on) return fn();
    hipEvent_t a = pool_event(c), b = pool_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, c->stream);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, c->stream);
    c->prof_pending.push_back({stage, a, b, pts});
    return e;
}

// Subsample of the E_F estimate: every s-th point, s at least 61 and grown
// on large grids so that about 2^18 points are sampled (the estimate only has
// to place the stored energy window, whose margin is 0.3 eV; 65,000 points
// already land within 2e-4 eV), s a prime that divides neither a row nor a
// plane of the grid, so the samples do not line up with its structure.
constexpr int64_t kEstStrideMin = 61;
constexpr int64_t kEstSamples = int64_t(1) << 18;

int64_t est_stride(const mala_cell_grid* cg) {
    const int64_t row = cg->N[2], plane = (int64_t)cg->N[1] * cg->N[2];
    const int64_t ntot = plane * cg->N[0];
    int64_t s = ntot / kEstSamples > kEstStrideMin ? ntot / kEstSamples : kEstStrideMin;
    auto prime = [](int64_t v) {
        for (int64_t d = 2; d * d <= v; ++d)
            if (v % d == 0) return false;
        return true;
    };
    while (!prime(s) || row % s == 0 || plane % s == 0) ++s;
    return s;
}

__global__ void k_set_covered(WindowRec* w, int v) {
    if (threadIdx.x == 0) {
        w->covered = v;
        w->valid = v;
    }
}

hipError_t set_covered(mala_ctx* c, int v) {
    hipLaunchKernelGGL(k_set_covered, dim3(1), dim3(64), 0, c->stream, c->win, v);
    return hipGetLastError();
}

mala_status ensure_tables(mala_ctx* c, int tj) {
    TjTables& t = c->tj[tj];
    if (t.ready) return MALA_OK;
    std::vector<float> tab(32768);
    std::vector<int> off(n_triples(tj));
    int n = build_cg_table(tj, tab.data(), off.data(), (int)tab.size());
    if (n < 0) return fail(MALA_E_UNSUPPORTED, "Clebsch-Gordan table too large");
    t.zb_waves = 12;      // three waves per SIMD share the LDS tile
    std::vector<int> waves(t.zb_waves * kMaxZbStride, 0);
    plan_zb_waves(tj, t.zb_waves, waves.data(), kMaxZbStride);
    c->n_allocs += 3;
    HIP_TRY(hipMalloc(&t.cg, sizeof(float) * (n > 0 ? n : 1)));
    HIP_TRY(hipMalloc(&t.cg_off, sizeof(int) * off.size()));
    HIP_TRY(hipMalloc(&t.waves, sizeof(int) * waves.size()));
    HIP_TRY(hipMemcpy(t.cg, tab.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t.cg_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t.waves, waves.data(), sizeof(int) * waves.size(), hipMemcpyHostToDevice));
    t.ready = true;
    return MALA_OK;
}

mala_status ensure_adjoint_tables(mala_ctx* c, int tj) {
    TjTables& t = c->tj[tj];
    if (t.adj_ready) return MALA_OK;
    std::vector<float> tab(65536);
    std::vector<int> off(n_combos(tj));
    const int n = build_cg_table_adjoint(tj, tab.data(), off.data(), (int)tab.size());
    if (n < 0) return fail(MALA_E_UNSUPPORTED, "Clebsch-Gordan table of the adjoint too large");
    const int nw = y_max_waves(), ng = y_group_count(tj);
    std::vector<int> units((size_t)ng * nw * kMaxYStride, 0);       // one plan per level group
    for (int g = 0; g < ng; ++g)
        plan_y_units(tj, y_group_first(tj, g), y_group_last(tj, g), y_group_wave_count(tj, g),
                     units.data() + (size_t)g * nw * kMaxYStride, kMaxYStride);
    c->n_allocs += 3;
    HIP_TRY(hipMalloc(&t.cgy, sizeof(float) * (n > 0 ? n : 1)));
    HIP_TRY(hipMalloc(&t.cgy_off, sizeof(int) * off.size()));
    HIP_TRY(hipMalloc(&t.yunits, sizeof(int) * units.size()));
    HIP_TRY(hipMemcpy(t.cgy, tab.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t.cgy_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t.yunits, units.data(), sizeof(int) * units.size(), hipMemcpyHostToDevice));
    t.adj_ready = true;
    return MALA_OK;
}

bool finite3(const double* v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

mala_status check_geometry(const double* positions, int32_t n_atoms, const mala_cell_grid* cg,
                           double rcut, int32_t twojmax) {
    if (!cg) return fail(MALA_E_INVALID_ARG, "cell_grid is NULL");
    if (n_atoms < 0) return fail(MALA_E_INVALID_ARG, "n_atoms < 0");
    if (n_atoms > 0 && !positions) return fail(MALA_E_INVALID_ARG, "positions is NULL");
    for (int d = 0; d < 3; ++d) {
        if (!(cg->L[d] > 0.0) || !isfinite(cg->L[d])) return fail(MALA_E_INVALID_ARG, "cell edge not positive");
        if (cg->N[d] < 1) return fail(MALA_E_INVALID_ARG, "grid size < 1");
    }
    if (!(rcut > 0.0) || !isfinite(rcut)) return fail(MALA_E_INVALID_ARG, "rcut not positive");
    if (twojmax < 2 || twojmax > kMaxTwojmax || (twojmax & 1))
        return fail(MALA_E_UNSUPPORTED, "twojmax must be one of 2, 4, 6, 8, 10");
    for (int i = 0; i < n_atoms; ++i)
        if (!finite3(positions + 3 * i)) return fail(MALA_E_INVALID_ARG, "non-finite atom position");
    return MALA_OK;
}

mala_status upload_positions(mala_ctx* c, const double* positions, int32_t n_atoms) {
    const size_t n = (size_t)3 * (n_atoms > 0 ? n_atoms : 1);
    HIP_TRY(ensure(c->n_allocs, c->pos, n));
    if (n_atoms == 0) return MALA_OK;
    HIP_TRY(hipEventSynchronize(c->stage_ev));          // previous copy out of the stage is done
    if (c->pos_stage_cap < n) {
        if (c->pos_stage) HIP_TRY(hipHostFree(c->pos_stage));
        c->pos_stage = nullptr;
        ++c->n_allocs;
        HIP_TRY(hipHostMalloc(&c->pos_stage, sizeof(double) * n, hipHostMallocDefault));
        c->pos_stage_cap = n;
    }
    memcpy(c->pos_stage, positions, sizeof(double) * 3 * n_atoms);
    HIP_TRY(hipMemcpyAsync(c->pos.p, c->pos_stage, sizeof(double) * 3 * n_atoms, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipEventRecord(c->stage_ev, c->stream));
    return MALA_OK;
}

// Entries of the cell-count arrays of a cell list for cutoff rcut (cells of
// edge >= rcut / 2, at most 256 per edge, plus one).
size_t cell_entries(const mala_cell_grid* cg, double rcut) {
    size_t nc_est = 1;
    for (int d = 0; d < 3; ++d) {
        int nc = (int)floor(cg->L[d] / (0.5 * rcut));
        nc = nc < 1 ? 1 : (nc > 256 ? 256 : nc);
        nc_est *= nc;
    }
    return nc_est + 1;
}

// u scratch elements of one descriptor chunk (at most chunk_max points) of a
// grid of ntot points.
size_t u_elements(int64_t ntot, int twojmax, int64_t chunk_max = kChunk) {
    const int64_t chunk = ntot < chunk_max ? ntot : chunk_max;
    return (size_t)((chunk + kTile - 1) / kTile) * n_half(twojmax) * kTile;
}

// Energies of the stored LDOS window of the single-pass density.
int window_width(const mala_egrid* eg, double T) {
    const double kT = kBoltzmannEv * T;
    return std::min(eg->n, (int)ceil(2.0 * (40.0 * kT + kWindowMargin) / eg->de) + 3);
}

// Cell list of the uploaded atoms for neighbour searches within rcut.
mala_status bin_atoms(mala_ctx* c, int32_t n_atoms, const mala_cell_grid* cg, double rcut, BinState* bs) {
    const size_t ncell = cell_entries(cg, rcut);
    const size_t na = n_atoms > 0 ? n_atoms : 1;
    HIP_TRY(ensure(c->n_allocs, c->cell_count, ncell));
    HIP_TRY(ensure(c->n_allocs, c->cell_start, ncell));
    HIP_TRY(ensure(c->n_allocs, c->cell_fill, ncell));
    HIP_TRY(ensure(c->n_allocs, c->atom_cell, na));
    HIP_TRY(ensure(c->n_allocs, c->atoms_tmp, na));
    HIP_TRY(ensure(c->n_allocs, c->atoms_sorted, na));
    HIP_TRY(staged(c, MALA_STAGE_BIN, 0, [&] {
        return launch_bin(c->stream, c->pos.p, n_atoms, cg->L, rcut, c->cell_count.p, c->cell_start.p,
                          c->cell_fill.p, c->atoms_tmp.p, c->atom_cell.p, c->atoms_sorted.p, bs);
    }));
    return MALA_OK;
}

mala_status run_descriptors(mala_ctx* c, int32_t n_atoms, const mala_cell_grid* cg, double rcut,
                            int32_t twojmax, int64_t pt_begin, int64_t pt_end, float* B_out,
                            int64_t chunk_max = kChunk) {
    BinState bs{};
    mala_status st = bin_atoms(c, n_atoms, cg, rcut, &bs);
    if (st) return st;
    const int nB = n_triples(twojmax);
    const int64_t total = pt_end - pt_begin;
    const int64_t chunk = total < chunk_max ? total : chunk_max;
    HIP_TRY(ensure(c->n_allocs, c->u, u_elements(total, twojmax, chunk_max)));
    const TjTables& t = c->tj[twojmax];
    for (int64_t off = 0; off < total; off += chunk) {
        const int64_t n = (total - off) < chunk ? (total - off) : chunk;
        HIP_TRY(staged(c, MALA_STAGE_UI, n, [&] {
            return launch_ui(c->stream, twojmax, bs, cg->N, rcut, pt_begin + off, n, c->u.p, c->err);
        }));
        HIP_TRY(staged(c, MALA_STAGE_ZB, n, [&] {
            return launch_zb(c->stream, twojmax, n, c->u.p, B_out + off * nB, t.cg, t.cg_off, t.waves,
                             t.zb_waves);
        }));
    }
    return MALA_OK;
}

// Partial rows of the stored-LDOS column sums: one per point up to
// kIntegrateMaxParts (the same partition in both integrate entry points).
int integrate_parts(int64_t n_pts) {
    return n_pts < kIntegrateMaxParts ? (int)(n_pts > 0 ? n_pts : 1) : kIntegrateMaxParts;
}

mala_status check_egrid(const mala_egrid* eg, double T, double ne) {
    if (!eg) return fail(MALA_E_INVALID_ARG, "egrid is NULL");
    if (eg->n < 2 || eg->n > kMlpMaxOut) return fail(MALA_E_UNSUPPORTED, "energy grid size must be 2..256");
    if (!(eg->de > 0.0) || !isfinite(eg->de) || !isfinite(eg->e0))
        return fail(MALA_E_INVALID_ARG, "bad energy grid");
    if (!(T > 0.0) || !isfinite(T)) return fail(MALA_E_INVALID_ARG, "temperature must be positive");
    if (!(ne > 0.0) || !isfinite(ne)) return fail(MALA_E_INVALID_ARG, "n_electrons must be positive");
    return MALA_OK;
}

mala_status check_integrate_args(mala_ctx* c, const float* ldos, int64_t n_pts, double dV, const mala_egrid* eg,
                                 double T, double ne, double* dos_out, mala_result* result) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    mala_status st = check_egrid(eg, T, ne);
    if (st) return st;
    if (n_pts < 0) return fail(MALA_E_INVALID_ARG, "n_pts < 0");
    if (!(dV > 0.0) || !isfinite(dV)) return fail(MALA_E_INVALID_ARG, "dV must be positive");
    if (!dos_out || !result || (n_pts > 0 && !ldos)) return fail(MALA_E_INVALID_ARG, "NULL buffer");
    return MALA_OK;
}

}  // namespace

namespace mala {

template <typename T>
static size_t bytes_of(const DevBuf<T>& b) {
    return b.cap * sizeof(T);
}

size_t ctx_device_bytes(mala_ctx* c) {
    return bytes_of(c->pos) + bytes_of(c->cell_count) + bytes_of(c->cell_start) + bytes_of(c->cell_fill) +
           bytes_of(c->atom_cell) + bytes_of(c->atoms_tmp) + bytes_of(c->atoms_sorted) + bytes_of(c->u) +
           bytes_of(c->Bbuf) + bytes_of(c->partials) + bytes_of(c->est_partials) + bytes_of(c->fermi_w) +
           bytes_of(c->window) + bytes_of(c->prefix);
}

uint64_t ctx_alloc_count(mala_ctx* c) { return c->n_allocs; }

int* ctx_error_flags(mala_ctx* c) { return c->err; }

// Elements of every context buffer mala_predict uses for one request
// (positions, cell list, u scratch, B cache unless the caller owns it,
// partial rows, window and prefix of the single-pass density).
PredictPlan plan_predict(const mala_cell_grid* cg, int32_t n_atoms, double rcut, int32_t twojmax,
                         const mala_egrid* eg, double T, bool density, int density_mode, bool caller_b_cache) {
    PredictPlan p{};
    const int64_t ntot = (int64_t)cg->N[0] * cg->N[1] * cg->N[2];
    const size_t na = n_atoms > 0 ? (size_t)n_atoms : 1;
    p.twojmax = twojmax;
    p.pos = 3 * na;
    p.cells = cell_entries(cg, rcut);
    p.atoms = na;
    p.u = u_elements(ntot, twojmax, kPredictChunk);
    p.B = caller_b_cache ? 0 : (size_t)ntot * n_triples(twojmax);
    p.partials = (size_t)mlp_blocks(ntot) * kMlpMaxOut;
    p.fermi_w = kMlpMaxOut;
    if (density && density_mode == 0) {
        const int64_t stride = est_stride(cg);
        const int64_t n_est = (ntot + stride - 1) / stride;
        p.est_partials = (size_t)mlp_blocks(n_est) * kMlpMaxOut;
        p.window = (size_t)ntot * window_width(eg, T);
        p.prefix = (size_t)ntot;
    }
    return p;
}

PredictPlan plan_max(const PredictPlan& a, const PredictPlan& b) {
    PredictPlan p{};
    p.twojmax = a.twojmax > b.twojmax ? a.twojmax : b.twojmax;
#define MALA_PLAN_MAX(f) p.f = a.f > b.f ? a.f : b.f
    MALA_PLAN_MAX(pos); MALA_PLAN_MAX(cells); MALA_PLAN_MAX(atoms); MALA_PLAN_MAX(u); MALA_PLAN_MAX(B);
    MALA_PLAN_MAX(partials); MALA_PLAN_MAX(fermi_w); MALA_PLAN_MAX(est_partials); MALA_PLAN_MAX(window);
    MALA_PLAN_MAX(prefix);
#undef MALA_PLAN_MAX
    return p;
}

// Device bytes the context would add to run a request of this plan: the sum
// over buffers of what each one grows by (a buffer that already holds enough
// adds nothing; one that grows is reallocated at grown_size).
size_t plan_growth_bytes(mala_ctx* c, const PredictPlan& p) {
    size_t g = 0;
    auto add = [&](const auto& b, size_t n, size_t elem) {
        if (n > b.cap) g += grown_size(n) * elem - b.cap * elem;
    };
    add(c->pos, p.pos, 8);
    add(c->cell_count, p.cells, 4); add(c->cell_start, p.cells, 4); add(c->cell_fill, p.cells, 4);
    add(c->atom_cell, p.atoms, 4); add(c->atoms_tmp, p.atoms, 32); add(c->atoms_sorted, p.atoms, 32);
    add(c->u, p.u, 8); add(c->Bbuf, p.B, 4); add(c->partials, p.partials, 8); add(c->fermi_w, p.fermi_w, 8);
    add(c->est_partials, p.est_partials, 8); add(c->window, p.window, 4); add(c->prefix, p.prefix, 8);
    return g;
}

// Grow every buffer of the plan now (and upload the Clebsch-Gordan tables
// and size the pinned position stage), so that later requests within the
// plan allocate nothing.
mala_status ctx_reserve(mala_ctx* c, const PredictPlan& p) {
    DeviceGuard g(c->device);
    mala_status st = ensure_tables(c, p.twojmax);
    if (st) return st;
    HIP_TRY(ensure(c->n_allocs, c->pos, p.pos));
    HIP_TRY(ensure(c->n_allocs, c->cell_count, p.cells));
    HIP_TRY(ensure(c->n_allocs, c->cell_start, p.cells));
    HIP_TRY(ensure(c->n_allocs, c->cell_fill, p.cells));
    HIP_TRY(ensure(c->n_allocs, c->atom_cell, p.atoms));
    HIP_TRY(ensure(c->n_allocs, c->atoms_tmp, p.atoms));
    HIP_TRY(ensure(c->n_allocs, c->atoms_sorted, p.atoms));
    HIP_TRY(ensure(c->n_allocs, c->u, p.u));
    if (p.B) HIP_TRY(ensure(c->n_allocs, c->Bbuf, p.B));
    HIP_TRY(ensure(c->n_allocs, c->partials, p.partials));
    HIP_TRY(ensure(c->n_allocs, c->fermi_w, p.fermi_w));
    if (p.window) {
        HIP_TRY(ensure(c->n_allocs, c->est_partials, p.est_partials));
        HIP_TRY(ensure(c->n_allocs, c->window, p.window));
        HIP_TRY(ensure(c->n_allocs, c->prefix, p.prefix));
    }
    if (c->pos_stage_cap < p.pos) {
        HIP_TRY(hipEventSynchronize(c->stage_ev));
        if (c->pos_stage) HIP_TRY(hipHostFree(c->pos_stage));
        c->pos_stage = nullptr;
        ++c->n_allocs;
        HIP_TRY(hipHostMalloc(&c->pos_stage, sizeof(double) * p.pos, hipHostMallocDefault));
        c->pos_stage_cap = p.pos;
    }
    return MALA_OK;
}

void ctx_trim(mala_ctx* c) {
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    release(c->u);
    release(c->yadj);
    release(c->aceA);
    release(c->ace4S);
    release(c->Bbuf);
    release(c->window);
    release(c->prefix);
    release(c->partials);
    release(c->est_partials);
}

}  // namespace mala

// ====================================================================== ABI
extern "C" {

const char* mala_last_error(void) { return g_err.c_str(); }
const char* mala_version(void) { return "mala-gfx950 0.1.0"; }

int32_t mala_n_descriptors(int32_t twojmax) {
    if (twojmax < 0) return -1;
    return (twojmax + 2) * (twojmax + 3) * (twojmax + 4) / 24;
}

mala_status mala_create(int32_t device, void* stream, mala_ctx** out) {
    if (!out) return fail(MALA_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(MALA_E_INVALID_ARG, "no such device");
    DeviceGuard g(device);
    mala_ctx* c = new mala_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&c->err, sizeof(int));
    if (e == hipSuccess) e = hipMemset(c->err, 0, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&c->li_coef, sizeof(double) * kLiCoef);
    if (e == hipSuccess) e = hipMalloc(&c->win, sizeof(WindowRec));
    if (e == hipSuccess) {      // this device's fixed scratch of mala_integrate_noalloc
        double* scr = nullptr;
        e = scratch_device_ptr(device, &scr);
    }
    if (e == hipSuccess) {
        double coef[kLiCoef];
        polylog_coefficients(coef);
        e = hipMemcpy(c->li_coef, coef, sizeof(coef), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipEventRecord(c->stage_ev, c->stream);
    if (e != hipSuccess) {
        mala_destroy(c);
        return fail(MALA_E_HIP, std::string("context setup: ") + hipGetErrorString(e));
    }
    *out = c;
    return MALA_OK;
}

mala_status mala_destroy(mala_ctx* c) {
    if (!c) return MALA_OK;
    DeviceGuard g(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    release(c->pos);
    release(c->cell_count);
    release(c->cell_start);
    release(c->cell_fill);
    release(c->atom_cell);
    release(c->atoms_tmp);
    release(c->atoms_sorted);
    release(c->u);
    release(c->yadj);
    release(c->aceA);
    release(c->ace4S);
    release(c->Bbuf);
    release(c->partials);
    release(c->est_partials);
    release(c->fermi_w);
    release(c->window);
    release(c->prefix);
    if (c->win) (void)hipFree(c->win);
    if (c->pos_stage) (void)hipHostFree(c->pos_stage);
    if (c->err) (void)hipFree(c->err);
    if (c->li_coef) (void)hipFree(c->li_coef);
    for (auto& row : c->ace)
        for (auto& a : row) {
            if (a.groups) (void)hipFree(a.groups);
            if (a.groups_dm) (void)hipFree(a.groups_dm);
            if (a.coef) (void)hipFree(a.coef);
        }
    for (auto& row : c->ace4)
        for (auto& a : row) {
            if (a.l_units) (void)hipFree(a.l_units);
            if (a.units) (void)hipFree(a.units);
            if (a.coef) (void)hipFree(a.coef);
            if (a.l_descs) (void)hipFree(a.l_descs);
            if (a.descs) (void)hipFree(a.descs);
        }
    for (auto& t : c->tj) {
        if (t.cg) (void)hipFree(t.cg);
        if (t.cg_off) (void)hipFree(t.cg_off);
        if (t.waves) (void)hipFree(t.waves);
        if (t.cgy) (void)hipFree(t.cgy);
        if (t.cgy_off) (void)hipFree(t.cgy_off);
        if (t.yunits) (void)hipFree(t.yunits);
    }
    if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
    for (auto& r : c->prof_pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
    return MALA_OK;
}

mala_status mala_set_stream(mala_ctx* c, void* stream) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    c->stream = static_cast<hipStream_t>(stream);
    return MALA_OK;
}

mala_status mala_synchronize(mala_ctx* c) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    DeviceGuard g(c->device);
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MALA_OK;
}

mala_status mala_check_device_errors(mala_ctx* c) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    DeviceGuard g(c->device);
    HIP_TRY(hipStreamSynchronize(c->stream));
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, c->err, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(c->err, 0, sizeof(int)));
    if (flag & kErrCand) return fail(MALA_E_CAPACITY, "more than 1024 atom images near one 64-point tile");
    if (flag & kErrNbr) return fail(MALA_E_CAPACITY, "more than 128 neighbours within rcut of a grid point");
    return MALA_OK;
}

mala_status mala_set_density_mode(mala_ctx* c, int32_t mode) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    if (mode != MALA_DENSITY_WINDOW && mode != MALA_DENSITY_RECOMPUTE) return fail(MALA_E_INVALID_ARG, "unknown density mode");
    c->density_mode = mode;
    return MALA_OK;
}

mala_status mala_profile_enable(mala_ctx* c, int32_t on) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    DeviceGuard g(c->device);
    if (on) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (auto& r : c->prof_pending) {
            c->ev_pool.push_back(r.a);
            c->ev_pool.push_back(r.b);
        }
        c->prof_pending.clear();
        for (int i = 0; i < MALA_N_STAGES; ++i) {
            c->prof_ms[i] = 0.0;
            c->prof_n[i] = c->prof_pts[i] = 0;
        }
    }
    c->prof_on = on != 0;
    return MALA_OK;
}

mala_status mala_profile_read(mala_ctx* c, double* ms, int64_t* launches, int64_t* points) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    DeviceGuard g(c->device);
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& r : c->prof_pending) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        c->prof_ms[r.stage] += t;
        c->prof_n[r.stage] += 1;
        c->prof_pts[r.stage] += r.pts;
        c->ev_pool.push_back(r.a);
        c->ev_pool.push_back(r.b);
    }
    c->prof_pending.clear();
    for (int i = 0; i < MALA_N_STAGES; ++i) {
        if (ms) ms[i] = c->prof_ms[i];
        if (launches) launches[i] = c->prof_n[i];
        if (points) points[i] = c->prof_pts[i];
    }
    return MALA_OK;
}

// ---------------------------------------------------------------- weights
mala_status mala_weights_load(mala_ctx* c, const void* blob, size_t bytes, int32_t precision,
                              mala_weights** out) {
    if (!c || !blob || !out) return fail(MALA_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (precision != MALA_PREC_FP32 && precision != MALA_PREC_BF16)
        return fail(MALA_E_INVALID_ARG, "unknown precision");
    const unsigned char* b = static_cast<const unsigned char*>(blob);
    size_t pos = 0;
    auto take = [&](void* dst, size_t n) {
        if (pos + n > bytes) return false;
        memcpy(dst, b + pos, n);
        pos += n;
        return true;
    };
    char magic[8];
    int32_t hdr[4];
    double slope;
    if (!take(magic, 8) || memcmp(magic, "MALANET1", 8) != 0) return fail(MALA_E_INVALID_ARG, "bad blob magic");
    if (!take(hdr, sizeof(hdr)) || hdr[0] != 1) return fail(MALA_E_INVALID_ARG, "bad blob version");
    const int nl = hdr[1], out_act = hdr[2];
    if (nl != 3) return fail(MALA_E_UNSUPPORTED, "only networks with 3 affine layers are supported");
    if (!take(&slope, 8) || !isfinite(slope)) return fail(MALA_E_INVALID_ARG, "bad slope");
    int32_t wid[4];
    if (!take(wid, sizeof(int32_t) * 4)) return fail(MALA_E_INVALID_ARG, "truncated blob");
    // 4 widths: (nl+1) even, no padding int
    for (int i = 0; i < 4; ++i)
        if (wid[i] < 1) return fail(MALA_E_INVALID_ARG, "bad layer width");
    const int n_in = wid[0], h1 = wid[1], h2 = wid[2], n_out = wid[3];
    if (n_in > kMlpMaxIn || h1 > kMlpMaxHidden || h2 > kMlpMaxHidden || n_out > kMlpMaxOut)
        return fail(MALA_E_UNSUPPORTED, "layer width beyond the library's limits");
    std::vector<double> mean(n_in), sd(n_in), W1((size_t)h1 * n_in), b1(h1), W2((size_t)h2 * h1), b2(h2),
        W3((size_t)n_out * h2), b3(n_out), osc(n_out), osh(n_out);
    bool ok = take(mean.data(), 8 * n_in) && take(sd.data(), 8 * n_in) && take(W1.data(), 8 * W1.size()) &&
              take(b1.data(), 8 * h1) && take(W2.data(), 8 * W2.size()) && take(b2.data(), 8 * h2) &&
              take(W3.data(), 8 * W3.size()) && take(b3.data(), 8 * n_out) && take(osc.data(), 8 * n_out) &&
              take(osh.data(), 8 * n_out);
    if (!ok) return fail(MALA_E_INVALID_ARG, "truncated blob");
    for (double v : sd)
        if (!(v > 0.0) || !isfinite(v)) return fail(MALA_E_INVALID_ARG, "input std must be positive");

    // padded shape for the precision: K multiple of the MFMA K (4 or 32)
    const bool bf = precision == MALA_PREC_BF16;
    auto ceil_div = [](int a, int b) { return (a + b - 1) / b; };
    const int KK = bf ? 32 : 4;
    // fp32 batches 4 K-steps (16 units): input padded to a multiple of 16
    const int in_pad = bf ? 32 * ceil_div(n_in, 32) : 16 * ceil_div(n_in, 16);
    const int h1t = bf ? 2 * ceil_div(h1, 32) : ceil_div(h1, 16);
    const int h2t = bf ? 2 * ceil_div(h2, 32) : ceil_div(h2, 16);
    const int ot = ceil_div(n_out, 16);
    const int KS1 = in_pad / KK, KS2 = h1t * 16 / KK, KS3 = h2t * 16 / KK;
    // A operand of MFMA tile (mt, s): lane l holds row 16 mt + l%16 and, for
    // bf16, k = 32 s + 8 (l/16) + q, q < 8; for fp32 the K order that makes
    // four consecutive K-steps contiguous per lane: k = 16 (s/4) + 4 (l/16) + s%4.
    auto pack = [&](const std::vector<double>& W, int fout, int fin, int mtiles, int ks, std::vector<float>& o) {
        const int per = KK / 4;
        o.assign((size_t)mtiles * ks * 64 * per, 0.f);
        for (int mt = 0; mt < mtiles; ++mt)
            for (int s = 0; s < ks; ++s)
                for (int lane = 0; lane < 64; ++lane)
                    for (int q = 0; q < per; ++q) {
                        const int row = 16 * mt + (lane & 15);
                        const int k = bf ? 32 * s + 8 * (lane >> 4) + q
                                         : 16 * (s / 4) + 4 * (lane >> 4) + (s % 4);
                        float v = 0.f;
                        if (row < fout && k < fin) v = (float)W[(size_t)row * fin + k];
                        o[(((size_t)mt * ks + s) * 64 + lane) * per + q] = v;
                    }
    };
    std::vector<float> P1, P2, P3;
    pack(W1, h1, n_in, h1t, KS1, P1);
    pack(W2, h2, h1, h2t, KS2, P2);
    pack(W3, n_out, h2, ot, KS3, P3);
    // transposed weights for the network's vector-Jacobian product (FP32
    // only): W^T is [in][out] row-major, packed like a layer with the widths
    // swapped; its K runs over the padded output units of the forward layer
    auto transpose = [](const std::vector<double>& W, int fout, int fin) {
        std::vector<double> t((size_t)fin * fout);
        for (int o = 0; o < fout; ++o)
            for (int i = 0; i < fin; ++i) t[(size_t)i * fout + o] = W[(size_t)o * fin + i];
        return t;
    };
    std::vector<float> T1, T2, T3;
    if (!bf) {
        pack(transpose(W1, h1, n_in), n_in, h1, in_pad / 16, h1t * 16 / KK, T1);
        pack(transpose(W2, h2, h1), h1, h2, h1t, h2t * 16 / KK, T2);
        pack(transpose(W3, n_out, h2), h2, n_out, h2t, ot * 16 / KK, T3);
    }
    auto padv = [](const std::vector<double>& v, int n) {
        std::vector<float> o(n, 0.f);
        for (size_t i = 0; i < v.size() && (int)i < n; ++i) o[i] = (float)v[i];
        return o;
    };
    std::vector<float> pb1 = padv(b1, 16 * h1t), pb2 = padv(b2, 16 * h2t), pb3 = padv(b3, 16 * ot);
    std::vector<float> pm = padv(mean, n_in), prs(n_in), psc = padv(osc, kMlpMaxOut), psh = padv(osh, kMlpMaxOut);
    for (int i = 0; i < n_in; ++i) prs[i] = (float)(1.0 / sd[i]);

    DeviceGuard g(c->device);
    mala_weights* w = new mala_weights();
    w->device = c->device;
    auto upload_f = [&](const std::vector<float>& v) -> void* {
        void* d = nullptr;
        if (hipMalloc(&d, sizeof(float) * (v.size() ? v.size() : 1)) != hipSuccess) return nullptr;
        w->allocs.push_back(d);
        if (hipMemcpy(d, v.data(), sizeof(float) * v.size(), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
        return d;
    };
    auto upload_bf = [&](const std::vector<float>& v) -> void* {
        std::vector<uint16_t> h(v.size());
        for (size_t i = 0; i < v.size(); ++i) {   // round to nearest even
            uint32_t x;
            memcpy(&x, &v[i], 4);
            const uint32_t lsb = (x >> 16) & 1u;
            h[i] = (uint16_t)((x + 0x7FFFu + lsb) >> 16);
        }
        void* d = nullptr;
        if (hipMalloc(&d, sizeof(uint16_t) * (h.size() ? h.size() : 1)) != hipSuccess) return nullptr;
        w->allocs.push_back(d);
        if (hipMemcpy(d, h.data(), sizeof(uint16_t) * h.size(), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
        return d;
    };
    MlpArgs& a = w->args;
    a.precision = bf ? 1 : 0;
    a.n_in = n_in; a.n_h1 = h1; a.n_h2 = h2; a.n_out = n_out;
    a.in_pad = in_pad; a.h1_tiles = h1t; a.h2_tiles = h2t; a.out_tiles = ot;
    a.slope = (float)slope;
    a.out_act = out_act ? 1 : 0;
    a.W1 = bf ? upload_bf(P1) : upload_f(P1);
    a.W2 = bf ? upload_bf(P2) : upload_f(P2);
    a.W3 = bf ? upload_bf(P3) : upload_f(P3);
    a.W1T = bf ? nullptr : upload_f(T1);
    a.W2T = bf ? nullptr : upload_f(T2);
    a.W3T = bf ? nullptr : upload_f(T3);
    a.b1 = (const float*)upload_f(pb1);
    a.b2 = (const float*)upload_f(pb2);
    a.b3 = (const float*)upload_f(pb3);
    a.in_mean = (const float*)upload_f(pm);
    a.in_rstd = (const float*)upload_f(prs);
    a.out_scale = (const float*)upload_f(psc);
    a.out_shift = (const float*)upload_f(psh);
    if (!a.W1 || !a.W2 || !a.W3 || (!bf && (!a.W1T || !a.W2T || !a.W3T)) || !a.b1 || !a.b2 || !a.b3 || !a.in_mean || !a.in_rstd || !a.out_scale ||
        !a.out_shift) {
        mala_weights_free(w);
        return fail(MALA_E_OOM, "weight upload failed");
    }
    *out = w;
    return MALA_OK;
}

mala_status mala_weights_free(mala_weights* w) {
    if (!w) return MALA_OK;
    DeviceGuard g(w->device);
    (void)hipDeviceSynchronize();     // no kernel of any stream may still read the weights
    for (void* p : w->allocs) (void)hipFree(p);
    delete w;
    return MALA_OK;
}

// ---------------------------------------------------------------- compute
mala_status mala_descriptors(mala_ctx* c, const double* positions, int32_t n_atoms, const mala_cell_grid* cg,
                             double rcut, int32_t twojmax, int64_t pt_begin, int64_t pt_end, float* B_out) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    mala_status st = check_geometry(positions, n_atoms, cg, rcut, twojmax);
    if (st) return st;
    const int64_t ntot = (int64_t)cg->N[0] * cg->N[1] * cg->N[2];
    if (pt_begin < 0 || pt_end < pt_begin || pt_end > ntot) return fail(MALA_E_INVALID_ARG, "bad point range");
    if (pt_end == pt_begin) return MALA_OK;
    if (!B_out) return fail(MALA_E_INVALID_ARG, "B_out is NULL");
    DeviceGuard g(c->device);
    if ((st = ensure_tables(c, twojmax))) return st;
    if ((st = upload_positions(c, positions, n_atoms))) return st;
    return run_descriptors(c, n_atoms, cg, rcut, twojmax, pt_begin, pt_end, B_out);
}

mala_status mala_descriptors_vjp(mala_ctx* c, const double* positions, int32_t n_atoms, const mala_cell_grid* cg,
                                 double rcut, int32_t twojmax, int64_t pt_begin, int64_t pt_end, const float* gB,
                                 double* dLdR_out) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    mala_status st = check_geometry(positions, n_atoms, cg, rcut, twojmax);
    if (st) return st;
    const int64_t ntot = (int64_t)cg->N[0] * cg->N[1] * cg->N[2];
    if (pt_begin < 0 || pt_end < pt_begin || pt_end > ntot) return fail(MALA_E_INVALID_ARG, "bad point range");
    if (n_atoms == 0) return MALA_OK;
    if (!dLdR_out) return fail(MALA_E_INVALID_ARG, "dLdR_out is NULL");
    if (pt_end > pt_begin && !gB) return fail(MALA_E_INVALID_ARG, "gB is NULL");
    DeviceGuard g(c->device);
    HIP_TRY(launch_zero_f64(c->stream, dLdR_out, (int64_t)3 * n_atoms));
    if (pt_end == pt_begin) return MALA_OK;
    if ((st = ensure_adjoint_tables(c, twojmax))) return st;
    if ((st = upload_positions(c, positions, n_atoms))) return st;
    BinState bs{};
    if ((st = bin_atoms(c, n_atoms, cg, rcut, &bs))) return st;
    const int nB = n_triples(twojmax);
    const int64_t total = pt_end - pt_begin;
    const int64_t chunk = total < kChunk ? total : kChunk;
    const int64_t tiles = (chunk + kTile - 1) / kTile;
    HIP_TRY(ensure(c->n_allocs, c->u, (size_t)tiles * n_half(twojmax) * kTile));
    HIP_TRY(ensure(c->n_allocs, c->yadj, (size_t)tiles * n_half(twojmax) * kTile));
    const TjTables& t = c->tj[twojmax];
    for (int64_t off = 0; off < total; off += chunk) {
        const int64_t n = (total - off) < chunk ? (total - off) : chunk;
        HIP_TRY(staged(c, MALA_STAGE_UI, n, [&] {
            return launch_ui(c->stream, twojmax, bs, cg->N, rcut, pt_begin + off, n, c->u.p, c->err);
        }));
        HIP_TRY(staged(c, MALA_STAGE_ADJ_Y, n, [&] {
            return launch_yi(c->stream, twojmax, n, c->u.p, gB + off * nB, c->yadj.p, t.cgy, t.cgy_off, t.yunits);
        }));
        HIP_TRY(staged(c, MALA_STAGE_ADJ_DEDR, n, [&] {
            return launch_dedr(c->stream, twojmax, bs, cg->N, rcut, pt_begin + off, n, c->yadj.p, dLdR_out, c->err);
        }));
    }
    return MALA_OK;
}

int32_t mala_ace_count(int32_t nmax, int32_t lmax) {
    if (nmax < 1 || nmax > kAceMaxN || lmax < 0 || lmax > kAceMaxL) return MALA_E_UNSUPPORTED;
    std::vector<int> groups, groups_dm;
    std::vector<float> coef;
    const int n3 = build_ace_tables(nmax, lmax, groups, groups_dm, coef);
    return n3 < 0 ? MALA_E_UNSUPPORTED : ace_count_ranks12(nmax, lmax) + n3;
}

mala_status mala_ace_descriptors(mala_ctx* c, const double* positions, int32_t n_atoms, const mala_cell_grid* cg,
                                 double rcut, int32_t nmax, int32_t lmax, int64_t pt_begin, int64_t pt_end,
                                 int32_t layout, float* out) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    if (nmax < 1 || nmax > kAceMaxN || lmax < 0 || lmax > kAceMaxL)
        return fail(MALA_E_UNSUPPORTED, "grid ACE: nmax must be 1..4 and lmax 0..4");
    if (layout != MALA_LAYOUT_POINT_MAJOR && layout != MALA_LAYOUT_DESCRIPTOR_MAJOR)
        return fail(MALA_E_INVALID_ARG, "unknown output layout");
    mala_status st = check_geometry(positions, n_atoms, cg, rcut, 2);
    if (st) return st;
    const int64_t ntot = (int64_t)cg->N[0] * cg->N[1] * cg->N[2];
    if (pt_begin < 0 || pt_end < pt_begin || pt_end > ntot) return fail(MALA_E_INVALID_ARG, "bad point range");
    if (pt_end == pt_begin) return MALA_OK;
    if (!out) return fail(MALA_E_INVALID_ARG, "out is NULL");
    DeviceGuard g(c->device);
    AceTables& t = c->ace[nmax][lmax];
    if (!t.ready) {
        std::vector<int> groups, groups_dm;
        std::vector<float> coef;
        t.n3 = build_ace_tables(nmax, lmax, groups, groups_dm, coef);
        if (t.n3 < 0) return fail(MALA_E_UNSUPPORTED, "grid ACE: a pair's outputs exceed the staging columns");
        t.n_groups = (int)(groups.size() / kAceGroupInts);
        t.n_groups_dm = (int)(groups_dm.size() / kAceGroupInts);
        c->n_allocs += 3;
        HIP_TRY(hipMalloc(&t.groups, sizeof(int) * (groups.size() ? groups.size() : 1)));
        HIP_TRY(hipMalloc(&t.groups_dm, sizeof(int) * (groups_dm.size() ? groups_dm.size() : 1)));
        HIP_TRY(hipMalloc(&t.coef, sizeof(float) * (coef.size() ? coef.size() : 1)));
        HIP_TRY(hipMemcpy(t.groups, groups.data(), sizeof(int) * groups.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(t.groups_dm, groups_dm.data(), sizeof(int) * groups_dm.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(t.coef, coef.data(), sizeof(float) * coef.size(), hipMemcpyHostToDevice));
        t.ready = true;
    }
    const int n_desc = ace_count_ranks12(nmax, lmax) + t.n3;
    // point-major [point][descriptor] or descriptor-major [descriptor][point]
    const int64_t ps = layout == MALA_LAYOUT_POINT_MAJOR ? n_desc : 1;
    const int64_t ds = layout == MALA_LAYOUT_POINT_MAJOR ? 1 : pt_end - pt_begin;
    if ((st = upload_positions(c, positions, n_atoms))) return st;
    BinState bs{};
    if ((st = bin_atoms(c, n_atoms, cg, rcut, &bs))) return st;
    const int64_t total = pt_end - pt_begin;
    const int64_t chunk = total < kChunk ? total : kChunk;
    HIP_TRY(ensure(c->n_allocs, c->aceA, (size_t)((chunk + kTile - 1) / kTile) * kAceAPerPoint * kTile));
    for (int64_t off = 0; off < total; off += chunk) {
        const int64_t n = (total - off) < chunk ? (total - off) : chunk;
        HIP_TRY(staged(c, MALA_STAGE_ACE, n, [&] {
            hipError_t e = launch_ace_proj(c->stream, bs, cg->N, rcut, pt_begin + off, n, c->aceA.p, c->err);
            if (e != hipSuccess) return e;
            const bool pm = ds == 1;              // staged point-major rows, else plain stores
            return launch_ace(c->stream, c->aceA.p, nmax, lmax, n, pm ? t.groups : t.groups_dm,
                              pm ? t.n_groups : t.n_groups_dm, t.coef, n_desc, out + off * ps, ps, ds);
        }));
    }
    return MALA_OK;
}

int32_t mala_ace4_count(int32_t nmax4, int32_t lmax4) {
    if (nmax4 < 1 || nmax4 > kAce4MaxN || lmax4 < 0 || lmax4 > kAce4MaxL) return MALA_E_UNSUPPORTED;
    std::vector<int> set;
    return ace4_descriptor_set(nmax4, lmax4, set);
}

int32_t mala_ace4_list(int32_t nmax4, int32_t lmax4, int32_t* out, int32_t cap) {
    if (nmax4 < 1 || nmax4 > kAce4MaxN || lmax4 < 0 || lmax4 > kAce4MaxL) return MALA_E_UNSUPPORTED;
    std::vector<int> set;
    const int n = ace4_descriptor_set(nmax4, lmax4, set);
    if (!out || cap < n) return MALA_E_INVALID_ARG;
    for (size_t i = 0; i < set.size(); ++i) out[i] = set[i];
    return n;
}

mala_status mala_ace4_descriptors(mala_ctx* c, const double* positions, int32_t n_atoms, const mala_cell_grid* cg,
                                  double rcut, int32_t nmax4, int32_t lmax4, int64_t pt_begin, int64_t pt_end,
                                  int32_t layout, float* out) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    if (nmax4 < 1 || nmax4 > kAce4MaxN || lmax4 < 0 || lmax4 > kAce4MaxL)
        return fail(MALA_E_UNSUPPORTED, "rank-4 grid ACE: nmax4 must be 1..3 and lmax4 0..3");
    if (layout != MALA_LAYOUT_POINT_MAJOR && layout != MALA_LAYOUT_DESCRIPTOR_MAJOR)
        return fail(MALA_E_INVALID_ARG, "unknown output layout");
    mala_status st = check_geometry(positions, n_atoms, cg, rcut, 2);
    if (st) return st;
    const int64_t ntot = (int64_t)cg->N[0] * cg->N[1] * cg->N[2];
    if (pt_begin < 0 || pt_end < pt_begin || pt_end > ntot) return fail(MALA_E_INVALID_ARG, "bad point range");
    if (pt_end == pt_begin) return MALA_OK;
    if (!out) return fail(MALA_E_INVALID_ARG, "out is NULL");
    DeviceGuard g(c->device);
    Ace4Tables& t = c->ace4[nmax4][lmax4];
    if (!t.ready) {
        std::vector<int> l_units, l_descs;
        std::vector<int4> units, descs;
        std::vector<float> coef;
        t.n4 = build_ace4_tables(nmax4, lmax4, l_units, units, coef, l_descs, descs, t.max_slots);
        if ((size_t)t.max_slots * kTile * sizeof(float2) > kAce4LdsBudget)
            return fail(MALA_E_UNSUPPORTED, "rank-4 grid ACE: pair vectors exceed the LDS budget");
        for (size_t ph = 0; ph + 1 < l_descs.size(); ++ph)
            if (l_descs[ph + 1] - l_descs[ph] > kAce4MaxDescsL)
                return fail(MALA_E_UNSUPPORTED, "rank-4 grid ACE: more descriptors of one L than staged in LDS");
        t.n_phases = (int)l_descs.size() - 1;
        c->n_allocs += 5;
        HIP_TRY(hipMalloc(&t.l_units, sizeof(int) * l_units.size()));
        HIP_TRY(hipMalloc(&t.units, sizeof(int4) * (units.size() ? units.size() : 1)));
        HIP_TRY(hipMalloc(&t.coef, sizeof(float) * (coef.size() ? coef.size() : 1)));
        HIP_TRY(hipMalloc(&t.l_descs, sizeof(int) * l_descs.size()));
        HIP_TRY(hipMalloc(&t.descs, sizeof(int4) * (descs.size() ? descs.size() : 1)));
        HIP_TRY(hipMemcpy(t.l_units, l_units.data(), sizeof(int) * l_units.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(t.units, units.data(), sizeof(int4) * units.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(t.coef, coef.data(), sizeof(float) * coef.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(t.l_descs, l_descs.data(), sizeof(int) * l_descs.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(t.descs, descs.data(), sizeof(int4) * descs.size(), hipMemcpyHostToDevice));
        t.ready = true;
    }
    if ((st = upload_positions(c, positions, n_atoms))) return st;
    BinState bs{};
    if ((st = bin_atoms(c, n_atoms, cg, rcut, &bs))) return st;
    const int64_t total = pt_end - pt_begin;
    const bool pm = layout == MALA_LAYOUT_POINT_MAJOR;
    // point-major: descriptor planes of each chunk into ace4S, then rows
    const int64_t chunk_max = pm ? kAce4RowChunk : kChunk;
    const int64_t chunk = total < chunk_max ? total : chunk_max;
    HIP_TRY(ensure(c->n_allocs, c->aceA, (size_t)((chunk + kTile - 1) / kTile) * kAceAPerPoint * kTile));
    if (pm) HIP_TRY(ensure(c->n_allocs, c->ace4S, (size_t)chunk * t.n4));
    for (int64_t off = 0; off < total; off += chunk) {
        const int64_t n = (total - off) < chunk ? (total - off) : chunk;
        HIP_TRY(staged(c, MALA_STAGE_ACE4, n, [&] {
            hipError_t e = launch_ace_proj(c->stream, bs, cg->N, rcut, pt_begin + off, n, c->aceA.p, c->err);
            if (e != hipSuccess) return e;
            if (!pm)
                return launch_ace4(c->stream, c->aceA.p, lmax4, t.n_phases, n, t.l_units, t.units, t.coef, t.l_descs, t.descs,
                                   t.max_slots, t.n4, out + off, 1, total);
            e = launch_ace4(c->stream, c->aceA.p, lmax4, t.n_phases, n, t.l_units, t.units, t.coef, t.l_descs, t.descs,
                            t.max_slots, t.n4, c->ace4S.p, 1, chunk);
            if (e != hipSuccess) return e;
            return launch_planes_to_rows(c->stream, c->ace4S.p, chunk, n, t.n4, out + off * t.n4);
        }));
    }
    return MALA_OK;
}

mala_status mala_gaussian_descriptors(mala_ctx* c, const double* positions, int32_t n_atoms,
                                      const mala_cell_grid* cg, double sigma, double cutoff, int64_t pt_begin,
                                      int64_t pt_end, float* G_out) {
    if (!c) return fail(MALA_E_INVALID_ARG, "ctx is NULL");
    if (!(sigma > 0.0) || !isfinite(sigma)) return fail(MALA_E_INVALID_ARG, "sigma not positive");
    mala_status st = check_geometry(positions, n_atoms, cg, cutoff, 2);
    if (st) return st;
    const int64_t ntot = (int64_t)cg->N[0] * cg->N[1] * cg->N[2];
    if (pt_begin < 0 || pt_end < pt_begin || pt_end > ntot) return fail(MALA_E_INVALID_ARG, "bad point range");
    if (pt_end == pt_begin) return MALA_OK;
    if (!G_out) return fail(MALA_E_INVALID_ARG, "G_out is NULL");
    DeviceGuard g(c->device);
    if ((st = upload_positions(c, positions, n_atoms))) return st;
    BinState bs{};
    if ((st = bin_atoms(c, n_atoms, cg, cutoff, &bs))) return st;
    HIP_TRY(staged(c, MALA_STAGE_GAUSS, pt_end - pt_begin, [&] {
        return launch_gauss(c->stream, bs, cg->N, sigma, cutoff, pt_begin, pt_end - pt_begin, G_out, c->err);
    }));
    return MALA_OK;
}

mala_status mala_ldos_infer(mala_ctx* c, const mala_weights* w, const float* B, int64_t n_pts, float* ldos_out) {
    if (!c || !w) return fail(MALA_E_INVALID_ARG, "NULL argument");
    if (n_pts < 0) return fail(MALA_E_INVALID_ARG, "n_pts < 0");
    if (n_pts == 0) return MALA_OK;
    if (!B || !ldos_out) return fail(MALA_E_INVALID_ARG, "NULL buffer");
    DeviceGuard g(c->device);
    MlpOut o;
    o.ldos = ldos_out;
    HIP_TRY(staged(c, MALA_STAGE_MLP_LDOS, n_pts,
                   [&] { return launch_mlp(c->stream, w->args, kModeLdos, B, n_pts, 1, mlp_blocks(n_pts), o); }));
    return MALA_OK;
}

mala_status mala_ldos_vjp(mala_ctx* c, const mala_weights* w, const float* B, const float* v, int64_t n_pts,
                          float* g_out) {
    if (!c || !w) return fail(MALA_E_INVALID_ARG, "NULL argument");
    if (w->args.precision != 0) return fail(MALA_E_UNSUPPORTED, "the network VJP needs FP32 weights");
    if (n_pts < 0) return fail(MALA_E_INVALID_ARG, "n_pts < 0");
    if (n_pts == 0) return MALA_OK;
    if (!B || !v || !g_out) return fail(MALA_E_INVALID_ARG, "NULL buffer");
    if (mlp_vjp_lds_bytes(w->args) > kMlpLdsBudget)
        return fail(MALA_E_UNSUPPORTED, "network too wide for the VJP kernel's LDS tile");
    DeviceGuard g(c->device);
    HIP_TRY(staged(c, MALA_STAGE_MLP_VJP, n_pts, [&] { return launch_mlp_vjp(c->stream, w->args, B, v, n_pts, g_out); }));
    return MALA_OK;
}

mala_status mala_integrate(mala_ctx* c, const float* ldos, int64_t n_pts, double dV, const mala_egrid* eg,
                           double T, double ne, double* dos_out, double* density_out, mala_result* result) {
    mala_status st = check_integrate_args(c, ldos, n_pts, dV, eg, T, ne, dos_out, result);
    if (st) return st;
    DeviceGuard g(c->device);
    const int nb = integrate_parts(n_pts);
    HIP_TRY(ensure(c->n_allocs, c->partials, (size_t)nb * kMlpMaxOut));
    HIP_TRY(ensure(c->n_allocs, c->fermi_w, kMlpMaxOut));
    HIP_TRY(staged(c, MALA_STAGE_INTEGRATE, n_pts,
                   [&] { return launch_ldos_colsum(c->stream, ldos, n_pts, eg->n, c->partials.p, nb); }));
    HIP_TRY(staged(c, MALA_STAGE_FERMI, 0, [&] {
        return launch_fermi(c->stream, c->partials.p, nb, eg->n, dV, eg->e0, eg->de, kBoltzmannEv * T, ne,
                            dos_out, c->fermi_w.p, result, nullptr, c->li_coef);
    }));
    if (density_out && n_pts > 0)
        HIP_TRY(staged(c, MALA_STAGE_INTEGRATE, n_pts, [&] {
            return launch_density_from_ldos(c->stream, ldos, n_pts, eg->n, c->fermi_w.p, result, density_out);
        }));
    return MALA_OK;
}

mala_status mala_integrate_noalloc(mala_ctx* c, const float* ldos, int64_t n_pts, double dV, const mala_egrid* eg,
                                   double T, double ne, double* dos_out, double* density_out, mala_result* result) {
    mala_status st = check_integrate_args(c, ldos, n_pts, dV, eg, T, ne, dos_out, result);
    if (st) return st;
    const int nb = integrate_parts(n_pts);
    if ((size_t)nb * kMlpMaxOut + kMlpMaxOut > (size_t)kNoallocScratchDoubles)
        return fail(MALA_E_UNSUPPORTED, "mala_integrate_noalloc: partial rows exceed the fixed scratch");
    DeviceGuard g(c->device);
    double* scr = nullptr;
    HIP_TRY(scratch_device_ptr(c->device, &scr));      // looked up by mala_create: no allocation here
    double* partials = scr;
    double* weights = scr + (size_t)kIntegrateMaxParts * kMlpMaxOut;
    // every partial row is written by the column sums, the weights by the
    // Fermi pass: nothing has to start at zero
    HIP_TRY(launch_ldos_colsum(c->stream, ldos, n_pts, eg->n, partials, nb));
    HIP_TRY(launch_fermi(c->stream, partials, nb, eg->n, dV, eg->e0, eg->de, kBoltzmannEv * T, ne, dos_out, weights,
                         result, nullptr, c->li_coef));
    if (density_out && n_pts > 0)
        HIP_TRY(launch_density_from_ldos(c->stream, ldos, n_pts, eg->n, weights, result, density_out));
    return MALA_OK;
}

mala_status mala_predict(mala_ctx* c, const mala_weights* w, const double* positions, int32_t n_atoms,
                         const mala_cell_grid* cg, double rcut, int32_t twojmax, const mala_egrid* eg, double T,
                         double ne, double* dos_out, double* density_out, mala_result* result, float* B_cache) {
    if (!c || !w) return fail(MALA_E_INVALID_ARG, "NULL argument");
    mala_status st = check_geometry(positions, n_atoms, cg, rcut, twojmax);
    if (st) return st;
    if ((st = check_egrid(eg, T, ne))) return st;
    if (!dos_out || !result) return fail(MALA_E_INVALID_ARG, "NULL buffer");
    if (w->args.n_in != n_triples(twojmax))
        return fail(MALA_E_INVALID_ARG, "network input width does not match twojmax");
    if (w->args.n_out != eg->n) return fail(MALA_E_INVALID_ARG, "network output width != energy grid size");
    const int64_t ntot = (int64_t)cg->N[0] * cg->N[1] * cg->N[2];
    DeviceGuard g(c->device);
    if ((st = ensure_tables(c, twojmax))) return st;
    float* B = B_cache;
    if (!B) {
        HIP_TRY(ensure(c->n_allocs, c->Bbuf, (size_t)ntot * n_triples(twojmax)));
        B = c->Bbuf.p;
    }
    if ((st = upload_positions(c, positions, n_atoms))) return st;
    if ((st = run_descriptors(c, n_atoms, cg, rcut, twojmax, 0, ntot, B, kPredictChunk))) return st;
    const int nb = mlp_blocks(ntot);
    HIP_TRY(ensure(c->n_allocs, c->partials, (size_t)nb * kMlpMaxOut));
    HIP_TRY(ensure(c->n_allocs, c->fermi_w, kMlpMaxOut));
    const double dV = cg->L[0] * cg->L[1] * cg->L[2] / (double)ntot;
    const double kT = kBoltzmannEv * T;
    MlpOut o;
    o.partials = c->partials.p;
    o.de = eg->de;
    const bool window = density_out && c->density_mode == 0;
    if (window) {
        // E_F estimate from every stride-th point -> energy window of the stored LDOS
        const int64_t stride = est_stride(cg);
        const int64_t n_est = (ntot + stride - 1) / stride;
        const int nbe = mlp_blocks(n_est);
        const double margin = kWindowMargin;            // eV, covers the estimate's error
        const int w_max = window_width(eg, T);
        HIP_TRY(ensure(c->n_allocs, c->est_partials, (size_t)nbe * kMlpMaxOut));
        HIP_TRY(ensure(c->n_allocs, c->window, (size_t)ntot * w_max));
        HIP_TRY(ensure(c->n_allocs, c->prefix, (size_t)ntot));
        MlpOut oe;
        oe.partials = c->est_partials.p;
        HIP_TRY(staged(c, MALA_STAGE_ESTIMATE, n_est, [&] {
            hipError_t e = launch_mlp(c->stream, w->args, kModeDos, B, n_est, (int)stride, nbe, oe);
            if (e != hipSuccess) return e;
            return launch_fermi_estimate(c->stream, c->est_partials.p, nbe, eg->n, dV * (double)stride, eg->e0, eg->de,
                                         kT, ne, c->win, c->li_coef, w_max, margin);
        }));
        o.win = c->win;
        o.window = c->window.p;
        o.prefix = c->prefix.p;
        HIP_TRY(staged(c, MALA_STAGE_MLP_DOS, ntot,
                       [&] { return launch_mlp(c->stream, w->args, kModeDosWindow, B, ntot, 1, nb, o); }));
    } else {
        HIP_TRY(staged(c, MALA_STAGE_MLP_DOS, ntot,
                       [&] { return launch_mlp(c->stream, w->args, kModeDos, B, ntot, 1, nb, o); }));
    }
    HIP_TRY(staged(c, MALA_STAGE_FERMI, 0, [&] {
        return launch_fermi(c->stream, c->partials.p, nb, eg->n, dV, eg->e0, eg->de, kT, ne, dos_out, c->fermi_w.p,
                            result, window ? c->win : nullptr, c->li_coef, c->err);
    }));
    if (density_out) {
        if (window)
            HIP_TRY(staged(c, MALA_STAGE_DENSITY_WINDOW, ntot, [&] {
                return launch_density_window(c->stream, c->prefix.p, c->window.p, ntot, c->win, result,
                                             c->fermi_w.p, density_out, window_width(eg, T));
            }));
        else
            HIP_TRY(set_covered(c, 0));
        // recompute pass: a no-op on the device when the window covered E_F
        MlpOut od;
        od.fermi_w = c->fermi_w.p;
        od.density = density_out;
        od.res = static_cast<const ResultRec*>(static_cast<const void*>(result));
        od.win = c->win;
        HIP_TRY(staged(c, MALA_STAGE_MLP_DENSITY, ntot,
                       [&] { return launch_mlp(c->stream, w->args, kModeDensity, B, ntot, 1, nb, od); }));
    }
    return MALA_OK;
}

}  // extern "C"
