// Internal declarations of the gfx950 library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include "mala.h"
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <utility>

struct mala_ctx;

namespace mala {

constexpr int kTile = 64;            // grid points per bispectrum tile (one per lane)
constexpr int kMaxTwojmax = 10;
constexpr int kMaxCand = 1024;       // candidate atom images per tile
constexpr int kMaxNbr = 128;         // neighbours per grid point
constexpr int kMlpBlocks = 256;      // fixed block count of the network kernels (one per CU; deterministic partials)
constexpr int kMaxZbStride = 64;     // per-wave triple list stride (count + indices)
constexpr int kMaxYStride = 64;      // per-wave unit list stride of the descriptor adjoint
constexpr int kMlpMaxIn = 128;       // padded input width limit
constexpr int kMlpMaxHidden = 512;   // hidden width limit
constexpr int kMlpMaxOut = 256;      // output width limit
// DOS partial rows of the stored-LDOS reductions (mala_integrate): one per
// block over a fixed contiguous range of points, at most this many.
constexpr int kIntegrateMaxParts = 2048;
// fixed scratch of mala_integrate_noalloc: the partial rows and the weights
constexpr int kNoallocScratchDoubles = kIntegrateMaxParts * kMlpMaxOut + kMlpMaxOut;
constexpr double kBoltzmannEv = 8.617333262e-5;
constexpr float kRfac0 = 0.99363f;

// Device-side error bits (OR-ed into a flag word in device memory).
constexpr int kErrCand = 1;          // tile candidate list overflow
constexpr int kErrNbr = 2;           // per-point neighbour list overflow

// ---------------------------------------------------------------- u indexing
// u^J is stored for rows ma = 0..J/2 (the other rows follow from
// u_{J-ma, J-mb} = (-1)^(ma-mb) conj(u_{ma, mb})), row-major, levels
// concatenated: element (J, ma, mb) -> half_off(J) + ma*(J+1) + mb.
__host__ __device__ constexpr int half_rows(int J) { return J / 2 + 1; }
__host__ __device__ constexpr int half_size(int J) { return half_rows(J) * (J + 1); }
__host__ __device__ constexpr int half_off(int J) {
    int o = 0;
    for (int k = 0; k < J; ++k) o += half_size(k);
    return o;
}
__host__ __device__ constexpr int n_half(int tj) { return half_off(tj + 1); }

// Descriptor triples (doubled indices) in output order.
__host__ __device__ constexpr int n_triples(int tj) {
    int n = 0;
    for (int j1 = 0; j1 <= tj; ++j1)
        for (int j2 = 0; j2 <= j1; ++j2)
            for (int j = j1 - j2; j <= j1 + j2 && j <= tj; j += 2)
                if (j >= j1) ++n;
    return n;
}

struct Triple {
    int j1, j2, j;
};
__host__ __device__ constexpr Triple triple_of(int tj, int idx) {
    int n = 0;
    for (int j1 = 0; j1 <= tj; ++j1)
        for (int j2 = 0; j2 <= j1; ++j2)
            for (int j = j1 - j2; j <= j1 + j2 && j <= tj; j += 2)
                if (j >= j1) {
                    if (n == idx) return Triple{j1, j2, j};
                    ++n;
                }
    return Triple{0, 0, 0};
}

// Index of a descriptor triple (j1 >= j2, j >= j1) in output order.
__host__ __device__ constexpr int triple_index(int tj, int j1, int j2, int j) {
    int n = 0;
    for (int a = 0; a <= tj; ++a)
        for (int b = 0; b <= a; ++b)
            for (int c = a - b; c <= a + b && c <= tj; c += 2)
                if (c >= a) {
                    if (a == j1 && b == j2 && c == j) return n;
                    ++n;
                }
    return -1;
}

// The derivative of sum_l g_l B_l with respect to u^C is a sum of Z^C(A, B)
// over coupled pairs A >= B: every (A, B, C) with |A-B| <= C <= A+B,
// A+B+C even (levels <= tj), ordered by C, then A, then B.  Its descriptor
// triple is the sorted {A, B, C} (j = largest, j1 = middle, j2 = smallest)
// and its weight mult * (j+1)/(C+1) counts the slots of that triple that
// hold level C (each such slot leaves exactly {A, B}); a slot holding the
// middle or smallest level enters through the identity
// B(j1,j2,j) = (j+1)/(j1+1) I(j, j2 -> j1) = (j+1)/(j2+1) I(j, j1 -> j2).
struct Combo {
    int a, b, c;      // coupled levels a >= b, output level c
    int triple;       // descriptor triple of {a, b, c}
    int mult;         // slots of that triple holding level c
    int jmax;
};
__host__ __device__ constexpr int n_combos(int tj) {
    int n = 0;
    for (int c = 0; c <= tj; ++c)
        for (int a = 0; a <= tj; ++a)
            for (int b = 0; b <= a; ++b)
                if (a - b <= c && c <= a + b && (a + b + c) % 2 == 0) ++n;
    return n;
}
__host__ __device__ constexpr Combo combo_of(int tj, int idx) {
    int n = 0;
    for (int c = 0; c <= tj; ++c)
        for (int a = 0; a <= tj; ++a)
            for (int b = 0; b <= a; ++b)
                if (a - b <= c && c <= a + b && (a + b + c) % 2 == 0) {
                    if (n == idx) {
                        const int hi = a > c ? a : c;                    // a >= b
                        const int lo = b < c ? b : c;
                        const int mid = a + b + c - hi - lo;
                        const int mult = (a == c) + (b == c) + 1;
                        return Combo{a, b, c, triple_index(tj, mid, lo, hi), mult, hi};
                    }
                    ++n;
                }
    return Combo{0, 0, 0, -1, 0, 0};
}
__host__ __device__ constexpr int combo_first(int tj, int c) {     // first combo of output level c
    int n = 0;
    for (int i = 0; i < n_combos(tj); ++i)
        if (combo_of(tj, i).c < c) ++n;
    return n;
}

// Pairs (row ma of the output level, row ma1 of level A) of the Z/B
// contraction with coupled levels (A, B) and output C: the row of level B is
// ma2 = ma - ma1 + (A+B-C)/2.  When A == B, exchanging the two coupled
// factors maps pair (ma, ma1) to (ma, ma2) and multiplies both its T sum and
// its row Clebsch-Gordan factor by the same sign (-1)^((A+B-C)/2), so only
// ma1 <= ma2 is formed and ma1 < ma2 counts twice.
__host__ __device__ constexpr bool zb_pair_ok(int A, int B, int C, int ma, int ma1) {
    const int ma2 = ma - ma1 + (A + B - C) / 2;
    return ma2 >= 0 && ma2 <= B && (A != B || ma1 <= ma2);
}
__host__ __device__ constexpr bool zb_pair_doubled(int A, int B, int C, int ma, int ma1) {
    return A == B && zb_pair_ok(A, B, C, ma, ma1) && ma1 < ma - ma1 + (A + B - C) / 2;
}

// Rows of u^A (ma1) and of u^B (r = ma2) that the pairs of a triple use.
__host__ __device__ constexpr bool zb_row1_used(int A, int B, int C, int ma1) {
    for (int ma = 0; ma <= C / 2; ++ma)
        if (zb_pair_ok(A, B, C, ma, ma1)) return true;
    return false;
}
__host__ __device__ constexpr bool zb_row2_used(int A, int B, int C, int r) {
    const int D = (A + B - C) / 2;
    for (int ma = 0; ma <= C / 2; ++ma)
        for (int ma1 = 0; ma1 <= A; ++ma1)
            if (zb_pair_ok(A, B, C, ma, ma1) && ma - ma1 + D == r) return true;
    return false;
}

// Per output-column work of a m1' column besides the complex FMAs.  The CG
// factor C(m1',m') scales the used rows of one of the two levels (2
// multiplies a row); a mirrored row (past J/2) is a signed conjugate of a
// stored one whose sign (-1)^(row - column) changes with the runtime column:
// on the scaled side it folds into the scalar factor, on the other side it
// costs 2 multiplies.  side 1 scales u^A, side 2 scales u^B.
struct ZbRows {
    int used1, mirr1, stor1, used2, mirr2, stor2;
};
__host__ __device__ constexpr ZbRows zb_rows(int A, int B, int C) {
    ZbRows r{0, 0, 0, 0, 0, 0};
    for (int i = 0; i <= A; ++i)
        if (zb_row1_used(A, B, C, i)) {
            ++r.used1;
            if (2 * i > A) ++r.mirr1; else ++r.stor1;
        }
    for (int i = 0; i <= B; ++i)
        if (zb_row2_used(A, B, C, i)) {
            ++r.used2;
            if (2 * i > B) ++r.mirr2; else ++r.stor2;
        }
    return r;
}
__host__ __device__ constexpr int zb_scale_ops(int A, int B, int C, int side) {
    const ZbRows r = zb_rows(A, B, C);
    return side == 1 ? 2 * r.used1 + 2 * r.mirr2 : 2 * r.used2 + 2 * r.mirr1;
}
__host__ __device__ constexpr bool zb_scale2(int A, int B, int C) {
    return zb_scale_ops(A, B, C, 2) < zb_scale_ops(A, B, C, 1);
}

// Operation count of the Z/B contraction with output index C and coupled
// pair (A, B): per output column, every m1' column updates the pairs of T
// (4 FMA) after its loads (one address add per level side in use) and
// scaling, then the row CG fold over the half rows; the middle row of an
// even C is formed for the columns mb <= C/2 only.
__host__ __device__ constexpr double zb_cost(int A, int B, int C) {
    const int D = (A + B - C) / 2, HR = C / 2;
    int terms = 0, mid = 0;
    for (int ma = 0; ma <= HR; ++ma)
        for (int ma1 = 0; ma1 <= A; ++ma1)
            if (zb_pair_ok(A, B, C, ma, ma1)) {
                if (C % 2 == 0 && ma == HR) ++mid;
                else ++terms;
            }
    const ZbRows r = zb_rows(A, B, C);
    const int s1 = zb_scale_ops(A, B, C, 1), s2 = zb_scale_ops(A, B, C, 2);
    const int col = (s1 < s2 ? s1 : s2) + (r.stor1 > 0) + (r.mirr1 > 0) + (r.stor2 > 0) + (r.mirr2 > 0) + 2;
    double tot = 0.0;
    for (int mb = 0; mb <= C; ++mb) {
        const int lo = mb + D - B > 0 ? mb + D - B : 0, hi = A < mb + D ? A : mb + D;
        const int t = terms + (mb <= HR ? mid : 0);
        tot += (hi - lo + 1) * (4.0 * t + col) + 2.0 * t + 3.0 * (HR + 1);
    }
    return tot;
}

// The triple product is invariant under moving the conjugated level:
// B(j1,j2,j) = (J+1)/(J1+1) I(j,j2 -> j1) = (J+1)/(J2+1) I(j,j1 -> j2), I
// the same contraction with the named output level.  Each triple is
// evaluated in the cheapest of the three orientations (first on ties).
struct ZbPerm {
    int a, b, c;          // coupled levels a >= b, output level c
};
__host__ __device__ constexpr ZbPerm zb_perm(int tj, int idx) {
    const Triple t = triple_of(tj, idx);
    ZbPerm best{t.j1, t.j2, t.j};
    double cbest = zb_cost(t.j1, t.j2, t.j);
    const ZbPerm alt[2] = {{t.j, t.j2, t.j1}, {t.j, t.j1, t.j2}};
    for (int i = 0; i < 2; ++i) {
        const double c = zb_cost(alt[i].a, alt[i].b, alt[i].c);
        if (c < cbest) {
            cbest = c;
            best = alt[i];
        }
    }
    return best;
}

// compile-time loop helper
template <int Begin, int End, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (Begin < End) {
        f(std::integral_constant<int, Begin>{});
        static_for<Begin + 1, End>(std::forward<F>(f));
    }
}

// ---------------------------------------------------------------- launches
struct BinState {
    int nc[3];            // cells per edge
    double cs[3];         // cell size
    double L[3];
    int ncell;
    int n_atoms;
    const int* cell_start;      // [ncell+1]
    const double4* atoms;       // [n_atoms] wrapped positions sorted by cell (w = index)
};

hipError_t launch_bin(hipStream_t s, const double* pos_dev, int n_atoms, const double L[3],
                      double rcut, int* cell_count, int* cell_start, int* cell_fill,
                      double4* atoms_tmp, int* atom_cell, double4* atoms_sorted, BinState* st);

hipError_t launch_ui(hipStream_t s, int twojmax, const BinState& bins, const int N[3], double rcut,
                     int64_t pt_begin, int64_t n_pts, float2* u_scratch, int* err_flag);
hipError_t launch_zb(hipStream_t s, int twojmax, int64_t n_pts, const float2* u_scratch, float* B_out,
                     const float* cg_table, const int* cg_offsets, const int* wave_triples, int zb_waves);
hipError_t launch_gauss(hipStream_t s, const BinState& bins, const int N[3], double sigma, double cutoff,
                        int64_t pt_begin, int64_t n_pts, float* out, int* err_flag);

struct MlpArgs {
    int precision;               // 0 fp32, 1 bf16
    int n_in, n_h1, n_h2, n_out; // logical widths
    int in_pad, h1_tiles, h2_tiles, out_tiles;
    float slope;
    int out_act;
    const void* W1;              // packed A operands
    const void* W2;
    const void* W3;
    const float* b1;             // padded biases (zeros in the padding)
    const float* b2;
    const float* b3;
    const float* in_mean;        // [n_in]
    const float* in_rstd;        // [n_in] 1/std
    const float* out_scale;      // [out_tiles*16] (zeros in the padding)
    const float* out_shift;
    const void* W1T;             // transposed weights packed as A operands (FP32 only;
    const void* W2T;             // null for BF16 weights): [in_pad] x h1, h1 x h2,
    const void* W3T;             // h2 x [out_tiles*16]
};

enum MlpMode { kModeLdos = 0, kModeDos = 1, kModeDensity = 2, kModeDosWindow = 3 };
constexpr size_t kMlpLdsBudget = 155000;   // dynamic LDS of one network block

// Mirrors mala_result of include/mala.h.
struct ResultRec {
    double e_fermi, e_band, n_found, n_target;
    int32_t iterations, status, density_from_window, reserved;
    double entropy, e_entropy;        // S_s / k_B, -tau S_s (eV)
};

// Energy window of the stored LDOS (device scratch).
struct WindowRec {
    int32_t lo, hi, valid, covered;
    double e_fermi_est;
};

struct MlpOut {
    float* ldos = nullptr;            // LDOS mode
    double* partials = nullptr;       // DOS modes: [blocks][kMlpMaxOut]
    const double* fermi_w = nullptr;  // density mode
    double* density = nullptr;
    const ResultRec* res = nullptr;
    const WindowRec* win = nullptr;   // window / density modes
    float* window = nullptr;          // [n][hi-lo+1]
    double* prefix = nullptr;         // [n]
    double de = 0.0;
};

int mlp_blocks(int64_t n_pts);
size_t mlp_vjp_lds_bytes(const MlpArgs& a);
hipError_t launch_mlp_vjp(hipStream_t s, const MlpArgs& a, const float* B, const float* v, int64_t n_pts,
                          float* g_out);
hipError_t launch_mlp(hipStream_t s, const MlpArgs& a, int mode, const float* B, int64_t n_pts, int row_stride,
                      int n_blocks, const MlpOut& o);

hipError_t launch_ldos_colsum(hipStream_t s, const float* ldos, int64_t n_pts, int n_e,
                              double* partials, int n_blocks);

hipError_t launch_fermi(hipStream_t s, const double* partials, int n_parts, int n_e, double dV,
                        double e0, double de, double kT, double n_target, double* dos_out,
                        double* weights_out, void* result, WindowRec* win, const double* li_coef,
                        const int* cap_err = nullptr);   // capacity flags: nonzero -> status MALA_E_CAPACITY
hipError_t launch_fermi_estimate(hipStream_t s, const double* partials, int n_parts, int n_e, double dV,
                                 double e0, double de, double kT, double n_target, WindowRec* win,
                                 const double* li_coef, int w_max, double margin);
constexpr int kDensityStageMax = 96;       // window energies per point the density kernel stages in LDS
hipError_t launch_density_window(hipStream_t s, const double* prefix, const float* window, int64_t n_pts,
                                 const WindowRec* win, const void* result, const double* weights,
                                 double* density, int w_max);

hipError_t launch_density_from_ldos(hipStream_t s, const float* ldos, int64_t n_pts, int n_e,
                                    const double* weights, const void* result, double* density);

// Device bytes held by a context's scratch, and releasing them (serving).
size_t ctx_device_bytes(mala_ctx* c);
uint64_t ctx_alloc_count(mala_ctx* c);      // device and pinned allocations so far
int* ctx_error_flags(mala_ctx* c);          // device word of the kernels' capacity flags
// Buffer sizes (elements) mala_predict needs for one request.
struct PredictPlan {
    int twojmax;
    size_t pos, cells, atoms, u, B, partials, fermi_w, est_partials, window, prefix;
};
PredictPlan plan_predict(const mala_cell_grid* cg, int32_t n_atoms, double rcut, int32_t twojmax,
                         const mala_egrid* eg, double T, bool density, int density_mode, bool caller_b_cache);
PredictPlan plan_max(const PredictPlan& a, const PredictPlan& b);
size_t plan_growth_bytes(mala_ctx* c, const PredictPlan& p);
mala_status ctx_reserve(mala_ctx* c, const PredictPlan& p);
hipError_t scratch_device_ptr(int device, double** out);   // noalloc.hip
void ctx_trim(mala_ctx* c);

// Host-side tables.
int build_cg_table(int twojmax, float* table, int* offsets, int cap);
int build_cg_table_adjoint(int twojmax, float* table, int* offsets, int cap);
int y_max_waves();
int y_group_wave_count(int tj, int g);
int y_group_count(int tj);      // kernels (groups of output levels) of the dL/du contraction
int y_group_first(int tj, int g);
int y_group_last(int tj, int g);
hipError_t launch_zero_f64(hipStream_t s, double* p, int64_t n);
hipError_t launch_yi(hipStream_t s, int twojmax, int64_t n_pts, const float2* u, const float* gB, float2* y,
                     const float* cg_tab, const int* cg_off, const int* wave_units);
hipError_t launch_dedr(hipStream_t s, int twojmax, const BinState& bins, const int N[3], double rcut,
                       int64_t pt_begin, int64_t n_pts, const float2* y, double* dLdR, int* err);
void plan_y_units(int twojmax, int c_lo, int c_hi, int n_waves, int* wave_units, int stride);
void plan_zb_waves(int twojmax, int n_waves, int* wave_triples, int stride);
constexpr int kLiTerms = 32;
constexpr int kLiPow = 64;
constexpr int kLiCoef = 2 * kLiTerms + 2 * kLiPow;
void polylog_coefficients(double* coef);   // [kLiCoef]: Taylor coefficients at y=1, inverse powers

}  // namespace mala
