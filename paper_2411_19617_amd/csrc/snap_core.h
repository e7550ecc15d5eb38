// Compile-time helpers of the bispectrum kernels (Sec. 3.2.2, Eq. SNAPExpansion,
// Eq. snap_dim) shared by the descriptor kernels and their adjoint: exact
// constants, the chain layout of the U recursion, the wave groups of the
// chains, and the (row, row) pairs of the Z contraction.
#pragma once
#include "mala_internal.h"

namespace mala {

__host__ __device__ constexpr double ce_sqrt(double x) {
    if (x <= 0.0) return 0.0;
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 64; ++i) r = 0.5 * (r + x / r);
    return r;
}

// ------------------------------------------------------------------ chains
// Chain q: rows k = 0..min(q, TJ-q) at level J = q + k, row index ma = k.
__host__ __device__ constexpr int chain_rows(int tj, int q) { return (q < tj - q ? q : tj - q) + 1; }
__host__ __device__ constexpr int chain_len(int tj, int q) {
    int n = 0;
    for (int k = 0; k < chain_rows(tj, q); ++k) n += q + k + 1;
    return n;
}
// Chains are split over four waves at twojmax 8 and 10 (operation counts
// balanced to within 4%, at most 75 complex accumulators per wave, and
// power tables small enough that every wave keeps its share in VGPRs with
// two waves per SIMD); one wave below that.
__host__ __device__ constexpr int n_groups(int tj) { return tj >= 8 ? 4 : 1; }
__host__ __device__ constexpr bool in_group(int tj, int g, int q) {
    if (tj == 10) return g == 0 ? (q == 0 || q == 5 || q == 10)
                       : g == 1 ? (q == 1 || q == 2 || q == 3 || q == 4)
                       : g == 2 ? (q == 6 || q == 9)
                                : (q == 7 || q == 8);
    if (tj == 8) return g == 0 ? (q <= 3) : g == 1 ? (q == 4) : g == 2 ? (q == 5 || q == 8) : (q == 6 || q == 7);
    return g == 0;
}
__host__ __device__ constexpr int group_size(int tj, int g) {
    int n = 0;
    for (int q = 0; q <= tj; ++q)
        if (in_group(tj, g, q)) n += chain_len(tj, q);
    return n;
}
__host__ __device__ constexpr int group_qmax(int tj, int g) {
    int m = 0;
    for (int q = 0; q <= tj; ++q)
        if (in_group(tj, g, q)) m = q;
    return m;
}
__host__ __device__ constexpr int chain_slot(int tj, int g, int q) {
    int n = 0;
    for (int p = 0; p < q; ++p)
        if (in_group(tj, g, p)) n += chain_len(tj, p);
    return n;
}
__host__ __device__ constexpr int row_slot(int q, int k) {
    int n = 0;
    for (int i = 0; i < k; ++i) n += q + i + 1;
    return n;
}

__host__ __device__ constexpr double ce_binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

__host__ __device__ constexpr double ce_fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// x * (-1)^k for wave-uniform x and k, as a sign-bit flip on the scalar unit
__device__ __forceinline__ float flip_odd(float x, int k) {
    return __int_as_float(__float_as_int(x) ^ (int)((unsigned)(k & 1) << 31));
}

// Number of (ma, ma1) row pairs of a triple (rows ma <= J/2), their index,
// and which rows of u^{J1} and u^{J2} they use.
__host__ __device__ constexpr int zb_pairs(int J1, int J2, int J) {
    int n = 0;
    for (int ma = 0; ma <= J / 2; ++ma)
        for (int ma1 = 0; ma1 <= J1; ++ma1)
            if (zb_pair_ok(J1, J2, J, ma, ma1)) ++n;
    return n;
}
__host__ __device__ constexpr int zb_pair_index(int J1, int J2, int J, int ma, int ma1) {
    int n = 0;
    for (int a = 0; a <= J / 2; ++a)
        for (int a1 = 0; a1 <= J1; ++a1)
            if (zb_pair_ok(J1, J2, J, a, a1)) {
                if (a == ma && a1 == ma1) return n;
                ++n;
            }
    return -1;
}
// Scaling side of the dL/du column (the Z contraction of the adjoint).  It
// keeps the mirrored rows of the unscaled level unsigned: their sign
// (-1)^(row - column) alternates with the m1' column, so the pairs using them
// accumulate R <- P - R (a negated addend) and take the sign once, on the
// row CG factor in the fold.  The per-column scaling cost is then 2
// multiplies per used row of the scaled level, the smaller one scaled (ties
// as zb_scale2).
__host__ __device__ constexpr bool zy_scale2(int A, int B, int C) {
    const ZbRows r = zb_rows(A, B, C);
    return r.used2 < r.used1 || (r.used2 == r.used1 && zb_scale2(A, B, C));
}
__host__ __device__ constexpr int zy_scale_ops(int A, int B, int C) {
    const ZbRows r = zb_rows(A, B, C);
    return 2 * (zy_scale2(A, B, C) ? r.used2 : r.used1);
}
// Pair (ma, ma1) uses a mirrored row of the unscaled level, and which row.
__host__ __device__ constexpr bool zy_alt(int A, int B, int C, int ma, int ma1) {
    return zy_scale2(A, B, C) ? 2 * ma1 > A : 2 * (ma - ma1 + (A + B - C) / 2) > B;
}
__host__ __device__ constexpr int zy_alt_row(int A, int B, int C, int ma, int ma1) {
    return zy_scale2(A, B, C) ? ma1 : ma - ma1 + (A + B - C) / 2;
}
}  // namespace mala
