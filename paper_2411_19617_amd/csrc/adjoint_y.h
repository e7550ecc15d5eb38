// Adjoint of the bispectrum descriptors, first step: the derivative of
// L = sum_p sum_l g_l(p) B_l(p) with respect to u (the descriptor factor of
// the force expression, Eq. forcesmala, applied through Eq. SNAPExpansion).
// With dL = sum_J sum_{m m'} Re(conj(Y^J_{m m'}) du^J_{m m'}),
//   Y^C = sum over coupled pairs (A >= B) of beta(A,B,C) Z^C(A,B),
//   beta = mult (j+1)/(C+1) g_l  (combo_of).
// The u tile of 64 points sits in LDS as for the Z/B contraction; every wave
// owns (level C, column mb) units (LPT plan) and forms the column of every
// Z^C(A,B) by the same T accumulation (one runtime loop over the pairs of the
// level, so one column body is live at a time), then writes the half rows of
// Y (the middle row of an even C for mb <= C/2 and its mirror, by the
// conjugate symmetry u and Z share).
#pragma once
#include "snap_core.h"

namespace mala {

typedef float fv2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) const fv2 lds_float2;      // the LDS u tile

constexpr int kYMaxWaves = 12;        // plan stride: waves of the widest group

// ------------------------------------------------------------------ Y
// Column mb of Z^C(A,B) (half rows; the middle row only for mb <= C/2),
// added to y with weight beta.  The mirrored rows of the unscaled level are
// used unsigned, their pairs accumulating T <- P - T, with the sign put on
// the row CG factor in the fold (zy_scale2).
template <int A, int B, int C, int YN>
__device__ __forceinline__ void zy_column(lds_float2* __restrict__ su, int lane, const float* __restrict__ cg,
                                          int mb, float beta, float (&yr)[YN], float (&yi)[YN]) {
    constexpr int D = (A + B - C) / 2;
    constexpr int HR = C / 2;
    constexpr bool MID = (C % 2 == 0);
    constexpr int HN = MID ? HR - 1 : HR;
    constexpr int W = C + 1;
    constexpr int NP = zb_pairs(A, B, C);
    constexpr bool S2 = zy_scale2(A, B, C);
    int off1 = half_off(A) * kTile, off2 = half_off(B) * kTile;
    asm volatile("" : "+s"(off1), "+s"(off2));
    lds_float2* l1 = su + lane + off1;
    lds_float2* l2 = su + lane + off2;
    const bool mid_on = mb <= HR;
    float tr[NP], ti[NP];
    auto pair_fma = [&](auto mac, auto ma1c, float wr, float wi, const float (&u2r)[B + 1],
                        const float (&u2i)[B + 1], auto first) {
        constexpr int ma = decltype(mac)::value, ma1 = decltype(ma1c)::value;
        constexpr int ma2 = ma - ma1 + D;
        constexpr int k = zb_pair_index(A, B, C, ma, ma1);
        if constexpr (decltype(first)::value) {
            tr[k] = fmaf(-wi, u2i[ma2], wr * u2r[ma2]);
            ti[k] = fmaf(wi, u2r[ma2], wr * u2i[ma2]);
        } else {
            constexpr float sa = zy_alt(A, B, C, ma, ma1) ? -1.f : 1.f;    // R <- P - R on alternating pairs
            tr[k] = fmaf(wr, u2r[ma2], sa * tr[k]);
            tr[k] = fmaf(-wi, u2i[ma2], tr[k]);
            ti[k] = fmaf(wr, u2i[ma2], sa * ti[k]);
            ti[k] = fmaf(wi, u2r[ma2], ti[k]);
        }
    };
    auto column = [&](int mb1, auto first) {
        const int mb2 = mb + D - mb1;
        const float c2 = cg[mb1 * W + mb];
        const float f1 = flip_odd(c2, mb1);          // the scaled level's mirrored rows
        const float f2 = flip_odd(c2, mb2);
        lds_float2* s1 = l1 + mb1 * kTile;
        lds_float2* m1 = l1 + (A - mb1) * kTile;
        lds_float2* s2 = l2 + mb2 * kTile;
        lds_float2* m2 = l2 + (B - mb2) * kTile;
        float u2r[B + 1], u2i[B + 1];
        static_for<0, B + 1>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            if constexpr (zb_row2_used(A, B, C, r)) {
                if constexpr (2 * r <= B) {
                    const fv2 v = s2[r * (B + 1) * kTile];
                    u2r[r] = S2 ? c2 * v.x : v.x;
                    u2i[r] = S2 ? c2 * v.y : v.y;
                } else if constexpr (S2) {
                    const fv2 v = m2[(B - r) * (B + 1) * kTile];
                    const float f = (r & 1) ? -f2 : f2;
                    u2r[r] = f * v.x;
                    u2i[r] = -f * v.y;
                } else {
                    const fv2 v = m2[(B - r) * (B + 1) * kTile];
                    u2r[r] = v.x;
                    u2i[r] = -v.y;
                }
            }
        });
        float wrs[A + 1], wis[A + 1];
        static_for<0, A + 1>([&](auto r1c) {
            constexpr int ma1 = decltype(r1c)::value;
            if constexpr (zb_row1_used(A, B, C, ma1)) {
                if constexpr (2 * ma1 <= A) {
                    const fv2 v = s1[ma1 * (A + 1) * kTile];
                    wrs[ma1] = S2 ? v.x : c2 * v.x;
                    wis[ma1] = S2 ? v.y : c2 * v.y;
                } else if constexpr (!S2) {
                    const fv2 v = m1[(A - ma1) * (A + 1) * kTile];
                    const float f = (ma1 & 1) ? -f1 : f1;
                    wrs[ma1] = f * v.x;
                    wis[ma1] = -f * v.y;
                } else {
                    const fv2 v = m1[(A - ma1) * (A + 1) * kTile];
                    wrs[ma1] = v.x;
                    wis[ma1] = -v.y;
                }
                static_for<0, HN + 1>([&](auto mc) {
                    if constexpr (zb_pair_ok(A, B, C, decltype(mc)::value, ma1))
                        pair_fma(mc, r1c, wrs[ma1], wis[ma1], u2r, u2i, first);
                });
            }
        });
        if constexpr (MID) {
            if (mid_on) {
                static_for<0, A + 1>([&](auto r1c) {
                    constexpr int ma1 = decltype(r1c)::value;
                    if constexpr (zb_pair_ok(A, B, C, HR, ma1))
                        pair_fma(std::integral_constant<int, HR>{}, r1c, wrs[ma1], wis[ma1], u2r, u2i, first);
                });
            }
        }
    };
    const int lo = max(0, mb + D - B), hi = min(A, mb + D);     // never empty
    column(lo, std::true_type{});
#pragma clang loop unroll(disable)
    for (int mb1 = lo + 1; mb1 <= hi; ++mb1) column(mb1, std::false_type{});
    const int par = S2 ? hi : mb + D + hi;         // sign parity of the alternating pairs, before the row's
    static_for<0, HR + 1>([&](auto mc) {
        constexpr int ma = decltype(mc)::value;
        constexpr bool MIDROW = MID && ma == HR;
        if (MIDROW && !mid_on) return;
        float zr = 0.f, zi = 0.f, zr2 = 0.f, zi2 = 0.f;
        static_for<0, A + 1>([&](auto r1c) {
            constexpr int ma1 = decltype(r1c)::value;
            if constexpr (zb_pair_ok(A, B, C, ma, ma1)) {
                constexpr int k = zb_pair_index(A, B, C, ma, ma1);
                float c1 = cg[ma1 * W + ma];
                if constexpr (zy_alt(A, B, C, ma, ma1)) c1 = flip_odd(c1, par + zy_alt_row(A, B, C, ma, ma1));
                if constexpr (zb_pair_doubled(A, B, C, ma, ma1)) {
                    zr2 = fmaf(c1, tr[k], zr2);
                    zi2 = fmaf(c1, ti[k], zi2);
                } else {
                    zr = fmaf(c1, tr[k], zr);
                    zi = fmaf(c1, ti[k], zi);
                }
            }
        });
        if constexpr (A == B) {
            zr = fmaf(2.f, zr2, zr);
            zi = fmaf(2.f, zi2, zi);
        }
        yr[ma] = fmaf(beta, zr, yr[ma]);
        yi[ma] = fmaf(beta, zi, yi[ma]);
    });
}

// the column of coupled pair k of level C (an if-chain over the level's
// combos, visited by one runtime loop: one column body is live at a time)
template <int TJ, int C, int K>
__device__ __forceinline__ void y_combo(int k, lds_float2* __restrict__ su, int lane,
                                        const float* __restrict__ cg_tab, const int* __restrict__ cg_off,
                                        const float* __restrict__ g, bool valid, int mb, float (&yr)[C / 2 + 1],
                                        float (&yi)[C / 2 + 1]) {
    if constexpr (K < n_combos(TJ)) {
        constexpr Combo cb = combo_of(TJ, K);
        if constexpr (cb.c == C) {
            if (k == K) {
                constexpr float fac = (float)(cb.mult * (cb.jmax + 1)) / (float)(C + 1);
                const float beta = valid ? fac * g[cb.triple] : 0.f;
                zy_column<cb.a, cb.b, C, C / 2 + 1>(su, lane, cg_tab + cg_off[K], mb, beta, yr, yi);
                return;
            }
            y_combo<TJ, C, K + 1>(k, su, lane, cg_tab, cg_off, g, valid, mb, yr, yi);
        }
    }
}

// Column mb of Y^C: every coupled pair of level C, then the half rows are
// written (middle row: mb <= C/2 and its mirror).
template <int TJ, int C>
__device__ __forceinline__ void y_level(int mb, lds_float2* __restrict__ su, int lane,
                                                   const float* __restrict__ cg_tab, const int* __restrict__ cg_off,
                                                   const float* __restrict__ g, bool valid, float2* __restrict__ yt) {
    constexpr int HR = C / 2;
    constexpr int K0 = combo_first(TJ, C), K1 = combo_first(TJ, C + 1);
    float yr[HR + 1], yi[HR + 1];
#pragma unroll
    for (int i = 0; i <= HR; ++i) yr[i] = yi[i] = 0.f;
#pragma clang loop unroll(disable)
    for (int k = K0; k < K1; ++k) y_combo<TJ, C, K0>(k, su, lane, cg_tab, cg_off, g, valid, mb, yr, yi);
    static_for<0, HR + 1>([&](auto mc) {
        constexpr int ma = decltype(mc)::value;
        constexpr int e = half_off(C) + ma * (C + 1);
        if constexpr (C % 2 == 0 && ma == HR) {
            if (mb <= HR) {
                yt[(e + mb) * kTile] = make_float2(yr[ma], yi[ma]);
                if (mb < HR) {       // Y[HR][C-mb] = (-1)^(HR-mb) conj(Y[HR][mb])
                    const float s = ((HR - mb) & 1) ? -1.f : 1.f;
                    yt[(e + C - mb) * kTile] = make_float2(s * yr[ma], -s * yi[ma]);
                }
            }
        } else {
            yt[(e + mb) * kTile] = make_float2(yr[ma], yi[ma]);
        }
    });
}

template <int TJ, int C, int CHI>
__device__ __forceinline__ void y_dispatch(int c, int mb, lds_float2* __restrict__ su, int lane,
                                           const float* __restrict__ cg_tab, const int* __restrict__ cg_off,
                                           const float* __restrict__ g, bool valid, float2* __restrict__ yt) {
    if constexpr (C <= CHI) {
        if (c == C) {
            y_level<TJ, C>(mb, su, lane, cg_tab, cg_off, g, valid, yt);
            return;
        }
        y_dispatch<TJ, C + 1, CHI>(c, mb, su, lane, cg_tab, cg_off, g, valid, yt);
    }
}

// Output levels are split into groups of contiguous levels, one kernel each
// (about 60 coupled pairs per kernel: the compile time of one fully inlined
// kernel grows faster than linearly with the pairs it holds; every group
// stages the u tile again).
__host__ __device__ constexpr int y_groups(int tj) { return tj == 10 ? 4 : tj == 8 ? 2 : 1; }
__host__ __device__ constexpr int y_group_lo(int tj, int g) {
    return tj == 10 ? (g == 0 ? 0 : g == 1 ? 4 : g == 2 ? 6 : 8) : tj == 8 ? (g == 0 ? 0 : 5) : 0;
}
__host__ __device__ constexpr int y_group_hi(int tj, int g) {
    return g + 1 < y_groups(tj) ? y_group_lo(tj, g + 1) - 1 : tj;
}

// Waves per block: three per SIMD (168 VGPRs) where the group's coupled pairs
// fit, two (256 VGPRs) for the two highest groups at twojmax 10.
__host__ __device__ constexpr int y_group_waves(int tj, int g) { return tj == 10 && g >= 2 ? 8 : 12; }

template <int TJ, int G>
__global__ __launch_bounds__(y_group_waves(TJ, G) * 64) void k_yi(const float2* __restrict__ u, int64_t n_pts,
                                                     const float* __restrict__ gB, float2* __restrict__ y_out,
                                                     const float* __restrict__ cg_tab, const int* __restrict__ cg_off,
                                                     const int* __restrict__ wave_units, int stride) {
    constexpr int NH = n_half(TJ);
    constexpr int NB = n_triples(TJ);
    extern __shared__ float2 su[];
    const int64_t tile = blockIdx.x;
    {
        const float4* src = reinterpret_cast<const float4*>(u + tile * NH * kTile);
        float4* dst = reinterpret_cast<float4*>(su);
        for (int i = threadIdx.x; i < NH * kTile / 2; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t idx = tile * kTile + lane;
    const bool valid = idx < n_pts;
    const float* g = gB + (valid ? idx : 0) * NB;

    float2* yt = y_out + tile * NH * kTile + lane;
    const int* list = wave_units + wave * stride;
    const int cnt = __builtin_amdgcn_readfirstlane(list[0]);
    for (int i = 0; i < cnt; ++i) {
        const int unit = __builtin_amdgcn_readfirstlane(list[1 + i]);
        y_dispatch<TJ, y_group_lo(TJ, G), y_group_hi(TJ, G)>(unit >> 5, unit & 31, (lds_float2*)su, lane,
                                                               cg_tab, cg_off, g, valid, yt);
    }
}

template <int TJ, int G>
hipError_t yi_group(hipStream_t s, int64_t n_pts, const float2* u, const float* gB, float2* y,
                    const float* cg_tab, const int* cg_off, const int* wave_units) {
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    if (n_tiles == 0) return hipSuccess;
    const size_t lds = sizeof(float2) * n_half(TJ) * kTile;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_yi<TJ, G>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_yi<TJ, G>), dim3((unsigned)n_tiles), dim3(y_group_waves(TJ, G) * 64), lds, s, u, n_pts, gB,
                       y, cg_tab, cg_off, wave_units + G * kYMaxWaves * kMaxYStride, kMaxYStride);
    return hipGetLastError();
}

}  // namespace mala
