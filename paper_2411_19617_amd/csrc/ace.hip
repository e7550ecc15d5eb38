// Grid-centred atomic cluster expansion descriptors (Sec. 3.2.3, Eqs.
// unweighted_ionicdensity, gridatom_basis, grid_base, product_grid_basis,
// ace_grid), one chemical element, ranks 1-3:
//   A_nlm = sum over atom images within rcut of R_n(r) Y_l^m(d/r), plus the
//   grid point's own delta on l = 0 (R_n(0) Y_0^0 = (-1)^n / sqrt(4 pi));
//   R_n(r) = T_n(2 r / rcut - 1) fc(r) (Chebyshev times the cosine cutoff);
//   rank 1: A_n00; rank 2: sum_m (-1)^m A_{n1 l m} A_{n2 l -m};
//   rank 3: sum (l1 l2 l3; m1 m2 m3) A A A over multisets of three (n, l).
// Four waves per 64-point tile (lane = point): the tile's candidate atom
// images are gathered into LDS (shared with the other neighbour kernels);
// wave w visits candidates w, w+4, ... and accumulates its part of the
// lane's A_nlm (m >= 0; A_{l,-m} = (-1)^m conj(A_{l,m})) in registers: T_n by
// the three-term recurrence, Y_l^m = N_lm Q_l^m(z/r) ((x + i y)/r)^m with
// Q_l^m = (-1)^m d^m P_l / dt^m by the associated Legendre recurrence in l.
// The parts are added into LDS (float atomics, so the last bits depend on
// the order), then wave 0 forms ranks 1 and 2 and every wave takes every
// fourth rank-3 group (p1, p2, l3): the partial sums
// P(m3) = sum_m1 (l1 l2 l3; m1 m2 m3) A_{n1 l1 m1} A_{n2 l2 m2} from a table of
// packed terms (storage indices, conjugation flags, 3j symbol with signs,
// sorted by m3) read with wave-uniform loads, then B = sum_m3 P(m3) A_{n3 l3 m3}
// for every n3 of the group.  Bound: LDS reads and the table loads.
#include <mutex>

#include "ace.h"
#include "tile_gather.h"

namespace mala {

constexpr int kAceN = kAceMaxN;          // radial functions held per point
constexpr int kAceL = kAceMaxL;          // largest l held
constexpr int kAceLm = 15;               // (l, m >= 0) entries per n: l(l+1)/2 + m
constexpr int kAceWaves = 4;

__host__ __device__ constexpr double ace_fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}
__host__ __device__ constexpr double ace_sqrt(double x) {
    if (x <= 0.0) return 0.0;
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 64; ++i) r = 0.5 * (r + x / r);
    return r;
}
// N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
__host__ __device__ constexpr float ace_norm(int l, int m) {
    return (float)ace_sqrt((2 * l + 1) / (4.0 * 3.14159265358979323846) * ace_fact(l - m) / ace_fact(l + m));
}

// The tile's own point (lane = point) relative to the tile origin, and its
// candidate atom images gathered into cand (whole block).
struct AceTile {
    int64_t idx;      // point index within the launch range
    bool valid;
    float px, py, pz;
    int ncand;
};

__device__ __forceinline__ AceTile ace_tile(const BinState& bins, int Nx, int Ny, int Nz, double rcut, int64_t pt_begin,
                                            int64_t n_pts, float4* cand, int* scan_tmp, int* err) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = blockIdx.x;
    AceTile t;
    t.idx = tile * kTile + lane;
    t.valid = t.idx < n_pts;
    const int64_t p = pt_begin + (t.valid ? t.idx : tile * kTile);
    const int64_t pk = p % Nz, pj = (p / Nz) % Ny, pi = p / ((int64_t)Ny * Nz);
    const double rx = (double)pi * bins.L[0] / Nx, ry = (double)pj * bins.L[1] / Ny,
                 rz = (double)pk * bins.L[2] / Nz;
    const int64_t p0 = pt_begin + tile * kTile;
    const int64_t qk = p0 % Nz, qj = (p0 / Nz) % Ny, qi = p0 / ((int64_t)Ny * Nz);
    const double ox = (double)qi * bins.L[0] / Nx, oy = (double)qj * bins.L[1] / Ny,
                 oz = (double)qk * bins.L[2] / Nz;
    const TileBoxes boxes = tile_boxes(p, p0, Ny, Nz, rx, ry, rz);
    const double org[3] = {ox, oy, oz};
    const int base = gather_candidates(bins, boxes, org, rcut, cand, kMaxCand, scan_tmp);
    if (base > kMaxCand && threadIdx.x == 0) atomicOr(err, kErrCand);
    t.ncand = base < kMaxCand ? base : kMaxCand;
    t.px = (float)(rx - ox);
    t.py = (float)(ry - oy);
    t.pz = (float)(rz - oz);
    return t;
}

// Adds the lane's A_nlm (n < 4, l <= 4, m >= 0) into sA (zeroed by the
// caller): wave w of nw visits candidates w, w + nw, ...; wave 0 adds the
// grid point's own delta.
__device__ __forceinline__ void ace_project(const float4* cand, const AceTile& tl, double rcut, int wave, int nw,
                                            int lane, float2 (*sA)[kTile]) {
    const int ncand = tl.ncand;
    const float px = tl.px, py = tl.py, pz = tl.pz;
    const float rcf = (float)rcut, rc2 = rcf * rcf;
    constexpr float kpi = 3.14159265358979323846f;
    float ar[kAceN][kAceLm], ai[kAceN][kAceLm];
#pragma unroll
    for (int n = 0; n < kAceN; ++n)
#pragma unroll
        for (int e = 0; e < kAceLm; ++e) ar[n][e] = ai[n][e] = 0.f;
    constexpr float y00 = 0.28209479177387814f;            // 1 / sqrt(4 pi)
    if (wave == 0) {
#pragma unroll
        for (int n = 0; n < kAceN; ++n) ar[n][0] = (n & 1) ? -y00 : y00;  // the grid point's own delta
    }
    for (int c = wave; c < ncand; c += nw) {
        const float4 q = cand[c];
        const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < rc2)) continue;
        const float r = sqrtf(r2);
        // radial: T_n(x) fc(r)
        const float x = 2.f * r / rcf - 1.f;
        const float fc = 0.5f * (cosf(kpi * r / rcf) + 1.f);
        float R[kAceN];
        R[0] = fc;
        R[1] = x * fc;
#pragma unroll
        for (int n = 2; n < kAceN; ++n) R[n] = 2.f * x * R[n - 1] - R[n - 2];
        if (r2 == 0.f) {                                   // an atom on the point: l = 0 only
#pragma unroll
            for (int n = 0; n < kAceN; ++n) ar[n][0] += R[n] * y00;
            continue;
        }
        const float inv = 1.f / r;
        const float t = dz * inv, ur = dx * inv, ui = dy * inv;
        // Q_l^m(t) for l <= 4, m >= 0, and ((x + i y)/r)^m
        float Q[kAceLm];
        float er[kAceL + 1], ei[kAceL + 1];
        er[0] = 1.f;
        ei[0] = 0.f;
#pragma unroll
        for (int m = 1; m <= kAceL; ++m) {
            er[m] = er[m - 1] * ur - ei[m - 1] * ui;
            ei[m] = er[m - 1] * ui + ei[m - 1] * ur;
        }
        static_for<0, kAceL + 1>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            // Q_m^m = (-1)^m (2m-1)!!
            constexpr float qmm = (float)(((m & 1) ? -1.0 : 1.0) * (ace_fact(2 * m) / (ace_fact(m) * (double)(1 << m))));
            Q[m * (m + 1) / 2 + m] = qmm;
            if constexpr (m + 1 <= kAceL) Q[(m + 1) * (m + 2) / 2 + m] = (2 * m + 1) * t * qmm;
            static_for<m + 2, kAceL + 1>([&](auto lc) {
                constexpr int l = decltype(lc)::value;
                Q[l * (l + 1) / 2 + m] = ((2 * l - 1) * t * Q[(l - 1) * l / 2 + m] -
                                          (float)(l + m - 1) * Q[(l - 2) * (l - 1) / 2 + m]) /
                                         (float)(l - m);
            });
        });
        static_for<0, kAceL + 1>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            static_for<0, l + 1>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                constexpr int e = l * (l + 1) / 2 + m;
                constexpr float nrm = ace_norm(l, m);
                const float yr = nrm * Q[e] * er[m], yi = nrm * Q[e] * ei[m];
#pragma unroll
                for (int n = 0; n < kAceN; ++n) {
                    ar[n][e] = fmaf(R[n], yr, ar[n][e]);
                    ai[n][e] = fmaf(R[n], yi, ai[n][e]);
                }
            });
        });
    }
#pragma unroll
    for (int n = 0; n < kAceN; ++n)
#pragma unroll
        for (int e = 0; e < kAceLm; ++e) {
            atomicAdd(&sA[n * kAceLm + e][lane].x, ar[n][e]);
            atomicAdd(&sA[n * kAceLm + e][lane].y, ai[n][e]);
        }
}

__global__ __launch_bounds__(64 * kAceWaves) void k_ace(BinState bins, int Nx, int Ny, int Nz, double rcut, int nmax, int lmax,
                                            int64_t pt_begin, int64_t n_pts, const int* __restrict__ groups,
                                            int n_groups, const int2* __restrict__ terms,
                                            const int* __restrict__ outputs, int n_desc, float* __restrict__ out,
                                            int* __restrict__ err) {
    __shared__ float4 cand[kMaxCand];
    __shared__ float2 sA[kAceN * kAceLm][kTile];
    __shared__ int scan_tmp[16];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const AceTile tl = ace_tile(bins, Nx, Ny, Nz, rcut, pt_begin, n_pts, cand, scan_tmp, err);
    const int64_t idx = tl.idx;
    const bool valid = tl.valid;
    for (int e = threadIdx.x; e < kAceN * kAceLm * kTile; e += blockDim.x)
        sA[e / kTile][e % kTile] = make_float2(0.f, 0.f);
    __syncthreads();
    ace_project(cand, tl, rcut, wave, kAceWaves, lane, sA);
    __syncthreads();

    float* o = out + (valid ? idx : 0) * n_desc;
    const int n12 = nmax + (lmax + 1) * nmax * (nmax + 1) / 2;
    int d = 0;
    if (wave == 0) {
    for (int n = 0; n < nmax; ++n, ++d)
        if (valid) o[d] = sA[n * kAceLm][lane].x;
    for (int l = 0; l <= lmax; ++l)
        for (int n1 = 0; n1 < nmax; ++n1)
            for (int n2 = n1; n2 < nmax; ++n2, ++d) {
                // sum_m (-1)^m A_{n1 l m} A_{n2 l -m} = A_{n1 l 0} A_{n2 l 0} + 2 sum_{m>0} Re(A_{n1 l m} conj(A_{n2 l m}))
                const int e0 = l * (l + 1) / 2;
                const float2 a0 = sA[n1 * kAceLm + e0][lane], b0 = sA[n2 * kAceLm + e0][lane];
                float s = a0.x * b0.x + a0.y * b0.y;
                for (int m = 1; m <= l; ++m) {
                    const float2 a = sA[n1 * kAceLm + e0 + m][lane], b = sA[n2 * kAceLm + e0 + m][lane];
                    s = fmaf(2.f, a.x * b.x + a.y * b.y, s);
                }
                if (valid) o[d] = s;
            }
    }
    // rank 3 by groups (p1, p2, l3): P(m3) once, then every n3 of the group
    // the next group's header is loaded while the current group is formed
    // (a wave past the last group re-reads group 0, unused)
    auto header = [&](int gi, int (&h)[6]) {
        const int* gr = groups + 8 * (gi < n_groups ? gi : 0);
#pragma unroll
        for (int i = 0; i < 6; ++i) h[i] = gr[i];
    };
    int nxt[6] = {0, 0, 0, 0, 0, 0};
    if (n_groups > 0) header(wave, nxt);
    for (int gi = wave; gi < n_groups; gi += kAceWaves) {
        int h[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) h[i] = nxt[i];
        header(gi + kAceWaves, nxt);
        int t = __builtin_amdgcn_readfirstlane(h[0]);
        const int l3 = __builtin_amdgcn_readfirstlane(h[1]);
        const int o0 = __builtin_amdgcn_readfirstlane(h[2]), oc = __builtin_amdgcn_readfirstlane(h[3]);
        const int cnt8 = __builtin_amdgcn_readfirstlane(h[4]), c8 = __builtin_amdgcn_readfirstlane(h[5]);
        float pr[9], pim[9];
        static_for<0, 9>([&](auto sc) {
            constexpr int slot = decltype(sc)::value;
            const int cnt = slot < 8 ? (cnt8 >> (4 * slot)) & 15 : c8;
            float xr = 0.f, xi = 0.f;
            auto term = [&](int2 e) {
                const int pk2 = __builtin_amdgcn_readfirstlane(e.x);
                const float cf = __int_as_float(__builtin_amdgcn_readfirstlane(e.y));
                const float2 a = sA[pk2 & 127][lane], b = sA[(pk2 >> 7) & 127][lane];
                const float ay = (pk2 & (1 << 14)) ? -a.y : a.y;
                const float by = (pk2 & (1 << 15)) ? -b.y : b.y;
                xr = fmaf(cf, a.x * b.x - ay * by, xr);
                xi = fmaf(cf, a.x * by + ay * b.x, xi);
            };
            // four terms per step: their table loads and LDS reads are issued
            // together, so a step waits once instead of once per term
            int k = 0;
            for (; k + 4 <= cnt; k += 4, t += 4) {
                int2 e[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) e[j] = terms[t + j];
#pragma unroll
                for (int j = 0; j < 4; ++j) term(e[j]);
            }
            if (k + 2 <= cnt) {
                const int2 e0 = terms[t], e1 = terms[t + 1];
                term(e0);
                term(e1);
                k += 2;
                t += 2;
            }
            if (k < cnt) term(terms[t++]);
            pr[slot] = xr;
            pim[slot] = xi;
        });
        for (int k = 0; k < oc; ++k) {
            const int ok = __builtin_amdgcn_readfirstlane(outputs[o0 + k]);
            const int base3 = ok & 127;
            float v = 0.f;
            static_for<0, 9>([&](auto sc) {
                constexpr int slot = decltype(sc)::value;
                constexpr int m3 = slot - 4, am = m3 < 0 ? -m3 : m3;
                if (am <= l3) {
                    // A_{l3,m3} = A_{l3,|m3|} for m3 >= 0, (-1)^|m3| conj(A_{l3,|m3|}) below
                    const float2 c = sA[base3 + am][lane];
                    constexpr float sg = (m3 < 0 && (am & 1)) ? -1.f : 1.f;
                    const float cy = m3 < 0 ? -c.y : c.y;
                    v = fmaf(sg, pr[slot] * c.x - pim[slot] * cy, v);    // Re(P A)
                }
            });
            if (valid) o[n12 + (ok >> 7)] = v;
        }
    }
}

// Rank 4 (one intermediate coupling L).  Eight waves per 64-point tile:
// after the projection, for every L the coupled pairs
// P_a(M) = sum_m1 <l1 m1 l2 m2|L M> A_p1 A_p2 (M = 0..L) the descriptors of
// that L need are formed into LDS (every wave takes every eighth unit
// (a, M)), then every wave evaluates a contiguous share of that L's
// descriptors, B = f (Re P_a(0) conj P_b(0) + 2 sum_{M>0} Re P_a(M) conj P_b(M))
// (f = (-1)^(l3+l4) / sqrt(2L+1)), keeping P_a in registers while consecutive
// descriptors share it.  Terms and descriptors come from wave-uniform loads.
constexpr int kAce4Waves = 8;

__global__ __launch_bounds__(64 * kAce4Waves) void k_ace4(BinState bins, int Nx, int Ny, int Nz, double rcut,
                                                          int lmax4, int64_t pt_begin, int64_t n_pts,
                                                          const int* __restrict__ l_units,
                                                          const int4* __restrict__ units,
                                                          const int2* __restrict__ terms,
                                                          const int* __restrict__ l_descs,
                                                          const int4* __restrict__ descs, int n4,
                                                          float* __restrict__ out, int* __restrict__ err) {
    __shared__ float4 cand[kMaxCand];
    __shared__ float2 sA[kAceN * kAceLm][kTile];
    __shared__ int scan_tmp[16];
    extern __shared__ float2 sP[];          // [slots][kTile]

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const AceTile tl = ace_tile(bins, Nx, Ny, Nz, rcut, pt_begin, n_pts, cand, scan_tmp, err);
    for (int e = threadIdx.x; e < kAceN * kAceLm * kTile; e += blockDim.x)
        sA[e / kTile][e % kTile] = make_float2(0.f, 0.f);
    __syncthreads();
    ace_project(cand, tl, rcut, wave, kAce4Waves, lane, sA);
    __syncthreads();

    float* o = out + (tl.valid ? tl.idx : 0) * n4;
    for (int L = 0; L <= 2 * lmax4; ++L) {
        // coupled pairs of this L into sP
        const int u0 = l_units[L], u1 = l_units[L + 1];
        for (int u = u0 + wave; u < u1; u += kAce4Waves) {
            const int4 h = units[u];
            int t = __builtin_amdgcn_readfirstlane(h.x);
            const int cnt = __builtin_amdgcn_readfirstlane(h.y), slot = __builtin_amdgcn_readfirstlane(h.z);
            float xr = 0.f, xi = 0.f;
            auto term = [&](int2 e) {
                const int pk2 = __builtin_amdgcn_readfirstlane(e.x);
                const float cf = __int_as_float(__builtin_amdgcn_readfirstlane(e.y));
                const float2 a = sA[pk2 & 127][lane], b = sA[(pk2 >> 7) & 127][lane];
                const float ay = (pk2 & (1 << 14)) ? -a.y : a.y;
                const float by = (pk2 & (1 << 15)) ? -b.y : b.y;
                xr = fmaf(cf, a.x * b.x - ay * by, xr);
                xi = fmaf(cf, a.x * by + ay * b.x, xi);
            };
            int k = 0;
            for (; k + 4 <= cnt; k += 4, t += 4) {
                int2 e[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) e[j] = terms[t + j];
#pragma unroll
                for (int j = 0; j < 4; ++j) term(e[j]);
            }
            for (; k < cnt; ++k) term(terms[t++]);
            sP[slot * kTile + lane] = make_float2(xr, xi);
        }
        __syncthreads();
        // this L's descriptors, a contiguous share per wave
        const int d0 = l_descs[L], nd = l_descs[L + 1] - d0;
        const int db = d0 + nd * wave / kAce4Waves, de = d0 + nd * (wave + 1) / kAce4Waves;
        int cached = -1;
        float2 pa[2 * kAce4MaxL + 1];
        for (int d = db; d < de; ++d) {
            const int4 q = descs[d];
            const int sa = __builtin_amdgcn_readfirstlane(q.x), sb = __builtin_amdgcn_readfirstlane(q.y);
            const int ok = __builtin_amdgcn_readfirstlane(q.z);
            const float f = __int_as_float(__builtin_amdgcn_readfirstlane(q.w));
            if (sa != cached) {
#pragma unroll
                for (int M = 0; M <= 2 * kAce4MaxL; ++M)
                    if (M <= L) pa[M] = sP[(sa + M) * kTile + lane];
                cached = sa;
            }
            const float2 b0 = sP[sb * kTile + lane];
            float acc = 0.f;
#pragma unroll
            for (int M = 1; M <= 2 * kAce4MaxL; ++M)
                if (M <= L) {
                    const float2 b = sP[(sb + M) * kTile + lane];
                    acc = fmaf(pa[M].x, b.x, fmaf(pa[M].y, b.y, acc));
                }
            const float v = f * fmaf(2.f, acc, pa[0].x * b0.x + pa[0].y * b0.y);
            if (tl.valid) o[ok] = v;
        }
        __syncthreads();
    }
}

hipError_t launch_ace4(hipStream_t s, const BinState& bins, const int N[3], double rcut, int lmax4, int64_t pt_begin,
                       int64_t n_pts, const int* l_units, const int4* units, const int2* terms, const int* l_descs,
                       const int4* descs, int max_slots, int n4, float* out, int* err) {
    if (n_pts <= 0 || n4 <= 0) return hipSuccess;
    if (lmax4 < 0 || lmax4 > kAce4MaxL) return hipErrorInvalidValue;
    const size_t lds = sizeof(float2) * (size_t)max_slots * kTile;
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(attr_once, [] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ace4),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kAce4LdsBudget);
    });
    if (attr_err != hipSuccess) return attr_err;
    if (lds > kAce4LdsBudget) return hipErrorInvalidValue;
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_ace4, dim3((unsigned)n_tiles), dim3(64 * kAce4Waves), lds, s, bins, N[0], N[1], N[2], rcut,
                       lmax4, pt_begin, n_pts, l_units, units, terms, l_descs, descs, n4, out, err);
    return hipGetLastError();
}

hipError_t launch_ace(hipStream_t s, const BinState& bins, const int N[3], double rcut, int nmax, int lmax,
                      int64_t pt_begin, int64_t n_pts, const int* groups, int n_groups, const int2* terms,
                      const int* outputs, int n_desc, float* out, int* err) {
    if (n_pts <= 0) return hipSuccess;
    if (nmax < 1 || nmax > kAceN || lmax < 0 || lmax > kAceL) return hipErrorInvalidValue;
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_ace, dim3((unsigned)n_tiles), dim3(64 * kAceWaves), 0, s, bins, N[0], N[1], N[2], rcut, nmax, lmax,
                       pt_begin, n_pts, groups, n_groups, terms, outputs, n_desc, out, err);
    return hipGetLastError();
}

}  // namespace mala
