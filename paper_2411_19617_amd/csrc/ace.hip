// Grid-centred atomic cluster expansion descriptors (Sec. 3.2.3, Eqs.
// unweighted_ionicdensity, gridatom_basis, grid_base, product_grid_basis,
// ace_grid), one chemical element:
//   A_nlm = sum over atom images within rcut of R_n(r) Y_l^m(d/r), plus the
//   grid point's own delta on l = 0 (R_n(0) Y_0^0 = (-1)^n / sqrt(4 pi));
//   R_n(r) = T_n(2 r / rcut - 1) fc(r) (Chebyshev times the cosine cutoff);
//   rank 1: A_n00; rank 2: sum_m (-1)^m A_{n1 l m} A_{n2 l -m};
//   rank 3: sum (l1 l2 l3; m1 m2 m3) A A A over multisets of three (n, l);
//   rank 4: the generalized Clebsch-Gordan contraction with one intermediate
//   coupling L (k_ace4 below).
// Two kernels per chunk of points.  k_ace_proj: per 64-point tile (lane =
// point) the candidate atom images are gathered into LDS (shared with the
// other neighbour kernels), wave 0 builds per-point neighbour lists, and wave
// n forms the rows A_{n l m} (m >= 0; A_{l,-m} = (-1)^m conj A_{l,m}) over its
// lane's list: T_n by the three-term recurrence, Y_l^m = N_lm Q_l^m(z/r)
// ((x + i y)/r)^m with Q_l^m = (-1)^m d^m P_l / dt^m by the associated
// Legendre recurrence in l; the tile's A goes to HBM (480 B per point,
// coalesced).  k_ace (ranks 1-3) and k_ace4 (rank 4) load a tile's A into
// LDS and contract it with few registers, so many waves share a CU.  Rank 3
// is grouped by (p1, p2, l3): the partial sums
// P(m3) = sum_m1 (l1 l2 l3; m1 m2 m3) A_{n1 l1 m1} A_{n2 l2 m2} from a table of
// packed terms (storage indices, conjugation flags, 3j symbol with signs,
// sorted by m3) read with wave-uniform loads, then B = sum_m3 P(m3) A_{n3 l3 m3}
// for every n3 of the group.  Outputs are written point-major or
// descriptor-major (one plane per descriptor, coalesced stores).
#include <mutex>

#include "ace.h"
#include "tile_gather.h"

namespace mala {

constexpr int kAceN = kAceMaxN;          // radial functions held per point
constexpr int kAceL = kAceMaxL;          // largest l held
constexpr int kAceLm = 15;               // (l, m >= 0) entries per n: l(l+1)/2 + m
constexpr int kAceWaves = 4;            // projection: one wave per radial index

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

// The tile's own point (lane = point) relative to the origins of its
// candidate atom images, gathered into cand (whole block).
struct AceTile {
    int64_t idx;      // point index within the launch range
    bool valid;
    PointFrame frame;
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
    const TileBoxes boxes = tile_boxes(p, p0, Ny, Nz, rx, ry, rz);
    int n0;
    const int base = gather_candidates(bins, boxes, rcut, cand, kMaxCand, scan_tmp, &n0);
    if (base > kMaxCand && threadIdx.x == 0) atomicOr(err, kErrCand);
    t.ncand = base < kMaxCand ? base : kMaxCand;
    t.frame = point_frame(boxes, n0, rx, ry, rz);
    return t;
}

// The lane's A_{n l m} for one radial index n (all l <= 4, m >= 0) over the
// lane's neighbour list (candidate indices within rcut, in candidate order),
// plus the grid point's own delta on l = 0; written to dst[lm][lane].
__device__ __forceinline__ void ace_project_n(const float4* cand, const unsigned short (*nbr)[kTile], int my_n,
                                              int n_iter, const AceTile& tl, double rcut, int n, int lane,
                                              float2* __restrict__ dst) {
    const float rcf = (float)rcut;
    constexpr float kpi = 3.14159265358979323846f;
    constexpr float y00 = 0.28209479177387814f;            // 1 / sqrt(4 pi)
    const float k2 = 2.f / rcf, kcut = kpi / rcf;          // per unit distance, formed once
    float ar[kAceLm], ai[kAceLm];
#pragma unroll
    for (int e = 0; e < kAceLm; ++e) ar[e] = ai[e] = 0.f;
    ar[0] = (n & 1) ? -y00 : y00;                          // the grid point's own delta: T_n(-1) Y_0^0
    for (int s = 0; s < n_iter; ++s) {
        if (s >= my_n) continue;
        const int c = nbr[s][lane];
        const float4 q = cand[c];
        const float3 o = tl.frame.at(c);
        const float dx = q.x - o.x, dy = q.y - o.y, dz = q.z - o.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        // 1/r and r from one hardware reciprocal square root (about 1 ulp)
        const bool at_point = !(r2 > kMinR2);
        const float inv = at_point ? 0.f : __builtin_amdgcn_rsqf(r2);
        const float r = r2 * inv;
        // radial: T_n(x) fc(r) by the three-term recurrence
        const float x = r * k2 - 1.f;
        const float fc = 0.5f * (cosf(kcut * r) + 1.f);
        float t0 = 1.f, t1 = x;
        for (int k = 2; k <= n; ++k) {
            const float t2 = 2.f * x * t1 - t0;
            t0 = t1;
            t1 = t2;
        }
        const float R = (n == 0 ? 1.f : t1) * fc;
        if (at_point) {                                    // an atom on the point: l = 0 only
            ar[0] += R * y00;
            continue;
        }
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
                const float y = R * nrm * Q[e];
                ar[e] = fmaf(y, er[m], ar[e]);
                ai[e] = fmaf(y, ei[m], ai[e]);
            });
        });
    }
#pragma unroll
    for (int e = 0; e < kAceLm; ++e) dst[e * kTile + lane] = make_float2(ar[e], ai[e]);
}

__global__ __launch_bounds__(64 * kAceWaves) void k_ace_proj(BinState bins, int Nx, int Ny, int Nz, double rcut,
                                                             int64_t pt_begin, int64_t n_pts,
                                                             float2* __restrict__ Ag, int* __restrict__ err) {
    __shared__ float4 cand[kMaxCand];
    __shared__ unsigned short nbr[kMaxNbr][kTile];
    __shared__ int nnbr[kTile];
    __shared__ int scan_tmp[16];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const AceTile tl = ace_tile(bins, Nx, Ny, Nz, rcut, pt_begin, n_pts, cand, scan_tmp, err);
    __syncthreads();
    // per-point neighbour lists (wave 0), in candidate order
    if (wave == 0) build_neighbour_lists(cand, tl.ncand, tl.frame, (float)rcut, tl.valid, lane, nbr, nnbr, err);
    __syncthreads();
    const int my_n = nnbr[lane];
    const int n_iter = wave_max_int(my_n);
    // wave n forms the rows of radial index n
    float2* dst = Ag + ((int64_t)blockIdx.x * kAceN * kAceLm + wave * kAceLm) * kTile;
    ace_project_n(cand, nbr, my_n, n_iter, tl, rcut, wave, lane, dst);
}

// The tile's A from the projection kernel into LDS (whole block).
__device__ __forceinline__ void ace_load_tile(const float2* __restrict__ Ag, float2 (*sA)[kTile]) {
    const float2* src = Ag + (int64_t)blockIdx.x * kAceN * kAceLm * kTile;
    for (int e = threadIdx.x; e < kAceN * kAceLm * kTile; e += blockDim.x) sA[e / kTile][e % kTile] = src[e];
}

// Position of the structural term (m3, m1) in the coefficient block of a
// rank-3 combination (l1, l2, l3): m3 = -l3..l3, m1 = -l1..l1 with
// |m1 + m3| <= l2 (the host builds the block in the same order).
__host__ __device__ constexpr int ace3_k(int L1, int L2, int L3, int m3, int m1) {
    int k = 0;
    for (int a = -L3; a <= L3; ++a)
        for (int b = -L1; b <= L1; ++b) {
            if (a == m3 && b == m1) return k;
            if (-b - a >= -L2 && -b - a <= L2) ++k;
        }
    return k;
}

// P(m3) = sum_m1 (l1 l2 l3; m1, m2 = -m1-m3, m3) A1(m1) A2(m2) of one group,
// code specialised for (L1, L2, L3): the group's A values are read from LDS
// once into registers (L1 + 1 and L2 + 1 of them, m >= 0), and every index,
// conjugation and sign of A_{l,-m} = (-1)^m conj A_{l,m} is resolved at
// compile time; the 3j symbols come from the combination's coefficient block.
template <int L1, int L2, int L3>
__device__ __forceinline__ void ace3_group(const float2 (*sA)[kTile], int b1, int b2, int lane,
                                           const float* __restrict__ cf, float (&pr)[9], float (&pim)[9]) {
    float2 a1[L1 + 1], a2[L2 + 1];
    static_for<0, L1 + 1>([&](auto mc) { a1[decltype(mc)::value] = sA[b1 + decltype(mc)::value][lane]; });
    static_for<0, L2 + 1>([&](auto mc) { a2[decltype(mc)::value] = sA[b2 + decltype(mc)::value][lane]; });
    static_for<0, 2 * L3 + 1>([&](auto ic) {
        constexpr int m3 = decltype(ic)::value - L3;
        // one slot's coefficients at a time (hoisting all of a group's loads
        // ahead would hold up to 81 of them in registers)
        __builtin_amdgcn_sched_barrier(0);
        float xr = 0.f, xi = 0.f;
        static_for<0, 2 * L1 + 1>([&](auto jc) {
            constexpr int m1 = decltype(jc)::value - L1, m2 = -m1 - m3;
            if constexpr (m2 >= -L2 && m2 <= L2) {
                constexpr int k = ace3_k(L1, L2, L3, m3, m1);
                constexpr int am1 = m1 < 0 ? -m1 : m1, am2 = m2 < 0 ? -m2 : m2;
                constexpr bool neg = ((m1 < 0 && (am1 & 1)) != (m2 < 0 && (am2 & 1)));
                const float c = neg ? -cf[k] : cf[k];
                const float ax = a1[am1].x, ay = m1 < 0 ? -a1[am1].y : a1[am1].y;
                const float bx = a2[am2].x, by = m2 < 0 ? -a2[am2].y : a2[am2].y;
                xr = fmaf(c, ax * bx - ay * by, xr);
                xi = fmaf(c, ax * by + ay * bx, xi);
            }
        });
        pr[m3 + 4] = xr;
        pim[m3 + 4] = xi;
    });
}

__host__ __device__ constexpr bool ace3_combo_valid(int c) {
    const int l1 = c / 25, l2 = (c / 5) % 5, l3 = c % 5;
    return l3 >= (l1 > l2 ? l1 - l2 : l2 - l1) && l3 <= l1 + l2 && (l1 + l2 + l3) % 2 == 0;
}

// Ranks 1-3 of one tile from its projected A (no register-heavy projection
// here, so many blocks share a CU).  STAGE: point-major output through LDS;
// the descriptor-major form stores directly and keeps the LDS for more blocks.
template <bool STAGE>
__global__ __launch_bounds__(64 * kAce3Waves) void k_ace(const float2* __restrict__ Ag, int nmax, int lmax,
                                                        int64_t n_pts, const int* __restrict__ groups,
                                                        int n_groups, const float* __restrict__ coef,
                                                        int n_desc,
                                                        float* __restrict__ out, int64_t ps, int64_t ds) {
    __shared__ float2 sA[kAceN * kAceLm][kTile];
    // point-major output: each wave gathers a pair's (contiguous) columns for
    // the tile's 64 points here, then writes them as row segments, several
    // rows per store instruction, instead of 64 values a row apart per store
    __shared__ float sO[STAGE ? kAce3Waves : 1][STAGE ? kAceMaxPairCols : 1][kTile + 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t idx = (int64_t)blockIdx.x * kTile + lane;
    const bool valid = idx < n_pts;
    constexpr bool stage = STAGE;
    ace_load_tile(Ag, sA);
    __syncthreads();

    float* o = out + (valid ? idx : 0) * ps;       // descriptor d at o[d * ds]
    const int n12 = nmax + (lmax + 1) * nmax * (nmax + 1) / 2;
    int d = 0;
    if (wave == 0) {
    for (int n = 0; n < nmax; ++n, ++d)
        if (valid) o[d * ds] = sA[n * kAceLm][lane].x;
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
                if (valid) o[d * ds] = s;
            }
    }
    // rank 3 by groups (p1, p2, l3): P(m3) once, then every n3 of the group
    // the next group's header is loaded while the current group is formed
    // (a wave past the last group re-reads group 0, unused)
    // (its outputs come with it: no load between the group and its LDS reads)
    auto header = [&](int gi, int (&h)[kAceGroupInts]) {
        const int* gr = groups + kAceGroupInts * (gi < n_groups ? gi : 0);
#pragma unroll
        for (int i = 0; i < kAceGroupInts; ++i) h[i] = gr[i];
    };
    int nxt[kAceGroupInts] = {};
    if (n_groups > 0) header(wave, nxt);
    for (int gi = wave; gi < n_groups; gi += kAce3Waves) {
        int h[kAceGroupInts];
#pragma unroll
        for (int i = 0; i < kAceGroupInts; ++i) h[i] = nxt[i];
        header(gi + kAce3Waves, nxt);
        const float* cf = coef + __builtin_amdgcn_readfirstlane(h[0]);
        const int l3 = __builtin_amdgcn_readfirstlane(h[1]);
        const int oc = __builtin_amdgcn_readfirstlane(h[2]);
        const int combo = __builtin_amdgcn_readfirstlane(h[3]);
        const int b1 = __builtin_amdgcn_readfirstlane(h[4]), b2 = __builtin_amdgcn_readfirstlane(h[5]);
        const int col0 = __builtin_amdgcn_readfirstlane(h[10]), pw = __builtin_amdgcn_readfirstlane(h[11]);
        float pr[9], pim[9];
        static_for<0, 125>([&](auto cc) {
            constexpr int C = decltype(cc)::value;
            if constexpr (ace3_combo_valid(C)) {
                if (combo == C) ace3_group<C / 25, (C / 5) % 5, C % 5>(sA, b1, b2, lane, cf, pr, pim);
            }
        });
        // every n3 of the group, by code specialised for l3: the A reads of
        // an output issue together, with no branch per m3 between them
        static_for<0, kAceMaxL + 1>([&](auto lc) {
            constexpr int L3 = decltype(lc)::value;
            if (l3 != L3) return;
            static_for<0, kAceN>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                if (k >= oc) return;
                const int ok = __builtin_amdgcn_readfirstlane(h[6 + k]);
                const int base3 = ok & 127;
                float2 c[L3 + 1];
#pragma unroll
                for (int am = 0; am <= L3; ++am) c[am] = sA[base3 + am][lane];
                float v = 0.f;
                static_for<4 - L3, 5 + L3>([&](auto sc) {
                    constexpr int slot = decltype(sc)::value;
                    constexpr int m3 = slot - 4, am = m3 < 0 ? -m3 : m3;
                    // A_{l3,m3} = A_{l3,|m3|} for m3 >= 0, (-1)^|m3| conj(A_{l3,|m3|}) below
                    constexpr float sg = (m3 < 0 && (am & 1)) ? -1.f : 1.f;
                    const float cy = m3 < 0 ? -c[am].y : c[am].y;
                    v = fmaf(sg, pr[slot] * c[am].x - pim[slot] * cy, v);    // Re(P A)
                });
                if constexpr (stage) sO[wave][(ok >> 7) - col0][lane] = v;
                else if (valid) o[(n12 + (ok >> 7)) * ds] = v;
            });
        });
        if (stage && (pw >> 8)) {                     // the pair's last group: write its columns
            const int ncol = pw & 255;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int rows = kTile / ncol, r_l = lane / ncol, c_l = lane - r_l * ncol;
            const int64_t t0 = (int64_t)blockIdx.x * kTile;
            for (int r0 = 0; r0 < kTile; r0 += rows) {
                const int r = r0 + r_l;
                if (r_l < rows && r < kTile && t0 + r < n_pts)
                    out[(t0 + r) * ps + (n12 + col0 + c_l)] = sO[wave][c_l][r];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Position of the term (M, m1) in the Clebsch-Gordan block of a rank-4
// pair combination (l1, l2, L): M = 0..L, m1 = -l1..l1 with |M - m1| <= l2
// (the host builds the block in the same order).
__host__ __device__ constexpr int ace4_k(int L1, int L2, int M, int m1) {
    int k = 0;
    for (int a = 0; a <= M; ++a)
        for (int b = -L1; b <= L1; ++b) {
            if (a == M && b == m1) return k;
            if (a - b >= -L2 && a - b <= L2) ++k;
        }
    return k;
}

// P_a(M) = sum_m1 <l1 m1 l2 m2|L M> A1(m1) A2(m2), m2 = M - m1, for M = 0..L,
// code specialised for (L1, L2, LL): the pair's A values in registers,
// indices, conjugations and signs at compile time; written to dst[M][lane].
template <int L1, int L2, int LL>
__device__ __forceinline__ void ace4_pair(const float2 (*sA)[kTile], int b1, int b2, int lane,
                                          const float* __restrict__ cf, float2* __restrict__ dst) {
    float2 a1[L1 + 1], a2[L2 + 1];
    static_for<0, L1 + 1>([&](auto mc) { a1[decltype(mc)::value] = sA[b1 + decltype(mc)::value][lane]; });
    static_for<0, L2 + 1>([&](auto mc) { a2[decltype(mc)::value] = sA[b2 + decltype(mc)::value][lane]; });
    static_for<0, LL + 1>([&](auto ic) {
        constexpr int M = decltype(ic)::value;
        __builtin_amdgcn_sched_barrier(0);
        float xr = 0.f, xi = 0.f;
        static_for<0, 2 * L1 + 1>([&](auto jc) {
            constexpr int m1 = decltype(jc)::value - L1, m2 = M - m1;
            if constexpr (m2 >= -L2 && m2 <= L2) {
                constexpr int k = ace4_k(L1, L2, M, m1);
                constexpr int am1 = m1 < 0 ? -m1 : m1, am2 = m2 < 0 ? -m2 : m2;
                constexpr bool neg = ((m1 < 0 && (am1 & 1)) != (m2 < 0 && (am2 & 1)));
                const float c = neg ? -cf[k] : cf[k];
                const float ax = a1[am1].x, ay = m1 < 0 ? -a1[am1].y : a1[am1].y;
                const float bx = a2[am2].x, by = m2 < 0 ? -a2[am2].y : a2[am2].y;
                xr = fmaf(c, ax * bx - ay * by, xr);
                xi = fmaf(c, ax * by + ay * bx, xi);
            }
        });
        dst[M * kTile + lane] = make_float2(xr, xi);
    });
}

__host__ __device__ constexpr bool ace4_combo_valid(int c) {
    const int l1 = c / 28, l2 = (c / 7) % 4, L = c % 7;
    return L >= (l1 > l2 ? l1 - l2 : l2 - l1) && L <= l1 + l2;
}

// Rank 4 (one intermediate coupling L).  Sixteen waves per 64-point tile
// (the projected A of the tile in LDS), in phases of one or more L: the
// coupled pairs P_a(M) = sum_m1 <l1 m1 l2 m2|L M> A_p1 A_p2 (M = 0..L) the
// descriptors of the phase need are formed into LDS (every wave takes every
// sixteenth pair, all its M by code specialised for (l1, l2, L)), then every
// wave evaluates a contiguous share of the phase's descriptors, B = f (Re P_a(0) conj P_b(0) + 2 sum_{M>0} Re P_a(M) conj P_b(M))
// (f = (-1)^(l3+l4) / sqrt(2L+1)), keeping P_a in registers while consecutive
// descriptors share it.  Terms and descriptors come from wave-uniform loads.
constexpr int kAce4Waves = 16;

__global__ __launch_bounds__(64 * kAce4Waves) void k_ace4(const float2* __restrict__ Ag, int n_phases, int64_t n_pts,
                                                          const int* __restrict__ l_units,
                                                          const int4* __restrict__ units,
                                                          const float* __restrict__ coef,
                                                          const int* __restrict__ l_descs,
                                                          const int4* __restrict__ descs, int n4,
                                                          float* __restrict__ out, int64_t ps, int64_t ds) {
    __shared__ float2 sA[kAceN * kAceLm][kTile];
    __shared__ int4 sD[kAce4MaxDescsL];     // this phase's descriptor entries
    extern __shared__ float2 sP[];          // [slots][kTile]

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    AceTile tl;
    tl.idx = (int64_t)blockIdx.x * kTile + lane;
    tl.valid = tl.idx < n_pts;
    ace_load_tile(Ag, sA);
    __syncthreads();

    float* o = out + (tl.valid ? tl.idx : 0) * ps;    // descriptor k at o[k * ds]
    for (int ph = 0; ph < n_phases; ++ph) {
        // this phase's descriptor entries into LDS, read back as broadcasts:
        // a scalar load per descriptor would hold every LDS wait of the loop
        // below until the scalar cache answered
        const int d0 = l_descs[ph], nd = l_descs[ph + 1] - d0;
        for (int i = threadIdx.x; i < nd; i += blockDim.x) sD[i] = descs[d0 + i];
        // coupled pairs of this phase's couplings L into sP
        const int u0 = l_units[ph], u1 = l_units[ph + 1];
        for (int u = u0 + wave; u < u1; u += kAce4Waves) {
            const int4 h = units[u];
            const float* cf = coef + __builtin_amdgcn_readfirstlane(h.x);
            const int combo = __builtin_amdgcn_readfirstlane(h.y), slot = __builtin_amdgcn_readfirstlane(h.z);
            const int bb = __builtin_amdgcn_readfirstlane(h.w);
            const int b1 = bb & 255, b2 = bb >> 8;
            static_for<0, 4 * 4 * 7>([&](auto cc) {
                constexpr int C = decltype(cc)::value;
                if constexpr (ace4_combo_valid(C)) {
                    if (combo == C) ace4_pair<C / 28, (C / 7) % 4, C % 7>(sA, b1, b2, lane, cf, sP + slot * kTile);
                }
            });
        }
        __syncthreads();
        // this phase's descriptors, a contiguous share per wave
        const int db = nd * wave / kAce4Waves, de = nd * (wave + 1) / kAce4Waves;
        int cached = -1;
        float2 pa[2 * kAce4MaxL + 1];
        for (int d = db; d < de; ++d) {
            const int4 q = sD[d];
            const int sx = __builtin_amdgcn_readfirstlane(q.x), sb = __builtin_amdgcn_readfirstlane(q.y);
            const int sa = sx & 0xffff, L = sx >> 16;             // a slot identifies its L too
            const int ok = __builtin_amdgcn_readfirstlane(q.z);
            const float f = __int_as_float(__builtin_amdgcn_readfirstlane(q.w));
            // code per L: a descriptor's LDS reads issue together, with no
            // branch per M between them
            float v = 0.f;
            static_for<0, 2 * kAce4MaxL + 1>([&](auto lc) {
                constexpr int LL = decltype(lc)::value;
                if (L != LL) return;
                if (sa != cached) {
#pragma unroll
                    for (int M = 0; M <= LL; ++M) pa[M] = sP[(sa + M) * kTile + lane];
                    cached = sa;
                }
                float2 b[LL + 1];
#pragma unroll
                for (int M = 0; M <= LL; ++M) b[M] = sP[(sb + M) * kTile + lane];
                float acc = 0.f;
#pragma unroll
                for (int M = 1; M <= LL; ++M) acc = fmaf(pa[M].x, b[M].x, fmaf(pa[M].y, b[M].y, acc));
                v = f * fmaf(2.f, acc, pa[0].x * b[0].x + pa[0].y * b[0].y);
            });
            if (tl.valid) o[ok * ds] = v;
        }
        __syncthreads();
    }
}

// Point-major rows from descriptor planes: out[p * n_cols + k] = in[k * ld + p]
// for p < n_rows, k < n_cols, through a 64 x 64 LDS block (both sides
// coalesced); neighbouring blocks take neighbouring row tiles, so the reads
// of one plane stay together (one block per row tile walking every column
// block, or column blocks as neighbours, measured slower).
// Rank 4 writes its planes this way: the columns of one L are spread over
// the whole row, so its direct point-major stores put every lane's value in
// a line of its own.
__global__ __launch_bounds__(256) void k_planes_to_rows(const float* __restrict__ in, int64_t ld, int64_t n_rows,
                                                        int n_cols, float* __restrict__ out) {
    __shared__ float sT[64][kTile + 1];
    const int64_t p0 = (int64_t)blockIdx.x * kTile;
    const int c0 = blockIdx.y * 64;
    const int rows = (int)(n_rows - p0 < kTile ? n_rows - p0 : kTile);
    const int cols = n_cols - c0 < 64 ? n_cols - c0 : 64;
    for (int e = threadIdx.x; e < 64 * kTile; e += blockDim.x) {
        const int c = e / kTile, r = e % kTile;
        if (c < cols && r < rows) sT[c][r] = in[(int64_t)(c0 + c) * ld + p0 + r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTile * 64; e += blockDim.x) {
        const int r = e / 64, c = e % 64;
        if (c < cols && r < rows) out[(p0 + r) * n_cols + c0 + c] = sT[c][r];
    }
}

hipError_t launch_ace_proj(hipStream_t s, const BinState& bins, const int N[3], double rcut, int64_t pt_begin,
                           int64_t n_pts, float2* Ag, int* err) {
    if (n_pts <= 0) return hipSuccess;
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_ace_proj, dim3((unsigned)n_tiles), dim3(64 * kAceWaves), 0, s, bins, N[0], N[1], N[2], rcut,
                       pt_begin, n_pts, Ag, err);
    return hipGetLastError();
}

hipError_t launch_ace4(hipStream_t s, const float2* Ag, int lmax4, int n_phases, int64_t n_pts, const int* l_units,
                       const int4* units, const float* coef, const int* l_descs, const int4* descs, int max_slots,
                       int n4, float* out, int64_t ps, int64_t ds) {
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
    hipLaunchKernelGGL(k_ace4, dim3((unsigned)n_tiles), dim3(64 * kAce4Waves), lds, s, Ag, n_phases, n_pts, l_units,
                       units, coef, l_descs, descs, n4, out, ps, ds);
    return hipGetLastError();
}

hipError_t launch_planes_to_rows(hipStream_t s, const float* in, int64_t ld, int64_t n_rows, int n_cols, float* out) {
    if (n_rows <= 0 || n_cols <= 0) return hipSuccess;
    if (ld < n_rows) return hipErrorInvalidValue;
    const int64_t row_tiles = (n_rows + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_planes_to_rows, dim3((unsigned)row_tiles, (unsigned)((n_cols + 63) / 64)), dim3(256), 0, s,
                       in, ld, n_rows, n_cols, out);
    return hipGetLastError();
}

hipError_t launch_ace(hipStream_t s, const float2* Ag, int nmax, int lmax, int64_t n_pts, const int* groups,
                      int n_groups, const float* coef, int n_desc, float* out, int64_t ps,
                      int64_t ds) {
    if (n_pts <= 0) return hipSuccess;
    if (nmax < 1 || nmax > kAceN || lmax < 0 || lmax > kAceL) return hipErrorInvalidValue;
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    if (ds == 1)
        hipLaunchKernelGGL(k_ace<true>, dim3((unsigned)n_tiles), dim3(64 * kAce3Waves), 0, s, Ag, nmax, lmax, n_pts,
                           groups, n_groups, coef, n_desc, out, ps, ds);
    else
        hipLaunchKernelGGL(k_ace<false>, dim3((unsigned)n_tiles), dim3(64 * kAce3Waves), 0, s, Ag, nmax, lmax, n_pts,
                           groups, n_groups, coef, n_desc, out, ps, ds);
    return hipGetLastError();
}

}  // namespace mala
