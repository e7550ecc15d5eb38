// Adjoint of the bispectrum descriptors, second step: dL/dR from Y = dL/du
// (the descriptor factor of the force expression, Eq. forcesmala).  With
// u^J = I + sum_k fc(r_k) U^J(Delta_k) (Eq. SNAPExpansion), per grid point
// and neighbour image k,
//   dL/dDelta_k = fc sum Re(conj(Y) dU/dDelta) + fc' n_k sum Re(conj(Y) U)
// (rows below the middle of a level twice, by the shared conjugate symmetry).
// U and its derivative along the three directions follow the chain recursion
// of the U kernel: row 0 of chain q from powers of b and conj(a), every later
// row by one more factor (a xi - conj(b) eta); each row is contracted with Y
// as soon as it is formed.  The chains are split over the waves of a block as
// in the U kernel; each wave makes one pass per derivative direction.  Per
// candidate image the lanes' and waves' terms are
// summed in LDS, then added to its atom's gradient with one FP64 atomic per
// component (the order of those additions is not fixed).  An atom sitting
// exactly on a grid point is left out of that point's gradient: the map from
// the displacement to U has no derivative at r = 0.
#include "snap_core.h"
#include "tile_gather.h"

namespace mala {
// ------------------------------------------------------------------ dL/dDelta
// One chain q of U rows for one neighbour: value c and its derivative dc
// along direction DIR (unnormalised coefficients, see the U kernel), each row
// contracted with Y: gu += sum Re(conj Y' c), gd += sum Re(conj Y' dc),
// Y' = w N Y (w = 2 below the middle row, N the normalisation of U).
template <int TJ, int Q>
__device__ __forceinline__ void dedr_chain(const float2* __restrict__ yt, float ar, float ai, float br, float bi,
                                           float dar, float dai, float dbr, float dbi, float& gu, float& gd) {
    constexpr int NR = chain_rows(TJ, Q);
    constexpr int JM = Q + NR - 1;          // last level of the chain
    float cr[JM + 1], ci[JM + 1], dcr[JM + 1], dci[JM + 1];
    // row 0 of level Q: binom(Q, mb) b^mb conj(a)^(Q-mb)
    {
        float pbr[Q + 1], pbi[Q + 1], par[Q + 1], pai[Q + 1];     // b^i, conj(a)^i
        pbr[0] = 1.f; pbi[0] = 0.f; par[0] = 1.f; pai[0] = 0.f;
        static_for<1, Q + 1>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            pbr[i] = pbr[i - 1] * br - pbi[i - 1] * bi;
            pbi[i] = pbr[i - 1] * bi + pbi[i - 1] * br;
            par[i] = par[i - 1] * ar + pai[i - 1] * ai;      // times conj(a) = (ar, -ai)
            pai[i] = pai[i - 1] * ar - par[i - 1] * ai;
        });
        static_for<0, Q + 1>([&](auto mc) {
            constexpr int mb = decltype(mc)::value;
            constexpr float bin = (float)ce_binom(Q, mb);
            const float vr = pbr[mb] * par[Q - mb] - pbi[mb] * pai[Q - mb];
            const float vi = pbr[mb] * pai[Q - mb] + pbi[mb] * par[Q - mb];
            cr[mb] = bin * vr;
            ci[mb] = bin * vi;
            float xr = 0.f, xi = 0.f;
            if constexpr (mb > 0) {       // mb b^(mb-1) db conj(a)^(Q-mb)
                const float tr = pbr[mb - 1] * par[Q - mb] - pbi[mb - 1] * pai[Q - mb];
                const float ti = pbr[mb - 1] * pai[Q - mb] + pbi[mb - 1] * par[Q - mb];
                xr += (float)mb * (tr * dbr - ti * dbi);
                xi += (float)mb * (tr * dbi + ti * dbr);
            }
            if constexpr (Q - mb > 0) {   // (Q-mb) b^mb conj(a)^(Q-mb-1) conj(da)
                const float tr = pbr[mb] * par[Q - mb - 1] - pbi[mb] * pai[Q - mb - 1];
                const float ti = pbr[mb] * pai[Q - mb - 1] + pbi[mb] * par[Q - mb - 1];
                xr += (float)(Q - mb) * (tr * dar + ti * dai);
                xi += (float)(Q - mb) * (ti * dar - tr * dai);
            }
            dcr[mb] = bin * xr;
            dci[mb] = bin * xi;
        });
    }
    static_for<0, NR>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int J = Q + k;
        if constexpr (k > 0) {
            // row k of level J from row k-1 of level J-1: c'[mb] = a c[mb-1] - conj(b) c[mb]
            static_for<0, J + 1>([&](auto mcr) {
                constexpr int mb = J - decltype(mcr)::value;      // descending: in place
                const float o0r = mb >= 1 ? cr[mb - 1] : 0.f, o0i = mb >= 1 ? ci[mb - 1] : 0.f;
                const float o1r = mb <= J - 1 ? cr[mb] : 0.f, o1i = mb <= J - 1 ? ci[mb] : 0.f;
                const float e0r = mb >= 1 ? dcr[mb - 1] : 0.f, e0i = mb >= 1 ? dci[mb - 1] : 0.f;
                const float e1r = mb <= J - 1 ? dcr[mb] : 0.f, e1i = mb <= J - 1 ? dci[mb] : 0.f;
                // da c0 + a dc0 - conj(db) c1 - conj(b) dc1
                float xr = dar * o0r - dai * o0i + ar * e0r - ai * e0i;
                float xi = dar * o0i + dai * o0r + ar * e0i + ai * e0r;
                xr -= dbr * o1r + dbi * o1i + br * e1r + bi * e1i;
                xi -= dbr * o1i - dbi * o1r + br * e1i - bi * e1r;
                dcr[mb] = xr;
                dci[mb] = xi;
                cr[mb] = ar * o0r - ai * o0i - (br * o1r + bi * o1i);
                ci[mb] = ar * o0i + ai * o0r - (br * o1i - bi * o1r);
            });
        }
        // contract row k of level J with Y (rows below the middle count twice);
        // the barrier keeps this row's loads of Y from being hoisted above the
        // recursion, where they would all be live at once
        asm volatile("" ::: "memory");
        constexpr float w = (2 * k == J) ? 1.f : 2.f;
        static_for<0, J + 1>([&](auto mc) {
            constexpr int mb = decltype(mc)::value;
            constexpr float nrm =
                w * (float)ce_sqrt(ce_fact(mb) * ce_fact(J - mb) / (ce_fact(k) * ce_fact(J - k)));
            const float2 y = yt[(half_off(J) + k * (J + 1) + mb) * kTile];
            const float yr = nrm * y.x, yi = nrm * y.y;
            gu = fmaf(yr, cr[mb], fmaf(yi, ci[mb], gu));
            gd = fmaf(yr, dcr[mb], fmaf(yi, dci[mb], gd));
        });
    });
}

template <int TJ, int G>
__device__ __forceinline__ void dedr_group(const float2* __restrict__ yt, float ar, float ai, float br, float bi,
                                           float dar, float dai, float dbr, float dbi, float& gu, float& gd) {
    static_for<0, TJ + 1>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (in_group(TJ, G, q)) dedr_chain<TJ, q>(yt, ar, ai, br, bi, dar, dai, dbr, dbi, gu, gd);
    });
}

// n_groups waves: wave w takes the chains of group w, in three passes (one
// per derivative direction)
template <int TJ>
__global__ __launch_bounds__(64 * n_groups(TJ)) void k_dedr(BinState bins, int Nx, int Ny, int Nz,
                                                               double rcut, int64_t pt_begin, int64_t n_pts,
                                                               const float2* __restrict__ y_in,
                                                               double* __restrict__ dLdR, int* __restrict__ err) {
    constexpr int NH = n_half(TJ);
    constexpr int NG = n_groups(TJ);
    __shared__ float4 cand[kMaxCand];
    __shared__ unsigned short nbr[kMaxNbr][kTile];
    __shared__ int nnbr[kTile];
    __shared__ int scan_tmp[16];
    __shared__ float cgrad[kMaxCand][3];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tile = blockIdx.x;
    const int64_t idx = tile * kTile + lane;
    const bool valid = idx < n_pts;
    const int64_t p = pt_begin + (valid ? idx : tile * kTile);
    const int64_t pk = p % Nz, pj = (p / Nz) % Ny, pi = p / ((int64_t)Ny * Nz);
    const double rx = (double)pi * bins.L[0] / Nx, ry = (double)pj * bins.L[1] / Ny,
                 rz = (double)pk * bins.L[2] / Nz;
    const int64_t p0 = pt_begin + tile * kTile;
    const int64_t qk = p0 % Nz, qj = (p0 / Nz) % Ny, qi = p0 / ((int64_t)Ny * Nz);
    const double ox = (double)qi * bins.L[0] / Nx, oy = (double)qj * bins.L[1] / Ny,
                 oz = (double)qk * bins.L[2] / Nz;
    const double lo[3] = {wave_min_d(rx), wave_min_d(ry), wave_min_d(rz)};
    const double hi[3] = {wave_max_d(rx), wave_max_d(ry), wave_max_d(rz)};
    const double org[3] = {ox, oy, oz};

    const int base = gather_candidates(bins, lo, hi, org, rcut, cand, kMaxCand, scan_tmp);
    if (base > kMaxCand && threadIdx.x == 0) atomicOr(err, kErrCand);
    const int ncand = base < kMaxCand ? base : kMaxCand;
    for (int c = threadIdx.x; c < ncand; c += blockDim.x) cgrad[c][0] = cgrad[c][1] = cgrad[c][2] = 0.f;
    __syncthreads();

    const float px = (float)(rx - ox), py = (float)(ry - oy), pz = (float)(rz - oz);
    const float rcf = (float)rcut;
    if (wave == 0) {
        int cnt = 0;
        for (int c = 0; c < ncand; ++c) {
            const float4 q = cand[c];
            const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
            if (dx * dx + dy * dy + dz * dz < rcf * rcf) {
                if (cnt < kMaxNbr) nbr[cnt][lane] = (unsigned short)c;
                ++cnt;
            }
        }
        if (cnt > kMaxNbr) atomicOr(err, kErrNbr);
        nnbr[lane] = valid ? (cnt < kMaxNbr ? cnt : kMaxNbr) : 0;
    }
    __syncthreads();

    const float2* yt = y_in + tile * NH * kTile + lane;
    const int nn = nnbr[lane];
    const int nmax = wave_max_int(nn);
    // wave w: chain group w, one pass over its neighbours per derivative
    // direction (the value recursion is repeated per pass, which keeps one
    // derivative row in registers); each pass is a branch of its own
    static_for<0, 3 * NG>([&](auto wc) {
        constexpr int WV = decltype(wc)::value;
        constexpr int G = WV % NG, DIR = WV / NG;
        if (wave != G) return;
        constexpr float kpi = 3.14159265358979323846f;
        constexpr float kRfac0 = 0.99363f;
        const float kth = kRfac0 * kpi / rcf;
        for (int s = 0; s < nmax; ++s) {
            const bool act = s < nn;
            const int c = act ? nbr[s][lane] : 0;
            const float4 q = cand[c];
            const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const bool on = act && r2 > 0.f;       // an atom on the point has no derivative: left out
            const float r = on ? sqrtf(r2) : 1.f;
            const float inv = 1.f / r;
            const float n[3] = {dx * inv, dy * inv, dz * inv};
            const float nd = n[DIR];
            float sn, cs;
            sincosf(kth * r, &sn, &cs);
            const float ar = cs, ai = -n[2] * sn, br = -n[1] * sn, bi = -n[0] * sn;
            // derivatives along DIR: theta = kth r, n_i' = (delta_i,DIR - n_i n_DIR) / r
            const float dth = kth * nd;
            const float dnx = ((DIR == 0 ? 1.f : 0.f) - n[0] * nd) * inv;
            const float dny = ((DIR == 1 ? 1.f : 0.f) - n[1] * nd) * inv;
            const float dnz = ((DIR == 2 ? 1.f : 0.f) - n[2] * nd) * inv;
            const float dar = -sn * dth;
            const float dai = -(dnz * sn + n[2] * cs * dth);
            const float dbr = -(cs * dth * n[1] + sn * dny);
            const float dbi = -(cs * dth * n[0] + sn * dnx);
            float gu = 0.f, gd = 0.f;
            dedr_group<TJ, G>(yt, ar, ai, br, bi, dar, dai, dbr, dbi, gu, gd);
            if (on) {
                const float x = kpi * r / rcf;
                const float fc = 0.5f * (cosf(x) + 1.f), dfc = -0.5f * kpi / rcf * sinf(x);
                atomicAdd(&cgrad[c][DIR], fc * gd + dfc * nd * gu);
            }
        }
    });
    __syncthreads();
    for (int c = threadIdx.x; c < ncand; c += blockDim.x) {
        const int atom = __float_as_int(cand[c].w);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float v = cgrad[c][d];
            if (v != 0.f) atomicAdd(&dLdR[3 * atom + d], (double)v);
        }
    }
}

// ------------------------------------------------------------------ launch
__global__ void k_zero_f64(double* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

hipError_t launch_zero_f64(hipStream_t s, double* p, int64_t n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <int TJ>
static hipError_t dedr_tj(hipStream_t s, const BinState& bins, const int N[3], double rcut, int64_t pt_begin,
                          int64_t n_pts, const float2* y, double* dLdR, int* err) {
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dedr<TJ>, dim3((unsigned)n_tiles), dim3(64 * n_groups(TJ)), 0, s, bins, N[0], N[1], N[2],
                       rcut, pt_begin, n_pts, y, dLdR, err);
    return hipGetLastError();
}

hipError_t launch_dedr(hipStream_t s, int twojmax, const BinState& bins, const int N[3], double rcut,
                       int64_t pt_begin, int64_t n_pts, const float2* y, double* dLdR, int* err) {
    switch (twojmax) {
    case 2: return dedr_tj<2>(s, bins, N, rcut, pt_begin, n_pts, y, dLdR, err);
    case 4: return dedr_tj<4>(s, bins, N, rcut, pt_begin, n_pts, y, dLdR, err);
    case 6: return dedr_tj<6>(s, bins, N, rcut, pt_begin, n_pts, y, dLdR, err);
    case 8: return dedr_tj<8>(s, bins, N, rcut, pt_begin, n_pts, y, dLdR, err);
    case 10: return dedr_tj<10>(s, bins, N, rcut, pt_begin, n_pts, y, dLdR, err);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mala
