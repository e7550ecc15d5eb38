// Adjoint of the bispectrum descriptors, second step: dL/dR from Y = dL/du
// (the descriptor factor of the force expression, Eq. forcesmala).  With
// u^J = I + sum_k fc(r_k) U^J(Delta_k) (Eq. SNAPExpansion), per grid point
// and neighbour image k,
//   dL/dDelta_k = fc sum Re(conj(Y) dU/dDelta) + fc' n_k sum Re(conj(Y) U)
// (rows below the middle of a level twice, by the shared conjugate symmetry).
// U follows the chain recursion of the U kernel: row 0 of chain q from powers
// of b and conj(a), every later row by one more factor (a xi - conj(b) eta).
// Its derivative comes from the rows of the level below through the
// homogeneity of the polynomial (see dedr_chain), so every row is contracted
// with Y once and the three directions are formed per neighbour at the end.
// The chains are split over the waves of a block as in the U kernel.  Per
// candidate image the lanes' and waves' terms are
// summed in LDS, then added to its atom's gradient with one FP64 atomic per
// component (the order of those additions is not fixed).  An atom sitting
// exactly on a grid point is left out of that point's gradient: the map from
// the displacement to U has no derivative at r = 0.
#include "snap_core.h"
#include "tile_gather.h"

namespace mala {
// ------------------------------------------------------------------ dL/dDelta
// One chain q of U rows for one neighbour, contracted with Y.  c^J_k is the
// unnormalised coefficient row of U^J (see the U kernel); as a homogeneous
// polynomial in (a, conj a, b, conj b) it has
//   dc^J_k[m] = k (da c^{J-1}_{k-1}[m-1] - d(conj b) c^{J-1}_{k-1}[m])
//             + (J-k) (db c^{J-1}_k[m-1] + d(conj a) c^{J-1}_k[m]),
// so the direction enters only through (da, db) and
//   sum_m Re(conj(Y'[m]) dc^J_k[m]) = Re(da A1 + conj(db) A2 + db A3 + conj(da) A4)
// with A1 = k sum conj(Y') c^{J-1}_{k-1}[m-1], A2 = -k sum conj(Y') c^{J-1}_{k-1}[m],
// A3 = (J-k) sum conj(Y') c^{J-1}_k[m-1], A4 = (J-k) sum conj(Y') c^{J-1}_k[m],
// Y' = w N Y (w = 2 below the middle row, N the normalisation of U).
// c^{J-1}_{k-1} is the chain's previous row; c^{J-1}_k is row k of chain
// q-1, advanced in step (or, for the middle row of an even J, the mirror of
// the previous row).  gu += sum Re(conj(Y') c^J_k).  A = (A1, A2, A3, A4) as
// (re, im) pairs.
template <int TJ, int Q>
__device__ __forceinline__ void dedr_chain(const float2* __restrict__ yt, float ar, float ai, float br, float bi,
                                           float (&A)[8], float& gu) {
    constexpr int NR = chain_rows(TJ, Q);
    constexpr int JM = Q + NR - 1;          // last level of the chain
    float cr[JM + 1], ci[JM + 1];           // this chain's row (level J-1 before the step, J after)
    float orr[JM + 1], oi[JM + 1];          // row k of chain Q-1 (level J-1)
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
        // row 0 of level Q: binom(Q, m) b^m conj(a)^(Q-m); of level Q-1 likewise
        static_for<0, Q + 1>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr float bin = (float)ce_binom(Q, m);
            cr[m] = bin * (pbr[m] * par[Q - m] - pbi[m] * pai[Q - m]);
            ci[m] = bin * (pbr[m] * pai[Q - m] + pbi[m] * par[Q - m]);
            if constexpr (Q >= 1 && m <= Q - 1) {
                constexpr float bo = (float)ce_binom(Q - 1, m);
                orr[m] = bo * (pbr[m] * par[Q - 1 - m] - pbi[m] * pai[Q - 1 - m]);
                oi[m] = bo * (pbr[m] * pai[Q - 1 - m] + pbi[m] * par[Q - 1 - m]);
            }
        });
    }
    // one a-step: row k of level L -> row k+1 of level L+1, in place (descending m)
    auto a_step = [&](float (&xr)[JM + 1], float (&xi)[JM + 1], auto lc) {
        constexpr int L = decltype(lc)::value;          // new level, entries 0..L
        static_for<0, L + 1>([&](auto mcr) {
            constexpr int m = L - decltype(mcr)::value;
            const float o0r = m >= 1 ? xr[m - 1] : 0.f, o0i = m >= 1 ? xi[m - 1] : 0.f;
            const float o1r = m <= L - 1 ? xr[m] : 0.f, o1i = m <= L - 1 ? xi[m] : 0.f;
            xr[m] = ar * o0r - ai * o0i - (br * o1r + bi * o1i);
            xi[m] = ar * o0i + ai * o0r - (br * o1i - bi * o1r);
        });
    };
    static_for<0, NR>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int J = Q + k;
        constexpr bool MIDROW = (2 * k == J);
        // the barrier keeps this row's loads of Y from being hoisted above the
        // previous row's work, where they would all be live at once
        asm volatile("" ::: "memory");
        float p1r = 0.f, p1i = 0.f, p2r = 0.f, p2i = 0.f, p3r = 0.f, p3i = 0.f, p4r = 0.f, p4i = 0.f;
        float yr[J + 1], yi[J + 1];
        static_for<0, J + 1>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr float nrm = (MIDROW ? 1.f : 2.f) *
                                  (float)ce_sqrt(ce_fact(m) * ce_fact(J - m) / (ce_fact(k) * ce_fact(J - k)));
            const float2 y = yt[(half_off(J) + k * (J + 1) + m) * kTile];
            yr[m] = nrm * y.x;
            yi[m] = nrm * y.y;
        });
        // conj(y) x = (yr xr + yi xi) + i (yr xi - yi xr)
        static_for<0, J + 1>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            if constexpr (k > 0) {                 // previous row c^{J-1}_{k-1} (in cr)
                if constexpr (m >= 1) {
                    p1r = fmaf(yr[m], cr[m - 1], fmaf(yi[m], ci[m - 1], p1r));
                    p1i = fmaf(yr[m], ci[m - 1], fmaf(-yi[m], cr[m - 1], p1i));
                }
                if constexpr (m <= J - 1) {
                    p2r = fmaf(yr[m], cr[m], fmaf(yi[m], ci[m], p2r));
                    p2i = fmaf(yr[m], ci[m], fmaf(-yi[m], cr[m], p2i));
                }
            }
            if constexpr (J - k > 0) {             // c^{J-1}_k: chain Q-1 row k, or the mirror
                float x0r = 0.f, x0i = 0.f, x1r = 0.f, x1i = 0.f;      // entries m-1 and m
                if constexpr (MIDROW) {
                    // c^{J-1}_k[n] = (-1)^(k-n) conj(c^{J-1}_{k-1}[J-1-n])
                    if constexpr (m >= 1) {
                        constexpr float sg = ((k - (m - 1)) & 1) ? -1.f : 1.f;
                        x0r = sg * cr[J - m];
                        x0i = -sg * ci[J - m];
                    }
                    if constexpr (m <= J - 1) {
                        constexpr float sg = ((k - m) & 1) ? -1.f : 1.f;
                        x1r = sg * cr[J - 1 - m];
                        x1i = -sg * ci[J - 1 - m];
                    }
                } else {
                    if constexpr (m >= 1) { x0r = orr[m - 1]; x0i = oi[m - 1]; }
                    if constexpr (m <= J - 1) { x1r = orr[m]; x1i = oi[m]; }
                }
                if constexpr (m >= 1) {
                    p3r = fmaf(yr[m], x0r, fmaf(yi[m], x0i, p3r));
                    p3i = fmaf(yr[m], x0i, fmaf(-yi[m], x0r, p3i));
                }
                if constexpr (m <= J - 1) {
                    p4r = fmaf(yr[m], x1r, fmaf(yi[m], x1i, p4r));
                    p4i = fmaf(yr[m], x1i, fmaf(-yi[m], x1r, p4i));
                }
            }
        });
        constexpr float fk = (float)k, fj = (float)(J - k);
        A[0] = fmaf(fk, p1r, A[0]);
        A[1] = fmaf(fk, p1i, A[1]);
        A[2] = fmaf(-fk, p2r, A[2]);
        A[3] = fmaf(-fk, p2i, A[3]);
        A[4] = fmaf(fj, p3r, A[4]);
        A[5] = fmaf(fj, p3i, A[5]);
        A[6] = fmaf(fj, p4r, A[6]);
        A[7] = fmaf(fj, p4i, A[7]);
        if constexpr (k > 0) a_step(cr, ci, std::integral_constant<int, J>{});   // c^J_k
        static_for<0, J + 1>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            gu = fmaf(yr[m], cr[m], fmaf(yi[m], ci[m], gu));
        });
        // advance chain Q-1 to row k+1 (level J) unless the next row is a middle row
        if constexpr (Q >= 1 && k + 1 < NR && 2 * (k + 1) != J + 1) a_step(orr, oi, std::integral_constant<int, J>{});
    });
}

template <int TJ, int G>
__device__ __forceinline__ void dedr_group(const float2* __restrict__ yt, float ar, float ai, float br, float bi,
                                           float (&A)[8], float& gu) {
    static_for<0, TJ + 1>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (in_group(TJ, G, q)) dedr_chain<TJ, q>(yt, ar, ai, br, bi, A, gu);
    });
}

// n_groups waves: wave w takes the chains of group w
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
    const TileBoxes boxes = tile_boxes(p, p0, Ny, Nz, rx, ry, rz);

    int n0;
    const int base = gather_candidates(bins, boxes, rcut, cand, kMaxCand, scan_tmp, &n0);
    if (base > kMaxCand && threadIdx.x == 0) atomicOr(err, kErrCand);
    const int ncand = base < kMaxCand ? base : kMaxCand;
    for (int c = threadIdx.x; c < ncand; c += blockDim.x) cgrad[c][0] = cgrad[c][1] = cgrad[c][2] = 0.f;
    __syncthreads();

    const PointFrame frame = point_frame(boxes, n0, rx, ry, rz);
    const float rcf = (float)rcut;
    if (wave == 0) build_neighbour_lists(cand, ncand, frame, rcf, valid, lane, nbr, nnbr, err);
    __syncthreads();

    const float2* yt = y_in + tile * NH * kTile + lane;
    const int nn = nnbr[lane];
    const int nmax = wave_max_int(nn);
    // wave w: chain group w, one pass over its neighbours for all three
    // directions (each group's loop is a branch of its own)
    static_for<0, NG>([&](auto gc) {
        constexpr int G = decltype(gc)::value;
        if (wave != G) return;
        constexpr float kpi = 3.14159265358979323846f;
        constexpr float kRfac0 = 0.99363f;
        const float kth = kRfac0 * kpi / rcf, kcut = kpi / rcf;     // per unit distance, formed once
        for (int s = 0; s < nmax; ++s) {
            const bool act = s < nn;
            const int c = act ? nbr[s][lane] : 0;
            const float4 q = cand[c];
            const float3 o = frame.at(c);
            const float dx = q.x - o.x, dy = q.y - o.y, dz = q.z - o.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const bool on = act && r2 > kMinR2;    // an atom on the point has no derivative: left out
            // 1/r and r from one hardware reciprocal square root (about 1 ulp)
            const float inv = on ? __builtin_amdgcn_rsqf(r2) : 1.f;
            const float r = on ? r2 * inv : 1.f;
            const float n[3] = {dx * inv, dy * inv, dz * inv};
            float sn, cs;
            sincosf(kth * r, &sn, &cs);
            const float ar = cs, ai = -n[2] * sn, br = -n[1] * sn, bi = -n[0] * sn;
            float A[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, gu = 0.f;
            dedr_group<TJ, G>(yt, ar, ai, br, bi, A, gu);
            if (on) {
                const float x = kcut * r;
                const float fc = 0.5f * (cosf(x) + 1.f), dfc = -0.5f * kcut * sinf(x);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    // theta = kth r, n_i' = (delta_id - n_i n_d) / r
                    const float dth = kth * n[d];
                    const float dnx = ((d == 0 ? 1.f : 0.f) - n[0] * n[d]) * inv;
                    const float dny = ((d == 1 ? 1.f : 0.f) - n[1] * n[d]) * inv;
                    const float dnz = ((d == 2 ? 1.f : 0.f) - n[2] * n[d]) * inv;
                    const float dar = -sn * dth;
                    const float dai = -(dnz * sn + n[2] * cs * dth);
                    const float dbr = -(cs * dth * n[1] + sn * dny);
                    const float dbi = -(cs * dth * n[0] + sn * dnx);
                    // Re(da A1 + conj(db) A2 + db A3 + conj(da) A4)
                    const float gd = dar * (A[0] + A[6]) + dai * (A[7] - A[1]) + dbr * (A[2] + A[4]) +
                                     dbi * (A[3] - A[5]);
                    atomicAdd(&cgrad[c][d], fc * gd + dfc * n[d] * gu);
                }
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
