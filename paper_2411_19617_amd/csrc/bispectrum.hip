// Grid bispectrum descriptors on gfx950 (Sec. 3.2.2: Eqs. ionicdensity,
// SNAPExpansion and the triple products that give B(r, j), Eq. snap_dim).
//
// Two kernels per tile of 64 consecutive grid points (one point per lane):
//
//  k_ui  -- neighbour gather and the expansion coefficients
//           u^J = I + sum_k f_c(r_k) U^J(g_k).  U^J is the spin-J/2 irrep of
//           g written as a polynomial action on (xi, eta); its unnormalised
//           coefficients are products of powers of a, b and their conjugates.
//           The rows that share J-ma form independent chains: the first row
//           of a chain comes from powers of b and f_c conj(a), each later row
//           from the previous one (one more factor), and everything is
//           normalised once after the neighbour sum.  The chains are split
//           over the waves of the block so that each wave keeps its share of
//           u in registers over the whole neighbour loop.  Only rows
//           ma <= J/2 are formed; the rest follow from
//           u_{J-ma,J-mb} = (-1)^(ma-mb) conj(u_{ma,mb}).
//
//  k_zb  -- the tile's half-u (271 complex per point at twojmax 10, 139 KB
//           for 64 points) is staged in LDS; every wave of the block owns a
//           balanced subset of the (j1,j2,j) triples and contracts
//           Z^j_{m m'} = sum C C u^{j1} u^{j2} one output column m' at a time
//           (columns of u^{j1} and u^{j2} in registers, the row CG factor
//           applied after the m1' sum), then B = sum Re(conj(u^j) Z) over the
//           half rows.
//           Each triple is contracted in whichever of its three
//           orientations (which level is the conjugated output) costs
//           least, and when its two coupled levels are equal only one of
//           each exchanged pair of rows is formed.  Clebsch-Gordan values of
//           the coupling come from a per-triple table in global memory read
//           with wave-uniform (scalar) loads.
#include <mutex>

#include "snap_core.h"
#include "tile_gather.h"

namespace mala {

// Accumulate f_c * c(g) of one neighbour into the group's registers, where
// c^J[ma][mb] is the coefficient of xi^mb eta^(J-mb) in
// (a xi - conj(b) eta)^ma (b xi + conj(a) eta)^(J-ma); U^J = N c^J with
// N = sqrt(mb! (J-mb)! / (ma! (J-ma)!)) applied once at write-out.
// Row 0 of level q is binom(q, mb) b^mb conj(a)^(q-mb) (from powers of b
// and f_c conj(a) shared by the group's chains); the later rows of a chain
// follow from multiplying by one more factor:
//   row k:   c^J[k][mb]  = a c^{J-1}[k-1][mb-1] - conj(b) c^{J-1}[k-1][mb]
// and the chain's last row is summed into the accumulators directly.
template <int TJ, int G, int NACC>
__device__ __forceinline__ void ui_neighbour(float ar, float ai, float br, float bi, float fc,
                                             float (&accr)[NACC], float (&acci)[NACC]) {
    constexpr int QMAX = group_qmax(TJ, G);
    float pbr[QMAX + 1], pbi[QMAX + 1], par[QMAX + 1], pai[QMAX + 1];   // b^k, fc conj(a)^k
    par[0] = fc;
    pai[0] = 0.f;
    static_for<1, QMAX + 1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if constexpr (k == 1) {
            pbr[1] = br;
            pbi[1] = bi;
            par[1] = fc * ar;
            pai[1] = -fc * ai;
        } else {
            pbr[k] = fmaf(pbr[k - 1], br, -pbi[k - 1] * bi);
            pbi[k] = fmaf(pbr[k - 1], bi, pbi[k - 1] * br);
            par[k] = fmaf(par[k - 1], ar, pai[k - 1] * ai);
            pai[k] = fmaf(pai[k - 1], ar, -par[k - 1] * ai);
        }
    });
    static_for<0, TJ + 1>([&](auto qc) {
        constexpr int Q = decltype(qc)::value;
        if constexpr (in_group(TJ, G, Q)) {
            constexpr int base = chain_slot(TJ, G, Q);
            constexpr int NR = chain_rows(TJ, Q);
            float cr[TJ + 1], ci[TJ + 1];
            static_for<0, Q + 1>([&](auto mc) {
                constexpr int mb = decltype(mc)::value;
                constexpr float bin = (float)ce_binom(Q, mb);
                float xr, xi;
                if constexpr (mb == 0) {
                    xr = par[Q];
                    xi = pai[Q];
                } else if constexpr (mb == Q) {
                    xr = fc * pbr[Q];
                    xi = fc * pbi[Q];
                } else {
                    xr = fmaf(pbr[mb], par[Q - mb], -pbi[mb] * pai[Q - mb]);
                    xi = fmaf(pbr[mb], pai[Q - mb], pbi[mb] * par[Q - mb]);
                }
                if constexpr (bin != 1.f) {
                    xr *= bin;
                    xi *= bin;
                }
                cr[mb] = xr;
                ci[mb] = xi;
                accr[base + mb] += xr;
                if constexpr (Q > 0) acci[base + mb] += xi;     // level 0 is the real f_c
            });
            static_for<1, NR>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                constexpr int Jp = Q + k;
                constexpr int rb = base + row_slot(Q, k);
                if constexpr (k == NR - 1) {
                    static_for<0, Jp + 1>([&](auto mc) {
                        constexpr int mb = decltype(mc)::value;
                        float sr = accr[rb + mb], si = acci[rb + mb];
                        if constexpr (mb >= 1) {                // a * old[mb-1]
                            sr = fmaf(ar, cr[mb - 1], sr);
                            sr = fmaf(-ai, ci[mb - 1], sr);
                            si = fmaf(ar, ci[mb - 1], si);
                            si = fmaf(ai, cr[mb - 1], si);
                        }
                        if constexpr (mb <= Jp - 1) {           // - conj(b) * old[mb]
                            sr = fmaf(-br, cr[mb], sr);
                            sr = fmaf(-bi, ci[mb], sr);
                            si = fmaf(-br, ci[mb], si);
                            si = fmaf(bi, cr[mb], si);
                        }
                        accr[rb + mb] = sr;
                        acci[rb + mb] = si;
                    });
                } else {
                    static_for<0, Jp + 1>([&](auto ic) {
                        constexpr int mb = Jp - decltype(ic)::value;   // in place, high mb first
                        float nr = 0.f, ni = 0.f;
                        if constexpr (mb >= 1) {                // a * old[mb-1]
                            const float orr = cr[mb - 1], oi = ci[mb - 1];
                            nr = fmaf(ar, orr, -ai * oi);
                            ni = fmaf(ar, oi, ai * orr);
                        }
                        if constexpr (mb <= Jp - 1) {           // - conj(b) * old[mb]
                            const float orr = cr[mb], oi = ci[mb];
                            nr = fmaf(-br, orr, fmaf(-bi, oi, nr));
                            ni = fmaf(-br, oi, fmaf(bi, orr, ni));
                        }
                        cr[mb] = nr;
                        ci[mb] = ni;
                    });
                    static_for<0, Jp + 1>([&](auto mc) {
                        constexpr int mb = decltype(mc)::value;
                        accr[rb + mb] += cr[mb];
                        acci[rb + mb] += ci[mb];
                    });
                }
            });
        }
    });
}

template <int TJ>
__global__ __launch_bounds__(64 * n_groups(TJ), 2) void k_ui(BinState bins, int Nx, int Ny, int Nz,
                                                          double rcut, int64_t pt_begin, int64_t n_pts,
                                                          float2* __restrict__ u_out,
                                                          int* __restrict__ err) {
    constexpr int NG = n_groups(TJ);
    constexpr int NH = n_half(TJ);
    __shared__ float4 cand[kMaxCand];
    __shared__ unsigned short nbr[kMaxNbr][kTile];
    __shared__ int nnbr[kTile];
    __shared__ int scan_tmp[16];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t idx = tile * kTile + lane;
    const bool valid = idx < n_pts;
    const int64_t p = pt_begin + (valid ? idx : tile * kTile);
    const int64_t pk = p % Nz, pj = (p / Nz) % Ny, pi = p / ((int64_t)Ny * Nz);
    const double rx = (double)pi * bins.L[0] / Nx, ry = (double)pj * bins.L[1] / Ny,
                 rz = (double)pk * bins.L[2] / Nz;
    const int64_t p0 = pt_begin + tile * kTile;
    // bounding boxes of the tile's points
    const TileBoxes boxes = tile_boxes(p, p0, Ny, Nz, rx, ry, rz);

    // ---- candidate atom images within rcut of the boxes, in a fixed order
    int n0;
    const int base = gather_candidates(bins, boxes, rcut, cand, kMaxCand, scan_tmp, &n0);
    if (base > kMaxCand && threadIdx.x == 0) atomicOr(err, kErrCand);
    const int ncand = base < kMaxCand ? base : kMaxCand;
    __syncthreads();

    // ---- per-point neighbour lists (wave 0), in candidate order
    const PointFrame frame = point_frame(boxes, n0, rx, ry, rz);
    const float rcf = (float)rcut;
    if (wave == 0) build_neighbour_lists(cand, ncand, frame, rcf, valid, lane, nbr, nnbr, err);
    __syncthreads();

    // ---- expansion coefficients, this wave's chain group
    static_for<0, NG>([&](auto gc) {
        constexpr int G = decltype(gc)::value;
        if (wave != G) return;
        constexpr int NACC = group_size(TJ, G);
        float accr[NACC], acci[NACC];
        static_for<0, NACC>([&](auto ec) {
            accr[decltype(ec)::value] = 0.f;
            acci[decltype(ec)::value] = 0.f;
        });
        const int my_n = nnbr[lane];
        const int n_iter = wave_max_int(my_n);
        const float kpi = 3.14159265358979f;
        // angle and cutoff phase per unit distance, formed once: a quotient
        // per neighbour is a full-precision division (a dozen instructions)
        const float kth = kRfac0 * kpi / rcf, kcut = kpi / rcf;
        for (int s = 0; s < n_iter; ++s) {
            float ar = 1.f, ai = 0.f, br = 0.f, bi = 0.f, fc = 0.f;
            if (s < my_n) {
                const int c = nbr[s][lane];
                const float4 q = cand[c];
                const float3 o = frame.at(c);
                const float dx = q.x - o.x, dy = q.y - o.y, dz = q.z - o.z;
                const float r2 = dx * dx + dy * dy + dz * dz;
                // 1/r and r from one hardware reciprocal square root (about
                // 1 ulp; an atom on the point gives r = 0)
                const float inv = r2 > kMinR2 ? __builtin_amdgcn_rsqf(r2) : 0.f;
                const float r = r2 * inv;
                float sn, cs;
                sincosf(kth * r, &sn, &cs);
                ar = cs;
                ai = -dz * inv * sn;
                br = -dy * inv * sn;
                bi = -dx * inv * sn;
                fc = 0.5f * (cosf(kcut * r) + 1.f);
            }
            ui_neighbour<TJ, G, NACC>(ar, ai, br, bi, fc, accr, acci);
        }
        // normalisation, self term (identity on the diagonal, N = 1 there), write-out
        static_for<0, TJ + 1>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (in_group(TJ, G, q)) {
                static_for<0, chain_rows(TJ, q)>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    constexpr int J = q + k;
                    constexpr int rb = chain_slot(TJ, G, q) + row_slot(q, k);
                    static_for<0, J + 1>([&](auto mc) {
                        constexpr int mb = decltype(mc)::value;
                        constexpr float nrm =
                            (float)ce_sqrt(ce_fact(mb) * ce_fact(J - mb) / (ce_fact(k) * ce_fact(J - k)));
                        constexpr int e = half_off(J) + k * (J + 1) + mb;
                        const float re = nrm * accr[rb + mb] + (mb == k ? 1.f : 0.f);
                        u_out[(tile * NH + e) * kTile + lane] = make_float2(re, nrm * acci[rb + mb]);
                    });
                });
            }
        });
    });
}

// ------------------------------------------------------------------ Z / B
// B(j1,j2,j) of the lane's point.  For each output column mb:
//   T[ma][ma1] = sum_mb1 C(mb1,mb) u1[ma1][mb1] u2[ma-ma1+D][mb-mb1+D]
// (the CG factor scales the column of whichever level has fewer rows to
// scale, zb_scale2, and is shared by every row ma), then
//   Z[ma][mb] = sum_ma1 C(ma1,ma) T[ma][ma1],  B += w Re(conj(u[ma][mb]) Z[ma][mb]).
// Z has the symmetry of u, so rows ma < J/2 count twice (w = 2); the middle
// row of an even J is its own mirror image with columns mb and J-mb paired,
// so it is formed for mb <= J/2 only (w = 2, 1 at mb = J/2): its pairs come
// last in each column body behind one wave-uniform branch.  For J1 == J2
// only the pairs of zb_pair_ok are formed; the others equal their exchanged
// partner (zb_pair_doubled).
// A row past J/2 of a level is (-1)^(row - column) times the conjugate of
// the stored row J - row at column J - column.  The level offsets in the u
// tile are kept opaque in scalar registers, so that every column costs one
// address add per level side and all row offsets fit the LDS instruction's
// immediate field.
template <int J1, int J2, int J>
__device__ __forceinline__ float zb_triple(const float2* __restrict__ su, int lane,
                                           const float* __restrict__ cg) {
    constexpr int D = (J1 + J2 - J) / 2;   // ma2 = ma - ma1 + D
    constexpr int HR = J / 2;              // half rows 0..HR
    constexpr bool MID = (J % 2 == 0);     // row HR is the middle row
    constexpr int HN = MID ? HR - 1 : HR;  // last row formed for every column
    constexpr int W = J + 1;               // cg row stride: cg[ma1*W + ma]
    constexpr int NP = zb_pairs(J1, J2, J);
    constexpr bool S2 = zb_scale2(J1, J2, J);
    int off1 = half_off(J1) * kTile, off2 = half_off(J2) * kTile, off3 = half_off(J) * kTile;
    asm volatile("" : "+s"(off1), "+s"(off2), "+s"(off3));
    const float2* l1 = su + lane + off1;
    const float2* l2 = su + lane + off2;
    const float2* l3 = su + lane + off3;
    float bsum = 0.f;
#pragma clang loop unroll(disable)
    for (int mb = 0; mb <= J; ++mb) {
        float tr[NP], ti[NP];
        const bool mid_on = mb <= HR;      // wave-uniform
        auto pair_fma = [&](auto mac, auto ma1c, float wr, float wi, const float (&u2r)[J2 + 1],
                            const float (&u2i)[J2 + 1], auto first) {
            constexpr int ma = decltype(mac)::value, ma1 = decltype(ma1c)::value;
            constexpr int ma2 = ma - ma1 + D;
            constexpr int k = zb_pair_index(J1, J2, J, ma, ma1);
            if constexpr (decltype(first)::value) {
                tr[k] = fmaf(-wi, u2i[ma2], wr * u2r[ma2]);
                ti[k] = fmaf(wi, u2r[ma2], wr * u2i[ma2]);
            } else {
                tr[k] = fmaf(wr, u2r[ma2], tr[k]);
                tr[k] = fmaf(-wi, u2i[ma2], tr[k]);
                ti[k] = fmaf(wr, u2i[ma2], ti[k]);
                ti[k] = fmaf(wi, u2r[ma2], ti[k]);
            }
        };
        // one m1' column: the first one initialises T, the others accumulate
        auto column = [&](int mb1, auto first) {
            const int mb2 = mb + D - mb1;
            const float c2 = cg[mb1 * W + mb];
            // scalar factors of the mirrored rows: (-1)^column, times c2 on the scaled side
            const float f1 = flip_odd(S2 ? 1.f : c2, mb1);
            const float f2 = flip_odd(S2 ? c2 : 1.f, mb2);
            const float2* s1 = l1 + mb1 * kTile;             // stored rows of u^J1, column mb1
            const float2* m1 = l1 + (J1 - mb1) * kTile;      // their mirror column
            const float2* s2 = l2 + mb2 * kTile;
            const float2* m2 = l2 + (J2 - mb2) * kTile;
            float u2r[J2 + 1], u2i[J2 + 1];
            static_for<0, J2 + 1>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                if constexpr (zb_row2_used(J1, J2, J, r)) {
                    if constexpr (2 * r <= J2) {
                        const float2 v = s2[r * (J2 + 1) * kTile];
                        u2r[r] = S2 ? c2 * v.x : v.x;
                        u2i[r] = S2 ? c2 * v.y : v.y;
                    } else {
                        const float2 v = m2[(J2 - r) * (J2 + 1) * kTile];
                        const float f = (r & 1) ? -f2 : f2;
                        u2r[r] = f * v.x;
                        u2i[r] = -f * v.y;
                    }
                }
            });
            float wrs[J1 + 1], wis[J1 + 1];
            static_for<0, J1 + 1>([&](auto r1c) {
                constexpr int ma1 = decltype(r1c)::value;
                if constexpr (zb_row1_used(J1, J2, J, ma1)) {
                    if constexpr (2 * ma1 <= J1) {
                        const float2 v = s1[ma1 * (J1 + 1) * kTile];
                        wrs[ma1] = S2 ? v.x : c2 * v.x;
                        wis[ma1] = S2 ? v.y : c2 * v.y;
                    } else {
                        const float2 v = m1[(J1 - ma1) * (J1 + 1) * kTile];
                        const float f = (ma1 & 1) ? -f1 : f1;
                        wrs[ma1] = f * v.x;
                        wis[ma1] = -f * v.y;
                    }
                    static_for<0, HN + 1>([&](auto mc) {
                        if constexpr (zb_pair_ok(J1, J2, J, decltype(mc)::value, ma1))
                            pair_fma(mc, r1c, wrs[ma1], wis[ma1], u2r, u2i, first);
                    });
                }
            });
            if constexpr (MID) {
                if (mid_on) {
                    static_for<0, J1 + 1>([&](auto r1c) {
                        constexpr int ma1 = decltype(r1c)::value;
                        if constexpr (zb_pair_ok(J1, J2, J, HR, ma1))
                            pair_fma(std::integral_constant<int, HR>{}, r1c, wrs[ma1], wis[ma1], u2r, u2i, first);
                    });
                }
            }
        };
        const int lo = max(0, mb + D - J2), hi = min(J1, mb + D);   // never empty
        column(lo, std::true_type{});
        // runtime loops stay rolled: unrolling them spills (the whole triple
        // list is inlined into one kernel) and doubles the code size
#pragma clang loop unroll(disable)
        for (int mb1 = lo + 1; mb1 <= hi; ++mb1) column(mb1, std::false_type{});
        const float2* s3 = l3 + mb * kTile;
        static_for<0, HR + 1>([&](auto mc) {
            constexpr int ma = decltype(mc)::value;
            constexpr bool MIDROW = MID && ma == HR;
            if (MIDROW && !mid_on) return;
            float zr = 0.f, zi = 0.f, zr2 = 0.f, zi2 = 0.f;
            static_for<0, J1 + 1>([&](auto r1c) {
                constexpr int ma1 = decltype(r1c)::value;
                if constexpr (zb_pair_ok(J1, J2, J, ma, ma1)) {
                    constexpr int k = zb_pair_index(J1, J2, J, ma, ma1);
                    const float c1 = cg[ma1 * W + ma];
                    if constexpr (zb_pair_doubled(J1, J2, J, ma, ma1)) {
                        zr2 = fmaf(c1, tr[k], zr2);
                        zi2 = fmaf(c1, ti[k], zi2);
                    } else {
                        zr = fmaf(c1, tr[k], zr);
                        zi = fmaf(c1, ti[k], zi);
                    }
                }
            });
            if constexpr (J1 == J2) {
                zr = fmaf(2.f, zr2, zr);
                zi = fmaf(2.f, zi2, zi);
            }
            const float w = MIDROW ? (mb < HR ? 2.f : 1.f) : 2.f;
            const float2 uj = s3[ma * (J + 1) * kTile];
            bsum += w * (uj.x * zr + uj.y * zi);
        });
    }
    return bsum;
}

template <int TJ, int T>
__device__ __forceinline__ float zb_dispatch(int t, const float2* __restrict__ su, int lane,
                                             const float* __restrict__ cg_table,
                                             const int* __restrict__ cg_off) {
    if constexpr (T < n_triples(TJ)) {
        if (t == T) {
            constexpr Triple tr = triple_of(TJ, T);
            constexpr ZbPerm p = zb_perm(TJ, T);
            constexpr float scale = (float)(tr.j + 1) / (float)(p.c + 1);
            const float v = zb_triple<p.a, p.b, p.c>(su, lane, cg_table + cg_off[T]);
            if constexpr (p.c == tr.j) return v;
            else return scale * v;
        }
        return zb_dispatch<TJ, T + 1>(t, su, lane, cg_table, cg_off);
    } else {
        return 0.f;
    }
}

template <int TJ>
__global__ __launch_bounds__(768) void k_zb(const float2* __restrict__ u, int64_t n_pts,
                                             float* __restrict__ B, const float* __restrict__ cg_table,
                                             const int* __restrict__ cg_off,
                                             const int* __restrict__ wave_triples, int stride) {
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
    const int* list = wave_triples + wave * stride;
    const int cnt = __builtin_amdgcn_readfirstlane(list[0]);
    for (int i = 0; i < cnt; ++i) {
        const int t = __builtin_amdgcn_readfirstlane(list[1 + i]);
        const float b = zb_dispatch<TJ, 0>(t, su, lane, cg_table, cg_off);
        if (valid) B[idx * NB + t] = b;
    }
}

template <int TJ>
static hipError_t ui_tj(hipStream_t s, const BinState& bins, const int N[3], double rcut, int64_t pt_begin,
                        int64_t n_pts, float2* u_scratch, int* err_flag) {
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ui<TJ>, dim3((unsigned)n_tiles), dim3(64 * n_groups(TJ)), 0, s, bins, N[0], N[1],
                       N[2], rcut, pt_begin, n_pts, u_scratch, err_flag);
    return hipGetLastError();
}

template <int TJ>
static hipError_t zb_tj(hipStream_t s, int64_t n_pts, const float2* u_scratch, float* B_out,
                        const float* cg_table, const int* cg_offsets, const int* wave_triples, int zb_waves) {
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    if (n_tiles == 0) return hipSuccess;
    const size_t lds = sizeof(float2) * n_half(TJ) * kTile;
    // once per process for this instantiation, whichever thread launches first
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(attr_once, [&] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zb<TJ>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    if (attr_err != hipSuccess) return attr_err;
    hipLaunchKernelGGL(k_zb<TJ>, dim3((unsigned)n_tiles), dim3(64 * zb_waves), lds, s, u_scratch, n_pts, B_out,
                       cg_table, cg_offsets, wave_triples, kMaxZbStride);
    return hipGetLastError();
}

hipError_t launch_ui(hipStream_t s, int twojmax, const BinState& bins, const int N[3], double rcut,
                     int64_t pt_begin, int64_t n_pts, float2* u_scratch, int* err_flag) {
    switch (twojmax) {
    case 2: return ui_tj<2>(s, bins, N, rcut, pt_begin, n_pts, u_scratch, err_flag);
    case 4: return ui_tj<4>(s, bins, N, rcut, pt_begin, n_pts, u_scratch, err_flag);
    case 6: return ui_tj<6>(s, bins, N, rcut, pt_begin, n_pts, u_scratch, err_flag);
    case 8: return ui_tj<8>(s, bins, N, rcut, pt_begin, n_pts, u_scratch, err_flag);
    case 10: return ui_tj<10>(s, bins, N, rcut, pt_begin, n_pts, u_scratch, err_flag);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zb(hipStream_t s, int twojmax, int64_t n_pts, const float2* u_scratch, float* B_out,
                     const float* cg_table, const int* cg_offsets, const int* wave_triples, int zb_waves) {
    switch (twojmax) {
    case 2: return zb_tj<2>(s, n_pts, u_scratch, B_out, cg_table, cg_offsets, wave_triples, zb_waves);
    case 4: return zb_tj<4>(s, n_pts, u_scratch, B_out, cg_table, cg_offsets, wave_triples, zb_waves);
    case 6: return zb_tj<6>(s, n_pts, u_scratch, B_out, cg_table, cg_offsets, wave_triples, zb_waves);
    case 8: return zb_tj<8>(s, n_pts, u_scratch, B_out, cg_table, cg_offsets, wave_triples, zb_waves);
    case 10: return zb_tj<10>(s, n_pts, u_scratch, B_out, cg_table, cg_offsets, wave_triples, zb_waves);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mala
