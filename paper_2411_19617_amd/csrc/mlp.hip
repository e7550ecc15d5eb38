// Per-point feed-forward network (Sec. 2.4, Eq. ffnn) on MFMA, with the LDOS
// reductions of Sec. 2.3 / 3.4 fused into the output epilogue.
//
// A block of 8 waves takes NP = 16*NT grid points at a time from its fixed,
// contiguous range.  Layers are computed transposed, H_out^T = W H_in^T:
// output units are the MFMA M dimension, the points the N dimension (NT
// tiles of 16).  Wave w owns M-tiles w, w+8, ... for all NT point tiles, so
// every weight operand fetched from L2 feeds NT MFMAs; the tiles left over
// after the full rounds are split as (M-tile, point-tile) items so the waves
// stay balanced.  Weights stream through a small register ring (prefetch).
// Activations live in LDS as [point][unit] rows with a stride of 8 (mod 64)
// dwords: on gfx950 that makes the 128-bit B-operand reads (row = point,
// column = 4 units per lane group) and the result writes conflict-free,
// where a stride of 4, 12, 16 or 36 (mod 64) costs 4 extra cycles per read
// (measured with the SQ_LDS_BANK_CONFLICT counter).  Layer 2 is
// produced a chunk of M-tiles at a time and consumed by layer 3 at once.
//
// Epilogues:
//   LDOS       d = out_scale*y + out_shift stored as float32 [n][n_e]
//   DOS        d summed over points in FP64 into a per-block FP64 row
//              (fixed assignment: deterministic); optional row stride to run
//              on a strided subsample of the points
//   DOS_WINDOW DOS as above, plus per point the FP64 prefix sum of the fully
//              occupied part sum_{e<lo} tw_e d_e and the float32 LDOS values
//              of the energy window [lo, hi] around the estimated E_F
//   DENSITY    n(p) = sum_e w_e d_e(p) (FP64) with the solved Fermi weights;
//              runs only when the stored window did not cover E_F.
#include "mlp_core.h"

namespace mala {

// M-tiles a wave computes at once (each LDS activation operand then feeds MB
// MFMAs): BF16 reads four times more LDS bytes per MFMA flop than FP32 (a
// 16x16x32 operand is 16 B per lane against 4 B for 16x16x4 at twice the
// flops), so it takes two; FP32 stays at one, which measured faster there.
template <int PREC>
constexpr int mlp_mb() { return PREC == 1 ? 2 : 1; }
// M-tiles of layer 2 held in LDS at once: BF16 keeps the whole layer (half
// the bytes of FP32), so layer 3 runs once after it with no accumulators
// live during layer 2; FP32 produces it kWaves M-tiles at a time, each chunk
// consumed by layer 3 at once.
template <int PREC>
inline __host__ __device__ int mlp_h2_chunk(const MlpArgs& a) { return PREC == 1 ? a.h2_tiles : kWaves; }

template <int PREC, int MODE, int NT>
__global__ __launch_bounds__(kWaves * 64) void k_mlp(MlpArgs a, const float* __restrict__ B, int64_t n_pts,
                                                     int row_stride, MlpOut o) {
    using P = Prec<PREC>;
    using T = typename P::T;
    constexpr int NP = 16 * NT;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_dos[kMlpMaxOut];
    __shared__ double s_part[kWaves][NP];
    __shared__ double s_w[kMlpMaxOut];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    int lo = 0, W = 0;
    if constexpr (MODE == kModeDensity) {
        if (o.res->status != 0 || o.win->covered) return;      // nothing to recompute
    }
    if constexpr (MODE == kModeDosWindow) {
        lo = o.win->lo;
        W = o.win->valid ? o.win->hi - o.win->lo + 1 : 0;
    }
    constexpr int MB = mlp_mb<PREC>();
    const int CH = mlp_h2_chunk<PREC>(a);
    const int xs = P::stride(a.in_pad), hs = P::stride(a.h1_tiles * 16), cs = P::stride(16 * CH);
    T* H1 = reinterpret_cast<T*>(smem);
    T* X0 = H1 + NP * hs;          // layer-1 input, later layer 2 (or its chunk)
    T* H2 = X0;

    if constexpr (MODE == kModeDensity || MODE == kModeDosWindow) {
        // weights of the per-point energy sum: density -> Fermi weights w_e,
        // window prefix -> trapezoid weight de (de/2 at e = 0) below lo
        for (int e = threadIdx.x; e < kMlpMaxOut; e += blockDim.x) {
            double we = 0.0;
            if (MODE == kModeDensity) we = e < a.n_out ? o.fermi_w[e] : 0.0;
            else we = (e < lo) ? (e == 0 ? 0.5 * o.de : o.de) : 0.0;
            s_w[e] = we;
        }
    }
    if constexpr (MODE == kModeDos || MODE == kModeDosWindow)
        for (int e = threadIdx.x; e < kMlpMaxOut; e += blockDim.x) s_dos[e] = 0.0;
    __syncthreads();

    const int64_t n_it = (n_pts + NP - 1) / NP;
    const int nb = gridDim.x;
    const int64_t it_begin = n_it * blockIdx.x / nb, it_end = n_it * (blockIdx.x + 1) / nb;
    const int KS1 = a.in_pad / P::K, KS2 = a.h1_tiles * 16 / P::K, KS3 = a.h2_tiles * 16 / P::K;
    const int n_in = a.n_in;

    // DOS column sums: every lane keeps the FP64 sums of its 8 energies over
    // all of its points and iterations; the 16 point lanes are combined once
    // at the end (fixed order)
    double dacc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    // input staging: thread t owns column k_t of the [NP][in_pad] tile and
    // rows r_t, r_t + R, ... (R = blockDim / in_pad >= 4 rows per pass, as
    // in_pad <= 128). All of its loads are issued before any is used; a row
    // past the tile's last valid point re-reads that point (always in bounds)
    // and is stored as zero, and a pad column re-reads column n_in - 1.
    constexpr int SPT = NP / 4;
    const int R = (kWaves * 64) / a.in_pad;
    const int k_t = threadIdx.x % a.in_pad, r_t = threadIdx.x / a.in_pad;
    const bool col_in = k_t < n_in;
    const int k_c = col_in ? k_t : n_in - 1;
    const float mu_t = a.in_mean[k_c], rs_t = a.in_rstd[k_c];
    const int rsn = row_stride * n_in;                 // floats per tile row; NP * rsn * 4 < 2^31 (host check)

    for (int64_t it = it_begin; it < it_end; ++it) {
        const int64_t p0 = it * NP;
        const int rows = (int)((n_pts - p0) < NP ? (n_pts - p0) : NP);
        if (r_t < R) {
            // the empty asm makes the row index loop-variant, so the per-row
            // offsets are formed next to their loads and not held across the loop
            int row0 = r_t;
            asm volatile("" : "+v"(row0));
            const char* Bt = reinterpret_cast<const char*>(B + p0 * row_stride * n_in);
            float v[SPT];
#pragma unroll
            for (int q = 0; q < SPT; ++q) {
                const int row = min(row0 + q * R, rows - 1);
                v[q] = *reinterpret_cast<const float*>(Bt + (unsigned)((row * rsn + k_c) * 4));
            }
#pragma unroll
            for (int q = 0; q < SPT; ++q) {
                const int pj = row0 + q * R;
                if (pj < NP) X0[pj * xs + k_t] = P::cvt((col_in && pj < rows) ? (v[q] - mu_t) * rs_t : 0.f);
            }
        }
        __syncthreads();
        layer<PREC, NT, MB>(a.W1, a.b1, a.h1_tiles, 0, KS1, X0, xs, H1, hs, a.slope, wave, lane);
        __syncthreads();

        f4 acc3[2][NT];
        if constexpr (PREC == 1) {
            // the whole of layer 2, then layer 3 in one pass: each wave's two
            // output tiles share every LDS operand when both exist
            layer<PREC, NT, MB>(a.W2, a.b2, a.h2_tiles, 0, KS2, H1, hs, H2, cs, a.slope, wave, lane);
            __syncthreads();
            auto init3 = [&]() {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int ot = wave + kWaves * i;
                    const f4 b = ot < a.out_tiles ? bias4(a.b3, 16 * ot + 4 * g) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int n = 0; n < NT; ++n) acc3[i][n] = b;
                }
            };
            auto layer3 = [&](int ks0, int ksn) {
                const T* rows[NT];
#pragma unroll
                for (int n = 0; n < NT; ++n) rows[n] = H2 + (16 * n + j) * cs;
                bool both = false;
                if (wave + kWaves < a.out_tiles) {
                    const size_t bases[2] = {((size_t)wave * KS3 + ks0) * 64 + lane,
                                             ((size_t)(wave + kWaves) * KS3 + ks0) * 64 + lane};
                    kloop_mn<PREC, 2, NT>(a.W3, bases, ksn, rows, g, acc3);
                    both = true;
                }
                if (!both) {
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const int ot = wave + kWaves * i;
                        if (ot < a.out_tiles)
                            kloop<PREC, NT>(a.W3, ((size_t)ot * KS3 + ks0) * 64 + lane, ksn, rows, g, acc3[i]);
                    }
                }
            };
            init3();
            layer3(0, KS3);
            __syncthreads();
        } else {
            // layer 2 in chunks of CH M-tiles, each consumed by layer 3 at once
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int ot = wave + kWaves * i;
                const f4 b = ot < a.out_tiles ? bias4(a.b3, 16 * ot + 4 * g) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int n = 0; n < NT; ++n) acc3[i][n] = b;
            }
            for (int c0 = 0; c0 < a.h2_tiles; c0 += CH) {
                const int ct = (a.h2_tiles - c0) < CH ? (a.h2_tiles - c0) : CH;
                layer<PREC, NT, MB>(a.W2, a.b2, ct, c0, KS2, H1, hs, H2, cs, a.slope, wave, lane);
                __syncthreads();
                const int ks0 = c0 * 16 / P::K, ksn = ct * 16 / P::K;
                const T* rows[NT];
#pragma unroll
                for (int n = 0; n < NT; ++n) rows[n] = H2 + (16 * n + j) * cs;
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int ot = wave + kWaves * i;
                    if (ot < a.out_tiles) kloop<PREC, NT>(a.W3, ((size_t)ot * KS3 + ks0) * 64 + lane, ksn, rows, g, acc3[i]);
                }
                __syncthreads();
            }
        }

        // ---- epilogue
        double part[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) part[n] = 0.0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int ot = wave + kWaves * i;
            if (ot >= a.out_tiles) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = 16 * ot + 4 * g + r;
                const bool ev = e < a.n_out;
                // every mode forms the same float LDOS value d = s y + c (affine map
                // in FP64, rounded once), so that the stored LDOS, the DOS, the
                // window, its prefix and a recomputed density all use identical numbers
                // the scaler rows are zero-padded to kMlpMaxOut: loaded unconditionally,
                // so the sixteen loads of the epilogue issue together
                const float scf = a.out_scale[e], shf = a.out_shift[e];
                const double sc = ev ? (double)scf : 0.0, sh = ev ? (double)shf : 0.0;
                double dsum = 0.0;
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const int64_t p = p0 + 16 * n + j;
                    const bool pv = (16 * n + j) < rows;
                    float yv = acc3[i][n][r];
                    if (a.out_act) yv = leaky(yv, a.slope);
                    const float df = (float)(sc * (double)yv + sh);
                    if constexpr (MODE == kModeLdos) {
                        if (pv && ev) o.ldos[p * a.n_out + e] = df;
                    } else if constexpr (MODE == kModeDensity) {
                        if (ev) part[n] += s_w[e] * (double)df;
                    } else {
                        const double d = (pv && ev) ? (double)df : 0.0;
                        dsum += d;
                        if constexpr (MODE == kModeDosWindow) {
                            part[n] += s_w[e] * d;
                            if (pv && e >= lo && e < lo + W) o.window[p * W + (e - lo)] = df;
                        }
                    }
                }
                if constexpr (MODE == kModeDos || MODE == kModeDosWindow) dacc[i][r] += dsum;
            }
        }
        if constexpr (MODE == kModeDensity || MODE == kModeDosWindow) {
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                double v = part[n];
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                if (g == 0) s_part[wave][16 * n + j] = v;
            }
            __syncthreads();
            if (threadIdx.x < NP && (int)threadIdx.x < rows) {
                double v = 0.0;
                for (int w = 0; w < kWaves; ++w) v += s_part[w][threadIdx.x];
                const int64_t q = p0 + threadIdx.x;
                if constexpr (MODE == kModeDensity) o.density[q] = v;
                else o.prefix[q] = v;
            }
        }
        __syncthreads();
    }
    if constexpr (MODE == kModeDos || MODE == kModeDosWindow) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int ot = wave + kWaves * i;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = dacc[i][r];
                v += __shfl_xor(v, 1, 16);
                v += __shfl_xor(v, 2, 16);
                v += __shfl_xor(v, 4, 16);
                v += __shfl_xor(v, 8, 16);
                const int e = 16 * ot + 4 * g + r;
                if (j == 0 && ot < a.out_tiles && e < a.n_out) s_dos[e] = v;
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kMlpMaxOut; e += blockDim.x)
            o.partials[(size_t)blockIdx.x * kMlpMaxOut + e] = s_dos[e];
    }
}

template <int PREC, int NT>
static size_t lds_bytes(const MlpArgs& a) {
    using P = Prec<PREC>;
    const size_t el = PREC == 0 ? 4 : 2;
    const size_t x = (size_t)std::max(P::stride(a.in_pad), P::stride(16 * mlp_h2_chunk<PREC>(a)));
    return el * 16 * NT * ((size_t)P::stride(a.h1_tiles * 16) + x);
}

template <int PREC, int MODE, int NT>
static hipError_t launch_pmn(hipStream_t s, const MlpArgs& a, const float* B, int64_t n_pts, int row_stride,
                             int n_blocks, const MlpOut& o) {
    const size_t lds = lds_bytes<PREC, NT>(a);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp<PREC, MODE, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_mlp<PREC, MODE, NT>), dim3(n_blocks), dim3(kWaves * 64), lds, s, a, B, n_pts,
                       row_stride, o);
    return hipGetLastError();
}

// 64 points per block when the activations fit next to the epilogue's static
// LDS, else 32.
template <int PREC, int MODE>
static hipError_t launch_pm(hipStream_t s, const MlpArgs& a, const float* B, int64_t n_pts, int row_stride,
                            int n_blocks, const MlpOut& o) {
    if ((int64_t)row_stride * a.n_in * 4 * 64 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    if (lds_bytes<PREC, 4>(a) <= kMlpLdsBudget) return launch_pmn<PREC, MODE, 4>(s, a, B, n_pts, row_stride, n_blocks, o);
    return launch_pmn<PREC, MODE, 2>(s, a, B, n_pts, row_stride, n_blocks, o);
}

int mlp_blocks(int64_t n_pts) {
    const int64_t it = (n_pts + 63) / 64;
    return (int)(it < kMlpBlocks ? (it > 0 ? it : 1) : kMlpBlocks);
}

hipError_t launch_mlp(hipStream_t s, const MlpArgs& a, int mode, const float* B, int64_t n_pts, int row_stride,
                      int n_blocks, const MlpOut& o) {
    if (n_pts <= 0 || n_blocks <= 0) return hipSuccess;
#define MALA_MLP_CASE(P, M) return launch_pm<P, M>(s, a, B, n_pts, row_stride, n_blocks, o)
    if (a.precision == 0) {
        if (mode == kModeLdos) MALA_MLP_CASE(0, kModeLdos);
        if (mode == kModeDos) MALA_MLP_CASE(0, kModeDos);
        if (mode == kModeDosWindow) MALA_MLP_CASE(0, kModeDosWindow);
        if (mode == kModeDensity) MALA_MLP_CASE(0, kModeDensity);
    } else {
        if (mode == kModeLdos) MALA_MLP_CASE(1, kModeLdos);
        if (mode == kModeDos) MALA_MLP_CASE(1, kModeDos);
        if (mode == kModeDosWindow) MALA_MLP_CASE(1, kModeDosWindow);
        if (mode == kModeDensity) MALA_MLP_CASE(1, kModeDensity);
    }
#undef MALA_MLP_CASE
    return hipErrorInvalidValue;
}

}  // namespace mala
