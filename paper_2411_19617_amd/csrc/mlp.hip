// Per-point feed-forward network (Sec. 2.4, Eq. ffnn) on MFMA, with the LDOS
// reductions of Sec. 2.3 / 3.4 fused into the output epilogue.
//
// Each block of 8 waves takes 32 grid points at a time from its fixed,
// contiguous range.  Layers are computed transposed, H_out^T = W H_in^T:
// output units are the MFMA M dimension, the points the N dimension (two
// 16-point tiles).  Wave (mg, ng) of the 4 x 2 wave grid owns the M-tiles
// mg, mg+4, ... of every layer for point tile ng.  Activations live in LDS
// as [point][unit] rows padded to a stride of 4 (mod 64) dwords, so the B
// operand reads and the result writes are free of bank conflicts; weights
// are streamed from L2 in MFMA lane order (packed once at load time).
// Layer 2 is produced four M-tiles at a time and consumed by layer 3 at
// once, so only layer 1's activations stay resident.
//
// Epilogues (one per mode):
//   LDOS    -- d = out_scale * y + out_shift stored as float32 [n][n_e];
//   DOS     -- d summed over the 16 points of a tile in FP64 (lane shuffles)
//              into a per-block FP64 row in LDS; each block writes one partial
//              row for its fixed range, so the later fixed-order sum is
//              deterministic;
//   DENSITY -- n(p) = sum_e w_e d_e(p) in FP64 with the Fermi weights of the
//              solved E_F, reduced over lane groups and the four M-groups.
#include "mala_internal.h"

namespace mala {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

constexpr int kNP = 32;         // points per block iteration
constexpr int kWaves = 8;       // 4 M-groups x 2 point tiles
constexpr int kChunk = 4;       // layer-2 M-tiles per chunk (one per M-group)

__device__ __forceinline__ float leaky(float x, float s) { return x < 0.f ? s * x : x; }
__device__ __forceinline__ f4 act4(f4 v, float s) {
    return f4{leaky(v[0], s), leaky(v[1], s), leaky(v[2], s), leaky(v[3], s)};
}
__device__ __forceinline__ f4 bias4(const float* b, int off) {
    const float4 v = *reinterpret_cast<const float4*>(b + off);
    return f4{v.x, v.y, v.z, v.w};
}

// Precision traits: element type in LDS, K per MFMA, operand loads.
template <int PREC>
struct Prec;

template <>
struct Prec<0> {
    using T = float;
    static constexpr int K = 4;
    // row stride (elements) for a width w: >= w, and stride/dword = 4 mod 64
    __device__ static int stride(int w) { return ((w + 63) / 64) * 64 + 4; }
    __device__ static f4 mma(const void* A, size_t idx, const T* row, int k0, f4 c) {
        const float a = static_cast<const float*>(A)[idx];
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, row[k0], c, 0, 0, 0);
    }
    __device__ static void store4(T* dst, f4 v) { *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]); }
    __device__ static T cvt(float x) { return x; }
};

template <>
struct Prec<1> {
    using T = __bf16;
    static constexpr int K = 32;
    __device__ static int stride(int w) { return ((w + 127) / 128) * 128 + 8; }
    __device__ static f4 mma(const void* A, size_t idx, const T* row, int k0, f4 c) {
        const uint4 av = static_cast<const uint4*>(A)[idx];
        bf8 a, b;
        __builtin_memcpy(&a, &av, 16);
        const uint4 bv = *reinterpret_cast<const uint4*>(row + k0);
        __builtin_memcpy(&b, &bv, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static void store4(T* dst, f4 v) {
        bf4 h = {(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
        *reinterpret_cast<bf4*>(dst) = h;
    }
    __device__ static T cvt(float x) { return (__bf16)x; }
};

// k offset of lane group g inside K-step s: fp32 -> 4s + g, bf16 -> 32s + 8g
template <int PREC>
__device__ __forceinline__ int kofs(int s, int g) {
    return PREC == 0 ? 4 * s + g : 32 * s + 8 * g;
}

template <int PREC, int MODE>
__global__ __launch_bounds__(kWaves * 64) void k_mlp(MlpArgs a, const float* __restrict__ B, int64_t n_pts,
                                                     float* __restrict__ ldos, double* __restrict__ partials,
                                                     int n_blocks, const double* __restrict__ fermi_w,
                                                     double* __restrict__ density,
                                                     const ResultRec* __restrict__ res) {
    using P = Prec<PREC>;
    using T = typename P::T;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_dos[2][kMlpMaxOut];
    __shared__ double s_dens[4][kNP];
    __shared__ double s_ws[kMlpMaxOut];
    __shared__ double s_wc;

    if constexpr (MODE == kModeDensity) {
        if (res->status != 0) return;     // no Fermi level: density not written
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    const int mg = wave & 3, ng = wave >> 2;

    const int xs = P::stride(a.in_pad), hs = P::stride(a.h1_tiles * 16), cs = P::stride(kChunk * 16);
    T* X0 = reinterpret_cast<T*>(smem);
    T* H1 = X0 + kNP * xs;
    T* H2 = H1 + kNP * hs;

    if constexpr (MODE == kModeDensity) {
        for (int e = threadIdx.x; e < kMlpMaxOut; e += blockDim.x)
            s_ws[e] = e < a.n_out ? fermi_w[e] * (double)a.out_scale[e] : 0.0;
        if (threadIdx.x == 0) {
            double c = 0.0;
            for (int e = 0; e < a.n_out; ++e) c += fermi_w[e] * (double)a.out_shift[e];
            s_wc = c;
        }
    }
    if constexpr (MODE == kModeDos)
        for (int e = threadIdx.x; e < 2 * kMlpMaxOut; e += blockDim.x) (&s_dos[0][0])[e] = 0.0;
    __syncthreads();

    const int64_t n_it = (n_pts + kNP - 1) / kNP;
    const int64_t it_begin = n_it * blockIdx.x / n_blocks, it_end = n_it * (blockIdx.x + 1) / n_blocks;
    const int KS1 = a.in_pad / P::K, KS2 = a.h1_tiles * 16 / P::K, KS3 = a.h2_tiles * 16 / P::K;
    const int n_in = a.n_in;

    for (int64_t it = it_begin; it < it_end; ++it) {
        const int64_t p0 = it * kNP;
        const int rows = (int)((n_pts - p0) < kNP ? (n_pts - p0) : kNP);
        // ---- x0 = (B - mean)/std, zero padded, for the block's 32 points
        for (int e = threadIdx.x; e < kNP * a.in_pad; e += blockDim.x) {
            const int pj = e / a.in_pad, k = e - pj * a.in_pad;
            float v = 0.f;
            if (pj < rows && k < n_in) v = (B[(p0 + pj) * n_in + k] - a.in_mean[k]) * a.in_rstd[k];
            X0[pj * xs + k] = P::cvt(v);
        }
        __syncthreads();
        // ---- layer 1
        const T* xrow = X0 + (16 * ng + j) * xs;
        for (int mt = mg; mt < a.h1_tiles; mt += 4) {
            f4 acc = bias4(a.b1, 16 * mt + 4 * g);
            const size_t base = (size_t)mt * KS1 * 64 + lane;
#pragma unroll 4
            for (int s = 0; s < KS1; ++s) acc = P::mma(a.W1, base + (size_t)s * 64, xrow, kofs<PREC>(s, g), acc);
            P::store4(H1 + (16 * ng + j) * hs + 16 * mt + 4 * g, act4(acc, a.slope));
        }
        __syncthreads();
        // ---- layer 2 in chunks of 4 M-tiles, consumed by layer 3 at once
        f4 acc3[4];
        for (int i = 0; i < 4; ++i) {
            const int ot = mg + 4 * i;
            acc3[i] = ot < a.out_tiles ? bias4(a.b3, 16 * ot + 4 * g) : f4{0.f, 0.f, 0.f, 0.f};
        }
        const T* hrow = H1 + (16 * ng + j) * hs;
        const T* crow = H2 + (16 * ng + j) * cs;
        for (int c0 = 0; c0 < a.h2_tiles; c0 += kChunk) {
            const int mt = c0 + mg;
            if (mt < a.h2_tiles) {
                f4 acc = bias4(a.b2, 16 * mt + 4 * g);
                const size_t base = (size_t)mt * KS2 * 64 + lane;
#pragma unroll 4
                for (int s = 0; s < KS2; ++s) acc = P::mma(a.W2, base + (size_t)s * 64, hrow, kofs<PREC>(s, g), acc);
                P::store4(H2 + (16 * ng + j) * cs + 16 * mg + 4 * g, act4(acc, a.slope));
            } else {
                P::store4(H2 + (16 * ng + j) * cs + 16 * mg + 4 * g, f4{0.f, 0.f, 0.f, 0.f});
            }
            __syncthreads();
            const int ks0 = c0 * 16 / P::K, ksn = kChunk * 16 / P::K;
            for (int i = 0; i < 4; ++i) {
                const int ot = mg + 4 * i;
                if (ot >= a.out_tiles) break;
                const size_t base = ((size_t)ot * KS3 + ks0) * 64 + lane;
#pragma unroll
                for (int s = 0; s < ksn; ++s) {
                    if (ks0 + s < KS3) acc3[i] = P::mma(a.W3, base + (size_t)s * 64, crow, kofs<PREC>(s, g), acc3[i]);
                }
            }
            __syncthreads();
        }
        // ---- epilogue
        const int64_t p = p0 + 16 * ng + j;
        const bool pv = p < n_pts;
        double dens = 0.0;
        for (int i = 0; i < 4; ++i) {
            const int ot = mg + 4 * i;
            if (ot >= a.out_tiles) break;
            const f4 y = a.out_act ? act4(acc3[i], a.slope) : acc3[i];
            for (int r = 0; r < 4; ++r) {
                const int e = 16 * ot + 4 * g + r;
                const bool ev = e < a.n_out;
                if constexpr (MODE == kModeLdos) {
                    if (pv && ev) ldos[p * a.n_out + e] = a.out_scale[e] * y[r] + a.out_shift[e];
                } else if constexpr (MODE == kModeDos) {
                    double d = (pv && ev) ? (double)a.out_scale[e] * (double)y[r] + (double)a.out_shift[e] : 0.0;
                    d += __shfl_xor(d, 1, 16);
                    d += __shfl_xor(d, 2, 16);
                    d += __shfl_xor(d, 4, 16);
                    d += __shfl_xor(d, 8, 16);
                    if (j == 0 && ev) s_dos[ng][e] += d;
                } else {
                    if (ev) dens += s_ws[e] * (double)y[r];
                }
            }
        }
        if constexpr (MODE == kModeDensity) {
            dens += __shfl_xor(dens, 16, 64);
            dens += __shfl_xor(dens, 32, 64);
            if (g == 0) s_dens[mg][16 * ng + j] = dens;
            __syncthreads();
            if (threadIdx.x < kNP) {
                const int64_t q = p0 + threadIdx.x;
                if (q < n_pts)
                    density[q] = ((s_dens[0][threadIdx.x] + s_dens[1][threadIdx.x]) +
                                  (s_dens[2][threadIdx.x] + s_dens[3][threadIdx.x])) + s_wc;
            }
        }
        __syncthreads();
    }
    if constexpr (MODE == kModeDos) {
        for (int e = threadIdx.x; e < kMlpMaxOut; e += blockDim.x)
            partials[(size_t)blockIdx.x * kMlpMaxOut + e] = s_dos[0][e] + s_dos[1][e];
    }
}

template <int PREC>
static size_t lds_bytes(const MlpArgs& a) {
    const size_t el = PREC == 0 ? 4 : 2;
    auto stride = [&](int w) {
        return PREC == 0 ? (size_t)(((w + 63) / 64) * 64 + 4) : (size_t)(((w + 127) / 128) * 128 + 8);
    };
    return el * kNP * (stride(a.in_pad) + stride(a.h1_tiles * 16) + stride(kChunk * 16));
}

template <int PREC, int MODE>
static hipError_t launch_pm(hipStream_t s, const MlpArgs& a, const float* B, int64_t n_pts, float* ldos,
                            double* partials, int n_blocks, const double* fermi_w, double* density,
                            const ResultRec* res) {
    const size_t lds = lds_bytes<PREC>(a);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp<PREC, MODE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_mlp<PREC, MODE>), dim3(n_blocks), dim3(kWaves * 64), lds, s, a, B, n_pts, ldos,
                       partials, n_blocks, fermi_w, density, res);
    return hipGetLastError();
}

int mlp_blocks(int64_t n_pts) {
    const int64_t it = (n_pts + kNP - 1) / kNP;
    return (int)(it < kMlpBlocks ? (it > 0 ? it : 1) : kMlpBlocks);
}

hipError_t launch_mlp(hipStream_t s, const MlpArgs& a, int mode, const float* B, int64_t n_pts,
                      float* ldos_out, double* dos_partials, int n_blocks, const double* fermi_w,
                      double* density_out, const void* result) {
    if (n_pts <= 0 || n_blocks <= 0) return hipSuccess;
    const ResultRec* res = static_cast<const ResultRec*>(result);
#define MALA_MLP_CASE(P, M) \
    return launch_pm<P, M>(s, a, B, n_pts, ldos_out, dos_partials, n_blocks, fermi_w, density_out, res)
    if (a.precision == 0) {
        if (mode == kModeLdos) MALA_MLP_CASE(0, kModeLdos);
        if (mode == kModeDos) MALA_MLP_CASE(0, kModeDos);
        if (mode == kModeDensity) MALA_MLP_CASE(0, kModeDensity);
    } else {
        if (mode == kModeLdos) MALA_MLP_CASE(1, kModeLdos);
        if (mode == kModeDos) MALA_MLP_CASE(1, kModeDos);
        if (mode == kModeDensity) MALA_MLP_CASE(1, kModeDensity);
    }
#undef MALA_MLP_CASE
    return hipErrorInvalidValue;
}

}  // namespace mala
