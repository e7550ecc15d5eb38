// MFMA building blocks of the per-point network (Sec. 2.4, Eq. ffnn): the
// precision traits, the K-loop with its register prefetch ring and the dense
// layer over the waves of a block.  Shared by the forward kernel and its
// vector-Jacobian product.
#pragma once
#include "mala_internal.h"

namespace mala {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;

__device__ __forceinline__ float leaky(float x, float s) { return x < 0.f ? s * x : x; }
__device__ __forceinline__ f4 act4(f4 v, float s) {
    return f4{leaky(v[0], s), leaky(v[1], s), leaky(v[2], s), leaky(v[3], s)};
}
__device__ __forceinline__ f4 bias4(const float* b, int off) {
    const float4 v = *reinterpret_cast<const float4*>(b + off);
    return f4{v.x, v.y, v.z, v.w};
}

template <int PREC>
struct Prec;

// FP32: MFMA 16x16x4.  K-step s of lane group g uses unit
// 16*(s/4) + 4*g + s%4, so a batch of 4 K-steps reads 4 contiguous floats
// per lane (one ds_read_b128); the weights are packed in the same order.
template <>
struct Prec<0> {
    using T = float;
    static constexpr int K = 4;      // units per K-step
    static constexpr int PF = 4;     // K-steps per batch
    static constexpr int DA = 2;     // weight batches fetched ahead
    struct BatchA { float v[4]; };
    struct BatchB { float4 v; };
    __host__ __device__ static int stride(int w) { return ((w + 63) / 64) * 64 + 8; }
    __device__ static void loadA(BatchA& a, const void* A, size_t base, int q) {
        const float* p = static_cast<const float*>(A) + base + (size_t)q * PF * 64;
#pragma unroll
        for (int i = 0; i < 4; ++i) a.v[i] = p[i * 64];
    }
    __device__ static void loadB(BatchB& b, const T* row, int q, int g) {
        b.v = *reinterpret_cast<const float4*>(row + 16 * q + 4 * g);
    }
    template <int S>
    __device__ static f4 mma_step(const BatchA& a, const BatchB& b, f4 c) {
        const float bv = S == 0 ? b.v.x : S == 1 ? b.v.y : S == 2 ? b.v.z : b.v.w;
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[S], bv, c, 0, 0, 0);
    }
    __device__ static void store4(T* dst, f4 v) {
        *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
    }
    __device__ static T cvt(float x) { return x; }
};

// BF16: MFMA 16x16x32, K-step s of lane group g uses units 32 s + 8 g + 0..7.
// One K-step per batch (a 16x16x32 MFMA is short, so the weights are fetched
// five batches ahead instead of holding larger batches).
template <>
struct Prec<1> {
    using T = __bf16;
    static constexpr int K = 32;
    static constexpr int PF = 1;
    static constexpr int DA = 5;
    struct BatchA { uint4 v; };
    struct BatchB { uint4 v; };
    __host__ __device__ static int stride(int w) { return ((w + 127) / 128) * 128 + 16; }
    __device__ static void loadA(BatchA& a, const void* A, size_t base, int q) {
        a.v = static_cast<const uint4*>(A)[base + (size_t)q * 64];
    }
    __device__ static void loadB(BatchB& b, const T* row, int q, int g) {
        b.v = *reinterpret_cast<const uint4*>(row + 32 * q + 8 * g);
    }
    template <int S>
    __device__ static f4 mma_step(const BatchA& a, const BatchB& b, f4 c) {
        bf8 x, y;
        __builtin_memcpy(&x, &a.v, 16);
        __builtin_memcpy(&y, &b.v, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    }
    __device__ static void store4(T* dst, f4 v) {
        bf4 h = {(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
        *reinterpret_cast<bf4*>(dst) = h;
    }
    __device__ static T cvt(float x) { return (__bf16)x; }
};

// acc[m][n] += sum over K-steps s < KS of A_m(s) B_n(s), in batches of PF
// K-steps (KS is a multiple of PF): MB weight tiles (A_m at base[m]) against
// NA point tiles, so every weight operand feeds NA MFMAs and every LDS
// operand MB.  Weights (from L2) are fetched DA batches ahead into a ring of
// DA+1 register sets, LDS operands one batch ahead into a ring of two; the
// loop is unrolled by a multiple of both ring sizes so the sets rotate by
// name: no register copies and no wait on a load issued in the same batch.
// Within a batch the MFMAs go K-step by K-step over the MB x NA independent
// accumulators.  An MB-fold batch is MB times longer, so fewer batches ahead
// cover the same L2 latency.
template <int PREC, int MB, int NA>
__device__ __forceinline__ void kloop_mn(const void* A, const size_t (&base)[MB], int KS,
                                         const typename Prec<PREC>::T* const (&rows)[NA], int g,
                                         f4 (&acc)[MB][NA]) {
    using P = Prec<PREC>;
    using BA = typename P::BatchA;
    using BB = typename P::BatchB;
    constexpr int DA = (P::DA + MB - 1) / MB;
    constexpr int RA = DA + 1;
    constexpr int U = RA % 2 == 0 ? RA : 2 * RA;
    const int NQ = KS / P::PF;
    BA a[RA][MB];
    BB b[2][NA];
    auto fetchA = [&](int q, BA (&ad)[MB]) {
#pragma unroll
        for (int m = 0; m < MB; ++m) P::loadA(ad[m], A, base[m], q);
    };
    auto fetchB = [&](int q, BB (&bd)[NA]) {
#pragma unroll
        for (int n = 0; n < NA; ++n) P::loadB(bd[n], rows[n], q, g);
    };
    auto mma = [&](const BA (&as)[MB], const BB (&bs)[NA]) {
        static_for<0, P::PF>([&](auto sc) {
            constexpr int S = decltype(sc)::value;
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NA; ++n) acc[m][n] = P::template mma_step<S>(as[m], bs[n], acc[m][n]);
        });
    };
    // batch q + u (u < U) lives in a[u % RA] and b[u % 2].  Prefetches past
    // the last batch re-read the last batch (unused): every load is
    // unconditional, so the waits count exactly the loads still needed.
    auto step = [&](int q, auto uc) {
        constexpr int u = decltype(uc)::value;
        const int qa = q + u + DA < NQ ? q + u + DA : NQ - 1;
        const int qb = q + u + 1 < NQ ? q + u + 1 : NQ - 1;
        fetchA(qa, a[(u + DA) % RA]);
        fetchB(qb, b[(u + 1) % 2]);
        mma(a[u % RA], b[u % 2]);
    };
    if (NQ <= 0) return;
    static_for<0, DA>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        fetchA(i < NQ ? i : NQ - 1, a[i]);
    });
    fetchB(0, b[0]);
    int q = 0;
    for (; q + U <= NQ; q += U) static_for<0, U>([&](auto uc) { step(q, uc); });
    static_for<0, U>([&](auto uc) {
        if (q + decltype(uc)::value < NQ) step(q, uc);
    });
}

// One weight tile against NA point tiles.
template <int PREC, int NA>
__device__ __forceinline__ void kloop(const void* A, size_t base, int KS, const typename Prec<PREC>::T* const (&rows)[NA],
                                      int g, f4 (&acc)[NA]) {
    const size_t bases[1] = {base};
    f4 acc1[1][NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) acc1[0][n] = acc[n];
    kloop_mn<PREC, 1, NA>(A, bases, KS, rows, g, acc1);
#pragma unroll
    for (int n = 0; n < NA; ++n) acc[n] = acc1[0][n];
}

// One dense layer on the waves of the block: out[p][16 mt + u] = act(W x + b)
// for the M-tiles tile_base + mt, mt < tiles.  in: LDS rows (stride is), out:
// LDS rows (stride os), column 16 mt.  With MB > 1 the waves first take MB
// M-tiles each as long as every wave has a full set, then one each, then
// the (M-tile, point-tile) items left over, so the waves stay balanced.
template <int PREC, int NT, int MB = 1>
__device__ __forceinline__ void layer(const void* W, const float* bias, int tiles, int tile_base, int KS,
                                      const typename Prec<PREC>::T* in, int is, typename Prec<PREC>::T* out,
                                      int os, float slope, int wave, int lane) {
    using P = Prec<PREC>;
    using T = typename P::T;
    const int j = lane & 15, g = lane >> 4;
    int done = 0;
    if constexpr (MB > 1) {
        const int fullm = (tiles / (kWaves * MB)) * kWaves * MB;
        for (int r0 = 0; r0 < fullm; r0 += kWaves * MB) {
            f4 acc[MB][NT];
            size_t bases[MB];
            const T* rows[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) rows[n] = in + (16 * n + j) * is;
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int mt = r0 + MB * wave + m;
                const f4 b = bias4(bias, 16 * (tile_base + mt) + 4 * g);
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[m][n] = b;
                bases[m] = (size_t)(tile_base + mt) * KS * 64 + lane;
            }
            kloop_mn<PREC, MB, NT>(W, bases, KS, rows, g, acc);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int mt = r0 + MB * wave + m;
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    P::store4(out + (16 * n + j) * os + 16 * mt + 4 * g, act4(acc[m][n], slope));
            }
        }
        done = fullm;
    }
    const int full = done + ((tiles - done) / kWaves) * kWaves;
    for (int mt = done + wave; mt < full; mt += kWaves) {
        f4 acc[NT];
        const f4 b = bias4(bias, 16 * (tile_base + mt) + 4 * g);
        const T* rows[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            acc[n] = b;
            rows[n] = in + (16 * n + j) * is;
        }
        kloop<PREC, NT>(W, (size_t)(tile_base + mt) * KS * 64 + lane, KS, rows, g, acc);
#pragma unroll
        for (int n = 0; n < NT; ++n) P::store4(out + (16 * n + j) * os + 16 * mt + 4 * g, act4(acc[n], slope));
    }
    const int rem_items = (tiles - full) * NT;
    for (int it = wave; it < rem_items; it += kWaves) {
        const int mt = full + it / NT, n = it % NT;
        f4 acc[1] = {bias4(bias, 16 * (tile_base + mt) + 4 * g)};
        const T* rows[1] = {in + (16 * n + j) * is};
        kloop<PREC, 1>(W, (size_t)(tile_base + mt) * KS * 64 + lane, KS, rows, g, acc);
        P::store4(out + (16 * n + j) * os + 16 * mt + 4 * g, act4(acc[0], slope));
    }
}


// Dense layer with a caller-supplied epilogue: acc = W x (+ bias when given)
// for every (point tile n, M-tile mt) the wave owns; ep(n, mt, acc) writes it.
template <int PREC, int NT, typename Ep>
__device__ __forceinline__ void layer_ep(const void* W, const float* bias, int tiles, int KS,
                                         const typename Prec<PREC>::T* in, int is, int wave, int lane, Ep&& ep) {
    using T = typename Prec<PREC>::T;
    const int j = lane & 15, g = lane >> 4;
    const int full = (tiles / kWaves) * kWaves;
    for (int mt = wave; mt < full; mt += kWaves) {
        f4 acc[NT];
        const f4 b = bias ? bias4(bias, 16 * mt + 4 * g) : f4{0.f, 0.f, 0.f, 0.f};
        const T* rows[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            acc[n] = b;
            rows[n] = in + (16 * n + j) * is;
        }
        kloop<PREC, NT>(W, (size_t)mt * KS * 64 + lane, KS, rows, g, acc);
#pragma unroll
        for (int n = 0; n < NT; ++n) ep(n, mt, acc[n]);
    }
    const int rem_items = (tiles - full) * NT;
    for (int it = wave; it < rem_items; it += kWaves) {
        const int mt = full + it / NT, n = it % NT;
        f4 acc[1] = {bias ? bias4(bias, 16 * mt + 4 * g) : f4{0.f, 0.f, 0.f, 0.f}};
        const T* rows[1] = {in + (16 * n + j) * is};
        kloop<PREC, 1>(W, (size_t)mt * KS * 64 + lane, KS, rows, g, acc);
        ep(n, mt, acc[0]);
    }
}

}  // namespace mala
