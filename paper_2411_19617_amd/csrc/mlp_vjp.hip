// Vector-Jacobian product of the per-point network: the network factor of
// the force expression (Eq. forcesmala).  For every grid point p and a given
// vector v(p) over the energies, g(p) = (dd(p)/dB(p))^T v(p), where
// d = s .* sigma(W3 sigma(W2 sigma(W1 x + b1) + b2) + b3) + c and
// x = (B - mean) / std (sigma on the output layer only with output
// activation).  Backpropagation, with sigma'(z) = 1 for z > 0 and slope
// otherwise:
//   delta3 = s .* v .* sigma'(z3),  delta2 = (W3^T delta3) .* sigma'(z2),
//   delta1 = (W2^T delta2) .* sigma'(z1),  g = (W1^T delta1) ./ std.
//
// A block of 8 waves takes 32 points at a time.  The forward pass is the
// same MFMA layer as the network kernel, with both hidden activations kept
// in LDS: sigma'(z) is read from the sign of the stored activation (z > 0
// exactly when sigma(z) > 0), so no pre-activations are stored.  The three
// backward layers are MFMA layers over the transposed weights (packed like
// the forward ones): delta3 overwrites the input tile, delta2 the layer-2
// activations and delta1 the layer-1 activations, each in place by the lane
// that reads the activation it replaces.  FP32 only.
#include "mlp_core.h"

namespace mala {

template <int NT>
__global__ __launch_bounds__(kWaves * 64) void k_mlp_vjp(MlpArgs a, const float* __restrict__ B,
                                                         const float* __restrict__ v, int64_t n_pts,
                                                         float* __restrict__ g_out) {
    using P = Prec<0>;
    constexpr int NP = 16 * NT;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    const int hs = P::stride(a.h1_tiles * 16), h2s = P::stride(a.h2_tiles * 16);
    const int xs = P::stride(a.in_pad > a.out_tiles * 16 ? a.in_pad : a.out_tiles * 16);
    float* H1 = reinterpret_cast<float*>(smem);
    float* H2 = H1 + NP * hs;
    float* X = H2 + NP * h2s;           // input tile, then delta3
    const int n_in = a.n_in, n_out = a.n_out;
    const float slope = a.slope;
    const int KS1 = a.in_pad / P::K, KS2 = a.h1_tiles * 16 / P::K, KS3 = a.h2_tiles * 16 / P::K;
    const int KB3 = a.out_tiles * 16 / P::K, KB2 = a.h2_tiles * 16 / P::K, KB1 = a.h1_tiles * 16 / P::K;
    const int in_tiles = a.in_pad / 16;

    const int64_t n_it = (n_pts + NP - 1) / NP;
    const int nb = gridDim.x;
    const int64_t it_begin = n_it * blockIdx.x / nb, it_end = n_it * (blockIdx.x + 1) / nb;
    auto mask4 = [&](const float* h) {       // sigma'(z) from the sign of sigma(z)
        return f4{h[0] > 0.f ? 1.f : slope, h[1] > 0.f ? 1.f : slope, h[2] > 0.f ? 1.f : slope,
                  h[3] > 0.f ? 1.f : slope};
    };

    for (int64_t it = it_begin; it < it_end; ++it) {
        const int64_t p0 = it * NP;
        const int rows = (int)((n_pts - p0) < NP ? (n_pts - p0) : NP);
        for (int e = threadIdx.x; e < NP * a.in_pad; e += blockDim.x) {
            const int pj = e / a.in_pad, k = e - pj * a.in_pad;
            float x = 0.f;
            if (pj < rows && k < n_in) x = (B[(p0 + pj) * n_in + k] - a.in_mean[k]) * a.in_rstd[k];
            X[pj * xs + k] = x;
        }
        __syncthreads();
        // forward: H1 = sigma(W1 x + b1), H2 = sigma(W2 H1 + b2)
        layer_ep<0, NT>(a.W1, a.b1, a.h1_tiles, KS1, X, xs, wave, lane, [&](int n, int mt, f4 acc) {
            P::store4(H1 + (16 * n + j) * hs + 16 * mt + 4 * g, act4(acc, slope));
        });
        __syncthreads();
        layer_ep<0, NT>(a.W2, a.b2, a.h2_tiles, KS2, H1, hs, wave, lane, [&](int n, int mt, f4 acc) {
            P::store4(H2 + (16 * n + j) * h2s + 16 * mt + 4 * g, act4(acc, slope));
        });
        __syncthreads();
        // output layer and delta3 = s .* v .* sigma'(z3) into the input tile
        layer_ep<0, NT>(a.W3, a.b3, a.out_tiles, KS3, H2, h2s, wave, lane, [&](int n, int mt, f4 acc) {
            const int pj = 16 * n + j;
            f4 d;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = 16 * mt + 4 * g + r;
                float x = 0.f;
                if (pj < rows && e < n_out) {
                    x = v[(p0 + pj) * n_out + e] * a.out_scale[e];
                    if (a.out_act && !(acc[r] > 0.f)) x *= slope;
                }
                d[r] = x;
            }
            P::store4(X + pj * xs + 16 * mt + 4 * g, d);
        });
        __syncthreads();
        // delta2 = (W3^T delta3) .* sigma'(z2), in place over H2
        layer_ep<0, NT>(a.W3T, nullptr, a.h2_tiles, KB3, X, xs, wave, lane, [&](int n, int mt, f4 acc) {
            float* h = H2 + (16 * n + j) * h2s + 16 * mt + 4 * g;
            P::store4(h, acc * mask4(h));
        });
        __syncthreads();
        // delta1 = (W2^T delta2) .* sigma'(z1), in place over H1
        layer_ep<0, NT>(a.W2T, nullptr, a.h1_tiles, KB2, H2, h2s, wave, lane, [&](int n, int mt, f4 acc) {
            float* h = H1 + (16 * n + j) * hs + 16 * mt + 4 * g;
            P::store4(h, acc * mask4(h));
        });
        __syncthreads();
        // g = (W1^T delta1) ./ std
        layer_ep<0, NT>(a.W1T, nullptr, in_tiles, KB1, H1, hs, wave, lane, [&](int n, int mt, f4 acc) {
            const int pj = 16 * n + j;
            if (pj >= rows) return;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * mt + 4 * g + r;
                if (k < n_in) g_out[(p0 + pj) * n_in + k] = acc[r] * a.in_rstd[k];
            }
        });
        // the next staging writes X only, which no wave reads after delta3 has
        // been consumed (the barrier after delta2 orders that)
    }
}

size_t mlp_vjp_lds_bytes(const MlpArgs& a) {
    using P = Prec<0>;
    const int x = a.in_pad > a.out_tiles * 16 ? a.in_pad : a.out_tiles * 16;
    return sizeof(float) * 32 * ((size_t)P::stride(a.h1_tiles * 16) + P::stride(a.h2_tiles * 16) + P::stride(x));
}

hipError_t launch_mlp_vjp(hipStream_t s, const MlpArgs& a, const float* B, const float* v, int64_t n_pts,
                          float* g_out) {
    if (n_pts <= 0) return hipSuccess;
    if (a.precision != 0 || !a.W1T || !a.W2T || !a.W3T) return hipErrorInvalidValue;
    const size_t lds = mlp_vjp_lds_bytes(a);
    if (lds > kMlpLdsBudget) return hipErrorInvalidValue;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_vjp<2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int64_t it = (n_pts + 31) / 32;
    const int n_blocks = (int)(it < kMlpBlocks ? it : kMlpBlocks);
    hipLaunchKernelGGL(k_mlp_vjp<2>, dim3(n_blocks), dim3(kWaves * 64), lds, s, a, B, v, n_pts, g_out);
    return hipGetLastError();
}

}  // namespace mala
