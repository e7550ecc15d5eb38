// Gaussian descriptors on the grid: the Gaussian representation of the ionic
// positions from which the structure factor follows (Eq.
// structurefactor_gaussian), a normalised Gaussian of width sigma on every
// atom and periodic image within the cutoff:
//   G(r) = (2 pi sigma^2)^(-3/2) sum_{|r-R| < cutoff} exp(-|r-R|^2 / (2 sigma^2)).
// One wave per tile of 64 consecutive grid points: the tile's candidate
// images are gathered into LDS from the cell list (as for the bispectrum),
// then every lane sums over them in the same fixed order.
#include <math.h>

#include "tile_gather.h"

namespace mala {

__global__ __launch_bounds__(64) void k_gauss(BinState bins, int Nx, int Ny, int Nz, float a, double norm,
                                              double cutoff, int64_t pt_begin, int64_t n_pts,
                                              float* __restrict__ out, int* __restrict__ err) {
    __shared__ float4 cand[kMaxCand];
    __shared__ int scan_tmp[16];
    const int lane = threadIdx.x;
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
    const int base = gather_candidates(bins, boxes, cutoff, cand, kMaxCand, scan_tmp, &n0);
    if (base > kMaxCand && lane == 0) atomicOr(err, kErrCand);
    const int ncand = base < kMaxCand ? base : kMaxCand;
    __syncthreads();

    const PointFrame frame = point_frame(boxes, n0, rx, ry, rz);
    const float rc2 = (float)(cutoff * cutoff);
    float acc = 0.f;
    auto scan = [&](int c0, int c1, float3 o) {
        for (int c = c0; c < c1; ++c) {
            const float4 q = cand[c];
            const float dx = q.x - o.x, dy = q.y - o.y, dz = q.z - o.z;
            const float d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < rc2) acc += expf(-a * d2);
        }
    };
    const int split = n0 < ncand ? n0 : ncand;
    scan(0, split, frame.p0);
    scan(split, ncand, frame.p1);
    if (valid) out[idx] = (float)(norm * (double)acc);
}

hipError_t launch_gauss(hipStream_t s, const BinState& bins, const int N[3], double sigma, double cutoff,
                        int64_t pt_begin, int64_t n_pts, float* out, int* err_flag) {
    const int64_t n_tiles = (n_pts + kTile - 1) / kTile;
    if (n_tiles == 0) return hipSuccess;
    const double norm = pow(2.0 * 3.14159265358979323846 * sigma * sigma, -1.5);   // unit integral
    const float a = (float)(0.5 / (sigma * sigma));
    hipLaunchKernelGGL(k_gauss, dim3((unsigned)n_tiles), dim3(64), 0, s, bins, N[0], N[1], N[2], a, norm, cutoff,
                       pt_begin, n_pts, out, err_flag);
    return hipGetLastError();
}

}  // namespace mala
