// Device helpers shared by the kernels that visit, for a tile of grid
// points, every atom image within a cutoff (the neighbour sums of
// Eq. ionicdensity and the Gaussian descriptors): wave reductions, a block
// scan, and the candidate gather over the cell list.
#pragma once

#include "mala_internal.h"

namespace mala {

__device__ __forceinline__ int wave_max_int(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_min_d(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide exclusive scan of one int per thread (blockDim <= 1024).
__device__ __forceinline__ int block_exclusive_scan(int v, int* tmp, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) tmp[wave] = x;
    __syncthreads();
    int wbase = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) wbase += tmp[w];
        tot += tmp[w];
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

// Bounding boxes of a tile of consecutive flat grid indices (lane = point,
// p0 the tile's first point): box 0 holds the points in p0's run (its z-row
// when a row has at least 64 points, else its x-plane), box 1 the others.
// A tile that crosses a row or a plane would otherwise get one box spanning
// the cell's whole cross-section, and with it far more candidate images.
struct TileBoxes {
    double lo[2][3], hi[2][3];
    int n;            // 1, or 2 when the tile crosses a run boundary
};

__device__ __forceinline__ TileBoxes tile_boxes(int64_t p, int64_t p0, int Ny, int Nz, double rx, double ry,
                                                double rz) {
    const int64_t run = Nz >= 64 ? (int64_t)Nz : (int64_t)Ny * Nz;
    const bool first = p / run == p0 / run;
    const double r[3] = {rx, ry, rz};
    TileBoxes b;
    for (int d = 0; d < 3; ++d) {
        b.lo[0][d] = wave_min_d(first ? r[d] : INFINITY);
        b.hi[0][d] = wave_max_d(first ? r[d] : -INFINITY);
        b.lo[1][d] = wave_min_d(first ? INFINITY : r[d]);
        b.hi[1][d] = wave_max_d(first ? -INFINITY : r[d]);
    }
    b.n = wave_max_int(first ? 0 : 1) ? 2 : 1;
    return b;
}

__device__ __forceinline__ bool near_box(const double lo[3], const double hi[3], double X, double Y, double Z,
                                         double rc2) {
    const double dx = fmax(0.0, fmax(lo[0] - X, X - hi[0]));
    const double dy = fmax(0.0, fmax(lo[1] - Y, Y - hi[1]));
    const double dz = fmax(0.0, fmax(lo[2] - Z, Z - hi[2]));
    return dx * dx + dy * dy + dz * dz < rc2;
}

// One pass of the candidate gather: every image in the cells overlapping box
// `k` grown by rcut that lies within rcut of that box (and, for k = 1, not
// within rcut of box 0, whose pass took it already), appended after `base`
// in a fixed order (cells in index order, atoms in cell order), relative to
// the box's lower corner.
__device__ __forceinline__ int gather_pass(const BinState& bins, const TileBoxes& tb, int k, double rcut,
                                           float4* cand, int cap, int* scan_tmp, int base) {
    const double rc2 = rcut * rcut;
    const double* lo = tb.lo[k];
    const double* hi = tb.hi[k];
    int c_lo[3], c_n[3];
    for (int d = 0; d < 3; ++d) {
        c_lo[d] = (int)floor((lo[d] - rcut) / bins.cs[d]);
        c_n[d] = (int)floor((hi[d] + rcut) / bins.cs[d]) - c_lo[d] + 1;
    }
    const int ncells = c_n[0] * c_n[1] * c_n[2];
    for (int c0 = 0; c0 < ncells; c0 += blockDim.x) {
        const int c = c0 + threadIdx.x;
        int cnt = 0, b = 0, e = 0;
        double sx = 0, sy = 0, sz = 0;
        if (c < ncells) {
            const int cz = c % c_n[2], cy = (c / c_n[2]) % c_n[1], cx = c / (c_n[2] * c_n[1]);
            const int gx = c_lo[0] + cx, gy = c_lo[1] + cy, gz = c_lo[2] + cz;
            const int wx = ((gx % bins.nc[0]) + bins.nc[0]) % bins.nc[0];
            const int wy = ((gy % bins.nc[1]) + bins.nc[1]) % bins.nc[1];
            const int wz = ((gz % bins.nc[2]) + bins.nc[2]) % bins.nc[2];
            sx = (double)((gx - wx) / bins.nc[0]) * bins.L[0];
            sy = (double)((gy - wy) / bins.nc[1]) * bins.L[1];
            sz = (double)((gz - wz) / bins.nc[2]) * bins.L[2];
            const int cell = (wx * bins.nc[1] + wy) * bins.nc[2] + wz;
            b = bins.cell_start[cell];
            e = bins.cell_start[cell + 1];
            for (int a = b; a < e; ++a) {
                const double4 at = bins.atoms[a];
                const double X = at.x + sx, Y = at.y + sy, Z = at.z + sz;
                cnt += near_box(lo, hi, X, Y, Z, rc2) && !(k == 1 && near_box(tb.lo[0], tb.hi[0], X, Y, Z, rc2));
            }
        }
        int total;
        int off = base + block_exclusive_scan(cnt, scan_tmp, &total);
        for (int a = b; a < e; ++a) {
            const double4 at = bins.atoms[a];
            const double X = at.x + sx, Y = at.y + sy, Z = at.z + sz;
            if (near_box(lo, hi, X, Y, Z, rc2) && !(k == 1 && near_box(tb.lo[0], tb.hi[0], X, Y, Z, rc2))) {
                if (off < cap)
                    cand[off] = make_float4((float)(X - lo[0]), (float)(Y - lo[1]), (float)(Z - lo[2]),
                                            __int_as_float((int)at.w));
                ++off;
            }
        }
        base += total;
    }
    return base;
}

// Candidate atom images of a tile with boxes `tb`: every image within rcut
// of one of its boxes, each once, as float4 in cand[0 .. cap) (w holds the
// bits of the atom's index).  Box 0's pass comes first and is stored
// relative to box 0's lower corner; box 1's pass, from index *n0 on, relative
// to box 1's, so that offsets stay as small as the boxes (a tile crossing a
// row spans the cell).  Called by the whole block; returns the total count,
// which exceeds cap when the list overflowed (only the first cap are
// stored).  scan_tmp holds blockDim/64 ints.
__device__ __forceinline__ int gather_candidates(const BinState& bins, const TileBoxes& tb, double rcut,
                                                 float4* cand, int cap, int* scan_tmp, int* n0) {
    int base = gather_pass(bins, tb, 0, rcut, cand, cap, scan_tmp, 0);
    *n0 = base;
    if (tb.n == 2) base = gather_pass(bins, tb, 1, rcut, cand, cap, scan_tmp, base);
    return base;
}

// Squared displacements below this (r < 1e-15 A) count as an atom on the
// point (r = 0): it keeps the hardware reciprocal square root away from
// denormal inputs, and the terms left out are below FP32 resolution.
constexpr float kMinR2 = 1e-30f;

// A lane's point relative to the two origins its candidates are stored
// against: candidate c is compared with at(c).
struct PointFrame {
    float3 p0, p1;
    int n0;
    __device__ __forceinline__ float3 at(int c) const { return c < n0 ? p0 : p1; }
};

__device__ __forceinline__ PointFrame point_frame(const TileBoxes& tb, int n0, double rx, double ry, double rz) {
    PointFrame f;
    f.p0 = make_float3((float)(rx - tb.lo[0][0]), (float)(ry - tb.lo[0][1]), (float)(rz - tb.lo[0][2]));
    f.p1 = tb.n == 2 ? make_float3((float)(rx - tb.lo[1][0]), (float)(ry - tb.lo[1][1]), (float)(rz - tb.lo[1][2]))
                     : f.p0;
    f.n0 = n0;
    return f;
}

// Wave 0's per-point neighbour lists: the indices of the candidates within
// rc of the lane's point, in candidate order, at most kMaxNbr (more sets
// kErrNbr in *err); invalid lanes get empty lists.
__device__ __forceinline__ void build_neighbour_lists(const float4* cand, int ncand, const PointFrame& f, float rc,
                                                      bool valid, int lane, unsigned short (*nbr)[kTile],
                                                      int* nnbr, int* err) {
    int cnt = 0;
    const int split = f.n0 < ncand ? f.n0 : ncand;
    auto scan = [&](int c0, int c1, float3 p) {
        for (int c = c0; c < c1; ++c) {
            const float4 q = cand[c];
            const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
            if (dx * dx + dy * dy + dz * dz < rc * rc) {
                if (cnt < kMaxNbr) nbr[cnt][lane] = (unsigned short)c;
                ++cnt;
            }
        }
    };
    scan(0, split, f.p0);
    scan(split, ncand, f.p1);
    if (cnt > kMaxNbr) atomicOr(err, kErrNbr);
    nnbr[lane] = valid ? (cnt < kMaxNbr ? cnt : kMaxNbr) : 0;
}

}  // namespace mala
