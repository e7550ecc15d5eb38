// Cell list of the atoms of one snapshot (the neighbour search of Sec. 3.2.2,
// Eq. ionicdensity: all atoms within the cutoff of a grid point).
//
// Atoms are wrapped into [0, L) and counting-sorted into a uniform grid of
// cells of edge >= rcut/2; inside a cell they are ordered by atom index, so
// the neighbour order (and with it every floating-point sum downstream) does
// not depend on atomic-operation timing.
#include "mala_internal.h"

namespace mala {

namespace {

__global__ void k_zero_int(int* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_wrap_count(const double* __restrict__ pos, int n, double Lx, double Ly, double Lz,
                             int ncx, int ncy, int ncz, double csx, double csy, double csz,
                             double4* __restrict__ tmp, int* __restrict__ atom_cell,
                             int* __restrict__ count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double L[3] = {Lx, Ly, Lz};
    double x[3];
    int c[3];
    const int nc[3] = {ncx, ncy, ncz};
    const double cs[3] = {csx, csy, csz};
    for (int d = 0; d < 3; ++d) {
        double v = pos[3 * i + d];
        v = v - floor(v / L[d]) * L[d];
        if (v >= L[d]) v -= L[d];
        if (v < 0.0) v = 0.0;
        x[d] = v;
        int ci = (int)(v / cs[d]);
        c[d] = ci < 0 ? 0 : (ci >= nc[d] ? nc[d] - 1 : ci);
    }
    int cell = (c[0] * ncy + c[1]) * ncz + c[2];
    tmp[i] = make_double4(x[0], x[1], x[2], (double)i);
    atom_cell[i] = cell;
    atomicAdd(&count[cell], 1);
}

// Exclusive scan of count[0..n) into start[0..n] by one block.
__global__ void k_scan(const int* __restrict__ count, int* __restrict__ start, int n) {
    __shared__ int buf[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        int i = base + threadIdx.x;
        int v = i < n ? count[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) start[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) start[n] = carry;
}

__global__ void k_scatter(const double4* __restrict__ tmp, const int* __restrict__ atom_cell, int n,
                          const int* __restrict__ start, int* __restrict__ fill,
                          double4* __restrict__ sorted) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = atom_cell[i];
    int slot = start[c] + atomicAdd(&fill[c], 1);
    sorted[slot] = tmp[i];
}

// Order each cell's atoms by atom index (insertion sort; cells hold a few atoms).
__global__ void k_sort_cells(const int* __restrict__ start, int ncell, double4* __restrict__ sorted) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int b = start[c], e = start[c + 1];
    for (int i = b + 1; i < e; ++i) {
        double4 v = sorted[i];
        int j = i - 1;
        while (j >= b && sorted[j].w > v.w) {
            sorted[j + 1] = sorted[j];
            --j;
        }
        sorted[j + 1] = v;
    }
}

}  // namespace

hipError_t launch_bin(hipStream_t s, const double* pos_dev, int n_atoms, const double L[3],
                      double rcut, int* cell_count, int* cell_start, int* cell_fill,
                      double4* atoms_tmp, int* atom_cell, double4* atoms_sorted, BinState* st) {
    for (int d = 0; d < 3; ++d) {
        int nc = (int)floor(L[d] / (0.5 * rcut));
        if (nc < 1) nc = 1;
        if (nc > 256) nc = 256;
        st->nc[d] = nc;
        st->cs[d] = L[d] / nc;
        st->L[d] = L[d];
    }
    st->ncell = st->nc[0] * st->nc[1] * st->nc[2];
    st->n_atoms = n_atoms;
    st->cell_start = cell_start;
    st->atoms = atoms_sorted;
    int nz = st->ncell + 1;
    hipLaunchKernelGGL(k_zero_int, dim3((nz + 255) / 256), dim3(256), 0, s, cell_count, nz);
    hipLaunchKernelGGL(k_zero_int, dim3((nz + 255) / 256), dim3(256), 0, s, cell_fill, nz);
    if (n_atoms > 0)
        hipLaunchKernelGGL(k_wrap_count, dim3((n_atoms + 255) / 256), dim3(256), 0, s, pos_dev, n_atoms,
                           L[0], L[1], L[2], st->nc[0], st->nc[1], st->nc[2], st->cs[0], st->cs[1],
                           st->cs[2], atoms_tmp, atom_cell, cell_count);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cell_count, cell_start, st->ncell);
    if (n_atoms > 0) {
        hipLaunchKernelGGL(k_scatter, dim3((n_atoms + 255) / 256), dim3(256), 0, s, atoms_tmp, atom_cell,
                           n_atoms, cell_start, cell_fill, atoms_sorted);
        hipLaunchKernelGGL(k_sort_cells, dim3((st->ncell + 255) / 256), dim3(256), 0, s, cell_start,
                           st->ncell, atoms_sorted);
    }
    return hipGetLastError();
}

}  // namespace mala
