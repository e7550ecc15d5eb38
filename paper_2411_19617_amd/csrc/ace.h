// Host interface of the grid ACE descriptor kernel (ace.hip) and its
// rank-3 term tables (tables.cpp).
#pragma once
#include <vector>
#include "mala_internal.h"

namespace mala {

constexpr int kAceMaxN = 4;      // radial functions
constexpr int kAceMaxL = 4;      // angular momentum

inline int ace_count_ranks12(int nmax, int lmax) { return nmax + (lmax + 1) * nmax * (nmax + 1) / 2; }
int build_ace_tables(int nmax, int lmax, std::vector<int>& groups, std::vector<int>& term_idx,
                     std::vector<float>& term_coef, std::vector<int>& outputs);
hipError_t launch_ace(hipStream_t s, const BinState& bins, const int N[3], double rcut, int nmax, int lmax,
                      int64_t pt_begin, int64_t n_pts, const int* groups, int n_groups, const int2* terms,
                      const int* outputs, int n_desc, float* out, int* err);

}  // namespace mala
