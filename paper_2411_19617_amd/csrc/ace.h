// Host interface of the grid ACE descriptor kernel (ace.hip) and its
// rank-3 term tables (tables.cpp).
#pragma once
#include <vector>
#include "mala_internal.h"

namespace mala {

constexpr int kAceMaxN = 4;      // radial functions
constexpr int kAceMaxL = 4;      // angular momentum

inline int ace_count_ranks12(int nmax, int lmax) { return nmax + (lmax + 1) * nmax * (nmax + 1) / 2; }
// rank-3 groups (p1, p2, l3): a header of kAceGroupInts ints each, its
// outputs (A row base of n3 | descriptor position << 7, at most kAceMaxN)
// inline, then the first rank-3 position of its pair (p1, p2) and the pair's
// width | (last group of the pair) << 8.  The outputs of a pair are
// contiguous (at most kAceMaxPairCols).  Two tables: `groups` for
// point-major output, laid out for kAce3Waves waves (entry k * kAce3Waves + w
// is wave w's k-th group, each wave holding whole pairs, balanced by their
// terms, padded with empty groups of combination -1), and `groups_dm` in
// (p1, p2, l3) order for descriptor-major output (the waves take every
// kAce3Waves-th group).
constexpr int kAceGroupInts = 12;
constexpr int kAce3Waves = 8;
constexpr int kAceMaxPairCols = kAceMaxN * (kAceMaxL + 1);
int build_ace_tables(int nmax, int lmax, std::vector<int>& groups, std::vector<int>& groups_dm,
                     std::vector<float>& coef);
// rank 4: descriptor set (p1, p2, p3, p4, L per entry) and its evaluation tables
constexpr int kAce4MaxN = 3;
constexpr int kAce4MaxL = 3;
constexpr size_t kAce4LdsBudget = 96 * 1024;     // dynamic LDS of the pair vectors of one L
constexpr int kAce4MaxDescsL = 1024;              // descriptors of one phase (364 for L = 2 at nmax4 = lmax4 = 3)
// point-major rank 4 runs in chunks of kAce4RowChunk points: descriptor
// planes of the chunk (246 MB at 939 per point), then rows
constexpr int64_t kAce4RowChunk = 1 << 16;
int ace4_descriptor_set(int nmax4, int lmax4, std::vector<int>& desc);
// The evaluation runs in phases, each one or more couplings L whose pair
// slots fit the LDS budget together: l_units / l_descs are offsets per
// phase; a descriptor entry is (first pair slot | L << 16, second pair slot,
// output, factor bits), slots counted within the phase.
int build_ace4_tables(int nmax4, int lmax4, std::vector<int>& l_units, std::vector<int4>& units,
                      std::vector<float>& coef, std::vector<int>& l_descs, std::vector<int4>& descs,
                      int& max_slots);
// A of every point of a chunk (n < 4, l <= 4, m >= 0: 60 complex per point),
// laid out [tile][60][64 lanes], written by the projection kernel and read by
// the contraction kernels.
constexpr int kAceAPerPoint = kAceMaxN * 15;
hipError_t launch_ace_proj(hipStream_t s, const BinState& bins, const int N[3], double rcut, int64_t pt_begin,
                           int64_t n_pts, float2* Ag, int* err);
hipError_t launch_ace4(hipStream_t s, const float2* Ag, int lmax4, int n_phases, int64_t n_pts, const int* l_units,
                       const int4* units, const float* coef, const int* l_descs, const int4* descs, int max_slots,
                       int n4, float* out, int64_t ps, int64_t ds);   // descriptor k of point p at out[p ps + k ds]
// out[p n_cols + k] = in[k ld + p] (p < n_rows <= ld, k < n_cols)
hipError_t launch_planes_to_rows(hipStream_t s, const float* in, int64_t ld, int64_t n_rows, int n_cols, float* out);
hipError_t launch_ace(hipStream_t s, const float2* Ag, int nmax, int lmax, int64_t n_pts, const int* groups,
                      int n_groups, const float* coef, int n_desc, float* out, int64_t ps,
                      int64_t ds);

}  // namespace mala
