// Launch of the descriptor adjoint's dL/du contraction (k_yi, adjoint_y.h):
// one kernel per group of output levels.  The twojmax-10 groups are
// instantiated in files of their own so that they compile in parallel.
#include "adjoint_y.h"

namespace mala {

extern template hipError_t yi_group<10, 0>(hipStream_t, int64_t, const float2*, const float*, float2*, const float*,
                                           const int*, const int*);
extern template hipError_t yi_group<10, 1>(hipStream_t, int64_t, const float2*, const float*, float2*, const float*,
                                           const int*, const int*);
extern template hipError_t yi_group<10, 2>(hipStream_t, int64_t, const float2*, const float*, float2*, const float*,
                                           const int*, const int*);
extern template hipError_t yi_group<10, 3>(hipStream_t, int64_t, const float2*, const float*, float2*, const float*,
                                           const int*, const int*);

int y_max_waves() { return kYMaxWaves; }
int y_group_wave_count(int tj, int g) { return y_group_waves(tj, g); }
int y_group_count(int tj) { return y_groups(tj); }
int y_group_first(int tj, int g) { return y_group_lo(tj, g); }
int y_group_last(int tj, int g) { return y_group_hi(tj, g); }

hipError_t launch_yi(hipStream_t s, int twojmax, int64_t n_pts, const float2* u, const float* gB, float2* y,
                     const float* cg_tab, const int* cg_off, const int* wave_units) {
    hipError_t e = hipSuccess;
#define MALA_YI(TJ, G)                                                                     \
    if (e == hipSuccess) e = yi_group<TJ, G>(s, n_pts, u, gB, y, cg_tab, cg_off, wave_units)
    switch (twojmax) {
    case 2: MALA_YI(2, 0); break;
    case 4: MALA_YI(4, 0); break;
    case 6: MALA_YI(6, 0); break;
    case 8: MALA_YI(8, 0); MALA_YI(8, 1); break;
    case 10: MALA_YI(10, 0); MALA_YI(10, 1); MALA_YI(10, 2); MALA_YI(10, 3); break;
    default: return hipErrorInvalidValue;
    }
#undef MALA_YI
    return e;
}

}  // namespace mala
