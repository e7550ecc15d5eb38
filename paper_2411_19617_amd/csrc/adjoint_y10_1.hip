// dL/du contraction of the descriptor adjoint at twojmax 10, output levels
// 4..5 (see adjoint_y.h).
#include "adjoint_y.h"

namespace mala {
template hipError_t yi_group<10, 1>(hipStream_t, int64_t, const float2*, const float*, float2*, const float*,
                                     const int*, const int*);
}  // namespace mala
