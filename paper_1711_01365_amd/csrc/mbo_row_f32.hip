// Row-pass kernels in float: every matrix size n = 1..4 and row length 2^3..2^11.
#include <hip/hip_ext.h>

#include "mbo_kernels.hpp"

namespace mbo {

template <int n>
static hipError_t row_n(int log2L, const RowArgs& a, dim3 g, dim3 bl, size_t lds, hipStream_t st,
                        bool prepare, hipEvent_t ev0, hipEvent_t ev1)
{
#define MBO_ROW_CASE(LG)                                                                       \
    {                                                                                          \
        if (prepare)                                                                           \
            return hipFuncSetAttribute(reinterpret_cast<const void*>(&row_pass<float, n, LG>), \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        if (ev0) hipExtLaunchKernelGGL((row_pass<float, n, LG>), g, bl, lds, st, ev0, ev1, 0, a);                  \
        else hipLaunchKernelGGL((row_pass<float, n, LG>), g, bl, lds, st, a);                        \
        return hipGetLastError();                                                              \
    }
    MBO_LOG2L_SWITCH(log2L, MBO_ROW_CASE)
#undef MBO_ROW_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_row_f32(int n, int log2L, const RowArgs& a, dim3 g, dim3 bl, size_t lds,
                          hipStream_t st, bool prepare, hipEvent_t ev0, hipEvent_t ev1)
{
    switch (n) {
    case 1: return row_n<1>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case 2: return row_n<2>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case 3: return row_n<3>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case 4: return row_n<4>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

}  // namespace mbo
