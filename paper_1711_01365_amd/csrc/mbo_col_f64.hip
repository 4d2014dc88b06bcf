// Strided-axis kernels in double: forward / inverse / heat / energy / tau-derivative / resolvent / Dirichlet modes for
// transform lengths 2^3..2^11.
#include <hip/hip_ext.h>

#include "mbo_kernels.hpp"

namespace mbo {

template <int MODE>
static hipError_t col_m(int log2L, const ColArgs& a, dim3 g, dim3 bl, size_t lds, hipStream_t st,
                        bool prepare, hipEvent_t ev0, hipEvent_t ev1)
{
#define MBO_COL_CASE(LG)                                                                       \
    {                                                                                          \
        if (prepare)                                                                           \
            return hipFuncSetAttribute(reinterpret_cast<const void*>(&col_pass<double, MODE, LG>), \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        if (ev0) hipExtLaunchKernelGGL((col_pass<double, MODE, LG>), g, bl, lds, st, ev0, ev1, 0, a);                  \
        else hipLaunchKernelGGL((col_pass<double, MODE, LG>), g, bl, lds, st, a);                     \
        return hipGetLastError();                                                              \
    }
    MBO_LOG2L_SWITCH(log2L, MBO_COL_CASE)
#undef MBO_COL_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_col_f64(int mode, int log2L, const ColArgs& a, dim3 g, dim3 bl, size_t lds,
                          hipStream_t st, bool prepare, hipEvent_t ev0, hipEvent_t ev1)
{
    switch (mode) {
    case CM_FORWARD: return col_m<CM_FORWARD>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case CM_INVERSE: return col_m<CM_INVERSE>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case CM_HEAT: return col_m<CM_HEAT>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case CM_ENERGY: return col_m<CM_ENERGY>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case CM_DTAU: return col_m<CM_DTAU>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case CM_RESOLVENT: return col_m<CM_RESOLVENT>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    case CM_DIRICHLET: return col_m<CM_DIRICHLET>(log2L, a, g, bl, lds, st, prepare, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

}  // namespace mbo
