// Row-pass kernels of the volume-preserving step in float: every matrix size
// n = 1..4 and row length 2^3..2^11.
#include "mbo_kernels.hpp"

namespace mbo {

template <int n>
static hipError_t vprow_n(int log2L, const RowArgs& a, dim3 g, dim3 bl, size_t lds, hipStream_t st,
                          bool prepare)
{
#define MBO_VPROW_CASE(LG)                                                                           \
    {                                                                                                \
        if (prepare)                                                                                 \
            return hipFuncSetAttribute(reinterpret_cast<const void*>(&row_pass<float, n, LG, RM_VOLUME>),    \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
        hipLaunchKernelGGL((row_pass<float, n, LG, RM_VOLUME>), g, bl, lds, st, a);                        \
        return hipGetLastError();                                                                    \
    }
    MBO_LOG2L_SWITCH(log2L, MBO_VPROW_CASE)
#undef MBO_VPROW_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_row_vp_f32(int n, int log2L, const RowArgs& a, dim3 g, dim3 bl, size_t lds,
                             hipStream_t st, bool prepare)
{
    switch (n) {
    case 1: return vprow_n<1>(log2L, a, g, bl, lds, st, prepare);
    case 2: return vprow_n<2>(log2L, a, g, bl, lds, st, prepare);
    case 3: return vprow_n<3>(log2L, a, g, bl, lds, st, prepare);
    case 4: return vprow_n<4>(log2L, a, g, bl, lds, st, prepare);
    }
    return hipErrorInvalidValue;
}

}  // namespace mbo
