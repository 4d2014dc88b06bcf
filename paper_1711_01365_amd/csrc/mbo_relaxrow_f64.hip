// Row-pass kernels of the relaxed gradient flows (reaction step) in double: every matrix size
// n = 1..4 and row length 2^3..2^11.
#include "mbo_kernels.hpp"

namespace mbo {

template <int n>
static hipError_t relaxrow_n(int log2L, const RowArgs& a, dim3 g, dim3 bl, size_t lds, hipStream_t st,
                          bool prepare)
{
#define MBO_RELAXROW_CASE(LG)                                                                           \
    {                                                                                                \
        if (prepare)                                                                                 \
            return hipFuncSetAttribute(reinterpret_cast<const void*>(&row_pass<double, n, LG, RM_RELAX>),    \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
        hipLaunchKernelGGL((row_pass<double, n, LG, RM_RELAX>), g, bl, lds, st, a);                        \
        return hipGetLastError();                                                                    \
    }
    MBO_LOG2L_SWITCH(log2L, MBO_RELAXROW_CASE)
#undef MBO_RELAXROW_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_row_relax_f64(int n, int log2L, const RowArgs& a, dim3 g, dim3 bl, size_t lds,
                             hipStream_t st, bool prepare)
{
    switch (n) {
    case 1: return relaxrow_n<1>(log2L, a, g, bl, lds, st, prepare);
    case 2: return relaxrow_n<2>(log2L, a, g, bl, lds, st, prepare);
    case 3: return relaxrow_n<3>(log2L, a, g, bl, lds, st, prepare);
    case 4: return relaxrow_n<4>(log2L, a, g, bl, lds, st, prepare);
    }
    return hipErrorInvalidValue;
}

}  // namespace mbo
