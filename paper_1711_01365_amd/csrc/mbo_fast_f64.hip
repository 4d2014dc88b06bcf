// Band-limited passes in double.
#include "mbo_fast_launch.hpp"

namespace mbo {

hipError_t launch_row_fast_f64(int n, int log2L, const FastRowArgs& a, dim3 g, hipStream_t st, bool prepare,
                               hipEvent_t ev0, hipEvent_t ev1)
{
    return row_fast_t<double>(n, log2L, a, g, st, prepare, ev0, ev1);
}

hipError_t launch_heat_fast_f64(int log2L, int TX, const FastColArgs& a, dim3 g, hipStream_t st, bool prepare,
                                hipEvent_t ev0, hipEvent_t ev1)
{
    return heat_fast_t<double>(log2L, TX, a, g, st, prepare, ev0, ev1);
}

}  // namespace mbo
