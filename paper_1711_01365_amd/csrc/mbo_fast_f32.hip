// Band-limited passes in float, and the precision dispatch of both launchers.
#include "mbo_fast_launch.hpp"

namespace mbo {

hipError_t launch_row_fast_f64(int n, int log2L, const FastRowArgs& a, dim3 g, hipStream_t st, bool prepare,
                               hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_heat_fast_f64(int log2L, int TX, const FastColArgs& a, dim3 g, hipStream_t st, bool prepare,
                                hipEvent_t ev0, hipEvent_t ev1);

hipError_t launch_row_fast(int prec, int n, int log2L, const FastRowArgs& a, dim3 grid, hipStream_t st,
                           bool prepare, hipEvent_t ev0, hipEvent_t ev1)
{
    if (prec == 1) return row_fast_t<float>(n, log2L, a, grid, st, prepare, ev0, ev1);
    return launch_row_fast_f64(n, log2L, a, grid, st, prepare, ev0, ev1);
}

hipError_t launch_heat_fast(int prec, int log2L, int TX, const FastColArgs& a, dim3 grid, hipStream_t st,
                            bool prepare, hipEvent_t ev0, hipEvent_t ev1)
{
    if (prec == 1) return heat_fast_t<float>(log2L, TX, a, grid, st, prepare, ev0, ev1);
    return launch_heat_fast_f64(log2L, TX, a, grid, st, prepare, ev0, ev1);
}

int row_fast_block(int prec, int n) { return prec == 1 && n == 3 ? row_fast_threads<float, 3>() : FAST_POINTS; }

size_t row_fast_lds_bytes(int prec, int n, int log2L)
{
    const int L = 1 << log2L;
    return (size_t)((n * n + 1) / 2) * (FAST_POINTS / L) * (L + L / 8) * 2 * (prec == 1 ? 4 : 8);
}

size_t heat_fast_lds_bytes(int prec, int log2L, int TX)
{
    const int L = 1 << log2L;
    return (size_t)TX * (L + L / 8) * 2 * (prec == 1 ? 4 : 8);
}

}  // namespace mbo
