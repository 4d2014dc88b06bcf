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

template <typename T>
static size_t row_lds_t(int n, int log2L)
{
#define MBO_ROW_LDS(NV, LG) \
    if (n == NV && log2L == LG) return RowFastShape<T, NV, LG>::LDS;
#define MBO_ROW_LDS_N(NV) \
    MBO_ROW_LDS(NV, 3) MBO_ROW_LDS(NV, 4) MBO_ROW_LDS(NV, 5) MBO_ROW_LDS(NV, 6) MBO_ROW_LDS(NV, 7) \
    MBO_ROW_LDS(NV, 8) MBO_ROW_LDS(NV, 9) MBO_ROW_LDS(NV, 10) MBO_ROW_LDS(NV, 11)
    MBO_ROW_LDS_N(1) MBO_ROW_LDS_N(2) MBO_ROW_LDS_N(3) MBO_ROW_LDS_N(4)
#undef MBO_ROW_LDS_N
#undef MBO_ROW_LDS
    return 0;
}

size_t row_fast_lds_bytes(int prec, int n, int log2L)
{
    return prec == 1 ? row_lds_t<float>(n, log2L) : row_lds_t<double>(n, log2L);
}

int row_fast_rows_per_group(int log2L) { return log2L >= 9 ? 1 : 512 >> log2L; }


}  // namespace mbo
