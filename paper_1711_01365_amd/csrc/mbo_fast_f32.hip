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

// planes of 64 or 128 points along y and z
hipError_t launch_plane_fast(int log2Y, int log2Z, const FastColArgs& a, dim3 grid, hipStream_t st, bool prepare,
                             hipEvent_t ev0, hipEvent_t ev1)
{
    if (log2Y == 6 && log2Z == 6) return plane_fast_go<float, 6, 6>(a, grid, st, prepare, ev0, ev1);
    if (log2Y == 6 && log2Z == 7) return plane_fast_go<float, 6, 7>(a, grid, st, prepare, ev0, ev1);
    if (log2Y == 7 && log2Z == 6) return plane_fast_go<float, 7, 6>(a, grid, st, prepare, ev0, ev1);
    if (log2Y == 7 && log2Z == 7) return plane_fast_go<float, 7, 7>(a, grid, st, prepare, ev0, ev1);
    return hipErrorInvalidValue;
}

int plane_fast_threads(int log2Y, int log2Z) { return (1 << (log2Y + log2Z)) / 16; }

size_t plane_fast_lds_bytes(int log2Y, int log2Z)
{
    const int ny = 1 << log2Y;
    return ((size_t)(1 << log2Z) * (ny + 1) + ny + (1 << log2Z)) * 2 * sizeof(float);
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
