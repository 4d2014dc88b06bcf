// Launchers of the band-limited passes (mbo_fast.hpp) for one precision T:
// row_fast for n = 1..4 and row lengths 2^3..2^11, heat_fast for column lengths
// 2^6..2^11 and tiles of TX = 1..16 columns with 64..1024 threads.
#pragma once

#include <hip/hip_ext.h>

#include "mbo_fast.hpp"

namespace mbo {

template <typename T, int n, int LG, bool PM>
static hipError_t row_fast_go(const FastRowArgs& a, dim3 g, hipStream_t st, bool prepare, hipEvent_t ev0,
                              hipEvent_t ev1)
{
    typedef RowFastShape<T, n, LG> S;
    const size_t lds = S::LDS;
    const void* f = reinterpret_cast<const void*>(&row_fast<T, n, LG, PM>);
    if (prepare) return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const dim3 bl(S::THREADS);
    if (ev0) hipExtLaunchKernelGGL((row_fast<T, n, LG, PM>), g, bl, lds, st, ev0, ev1, 0, a);
    else hipLaunchKernelGGL((row_fast<T, n, LG, PM>), g, bl, lds, st, a);
    return hipGetLastError();
}

// The row-major instance, and for float the plane-major one of the 3-D layout
// (both prepared together).
template <typename T, int n, int LG>
static hipError_t row_fast_pm(const FastRowArgs& a, dim3 g, hipStream_t st, bool prepare, hipEvent_t ev0,
                              hipEvent_t ev1)
{
    if constexpr (sizeof(T) == 4) {
        if (prepare) {
            const hipError_t e = row_fast_go<T, n, LG, true>(a, g, st, true, ev0, ev1);
            if (e != hipSuccess) return e;
        } else if (a.plane_major) {
            return row_fast_go<T, n, LG, true>(a, g, st, false, ev0, ev1);
        }
    } else {
        if (a.plane_major && !prepare) return hipErrorInvalidValue;  // float-only layout
    }
    return row_fast_go<T, n, LG, false>(a, g, st, prepare, ev0, ev1);
}

template <typename T, int n>
static hipError_t row_fast_n(int log2L, const FastRowArgs& a, dim3 g, hipStream_t st, bool prepare,
                             hipEvent_t ev0, hipEvent_t ev1)
{
    switch (log2L) {
    case 3: return row_fast_pm<T, n, 3>(a, g, st, prepare, ev0, ev1);
    case 4: return row_fast_pm<T, n, 4>(a, g, st, prepare, ev0, ev1);
    case 5: return row_fast_pm<T, n, 5>(a, g, st, prepare, ev0, ev1);
    case 6: return row_fast_pm<T, n, 6>(a, g, st, prepare, ev0, ev1);
    case 7: return row_fast_pm<T, n, 7>(a, g, st, prepare, ev0, ev1);
    case 8: return row_fast_pm<T, n, 8>(a, g, st, prepare, ev0, ev1);
    case 9: return row_fast_pm<T, n, 9>(a, g, st, prepare, ev0, ev1);
    case 10: return row_fast_pm<T, n, 10>(a, g, st, prepare, ev0, ev1);
    case 11: return row_fast_pm<T, n, 11>(a, g, st, prepare, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t row_fast_t(int n, int log2L, const FastRowArgs& a, dim3 g, hipStream_t st, bool prepare,
                             hipEvent_t ev0, hipEvent_t ev1)
{
    switch (n) {
    case 1: return row_fast_n<T, 1>(log2L, a, g, st, prepare, ev0, ev1);
    case 2: return row_fast_n<T, 2>(log2L, a, g, st, prepare, ev0, ev1);
    case 3: return row_fast_n<T, 3>(log2L, a, g, st, prepare, ev0, ev1);
    case 4: return row_fast_n<T, 4>(log2L, a, g, st, prepare, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

template <typename T, int LG, int TX>
static hipError_t heat_fast_go(const FastColArgs& a, dim3 g, hipStream_t st, bool prepare, hipEvent_t ev0,
                               hipEvent_t ev1)
{
    constexpr int NT = TX * (1 << LG) / 8;
    if constexpr (NT < 64 || NT > 1024) {
        return hipErrorInvalidValue;
    } else {
        const size_t lds = HeatFastShape<T, LG, TX>::LDS;
        const void* f = reinterpret_cast<const void*>(&heat_fast<T, LG, TX>);
        if (prepare) return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (ev0) hipExtLaunchKernelGGL((heat_fast<T, LG, TX>), g, dim3(NT), lds, st, ev0, ev1, 0, a);
        else hipLaunchKernelGGL((heat_fast<T, LG, TX>), g, dim3(NT), lds, st, a);
        return hipGetLastError();
    }
}

template <typename T, int LG>
static hipError_t heat_fast_l(int TX, const FastColArgs& a, dim3 g, hipStream_t st, bool prepare, hipEvent_t ev0,
                              hipEvent_t ev1)
{
    switch (TX) {
    case 1: return heat_fast_go<T, LG, 1>(a, g, st, prepare, ev0, ev1);
    case 2: return heat_fast_go<T, LG, 2>(a, g, st, prepare, ev0, ev1);
    case 4: return heat_fast_go<T, LG, 4>(a, g, st, prepare, ev0, ev1);
    case 8: return heat_fast_go<T, LG, 8>(a, g, st, prepare, ev0, ev1);
    case 16: return heat_fast_go<T, LG, 16>(a, g, st, prepare, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t heat_fast_t(int log2L, int TX, const FastColArgs& a, dim3 g, hipStream_t st, bool prepare,
                              hipEvent_t ev0, hipEvent_t ev1)
{
    switch (log2L) {
    case 6: return heat_fast_l<T, 6>(TX, a, g, st, prepare, ev0, ev1);
    case 7: return heat_fast_l<T, 7>(TX, a, g, st, prepare, ev0, ev1);
    case 8: return heat_fast_l<T, 8>(TX, a, g, st, prepare, ev0, ev1);
    case 9: return heat_fast_l<T, 9>(TX, a, g, st, prepare, ev0, ev1);
    case 10: return heat_fast_l<T, 10>(TX, a, g, st, prepare, ev0, ev1);
    case 11: return heat_fast_l<T, 11>(TX, a, g, st, prepare, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

template <typename T, int LY, int LZ>
static hipError_t plane_fast_go(const FastColArgs& a, dim3 g, hipStream_t st, bool prepare, hipEvent_t ev0,
                                hipEvent_t ev1)
{
    typedef PlaneFastShape<T, LY, LZ> S;
    const void* f = reinterpret_cast<const void*>(&plane_fast<T, LY, LZ>);
    if (prepare) return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::LDS);
    if (ev0) hipExtLaunchKernelGGL((plane_fast<T, LY, LZ>), g, dim3(S::THREADS), S::LDS, st, ev0, ev1, 0, a);
    else hipLaunchKernelGGL((plane_fast<T, LY, LZ>), g, dim3(S::THREADS), S::LDS, st, a);
    return hipGetLastError();
}

}  // namespace mbo
