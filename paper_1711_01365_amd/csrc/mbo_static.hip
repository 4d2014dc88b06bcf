// mbo_step_static: one step of Algorithm 1 for a 2-D field with no plan and no
// device allocation (declared in include/mbo.h).
//
// The step runs the band-limited kernels of mbo_step (forward row pass of the
// field, heat pass over the stored columns, row pass with the projection of
// Lemma 1.1).  Their working memory -- the kept row spectra of every packed
// plane, the twiddles of both axes and the two factors of the heat symbol --
// lives in one fixed device array per GPU, `scratch`, which the code object
// holds for the life of the process.  Every call on a GPU shares that GPU's
// array; calls that overlap on one GPU race.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "mbo.h"
#include "mbo_internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)MBO_STEP_STATIC_MAX_BYTES;
constexpr int kMaxDevices = 64;

// The working memory of mbo_step_static.  In host code this name is only a
// stand-in: kernels receive the address hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    bool ready = false;
    unsigned char* ptr = nullptr;  // device address of `scratch` on this GPU
    size_t lds_max = 0;            // dynamic LDS a workgroup may use
};
DeviceScratch g_dev[kMaxDevices];
std::mutex g_setup;

int ilog2i(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

bool pow2_in_range(int64_t v) { return v >= 8 && v <= 2048 && (v & (v - 1)) == 0; }

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Twiddles exp(-2 pi i m / L) of both axes and the heat-symbol factors of the
// band-limited layout, from the same double expressions the plans use, rounded
// to T: lrow[m] = exp(-4 pi^2 tau ky^2) / N0 (ky the wrapped index m), lcol[w] =
// exp(-4 pi^2 tau kx^2) / N1 for stored slot w (kx = w for w <= c, w - W for
// w >= W - c, every wrapped mode when W = N1; 0 in the unused slots).
template <typename T>
__global__ void static_tables(T* tw0, int N0, T* tw1, int N1, T* lrow, T* lcol, int W, int c, double tau)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const double two_pi = 6.283185307179586476925286766559;
    const double pi = 3.14159265358979323846;
    if (m < N0) {
        tw0[2 * m] = (T)cos(two_pi * (double)m / (double)N0);
        tw0[2 * m + 1] = (T)(-sin(two_pi * (double)m / (double)N0));
        const double k = (2 * m < N0) ? (double)m : (double)(m - N0);
        lrow[m] = (T)(exp(-4.0 * pi * pi * tau * k * k) / (double)N0);
    }
    if (m < N1) {
        tw1[2 * m] = (T)cos(two_pi * (double)m / (double)N1);
        tw1[2 * m + 1] = (T)(-sin(two_pi * (double)m / (double)N1));
    }
    if (m < W) {
        double k = 0.0;
        bool kept = true;
        if (W == N1) k = (2 * m < N1) ? (double)m : (double)(m - N1);
        else if (m <= c) k = (double)m;
        else if (m >= W - c) k = (double)(m - W);
        else kept = false;
        lcol[m] = kept ? (T)(exp(-4.0 * pi * pi * tau * k * k) / (double)N1) : (T)0;
    }
}

// Address of this GPU's array and the device limits, resolved once per device
// with that device current.
mbo_status device_scratch(int dev, DeviceScratch*& out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        mbo::report_static_error("device %d beyond the %d devices mbo_step_static serves", dev, kMaxDevices);
        return MBO_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_setup);
    DeviceScratch& d = g_dev[dev];
    if (!d.ready) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            mbo::report_static_error("hipGetSymbolAddress of the static working memory: %s", hipGetErrorString(e));
            return MBO_ERR_HIP;
        }
        int lds = 0;
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) {
            mbo::report_static_error("hipDeviceGetAttribute: %s", hipGetErrorString(e));
            return MBO_ERR_HIP;
        }
        d.ptr = static_cast<unsigned char*>(ptr);
        d.lds_max = lds > 4096 ? (size_t)lds - 2048 : 65536;  // as a plan sizes it
        d.ready = true;
    }
    out = &d;
    return MBO_OK;
}

#define STATIC_HIP(call)                                                                          \
    do {                                                                                          \
        const hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                                   \
            mbo::report_static_error("%s failed: %s", #call, hipGetErrorString(e_));              \
            return MBO_ERR_HIP;                                                                   \
        }                                                                                         \
    } while (0)

}  // namespace

extern "C" mbo_status mbo_step_static(int64_t N0, int64_t N1, int n, mbo_precision prec, double tau,
                                      double sigma_fallback, const void* A_prev, void* A_next, void* hip_stream)
{
    using namespace mbo;
    int pv = 0;
    static_assert(sizeof(prec) == sizeof(int), "enums of the ABI are int-sized");
    std::memcpy(&pv, &prec, sizeof pv);  // an out-of-range value is rejected, not read as the enum
    if (pv != MBO_F64 && pv != MBO_F32 && pv != MBO_F32_F64FALLBACK) {
        report_static_error("unknown precision %d", pv);
        return MBO_ERR_INVALID_ARG;
    }
    if (n < 1 || n > 4) {
        report_static_error("n = %d not in [1, 4]", n);
        return MBO_ERR_INVALID_ARG;
    }
    if (!(tau > 0.0) || !std::isfinite(tau)) {
        report_static_error("tau must be finite and > 0");
        return MBO_ERR_INVALID_ARG;
    }
    if (!A_prev || !A_next) {
        report_static_error("A_prev / A_next is NULL");
        return MBO_ERR_INVALID_ARG;
    }
    if (A_prev == (const void*)A_next) {
        report_static_error("A_next must not alias A_prev");
        return MBO_ERR_INVALID_ARG;
    }
    if (!pow2_in_range(N0) || !pow2_in_range(N1)) {
        report_static_error("grid %lld x %lld: each axis must be a power of two in [8, 2048]", (long long)N0,
                            (long long)N1);
        return MBO_ERR_UNSUPPORTED;
    }
    int dev = 0;
    STATIC_HIP(hipGetDevice(&dev));
    DeviceScratch* ds = nullptr;
    const mbo_status st = device_scratch(dev, ds);
    if (st != MBO_OK) return st;

    const int pk = pv == MBO_F64 ? 0 : 1;
    const size_t esz = pk ? sizeof(float) : sizeof(double);
    int c = 0, W = 0, tx = 0;
    if (!fast_layout(N0, N1, n, pk, &tau, 1, true, ds->lds_max, 0, &c, &W, &tx)) {
        report_static_error("the band-limited kernels do not serve a %lld x %lld grid with n = %d in this "
                            "precision (a first axis of at least 64 points is needed)",
                            (long long)N0, (long long)N1, n);
        return MBO_ERR_UNSUPPORTED;
    }

    // working memory: twiddles of both axes, the two symbol factors, the kept
    // spectra of the ceil(n^2 / 2) packed planes
    const int PL = (n * n + 1) / 2;
    const size_t o_tw0 = 0;
    const size_t o_tw1 = o_tw0 + align256(2 * esz * (size_t)N0);
    const size_t o_lrow = o_tw1 + align256(2 * esz * (size_t)N1);
    const size_t o_lcol = o_lrow + align256(esz * (size_t)N0);
    const size_t o_z = o_lcol + align256(esz * (size_t)W);
    const size_t need = o_z + 2 * esz * (size_t)PL * (size_t)N0 * (size_t)W;
    if (need > kScratchBytes) {
        report_static_error("a %lld x %lld field with n = %d needs %zu bytes of working memory; the fixed "
                            "array holds %zu (MBO_STEP_STATIC_MAX_BYTES)",
                            (long long)N0, (long long)N1, n, need, kScratchBytes);
        return MBO_ERR_SCRATCH;
    }
    unsigned char* base = ds->ptr;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);

    // dynamic-LDS limits of the two kernel instances (advisory, as for a plan)
    const int lg0 = ilog2i(N0), lg1 = ilog2i(N1);
    {
        FastRowArgs r;
        std::memset(&r, 0, sizeof r);
        (void)launch_row_fast(pk, n, lg1, r, dim3(1), nullptr, true);
        FastColArgs h;
        std::memset(&h, 0, sizeof h);
        (void)launch_heat_fast(pk, lg0, tx, h, dim3(1), nullptr, true);
        (void)hipGetLastError();
    }

    const int tn = (int)(N0 > N1 ? (N0 > W ? N0 : W) : (N1 > W ? N1 : W));
    if (pk) {
        hipLaunchKernelGGL(static_tables<float>, dim3((unsigned)((tn + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<float*>(base + o_tw0), (int)N0, reinterpret_cast<float*>(base + o_tw1),
                           (int)N1, reinterpret_cast<float*>(base + o_lrow),
                           reinterpret_cast<float*>(base + o_lcol), W, c, tau);
    } else {
        hipLaunchKernelGGL(static_tables<double>, dim3((unsigned)((tn + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<double*>(base + o_tw0), (int)N0,
                           reinterpret_cast<double*>(base + o_tw1), (int)N1,
                           reinterpret_cast<double*>(base + o_lrow), reinterpret_cast<double*>(base + o_lcol), W, c,
                           tau);
    }
    STATIC_HIP(hipGetLastError());

    // the kernels and arguments of mbo_step's band-limited path; the forward
    // row pass writes every stored slot, so nothing needs clearing
    FastRowArgs r;
    std::memset(&r, 0, sizeof r);
    r.L = (int)N1;
    r.band = c;
    r.W = W;
    r.rows = N0;
    r.npts = N0 * N1;
    r.tw = base + o_tw1;
    r.Z = base + o_z;
    r.sigma_fb = sigma_fallback > 0.0 ? sigma_fallback : 1e-3;
    r.K = 1;
    const int rpw = row_fast_rows_per_group(lg1);
    const dim3 rg((unsigned)((N0 + rpw - 1) / rpw), 1);
    FastRowArgs r0 = r;
    r0.Ain = A_prev;
    r0.flags = RF_LOAD_REAL | RF_FORWARD;
    STATIC_HIP(launch_row_fast(pk, n, lg1, r0, rg, s));

    FastColArgs h;
    std::memset(&h, 0, sizeof h);
    h.L = (int)N0;
    h.W = W;
    h.tiles = W / tx;
    h.field_elems = (int64_t)PL * N0 * W;
    h.tw = base + o_tw0;
    h.Z = base + o_z;
    h.lam_row = base + o_lrow;
    h.lam_col = base + o_lcol;
    h.xcd_remap = 1;
    h.apply = 1;
    STATIC_HIP(launch_heat_fast(pk, lg0, tx, h, dim3((unsigned)(PL * (W / tx)), 1), s));

    FastRowArgs r1 = r;
    r1.Aout = A_next;
    r1.flags = RF_INVERSE | RF_PROJECT | RF_STORE_REAL;
    if (pv == MBO_F32_F64FALLBACK) r1.flags |= RF_FALLBACK;
    STATIC_HIP(launch_row_fast(pk, n, lg1, r1, rg, s));
    return MBO_OK;
}
