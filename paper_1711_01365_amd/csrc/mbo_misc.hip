// Pointwise and utility kernels of libmbo (gfx950): standalone projection
// (Lemma 1.1) and its vector-Jacobian product, graph-capture-safe fills, the
// fixed-order energy and dot-product reductions, and
// the dispatch of the row / strided-axis passes to their translation units.
#include "mbo_kernels.hpp"

namespace mbo {

// ---------------------------------------------------------------------------
// Standalone projection, one point per thread
// ---------------------------------------------------------------------------
template <typename T, int n>
__global__ void __launch_bounds__(256) project_kernel(const ProjArgs a)
{
    constexpr int NN = n * n;
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ unsigned long long red_u[64];
    unsigned long long bad = 0, fb = 0;
    if (p < a.npts) {
        const T* A = reinterpret_cast<const T*>(a.A) + field_base(a.foff, b, NN * a.npts);
        T* Q = reinterpret_cast<T*>(a.Q) + field_base(a.foff, b, NN * a.npts);
        T av[NN], qv[NN];
#pragma unroll
        for (int k = 0; k < NN; ++k) av[k] = A[(int64_t)k * a.npts + p];
        bad = !all_finite<T, NN>(av);
        int ds;
        fb = project_point_fb<T, n>(av, qv, ds, a.fallback != 0, a.sigma_fb) ? 1ull : 0ull;
#pragma unroll
        for (int k = 0; k < NN; ++k) Q[(int64_t)k * a.npts + p] = qv[k];
        if (a.dsign) a.dsign[(size_t)b * a.npts + p] = (int8_t)ds;
    }
    bad = block_reduce<OpSum>(bad, red_u);
    if (threadIdx.x == 0 && bad) atomicAdd(a.nonfinite, bad);
    fb = block_reduce<OpSum>(fb, red_u);
    if (threadIdx.x == 0 && fb && a.fallbacks) atomicAdd(a.fallbacks, fb);
}

// ---------------------------------------------------------------------------
// Vector-Jacobian product of the projection, one point per thread.  Float
// plans with the double fallback redo points whose smallest singular value is
// below the threshold in double, as the forward projection does.
// ---------------------------------------------------------------------------
template <typename T, int n>
__global__ void __launch_bounds__(256) vjp_kernel(const VjpArgs a)
{
    constexpr int NN = n * n;
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ unsigned long long red_u[64];
    unsigned long long bad = 0;
    if (p < a.npts) {
        const T* A = reinterpret_cast<const T*>(a.A) + (size_t)b * NN * a.npts;
        const T* G = reinterpret_cast<const T*>(a.G) + (size_t)b * NN * a.npts;
        T* GA = reinterpret_cast<T*>(a.GA) + (size_t)b * NN * a.npts;
        T av[NN], gv[NN], ov[NN];
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            av[k] = A[(int64_t)k * a.npts + p];
            gv[k] = G[(int64_t)k * a.npts + p];
        }
        bad = !all_finite<T, NN>(av);
        if constexpr (n == 1) {
            ov[0] = 0;  // sign thresholding is locally constant
        } else {
            const T smin = polar_vjp<T, n>(av, gv, ov);
            if constexpr (sizeof(T) == 4) {
                if (a.fallback && (double)smin < a.sigma_fb) {
                    double ad[NN], gd[NN], od[NN];
#pragma unroll
                    for (int k = 0; k < NN; ++k) {
                        ad[k] = av[k];
                        gd[k] = gv[k];
                    }
                    (void)polar_vjp<double, n>(ad, gd, od);
#pragma unroll
                    for (int k = 0; k < NN; ++k) ov[k] = (T)od[k];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NN; ++k) GA[(int64_t)k * a.npts + p] = ov[k];
    }
    bad = block_reduce<OpSum>(bad, red_u);
    if (threadIdx.x == 0 && bad) atomicAdd(a.nonfinite, bad);
}

// out[b] (+)= fixed-order sum of the m partials of field b (one workgroup per field)
__global__ void __launch_bounds__(256) sum_rows(const double* part, int64_t m, double* out, int accumulate)
{
    __shared__ double red_d[64];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) acc += part[(int64_t)b * m + i];
    acc = block_reduce<OpSum>(acc, red_d);
    if (threadIdx.x == 0) out[b] = accumulate ? out[b] + acc : acc;
}

// ---------------------------------------------------------------------------
// Small utility kernels (graph-capture safe replacements for memset)
// ---------------------------------------------------------------------------
// Index of the first-column field of a 2-D O(2) field (Section 6.1): for loop
// l (axis 0: column l, the loop wrapping once in x; axis 1: row l, once in y),
// the sum over consecutive samples (the last joined to the first) of the angle
// from one first column to the next in (-pi, pi], divided by 2 pi.  One
// workgroup per loop and field; the FP64 sum runs in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) so2_index_kernel(const T* A, int64_t N0, int64_t N1, int axis, double* out)
{
    __shared__ double red_d[64];
    const int b = blockIdx.y;
    const int64_t loop = blockIdx.x;
    const int64_t npts = N0 * N1;
    const T* c0 = A + (size_t)b * 4 * npts;  // entry (0, 0)
    const T* c1 = c0 + 2 * npts;             // entry (1, 0)
    const int64_t L = axis == 0 ? N0 : N1;
    const int64_t stride = axis == 0 ? N1 : 1;
    const int64_t base = axis == 0 ? loop : loop * N1;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < L; k += blockDim.x) {
        const int64_t p = base + k * stride;
        const int64_t q = base + (k + 1 == L ? 0 : k + 1) * stride;
        const double u = (double)c0[p], v = (double)c1[p], un = (double)c0[q], vn = (double)c1[q];
        acc += atan2(u * vn - v * un, u * un + v * vn);
    }
    acc = block_reduce<OpSum>(acc, red_d);
    if (threadIdx.x == 0) out[(size_t)b * gridDim.x + loop] = acc / 6.283185307179586476925286766559;
}

// Pointwise penalty of the relaxed energies, summed per workgroup in double:
// kind 1 |A - U V^t|_F^2 / 2 (= sum (sigma_i - 1)^2 / 2, Lemma 1.1), kind 3
// |A^t A - I|_F^2 / 4.
template <typename T, int n>
__global__ void __launch_bounds__(256) penalty_kernel(const T* A, int64_t npts, int kind, double* part)
{
    __shared__ double red_d[64];
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (p < npts) {
        double a[n * n];
#pragma unroll
        for (int k = 0; k < n * n; ++k) a[k] = (double)A[((size_t)b * n * n + k) * npts + p];
        if (kind == 1) {
            double q[n * n], smin;
            int ds;
            project_point<double, n>(a, q, ds, smin);
#pragma unroll
            for (int k = 0; k < n * n; ++k) s += (a[k] - q[k]) * (a[k] - q[k]);
            s *= 0.5;
        } else {
#pragma unroll
            for (int i = 0; i < n; ++i)
#pragma unroll
                for (int j = 0; j < n; ++j) {
                    double m = 0.0;
#pragma unroll
                    for (int k = 0; k < n; ++k) m += a[k * n + i] * a[k * n + j];
                    m -= (i == j ? 1.0 : 0.0);
                    s += m * m;
                }
            s *= 0.25;
        }
    }
    s = block_reduce<OpSum>(s, red_d);
    if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = s;
}

__global__ void fill_u64(unsigned long long* p, int64_t count, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// splitmix64 (Steele, Lea and Flood, 2014) of seed + index, top 53 bits as a
// double in [0, 1), mapped to [-1, 1)
template <typename T>
__global__ void fill_uniform(T* p, int64_t count, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = (T)(2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0);
}

__global__ void fill_i32(int* p, int64_t count, int v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// E(A_s) = (1/tau) (n - (1/npts) sum_wg partial), the partials being
// sum_m symbol(m)/npts |Z(m)|^2 over each workgroup's modes.
// One workgroup per (field, iterate) slot; the partials are summed in a fixed
// order (strided per thread, then the fixed tree of block_reduce).
__global__ void __launch_bounds__(256) reduce_energy(const ReduceArgs a)
{
    __shared__ double red_d[64];
    const int64_t idx = blockIdx.x;
    const int b = (int)(idx / (a.K + 1));
    const int s = (int)(idx - (int64_t)b * (a.K + 1));
    if (a.stop_iter && s > a.stop_iter[b]) return;  // uniform per workgroup
    const double* p = a.epart + idx * a.nwg;
    double sum = 0.0;
    for (int i = threadIdx.x; i < a.nwg; i += blockDim.x) sum += p[i];
    sum = block_reduce<OpSum>(sum, red_d);
    if (threadIdx.x == 0)
        a.energy[idx] = ((double)a.n - sum / (double)a.npts) / (a.taus ? a.taus[b] : a.tau);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_row(int prec, int n, int log2L, const RowArgs& a, dim3 g, dim3 bl, size_t lds,
                      hipStream_t st, bool prepare, hipEvent_t ev0, hipEvent_t ev1)
{
    return prec == 0 ? launch_row_f64(n, log2L, a, g, bl, lds, st, prepare, ev0, ev1)
                     : launch_row_f32(n, log2L, a, g, bl, lds, st, prepare, ev0, ev1);
}

hipError_t launch_col(int prec, int mode, int log2L, const ColArgs& a, dim3 g, dim3 bl, size_t lds,
                      hipStream_t st, bool prepare, hipEvent_t ev0, hipEvent_t ev1)
{
    return prec == 0 ? launch_col_f64(mode, log2L, a, g, bl, lds, st, prepare, ev0, ev1)
                     : launch_col_f32(mode, log2L, a, g, bl, lds, st, prepare, ev0, ev1);
}

template <typename T>
static hipError_t proj_dispatch(int n, const ProjArgs& a, int batch, hipStream_t st)
{
    dim3 bl(256);
    dim3 g((unsigned)((a.npts + 255) / 256), (unsigned)batch);
    switch (n) {
    case 1: hipLaunchKernelGGL((project_kernel<T, 1>), g, bl, 0, st, a); break;
    case 2: hipLaunchKernelGGL((project_kernel<T, 2>), g, bl, 0, st, a); break;
    case 3: hipLaunchKernelGGL((project_kernel<T, 3>), g, bl, 0, st, a); break;
    case 4: hipLaunchKernelGGL((project_kernel<T, 4>), g, bl, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_project(int prec, int n, const ProjArgs& a, int batch, hipStream_t st)
{
    return prec == 0 ? proj_dispatch<double>(n, a, batch, st) : proj_dispatch<float>(n, a, batch, st);
}

template <typename T>
static hipError_t vjp_dispatch(int n, const VjpArgs& a, int batch, hipStream_t st)
{
    dim3 bl(256);
    dim3 g((unsigned)((a.npts + 255) / 256), (unsigned)batch);
    switch (n) {
    case 1: hipLaunchKernelGGL((vjp_kernel<T, 1>), g, bl, 0, st, a); break;
    case 2: hipLaunchKernelGGL((vjp_kernel<T, 2>), g, bl, 0, st, a); break;
    case 3: hipLaunchKernelGGL((vjp_kernel<T, 3>), g, bl, 0, st, a); break;
    case 4: hipLaunchKernelGGL((vjp_kernel<T, 4>), g, bl, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_vjp(int prec, int n, const VjpArgs& a, int batch, hipStream_t st)
{
    return prec == 0 ? vjp_dispatch<double>(n, a, batch, st) : vjp_dispatch<float>(n, a, batch, st);
}

hipError_t launch_penalty(int prec, int n, const void* A, int64_t npts, int batch, int kind, double* part,
                          hipStream_t st)
{
    const dim3 g((unsigned)((npts + 255) / 256), (unsigned)batch), bl(256);
#define MBO_PEN(T, N)                                                                          \
    hipLaunchKernelGGL((penalty_kernel<T, N>), g, bl, 0, st, (const T*)A, npts, kind, part); \
    break;
    if (prec == 0) {
        switch (n) {
        case 1: MBO_PEN(double, 1)
        case 2: MBO_PEN(double, 2)
        case 3: MBO_PEN(double, 3)
        case 4: MBO_PEN(double, 4)
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (n) {
        case 1: MBO_PEN(float, 1)
        case 2: MBO_PEN(float, 2)
        case 3: MBO_PEN(float, 3)
        case 4: MBO_PEN(float, 4)
        default: return hipErrorInvalidValue;
        }
    }
#undef MBO_PEN
    return hipGetLastError();
}

hipError_t launch_row_relax(int prec, int n, int log2L, const RowArgs& a, dim3 grid, dim3 block, size_t lds,
                            hipStream_t st, bool prepare)
{
    return prec == 0 ? launch_row_relax_f64(n, log2L, a, grid, block, lds, st, prepare)
                     : launch_row_relax_f32(n, log2L, a, grid, block, lds, st, prepare);
}

hipError_t launch_so2_index(int prec, const void* A, int64_t N0, int64_t N1, int batch, int axis, double* out,
                            hipStream_t st)
{
    const dim3 g((unsigned)(axis == 0 ? N1 : N0), (unsigned)batch), bl(256);
    if (prec == 0)
        hipLaunchKernelGGL((so2_index_kernel<double>), g, bl, 0, st, (const double*)A, N0, N1, axis, out);
    else
        hipLaunchKernelGGL((so2_index_kernel<float>), g, bl, 0, st, (const float*)A, N0, N1, axis, out);
    return hipGetLastError();
}

hipError_t launch_sum_rows(const double* part, int64_t m, int batch, double* out, hipStream_t st,
                           bool accumulate)
{
    hipLaunchKernelGGL(sum_rows, dim3((unsigned)batch), dim3(256), 0, st, part, m, out, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_uniform(int prec, void* p, int64_t count, uint64_t seed, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const dim3 g((unsigned)((count + 255) / 256));
    if (prec == 0) hipLaunchKernelGGL(fill_uniform<double>, g, dim3(256), 0, st, (double*)p, count, seed);
    else hipLaunchKernelGGL(fill_uniform<float>, g, dim3(256), 0, st, (float*)p, count, seed);
    return hipGetLastError();
}

// One workgroup per (field, iteration): the sums of the unpacked counts of
// every row-pass workgroup, in a fixed order.
__global__ void __launch_bounds__(256) sum_counts(const unsigned long long* part, int nwg, int K,
                                                  unsigned long long* flips, unsigned long long* fallbacks,
                                                  unsigned long long* nonfinite)
{
    __shared__ unsigned long long sh[3][256];
    const int64_t slot = blockIdx.x;  // b * K + s
    const unsigned long long* pp = part + slot * (int64_t)nwg;
    const unsigned long long m21 = (1ull << 21) - 1;
    unsigned long long f = 0, fb = 0, bad = 0;
    for (int i = threadIdx.x; i < nwg; i += 256) {
        const unsigned long long v = pp[i];
        f += v & m21;
        fb += (v >> 21) & m21;
        bad += v >> 42;
    }
    sh[0][threadIdx.x] = f;
    sh[1][threadIdx.x] = fb;
    sh[2][threadIdx.x] = bad;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        flips[slot] = sh[0][0];
        fallbacks[slot] = sh[1][0];
        nonfinite[slot] = sh[2][0];
    }
}

hipError_t launch_sum_counts(const unsigned long long* part, int nwg, int K, int batch, unsigned long long* flips,
                             unsigned long long* fallbacks, unsigned long long* nonfinite, hipStream_t st)
{
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(sum_counts, dim3((unsigned)((int64_t)batch * K)), dim3(256), 0, st, part, nwg, K, flips,
                       fallbacks, nonfinite);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st)
{
    const int64_t total = (int64_t)a.batch * (a.K + 1);
    hipLaunchKernelGGL(reduce_energy, dim3((unsigned)total), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace mbo
