// Volume-preserving MBO on a surface (Osting & Wang, arXiv:1711.01365,
// Section 7, Algorithm 3): Delta E per sample from the diffused field, the
// selection of the samples taken in descending Delta E order (equal values in
// ascending sample index) while their volume weights sum below V, and the
// reassignment of Lemma 7.2 (T+ on the selected samples, T- elsewhere).
//
// The selection is a radix search over the order-preserving keys of Delta E
// (vp_key), 8 bits per pass from the top, on integer weights (exact sums, so
// the cut does not depend on the order of the additions): a pass sums the
// weights of the keys that match the digits found so far per digit (LDS
// histogram per workgroup, non-zero bins added to a global histogram), and one
// workgroup picks the digit where the weight taken from the top reaches what
// is still needed, then clears the histogram.  After the last digit the key
// kstar of the last sample taken is known; a tie scan in ascending index over
// the samples with key kstar finds the last one taken (istar).
#include "mbo_kernels.hpp"

namespace mbo {

__device__ __forceinline__ bool wsel_member(const WSelState& s, unsigned long long key, int64_t idx)
{
    switch (s.mode) {
    case VS_ALL: return true;
    case VS_TIES_PART: return key > s.kstar || (key == s.kstar && idx <= s.istar);
    default: return false;  // VS_NONE (and an unfinished search)
    }
}

// Delta E of every sample from the diffused field D (entry-planar [n*n][m]).
template <typename T, int n>
__global__ void __launch_bounds__(256) surf_vp_key(const SurfVolArgs a)
{
    constexpr int NN = n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ unsigned long long red_u[64];
    unsigned long long bad = 0;
    if (q < a.m) {
        const T* D = reinterpret_cast<const T*>(a.D);
        T av[NN], tp[NN], tm[NN], de;
#pragma unroll
        for (int k = 0; k < NN; ++k) av[k] = D[(int64_t)k * a.m + q];
        bad = !all_finite<T, NN>(av);
        vp_point<T, n>(av, tp, tm, de, a.fallback != 0, a.sigma_fb);
        reinterpret_cast<T*>(a.de)[q] = de;
    }
    bad = block_reduce<OpSum>(bad, red_u);
    if (threadIdx.x == 0 && bad && a.nonfinite) atomicAdd(a.nonfinite, bad);
}

// Start of a selection: the target V and the mode it implies.
__global__ void wsel_init(WSelState* s, long long V, long long total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    s->prefix = 0ull;
    s->kstar = 0ull;
    s->istar = -1;
    s->vrem = V;
    s->mode = V <= 0 ? VS_NONE : (V > total ? VS_ALL : VS_SEARCH);
}

// Weights per next digit of the keys matching the digits found so far.
template <typename T>
__global__ void __launch_bounds__(256) wsel_hist(const SurfVolArgs a, int shift, int first)
{
    if (a.sel->mode != VS_SEARCH) return;
    __shared__ unsigned long long lh[256];
    lh[threadIdx.x] = 0ull;
    __syncthreads();
    const T* de = reinterpret_cast<const T*>(a.de);
    const unsigned long long hi = first ? 0ull : (a.sel->prefix >> (shift + 8));
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.m; q += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long key = vp_key(de[q]);
        if (first || (key >> (shift + 8)) == hi)
            atomicAdd(&lh[(key >> shift) & 255ull], (unsigned long long)a.W[q]);
    }
    __syncthreads();
    const unsigned long long v = lh[threadIdx.x];
    if (v) atomicAdd(&a.hist[threadIdx.x], v);
}

// One workgroup of 256 threads: the digit where the weight taken from the top
// reaches what is still needed; clears the histogram for the next pass.
__global__ void __launch_bounds__(256) wsel_pick(const SurfVolArgs a, int shift, int last)
{
    __shared__ unsigned long long h[256];
    h[threadIdx.x] = a.hist[threadIdx.x];
    a.hist[threadIdx.x] = 0ull;
    __syncthreads();
    if (threadIdx.x != 0 || a.sel->mode != VS_SEARCH) return;
    const long long need = a.sel->vrem;
    long long acc = 0;
    int d = 255;
    for (; d > 0; --d) {
        if (acc + (long long)h[d] >= need) break;
        acc += (long long)h[d];
    }
    a.sel->prefix |= (unsigned long long)d << shift;
    a.sel->vrem = need - acc;
    if (last) a.sel->kstar = a.sel->prefix;
}

// Tie scan, part 1: per chunk of WSEL_CHUNK samples the weight of those with key
// kstar.
template <typename T>
__global__ void __launch_bounds__(256) wsel_tie_sums(const SurfVolArgs a)
{
    __shared__ unsigned long long red_u[64];
    unsigned long long s = 0;
    if (a.sel->mode == VS_SEARCH) {
        const T* de = reinterpret_cast<const T*>(a.de);
        const unsigned long long ks = a.sel->kstar;
        const int64_t c0 = (int64_t)blockIdx.x * WSEL_CHUNK;
        for (int i = threadIdx.x; i < WSEL_CHUNK; i += blockDim.x) {
            const int64_t q = c0 + i;
            if (q < a.m && vp_key(de[q]) == ks) s += (unsigned long long)a.W[q];
        }
    }
    s = block_reduce<OpSum>(s, red_u);
    if (threadIdx.x == 0) a.csum[blockIdx.x] = (long long)s;
}

// Tie scan, part 2 (one workgroup of 256 threads): the chunk where the tie
// weight in ascending index reaches what is still needed, then the sample in
// it (16 consecutive samples per thread, a scan of the thread sums).
template <typename T>
__global__ void __launch_bounds__(256) wsel_tie_pick(const SurfVolArgs a, int nchunks)
{
    __shared__ long long part[256];
    __shared__ long long need_s;
    __shared__ int64_t chunk_s;
    if (a.sel->mode != VS_SEARCH) return;  // uniform
    if (threadIdx.x == 0) {
        long long need = a.sel->vrem, acc = 0;
        int c = 0;
        for (; c < nchunks - 1; ++c) {
            if (acc + a.csum[c] >= need) break;
            acc += a.csum[c];
        }
        need_s = need - acc;
        chunk_s = c;
    }
    __syncthreads();
    const T* de = reinterpret_cast<const T*>(a.de);
    const unsigned long long ks = a.sel->kstar;
    constexpr int PER = WSEL_CHUNK / 256;
    const int64_t q0 = chunk_s * WSEL_CHUNK + (int64_t)threadIdx.x * PER;
    long long s = 0;
    for (int i = 0; i < PER; ++i) {
        const int64_t q = q0 + i;
        if (q < a.m && vp_key(de[q]) == ks) s += a.W[q];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long acc = 0;
        for (int t = 0; t < 256; ++t) {
            const long long v = part[t];
            part[t] = acc;  // exclusive prefix
            acc += v;
        }
    }
    __syncthreads();
    const long long need = need_s, before = part[threadIdx.x];
    if (before < need && before + s >= need) {
        long long acc = before;
        for (int i = 0; i < PER; ++i) {
            const int64_t q = q0 + i;
            if (q < a.m && vp_key(de[q]) == ks) {
                acc += a.W[q];
                if (acc >= need) {
                    a.sel->istar = q;
                    a.sel->mode = VS_TIES_PART;
                    break;
                }
            }
        }
    }
}

// Reassignment: T+ on the selected samples, T- elsewhere, from the diffused
// field D (the candidates recomputed by the same code from the same values as
// the keys); sgn[q] = +1 / -1 records the component taken.
template <typename T, int n>
__global__ void __launch_bounds__(256) surf_vp_apply(const SurfVolArgs a)
{
    constexpr int NN = n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.m) return;
    const T* D = reinterpret_cast<const T*>(a.D);
    T* A = reinterpret_cast<T*>(a.A);
    T av[NN], tp[NN], tm[NN], de;
#pragma unroll
    for (int k = 0; k < NN; ++k) av[k] = D[(int64_t)k * a.m + q];
    vp_point<T, n>(av, tp, tm, de, a.fallback != 0, a.sigma_fb);
    const WSelState s = *a.sel;
    const bool in = wsel_member(s, vp_key(reinterpret_cast<const T*>(a.de)[q]), q);
#pragma unroll
    for (int k = 0; k < NN; ++k) A[(int64_t)k * a.m + q] = in ? tp[k] : tm[k];
    if (a.sgn) a.sgn[q] = in ? (int8_t)1 : (int8_t)-1;
}

template <typename T>
__global__ void __launch_bounds__(256) wsel_mark(const SurfVolArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.m) return;
    const WSelState s = *a.sel;
    a.selected[q] = wsel_member(s, vp_key(reinterpret_cast<const T*>(a.de)[q]), q) ? 1 : 0;
}

template <typename T>
static hipError_t select_t(const SurfVolArgs& a, long long V, long long total, hipStream_t st)
{
    const unsigned nb = (unsigned)((a.m + 255) / 256);
    const unsigned hb = nb < 2048u ? nb : 2048u;
    hipLaunchKernelGGL(wsel_init, dim3(1), dim3(64), 0, st, a.sel, V, total);
    constexpr int BITS = sizeof(T) * 8;
    for (int shift = BITS - 8; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL((wsel_hist<T>), dim3(hb), dim3(256), 0, st, a, shift, shift == BITS - 8 ? 1 : 0);
        hipLaunchKernelGGL(wsel_pick, dim3(1), dim3(256), 0, st, a, shift, shift == 0 ? 1 : 0);
    }
    const int nchunks = (int)((a.m + WSEL_CHUNK - 1) / WSEL_CHUNK);
    hipLaunchKernelGGL((wsel_tie_sums<T>), dim3((unsigned)nchunks), dim3(256), 0, st, a);
    hipLaunchKernelGGL((wsel_tie_pick<T>), dim3(1), dim3(256), 0, st, a, nchunks);
    return hipGetLastError();
}

hipError_t launch_wsel(int prec, const SurfVolArgs& a, long long V, long long total, hipStream_t st)
{
    if (a.m <= 0) return hipSuccess;
    return prec == 0 ? select_t<double>(a, V, total, st) : select_t<float>(a, V, total, st);
}

hipError_t launch_wsel_mark(int prec, const SurfVolArgs& a, hipStream_t st)
{
    if (a.m <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((a.m + 255) / 256);
    if (prec == 0) hipLaunchKernelGGL((wsel_mark<double>), dim3(nb), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((wsel_mark<float>), dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t keys_t(int n, const SurfVolArgs& a, bool apply, hipStream_t st)
{
    const unsigned nb = (unsigned)((a.m + 255) / 256);
#define MBO_SV_CASE(NV)                                                                            \
    case NV:                                                                                       \
        if (apply) hipLaunchKernelGGL((surf_vp_apply<T, NV>), dim3(nb), dim3(256), 0, st, a);     \
        else hipLaunchKernelGGL((surf_vp_key<T, NV>), dim3(nb), dim3(256), 0, st, a);             \
        return hipGetLastError();
    switch (n) {
        MBO_SV_CASE(1)
        MBO_SV_CASE(2)
        MBO_SV_CASE(3)
        MBO_SV_CASE(4)
    }
#undef MBO_SV_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_surf_vp_key(int prec, int n, const SurfVolArgs& a, hipStream_t st)
{
    if (a.m <= 0) return hipSuccess;
    return prec == 0 ? keys_t<double>(n, a, false, st) : keys_t<float>(n, a, false, st);
}

hipError_t launch_surf_vp_apply(int prec, int n, const SurfVolArgs& a, hipStream_t st)
{
    if (a.m <= 0) return hipSuccess;
    return prec == 0 ? keys_t<double>(n, a, true, st) : keys_t<float>(n, a, true, st);
}

}  // namespace mbo
