// Selection kernels of the volume-preserving step (Section 7 of Osting & Wang,
// arXiv:1711.01365): per field, the n_plus points with the largest Delta E
// (the flat-torus rule of choosing the first n_plus values in descending
// order), equal values taken in ascending point index.
//
// Radix search over order-preserving keys of Delta E (vp_key), SEL_BITS bits
// per pass from the top: a pass histograms the next digit of the keys that
// match the digits found so far (one workgroup per chunk of SEL_CHUNK points,
// LDS histogram, non-zero bins added to the field's global
// histogram), and one workgroup per field then finds the digit holding the
// n_plus-th largest key and clears the histogram.  After the last digit the
// key kstar is known; when only some of the points with key kstar are
// selected, per-chunk counts of those points and a walk through the chunk
// holding the last selected one give its index istar (sel_tie).  Every kernel
// reads the selection state first and returns at once when its field needs no
// more work.
#include <climits>

#include "mbo_kernels.hpp"

namespace mbo {

// Inclusive scan over a 256-thread workgroup (four waves); total receives the
// sum over the workgroup.  Every thread must call it.
__device__ __forceinline__ long long scan256(long long v, long long* sh /* >= 4 */, long long& total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) sh[w] = v;
    __syncthreads();
    long long add = 0;
    for (int i = 0; i < w; ++i) add += sh[i];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();  // sh is free for the next call
    return v + add;
}

template <typename T>
__global__ void __launch_bounds__(256) sel_hist(const SelArgs a, int shift, int bits, int pass)
{
    constexpr int KB = (int)sizeof(T) * 8;
    __shared__ unsigned h[1 << SEL_BITS];
    const int b = blockIdx.y;
    const long long np = a.nplus[b];
    if (np <= 0 || np >= a.npts) return;  // decided without a search
    if (pass > 0 && a.st[b].mode != VS_SEARCH) return;
    const int top = shift + bits;
    const unsigned long long pre = pass > 0 ? a.st[b].kstar : 0ull;
    const int nb = 1 << bits;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const T* v = reinterpret_cast<const T*>(a.dE) + (size_t)b * a.npts;
    const int64_t x0 = (int64_t)blockIdx.x * SEL_CHUNK + threadIdx.x;
    T val[SEL_PER];
#pragma unroll
    for (int k = 0; k < SEL_PER; ++k) {  // every load in flight at once
        const int64_t x = x0 + (int64_t)k * 256;
        val[k] = x < a.npts ? v[x] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < SEL_PER; ++k) {
        const unsigned long long key = vp_key(val[k]);
        if (x0 + (int64_t)k * 256 < a.npts && (top >= KB || (key >> top) == (pre >> top)))
            atomicAdd(&h[(key >> shift) & (unsigned)(nb - 1)], 1u);
    }
    __syncthreads();
    unsigned* g = a.hist + (size_t)b * (1 << SEL_BITS);
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        if (h[i]) atomicAdd(&g[i], h[i]);
}

__global__ void __launch_bounds__(256) sel_pick(const SelArgs a, int shift, int bits, int pass, int last)
{
    __shared__ long long sh[4];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    VpSel* st = a.st + b;
    const long long np = a.nplus[b];
    if (pass == 0) {
        if (np <= 0 || np >= a.npts) {
            if (tid == 0) {
                st->mode = np <= 0 ? VS_NONE : VS_ALL;
                st->kstar = 0ull;
                st->need = 0;
                st->ties = 0;
                st->istar = -1;
            }
            return;
        }
    } else if (st->mode != VS_SEARCH) {
        return;
    }
    const long long need = pass == 0 ? np : st->need;
    const unsigned long long pre = pass == 0 ? 0ull : st->kstar;
    unsigned* g = a.hist + (size_t)b * (1 << SEL_BITS);
    const int nb = 1 << bits;
    const int per = nb >> 8;  // bins per thread (bits >= 9)
    // thread t holds the t-th group of bins from the top, in descending order
    const int hi = nb - 1 - tid * per;
    unsigned c[8];
    long long sum = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        c[i] = i < per ? g[hi - i] : 0u;
        sum += c[i];
    }
    long long total;
    const long long incl = scan256(sum, sh, total);
    const long long excl = incl - sum;
    if (excl < need && need <= incl) {  // exactly one thread
        long long acc = excl;
        int d = hi;
        unsigned cnt = c[0];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i < per && acc + (long long)c[i] >= need) {
                d = hi - i;
                cnt = c[i];
                break;
            }
            acc += c[i];
        }
        const long long rem = need - acc;
        st->kstar = pre | ((unsigned long long)d << shift);
        st->need = rem;
        st->ties = cnt;
        st->mode = VS_SEARCH;
        if (last) {
            st->mode = rem == (long long)cnt ? VS_TIES_ALL : VS_TIES_PART;
            st->istar = rem == (long long)cnt ? LLONG_MAX : -1;
        }
    }
    __syncthreads();  // every bin has been read
    for (int i = tid; i < nb; i += 256) g[i] = 0u;
}

// Points whose key is kstar, per chunk; the workgroup of a field that finishes
// last then finds the chunk holding the need-th of them (in index order) and
// walks it for that point's index.  The per-chunk counts and the finished-
// workgroup counter are only touched by device-scope atomics, performed at the
// device's coherence point for workgroups on every XCD: a workgroup's count is
// performed once its returned value is in (before the barrier that precedes
// the counter), and the last workgroup's atomic reads come after the counter
// told it every other workgroup had counted; no cache write-back is needed.
template <typename T>
__global__ void __launch_bounds__(256) sel_tie(const SelArgs a)
{
    __shared__ long long sh[4];
    __shared__ long long s_chunk, s_rank;
    __shared__ int s_last;
    const int b = blockIdx.y;
    const int tid = threadIdx.x;
    VpSel* st = a.st + b;
    if (st->mode != VS_TIES_PART) return;
    const unsigned long long ks = st->kstar;
    const T* v = reinterpret_cast<const T*>(a.dE) + (size_t)b * a.npts;
    unsigned* tc = a.tcnt + (size_t)b * a.chunks;
    {
        const int64_t x0 = (int64_t)blockIdx.x * SEL_CHUNK + tid;
        T val[SEL_PER];
#pragma unroll
        for (int k = 0; k < SEL_PER; ++k) {
            const int64_t x = x0 + (int64_t)k * 256;
            val[k] = x < a.npts ? v[x] : (T)0;
        }
        long long cnt = 0;
#pragma unroll
        for (int k = 0; k < SEL_PER; ++k) cnt += (x0 + (int64_t)k * 256 < a.npts && vp_key(val[k]) == ks) ? 1 : 0;
        long long total;
        (void)scan256(cnt, sh, total);
        unsigned seen = 0u;
        if (tid == 0) seen = __hip_atomic_exchange(&tc[blockIdx.x], (unsigned)total, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (seen == 0xffffffffu) s_last = 2;  // consumes the returned value (overwritten below)
        __syncthreads();
        if (tid == 0)
            s_last = __hip_atomic_fetch_add(a.done + b, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                             gridDim.x - 1
                         ? 1
                         : 0;
        __syncthreads();
        if (s_last != 1) return;  // uniform
        if (tid == 0) (void)__hip_atomic_exchange(a.done + b, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the last workgroup: the chunk holding the need-th tie ...
    const long long need = st->need;
    const int64_t per = (a.chunks + 255) / 256;
    const int64_t c0 = (int64_t)tid * per;
    const int64_t c1 = c0 + per < a.chunks ? c0 + per : a.chunks;
    long long sum = 0;
    for (int64_t c = c0; c < c1; ++c)
        sum += __hip_atomic_load(&tc[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) {
        s_chunk = -1;
        s_rank = 0;
    }
    long long total;
    const long long incl = scan256(sum, sh, total);  // its barriers order the writes above
    const long long excl = incl - sum;
    if (excl < need && need <= incl) {
        long long acc = excl;
        for (int64_t c = c0; c < c1; ++c) {
            const long long k = __hip_atomic_load(&tc[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (acc + k >= need) {
                s_chunk = c;
                s_rank = need - acc;
                break;
            }
            acc += k;
        }
    }
    __syncthreads();
    const long long chunk = s_chunk, rank = s_rank;
    if (chunk < 0) return;  // uniform
    // ... and the point: walk the chunk in index order
    const int64_t x0 = chunk * SEL_CHUNK;
    const int64_t x1 = x0 + SEL_CHUNK < a.npts ? x0 + SEL_CHUNK : a.npts;
    long long run = 0;
    for (int64_t xb = x0; xb < x1; xb += 256) {
        const int64_t x = xb + tid;
        const long long eq = (x < x1 && vp_key(v[x]) == ks) ? 1 : 0;
        long long tot;
        const long long r = scan256(eq, sh, tot);
        if (eq && run + r == rank) st->istar = x;
        run += tot;
        if (run >= rank) break;  // uniform: tot is the same on every thread
    }
}

template <typename T>
__global__ void __launch_bounds__(256) sel_mark(const SelArgs a)
{
    const int b = blockIdx.y;
    const VpSel s = a.st[b];
    const T* v = reinterpret_cast<const T*>(a.dE) + (size_t)b * a.npts;
    const int64_t x0 = (int64_t)blockIdx.x * SEL_CHUNK;
    const int64_t x1 = x0 + SEL_CHUNK < a.npts ? x0 + SEL_CHUNK : a.npts;
    for (int64_t x = x0 + threadIdx.x; x < x1; x += blockDim.x)
        a.mask[(size_t)b * a.npts + x] = vp_member(s, vp_key(v[x]), x) ? 1 : 0;
}

__global__ void __launch_bounds__(256) count_pos(const int8_t* sgn, int64_t npts, long long* out)
{
    __shared__ long long sh[4];
    const int b = blockIdx.y;
    const int64_t x0 = (int64_t)blockIdx.x * SEL_CHUNK;
    const int64_t x1 = x0 + SEL_CHUNK < npts ? x0 + SEL_CHUNK : npts;
    long long cnt = 0;
    for (int64_t x = x0 + threadIdx.x; x < x1; x += blockDim.x) cnt += sgn[(size_t)b * npts + x] > 0 ? 1 : 0;
    long long total;
    (void)scan256(cnt, sh, total);
    if (threadIdx.x == 0 && total) atomicAdd(reinterpret_cast<unsigned long long*>(out + b), (unsigned long long)total);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t select_t(const SelArgs& a, int batch, hipStream_t st)
{
    // digits from the top: float keys 11 + 11 + 10 bits, double keys 5 x 11 + 9
    static const int fs[3] = {21, 10, 0}, fb[3] = {11, 11, 10};
    static const int ds[6] = {53, 42, 31, 20, 9, 0}, db[6] = {11, 11, 11, 11, 11, 9};
    const bool f = sizeof(T) == 4;
    const int passes = f ? 3 : 6;
    const dim3 gc((unsigned)a.chunks, (unsigned)batch), gb((unsigned)batch), bl(256);
    for (int p = 0; p < passes; ++p) {
        const int sh = f ? fs[p] : ds[p], bi = f ? fb[p] : db[p];
        hipLaunchKernelGGL((sel_hist<T>), gc, bl, 0, st, a, sh, bi, p);
        hipLaunchKernelGGL(sel_pick, gb, bl, 0, st, a, sh, bi, p, p == passes - 1 ? 1 : 0);
    }
    hipLaunchKernelGGL((sel_tie<T>), gc, bl, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_select(int prec, const SelArgs& a, int batch, hipStream_t st)
{
    if (a.chunks <= 0 || batch <= 0) return hipErrorInvalidValue;
    return prec == 0 ? select_t<double>(a, batch, st) : select_t<float>(a, batch, st);
}

hipError_t launch_sel_mark(int prec, const SelArgs& a, int batch, hipStream_t st)
{
    const dim3 gc((unsigned)a.chunks, (unsigned)batch), bl(256);
    if (prec == 0) hipLaunchKernelGGL((sel_mark<double>), gc, bl, 0, st, a);
    else hipLaunchKernelGGL((sel_mark<float>), gc, bl, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_count_pos(const int8_t* sgn, int64_t npts, int batch, long long* out, hipStream_t st)
{
    hipError_t e = launch_fill_u64(reinterpret_cast<unsigned long long*>(out), batch, 0ull, st);
    if (e != hipSuccess) return e;
    const dim3 gc((unsigned)((npts + SEL_CHUNK - 1) / SEL_CHUNK), (unsigned)batch), bl(256);
    hipLaunchKernelGGL(count_pos, gc, bl, 0, st, sgn, npts, out);
    return hipGetLastError();
}

hipError_t launch_row_vp(int prec, int n, int log2L, const RowArgs& a, dim3 grid, dim3 block, size_t lds,
                         hipStream_t st, bool prepare)
{
    return prec == 0 ? launch_row_vp_f64(n, log2L, a, grid, block, lds, st, prepare)
                     : launch_row_vp_f32(n, log2L, a, grid, block, lds, st, prepare);
}

}  // namespace mbo
