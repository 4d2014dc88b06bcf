// Spreading and interpolation kernels of the surface diffusion step (the
// closest point method of Osting & Wang, arXiv:1711.01365, Section 5.2, whose
// free-space heat convolution is evaluated here through a periodic Cartesian
// grid: spread the samples, transform, multiply, transform back, interpolate).
//
// Kernel psi(z) = exp(beta (sqrt(1 - (z / W)^2) - 1)) for |z| < W = w / 2 grid
// units ("exponential of semicircle", Barnett, Magland and af Klinteberg,
// SIAM J. Sci. Comput. 2019): a sample at grid coordinate u touches the w grid
// points i0 .. i0 + w - 1 per axis, i0 = ceil(u - W).  Work comes sorted by bin
// (SURF_BIN^3 grid points); the workgroup of a (bin, plane) accumulates into,
// or reads from, an LDS tile that covers every stencil of its bin's work.
// Spreading adds the tiles to the grid with atomics (tiles of neighbouring bins
// overlap).
#include "mbo_kernels.hpp"

namespace mbo {

template <typename T>
__device__ __forceinline__ T es_kernel(T z, T invW, T beta)
{
    const T r = z * invW;
    const T s = (T)1 - r * r;
    return s > (T)0 ? exp(beta * (sqrt(s) - (T)1)) : (T)0;
}

// Stencil start i0 and the w weights of one axis for grid coordinate u.
template <typename T, int W2>
__device__ __forceinline__ int es_weights(T u, T beta, T (&wt)[W2])
{
    const T half = (T)W2 * (T)0.5;
    const int i0 = (int)ceil(u - half);
    const T invW = (T)1 / half;
#pragma unroll
    for (int a = 0; a < W2; ++a) wt[a] = es_kernel<T>((T)(i0 + a) - u, invW, beta);
    return i0;
}

__device__ __forceinline__ int tile_off(int i) { return i < 0 ? 0 : (i > SURF_BIN ? SURF_BIN : i); }

__device__ __forceinline__ int64_t wrap(int64_t g, int64_t N) { return ((g % N) + N) % N; }

// Add the tile (planar re / im, z pitch TEz) of grid origin (ox, oy, oz) into
// plane pl of Z, wrapping periodically; zeros are skipped.
template <typename T>
__device__ __forceinline__ void flush_tile(const T* tre, const T* tim, int TE, int TEz, int ox, int oy, int oz,
                                           const SurfArgs& a, int pl)
{
    typedef typename cx<T>::type C;
    C* Z = reinterpret_cast<C*>(a.Z);
    const int64_t Ng = a.Ng, npts = Ng * Ng * Ng;
    const int TE3 = TE * TE * TE;
    for (int i = threadIdx.x; i < TE3; i += blockDim.x) {
        const int tx = i / (TE * TE), ty = (i / TE) % TE, tz = i % TE;
        const int li = (tx * TE + ty) * TEz + tz;
        const T vr = tre[li], vi = tim[li];
        const int64_t g = (wrap(ox + tx, Ng) * Ng + wrap(oy + ty, Ng)) * Ng + wrap(oz + tz, Ng);
        C* zp = Z + (size_t)pl * npts + g;
        if (vr != (T)0) atomicAdd(&zp->x, vr);
        if (vi != (T)0) atomicAdd(&zp->y, vi);
    }
}

// Spreading of whole band cells.  The p^3 samples of a cell are the tensor
// product of p nodes per axis and their weights factor per axis, so the cell's
// contribution to the grid,
//     G[i][j][k] = sum_{a,b,c} Wx[a][i] Wy[b][j] Wz[c][k] v[a][b][c]
// (W_d[a][i]: weight factor of node a times psi at grid point i of axis d),
// is contracted one axis at a time, z, then y, then x, over the U grid points
// per axis that cover the stencils of all its samples.  One wave per cell with
// a private LDS scratch (wave-level ordering only); the cell block is added
// into the bin's tile with LDS atomics on distinct addresses.
template <typename T>
__global__ void __launch_bounds__(256) surface_spread_cells(const SurfArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int PM = 8;  // nodes per axis at most
    const int TE = a.TE, TEz = a.TE | 1;
    const int U = a.U, p = a.p, p3 = p * p * p, pU = p * U, ppU = p * p * U, pUU = p * U * U;
    const size_t tsz = (size_t)TE * TE * TEz;
    T* tre = reinterpret_cast<T*>(smem_raw);
    T* tim = tre + tsz;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    T* Ws = tim + tsz + (size_t)wv * surface_cell_scratch(p, U);  // [3][p][U]
    T* Vs = Ws + 3 * pU;                                          // [2][p^3]
    T* T1 = Vs + 2 * p3;                                          // [2][p^2][U]
    T* T2 = T1 + 2 * ppU;                                         // [2][p][U][U]

    const int nb = blockIdx.x, pl = a.pl0 + (int)blockIdx.y;
    const int nn = a.n * a.n, e0 = 2 * pl, e1 = e0 + 1;
    const int hw = a.w / 2;
    const int o[3] = {a.bin[3 * nb] * SURF_BIN - hw, a.bin[3 * nb + 1] * SURF_BIN - hw,
                      a.bin[3 * nb + 2] * SURF_BIN - hw};
    const int64_t c0 = a.start[nb], c1 = a.start[nb + 1];
    const int64_t ncell = a.start[a.nbins];
    const T* corner = reinterpret_cast<const T*>(a.pos);
    const T* nodes = reinterpret_cast<const T*>(a.nodes);
    const T* nwts = reinterpret_cast<const T*>(a.nwts);
    const T* A = reinterpret_cast<const T*>(a.A);
    const T beta = (T)a.beta, invh = (T)(1.0 / a.h), y0 = (T)a.y0;
    const T W = (T)a.w * (T)0.5, invW = (T)1 / W;

    for (size_t i = threadIdx.x; i < 2 * tsz; i += blockDim.x) tre[i] = (T)0;
    __syncthreads();

    for (int64_t ci = c0 + wv; ci < c1; ci += nwv) {
        const int64_t q0 = a.perm[ci] * p3;
        const T cxyz[3] = {corner[ci], corner[ncell + ci], corner[2 * ncell + ci]};
        // union start per axis, relative to the tile: 0 .. SURF_BIN for a cell
        // listed in this bin (the host bins by the same first-node coordinate);
        // clamped so that no access leaves the tile whatever the input
        int r0[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T u0 = (cxyz[d] + nodes[0] - y0) * invh;
            const int rr = (int)ceil(u0 - W) - o[d];
            r0[d] = rr < 0 ? 0 : (rr > TE - U ? TE - U : rr);
        }
        for (int e = lane; e < 3 * pU; e += 64) {
            const int d = e / pU, r = e - d * pU, an = r / U, i = r - an * U;
            const T u = (cxyz[d] + nodes[an] - y0) * invh;
            Ws[e] = nwts[an] * es_kernel<T>((T)(o[d] + r0[d] + i) - u, invW, beta);
        }
        for (int e = lane; e < p3; e += 64) {
            Vs[e] = A[(size_t)e0 * a.m + q0 + e];
            Vs[p3 + e] = e1 < nn ? A[(size_t)e1 * a.m + q0 + e] : (T)0;
        }
        wave_lds_sync();
        // T1[ab][k] = sum_c Wz[c][k] v[ab][c]
        for (int e = lane; e < ppU; e += 64) {
            const int ab = e / U, k = e - ab * U;
            T s0 = 0, s1 = 0;
            for (int c = 0; c < p; ++c) {
                const T wz = Ws[(2 * p + c) * U + k];
                s0 += wz * Vs[ab * p + c];
                s1 += wz * Vs[p3 + ab * p + c];
            }
            T1[e] = s0;
            T1[ppU + e] = s1;
        }
        wave_lds_sync();
        // T2[a][j][k] = sum_b Wy[b][j] T1[a b][k]
        for (int e = lane; e < pUU; e += 64) {
            const int an = e / (U * U), r = e - an * U * U, j = r / U, k = r - j * U;
            T s0 = 0, s1 = 0;
            for (int b = 0; b < p; ++b) {
                const T wy = Ws[(p + b) * U + j];
                s0 += wy * T1[(an * p + b) * U + k];
                s1 += wy * T1[ppU + (an * p + b) * U + k];
            }
            T2[e] = s0;
            T2[pUU + e] = s1;
        }
        wave_lds_sync();
        // G[i][j][k] = sum_a Wx[a][i] T2[a][j][k] into the tile
        for (int e = lane; e < U * U; e += 64) {
            const int j = e / U, k = e - j * U;
            T t0[PM], t1[PM];
#pragma unroll
            for (int an = 0; an < PM; ++an) {
                t0[an] = an < p ? T2[an * U * U + e] : (T)0;
                t1[an] = an < p ? T2[pUU + an * U * U + e] : (T)0;
            }
            const size_t base = ((size_t)r0[0] * TE + (r0[1] + j)) * TEz + r0[2] + k;
            for (int i = 0; i < U; ++i) {
                T g0 = 0, g1 = 0;
#pragma unroll
                for (int an = 0; an < PM; ++an) {
                    if (an < p) {
                        const T wx = Ws[an * U + i];
                        g0 += wx * t0[an];
                        g1 += wx * t1[an];
                    }
                }
                const size_t li = base + (size_t)i * TE * TEz;
                if (g0 != (T)0) atomicAdd(&tre[li], g0);
                if (g1 != (T)0) atomicAdd(&tim[li], g1);
            }
        }
        wave_lds_sync();  // the scratch is read before the next cell writes it
    }
    __syncthreads();
    flush_tile<T>(tre, tim, TE, TEz, o[0], o[1], o[2], a, pl);
}

// Spreading one sample at a time (cells whose stencil union is too wide for
// the cell kernel's LDS): the w^3 stencil of each sample into the tile.
template <typename T, int W2>
__global__ void __launch_bounds__(256) surface_spread(const SurfArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TE = SURF_BIN + W2;
    constexpr int TEz = TE | 1;
    constexpr int TSZ = TE * TE * TEz;
    T* tre = reinterpret_cast<T*>(smem_raw);
    T* tim = tre + TSZ;
    const int nb = blockIdx.x, pl = a.pl0 + (int)blockIdx.y;
    const int ox = a.bin[3 * nb] * SURF_BIN - W2 / 2, oy = a.bin[3 * nb + 1] * SURF_BIN - W2 / 2,
              oz = a.bin[3 * nb + 2] * SURF_BIN - W2 / 2;
    const int nn = a.n * a.n, e0 = 2 * pl, e1 = e0 + 1;
    const int64_t s0 = a.start[nb], s1 = a.start[nb + 1];
    const T* pos = reinterpret_cast<const T*>(a.pos);
    const T* wts = reinterpret_cast<const T*>(a.wts);
    const T* A = reinterpret_cast<const T*>(a.A);
    const T beta = (T)a.beta, invh = (T)(1.0 / a.h), y0 = (T)a.y0;
    for (int i = threadIdx.x; i < 2 * TSZ; i += blockDim.x) tre[i] = (T)0;
    __syncthreads();
    for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const int64_t q = a.perm[s];
        T wx[W2], wy[W2], wz[W2];
        // stencil offsets in the tile: 0 .. SURF_BIN for a sample of this bin
        // (the host bins by the same coordinates); clamped so that no access
        // leaves the tile whatever the input
        const int ix = tile_off(es_weights<T, W2>((pos[s] - y0) * invh, beta, wx) - ox);
        const int iy = tile_off(es_weights<T, W2>((pos[a.m + s] - y0) * invh, beta, wy) - oy);
        const int iz = tile_off(es_weights<T, W2>((pos[2 * a.m + s] - y0) * invh, beta, wz) - oz);
        const T wq = wts ? wts[s] : (T)1;
        const T vr = wq * A[(size_t)e0 * a.m + q];
        const T vi = e1 < nn ? wq * A[(size_t)e1 * a.m + q] : (T)0;
#pragma unroll 1
        for (int i = 0; i < W2; ++i)
#pragma unroll
            for (int j = 0; j < W2; ++j) {
                const T wij = wx[i] * wy[j];
                const int base = ((ix + i) * TE + (iy + j)) * TEz + iz;
#pragma unroll
                for (int k = 0; k < W2; ++k) {
                    const T wt = wij * wz[k];
                    atomicAdd(&tre[base + k], wt * vr);
                    atomicAdd(&tim[base + k], wt * vi);
                }
            }
    }
    __syncthreads();
    flush_tile<T>(tre, tim, TE, TEz, ox, oy, oz, a, pl);
}

template <typename T, int W2>
__global__ void __launch_bounds__(256) surface_interp(const SurfArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TE = SURF_BIN + W2;
    constexpr int TE3 = TE * TE * TE;
    T* tile = reinterpret_cast<T*>(smem_raw);
    typedef typename cx<T>::type C;
    const int nb = blockIdx.x;
    const int bx = a.bin[3 * nb], by = a.bin[3 * nb + 1], bz = a.bin[3 * nb + 2];
    const int ox = bx * SURF_BIN - W2 / 2, oy = by * SURF_BIN - W2 / 2, oz = bz * SURF_BIN - W2 / 2;
    const int pl = a.pl0 + (int)blockIdx.y;
    const int nn = a.n * a.n;
    const int64_t Ng = a.Ng, npts = Ng * Ng * Ng;
    const C* Z = reinterpret_cast<const C*>(a.Z) + (size_t)pl * npts;
    for (int i = threadIdx.x; i < TE3; i += blockDim.x) {
        const int tx = i / (TE * TE), ty = (i / TE) % TE, tz = i % TE;
        const C v = Z[(wrap(ox + tx, Ng) * Ng + wrap(oy + ty, Ng)) * Ng + wrap(oz + tz, Ng)];
        tile[2 * i] = v.x;
        tile[2 * i + 1] = v.y;
    }
    __syncthreads();
    const int64_t s0 = a.start[nb], s1 = a.start[nb + 1];
    const T* pos = reinterpret_cast<const T*>(a.pos);
    T* out = reinterpret_cast<T*>(a.out);
    const T beta = (T)a.beta, invh = (T)(1.0 / a.h), y0 = (T)a.y0;
    for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const int64_t q = a.perm[s];
        T wx[W2], wy[W2], wz[W2];
        // stencil offsets in the tile: 0 .. SURF_BIN for a sample of this bin
        // (the host bins by the same coordinates); clamped so that no access
        // leaves the tile whatever the input
        const int ix = tile_off(es_weights<T, W2>((pos[s] - y0) * invh, beta, wx) - ox);
        const int iy = tile_off(es_weights<T, W2>((pos[a.m + s] - y0) * invh, beta, wy) - oy);
        const int iz = tile_off(es_weights<T, W2>((pos[2 * a.m + s] - y0) * invh, beta, wz) - oz);
        T sr = 0, si = 0;
#pragma unroll 1
        for (int i = 0; i < W2; ++i)
#pragma unroll
            for (int j = 0; j < W2; ++j) {
                const T wij = wx[i] * wy[j];
                const int base = ((ix + i) * TE + (iy + j)) * TE + iz;
#pragma unroll
                for (int k = 0; k < W2; ++k) {
                    const T wt = wij * wz[k];
                    sr += wt * tile[2 * (base + k)];
                    si += wt * tile[2 * (base + k) + 1];
                }
            }
        const int e0 = 2 * pl, e1 = e0 + 1;
        out[(size_t)e0 * a.m + q] = sr;
        if (e1 < nn) out[(size_t)e1 * a.m + q] = si;
    }
}

template <typename T, bool SPREAD>
static hipError_t surf_w(const SurfArgs& a, hipStream_t st)
{
    const size_t te = (size_t)(SURF_BIN + a.w);
    const size_t lds = (SPREAD ? 2 * te * te * (te | 1) : 2 * te * te * te) * sizeof(T);
    const dim3 g((unsigned)a.nbins, (unsigned)(a.pl1 - a.pl0)), bl(256);
#define MBO_SURF_CASE(WW)                                                                            \
    case WW: {                                                                                       \
        const void* f = SPREAD ? reinterpret_cast<const void*>(&surface_spread<T, WW>)              \
                               : reinterpret_cast<const void*>(&surface_interp<T, WW>);             \
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        if (e != hipSuccess) return e;                                                               \
        if (SPREAD) hipLaunchKernelGGL((surface_spread<T, WW>), g, bl, lds, st, a);                  \
        else hipLaunchKernelGGL((surface_interp<T, WW>), g, bl, lds, st, a);                         \
        return hipGetLastError();                                                                    \
    }
    switch (a.w) {
        MBO_SURF_CASE(3)
        MBO_SURF_CASE(4)
        MBO_SURF_CASE(5)
        MBO_SURF_CASE(6)
        MBO_SURF_CASE(7)
        MBO_SURF_CASE(8)
        MBO_SURF_CASE(9)
        MBO_SURF_CASE(10)
        MBO_SURF_CASE(11)
        MBO_SURF_CASE(12)
    }
#undef MBO_SURF_CASE
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t surf_cells(const SurfArgs& a, int waves, hipStream_t st)
{
    if (a.p < 1 || a.p > 8 || a.U < 1 || a.TE != SURF_BIN + a.U || waves < 1 || waves > 4)
        return hipErrorInvalidValue;
    const size_t lds = surface_cell_lds(a.p, a.U, waves, sizeof(T));
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&surface_spread_cells<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((surface_spread_cells<T>), dim3((unsigned)a.nbins, (unsigned)(a.pl1 - a.pl0)),
                       dim3(64 * waves), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_surface_spread(int prec, const SurfArgs& a, hipStream_t st)
{
    if (a.nbins <= 0 || a.pl1 <= a.pl0) return hipSuccess;
    return prec == 0 ? surf_w<double, true>(a, st) : surf_w<float, true>(a, st);
}

hipError_t launch_surface_spread_cells(int prec, const SurfArgs& a, int waves, hipStream_t st)
{
    if (a.nbins <= 0 || a.pl1 <= a.pl0) return hipSuccess;
    return prec == 0 ? surf_cells<double>(a, waves, st) : surf_cells<float>(a, waves, st);
}

hipError_t launch_surface_interp(int prec, const SurfArgs& a, hipStream_t st)
{
    if (a.nbins <= 0 || a.pl1 <= a.pl0) return hipSuccess;
    return prec == 0 ? surf_w<double, false>(a, st) : surf_w<float, false>(a, st);
}

}  // namespace mbo
