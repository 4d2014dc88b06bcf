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
// Spreading stores each (bin, plane) tile in a buffer of its own, and a gather
// kernel sums the overlapping tiles of neighbouring bins into the grid (no
// atomics on the grid).
#include "mbo_kernels.hpp"

namespace mbo {

template <typename T>
__device__ __forceinline__ T es_kernel(T z, T invW, T beta)
{
    const T r = z * invW;
    const T s = (T)1 - r * r;
    return s > (T)0 ? exp(beta * (sqrt(s) - (T)1)) : (T)0;
}

// Float: the hardware square root and power of two (about 1 ulp each), with
// exp(x) = 2^(x log2 e).  The exponent lies in [-beta log2 e, 0] (beta <= 28),
// where 2^x is a normal float; the weights' relative error stays near 1e-7,
// the size of the float gridding tolerance, at a third of the operations of
// the correctly rounded library calls.
template <>
__device__ __forceinline__ float es_kernel<float>(float z, float invW, float beta)
{
    const float r = z * invW;
    const float s = 1.0f - r * r;
    const float b2 = beta * 1.4426950408889634f;  // beta log2(e)
    return s > 0.0f ? __builtin_amdgcn_exp2f(b2 * __builtin_amdgcn_sqrtf(s) - b2) : 0.0f;
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

// Store the tile (planar re / im, z pitch TEz) of a (bin, plane) workgroup as
// complex values, natural order, into its slot of the tile buffer; the gather
// kernel sums the overlapping tiles into Z (no atomics on the grid).
template <typename T>
__device__ __forceinline__ void store_tile(const T* tre, const T* tim, int TE, int TEz, const SurfArgs& a, int nb,
                                           int pl)
{
    typedef typename cx<T>::type C;
    const int TE3 = TE * TE * TE;
    C* dst = reinterpret_cast<C*>(a.tiles) + ((size_t)nb * a.PL + pl) * TE3;
    for (int i = threadIdx.x; i < TE3; i += blockDim.x) {
        const int tx = i / (TE * TE), ty = (i / TE) % TE, tz = i % TE;
        const int li = (tx * TE + ty) * TEz + tz;
        C v;
        v.x = tre[li];
        v.y = tim[li];
        dst[i] = v;
    }
}

// One thread per grid point and plane: the sum of the tiles that cover it.
// Along an axis the tiles of bins b cover SURF_BIN b - w/2 .. + TE - 1 (mod Ng),
// so at most ceil(TE / SURF_BIN) bins per axis reach a point.
template <typename T>
__global__ void __launch_bounds__(256) surface_gather(const SurfArgs a, int TE)
{
    typedef typename cx<T>::type C;
    const int Ng = a.Ng, nbx = Ng / SURF_BIN, hw = a.w / 2;
    const int64_t npts = (int64_t)Ng * Ng * Ng;
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= npts) return;
    const int pl = a.pl0 + (int)blockIdx.y;
    const int g[3] = {(int)(gi / ((int64_t)Ng * Ng)), (int)((gi / Ng) % Ng), (int)(gi % Ng)};
    const int K = (TE + SURF_BIN - 1) / SURF_BIN;
    int bb[3][4], tt[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int dd = (g[d] + hw) % Ng;  // offset of the point past the tile start of bin dd / SURF_BIN
        const int b0 = dd / SURF_BIN;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int b = ((b0 - k) % nbx + nbx) % nbx;
            const int t = ((g[d] - (b * SURF_BIN - hw)) % Ng + Ng) % Ng;
            bb[d][k] = b;
            tt[d][k] = (k < K && t < TE) ? t : -1;
        }
    }
    const int TE3 = TE * TE * TE;
    const C* tiles = reinterpret_cast<const C*>(a.tiles);
    T sr = 0, si = 0;
    for (int i = 0; i < K; ++i) {
        if (tt[0][i] < 0) continue;
        for (int j = 0; j < K; ++j) {
            if (tt[1][j] < 0) continue;
            for (int k = 0; k < K; ++k) {
                if (tt[2][k] < 0) continue;
                const int slot = a.binmap[((int64_t)bb[0][i] * nbx + bb[1][j]) * nbx + bb[2][k]];
                if (slot < 0) continue;
                const C v = tiles[((size_t)slot * a.PL + pl) * TE3 + (tt[0][i] * TE + tt[1][j]) * TE + tt[2][k]];
                sr += v.x;
                si += v.y;
            }
        }
    }
    C out;
    out.x = sr;
    out.y = si;
    reinterpret_cast<C*>(a.Z)[(size_t)pl * npts + gi] = out;
}

// floor(n / d) for 0 <= n < 2^32 / d, 2 <= d, from M = ceil(2^32 / d): the
// product n M / 2^32 exceeds n / d by less than n d / 2^32 / d < 1 / d, which
// never reaches the next integer.  d = 1 is passed as M = 0.
__device__ __forceinline__ int fdiv(int n, unsigned M) { return M ? (int)__umulhi((unsigned)n, M) : n; }

// Spreading of whole band cells.  The p^3 samples of a cell are the tensor
// product of p nodes per axis and their weights factor per axis, so the cell's
// contribution to the grid,
//     G[i][j][k] = sum_{a,b,c} Wx[a][i] Wy[b][j] Wz[c][k] v[a][b][c]
// (W_d[a][i]: weight factor of node a times psi at grid point i of axis d),
// is contracted one axis at a time, z, then y, then x, over the U grid points
// per axis that cover the stencils of all its samples.  The workgroup stages a
// chunk of its bin's cells (corners and values) in LDS with coalesced loads;
// then one wave per cell with a private LDS scratch (wave-level ordering only)
// adds the cell block into the bin's tile with LDS atomics on distinct
// addresses.
template <typename T, int P>
__global__ void __launch_bounds__(256) surface_spread_cells(const SurfArgs a, unsigned Mp3, unsigned MU,
                                                            unsigned MpU, unsigned MUU)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int p = P, p3 = P * P * P;
    const int TE = a.TE, TEz = a.TE | 1;
    const int U = a.U, pU = p * U, ppU = p * p * U, pUU = p * U * U, UU = U * U;
    const int CH = a.chunk, cst = 3 + 2 * p3;
    const size_t tsz = (size_t)TE * TE * TEz;
    int64_t* ids = reinterpret_cast<int64_t*>(smem_raw);  // [CH] first sample of each staged cell
    T* tre = reinterpret_cast<T*>(ids + CH);
    T* tim = tre + tsz;
    T* stage = tim + tsz;  // [CH][3 + 2 p^3]: corner, re values, im values
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    T* Ws = stage + (size_t)CH * cst + (size_t)wv * surface_cell_scratch(p, U);  // [3][p][U]
    T* T1 = Ws + 3 * pU;                                                               // [2][p^2][U]
    T* T2 = T1 + 2 * ppU;                                                              // [2][p][U][U]

    const int nb = blockIdx.x, pl = a.pl0 + (int)blockIdx.y;
    const int nn = a.n * a.n, e0 = 2 * pl, e1 = e0 + 1;
    const int hw = a.w / 2;
    const int o[3] = {a.bin[3 * nb] * SURF_BIN - hw, a.bin[3 * nb + 1] * SURF_BIN - hw,
                      a.bin[3 * nb + 2] * SURF_BIN - hw};
    const int64_t c0 = a.start[nb], c1 = a.start[nb + 1];
    const int64_t ncell = a.start[a.nbins];
    const T* corner = reinterpret_cast<const T*>(a.pos);
    const T* A = reinterpret_cast<const T*>(a.A);
    const T* Are = A + (size_t)e0 * a.m;
    const T* Aim = A + (size_t)(e1 < nn ? e1 : e0) * a.m;
    const T beta = (T)a.beta, invh = (T)(1.0 / a.h), y0 = (T)a.y0;
    const T W = (T)a.w * (T)0.5, invW = (T)1 / W;
    T nd[P], nwt[P];
#pragma unroll
    for (int an = 0; an < P; ++an) {
        nd[an] = reinterpret_cast<const T*>(a.nodes)[an];
        nwt[an] = reinterpret_cast<const T*>(a.nwts)[an];
    }

    for (size_t i = threadIdx.x; i < 2 * tsz; i += blockDim.x) tre[i] = (T)0;

    for (int64_t cb = c0; cb < c1; cb += CH) {
        const int nch = (int)(c1 - cb < CH ? c1 - cb : CH);
        __syncthreads();  // the previous chunk is consumed (and the tile cleared)
        for (int i = threadIdx.x; i < nch; i += blockDim.x) ids[i] = a.perm[cb + i] * p3;
        for (int i = threadIdx.x; i < 3 * nch; i += blockDim.x) {
            const int d = i / nch, c = i - d * nch;
            stage[c * cst + d] = corner[d * ncell + cb + c];
        }
        __syncthreads();
        // values, several loads in flight per thread
        const int tot = nch * p3;
        for (int i0 = threadIdx.x; i0 < tot; i0 += 4 * blockDim.x) {
            T vr[4], vi[4];
            int dst[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                const int ii = i < tot ? i : tot - 1;
                const int c = fdiv(ii, Mp3), e = ii - c * p3;
                const int64_t q = ids[c] + e;
                vr[u] = Are[q];
                vi[u] = Aim[q];
                dst[u] = i < tot ? c * cst + 3 + e : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (dst[u] >= 0) {
                    stage[dst[u]] = vr[u];
                    stage[dst[u] + p3] = e1 < nn ? vi[u] : (T)0;
                }
            }
        }
        __syncthreads();
        for (int c = wv; c < nch; c += nwv) {
            const T* cs = stage + c * cst;
            const T* Vr = cs + 3;
            const T* Vi = cs + 3 + p3;
            // union start per axis, relative to the tile: 0 .. SURF_BIN for a
            // cell listed in this bin (the host bins by the same first-node
            // coordinate); clamped so that no access leaves the tile whatever
            // the input
            int r0[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T u0 = (cs[d] + nd[0] - y0) * invh;
                const int rr = (int)ceil(u0 - W) - o[d];
                r0[d] = rr < 0 ? 0 : (rr > TE - U ? TE - U : rr);
            }
            for (int e = lane; e < 3 * pU; e += 64) {
                const int d = fdiv(e, MpU), r = e - d * pU, an = fdiv(r, MU), i = r - an * U;
                T ndv = nd[0], nwv_ = nwt[0];
#pragma unroll
                for (int k = 1; k < P; ++k) {
                    ndv = an == k ? nd[k] : ndv;
                    nwv_ = an == k ? nwt[k] : nwv_;
                }
                const T u = (cs[d] + ndv - y0) * invh;
                Ws[e] = nwv_ * es_kernel<T>((T)(o[d] + r0[d] + i) - u, invW, beta);
            }
            wave_lds_sync();
            // T1[ab][k] = sum_c Wz[c][k] v[ab][c]
            for (int e = lane; e < ppU; e += 64) {
                const int ab = fdiv(e, MU), k = e - ab * U;
                T wz[P], xr[P], xi[P];
#pragma unroll
                for (int c3 = 0; c3 < P; ++c3) {
                    wz[c3] = Ws[(2 * p + c3) * U + k];
                    xr[c3] = Vr[ab * p + c3];
                    xi[c3] = Vi[ab * p + c3];
                }
                T s0 = 0, s1 = 0;
#pragma unroll
                for (int c3 = 0; c3 < P; ++c3) {
                    s0 += wz[c3] * xr[c3];
                    s1 += wz[c3] * xi[c3];
                }
                T1[e] = s0;
                T1[ppU + e] = s1;
            }
            wave_lds_sync();
            // T2[a][j][k] = sum_b Wy[b][j] T1[a b][k]
            for (int e = lane; e < pUU; e += 64) {
                const int an = fdiv(e, MUU), r = e - an * UU, j = fdiv(r, MU), k = r - j * U;
                T wy[P], xr[P], xi[P];
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    wy[b] = Ws[(p + b) * U + j];
                    xr[b] = T1[(an * p + b) * U + k];
                    xi[b] = T1[ppU + (an * p + b) * U + k];
                }
                T s0 = 0, s1 = 0;
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    s0 += wy[b] * xr[b];
                    s1 += wy[b] * xi[b];
                }
                T2[e] = s0;
                T2[pUU + e] = s1;
            }
            wave_lds_sync();
            // G[i][j][k] = sum_a Wx[a][i] T2[a][j][k] into the tile
            for (int e = lane; e < UU; e += 64) {
                const int j = fdiv(e, MU), k = e - j * U;
                T t0[P], t1[P];
#pragma unroll
                for (int an = 0; an < P; ++an) {
                    t0[an] = T2[an * UU + e];
                    t1[an] = T2[pUU + an * UU + e];
                }
                const int base = (r0[0] * TE + (r0[1] + j)) * TEz + r0[2] + k;
#pragma unroll 4
                for (int i = 0; i < U; ++i) {
                    T g0 = 0, g1 = 0;
#pragma unroll
                    for (int an = 0; an < P; ++an) {
                        const T wx = Ws[an * U + i];
                        g0 += wx * t0[an];
                        g1 += wx * t1[an];
                    }
                    const int li = base + i * TE * TEz;
                    atomicAdd(&tre[li], g0);
                    atomicAdd(&tim[li], g1);
                }
            }
            wave_lds_sync();  // the scratch is read before the next cell writes it
        }
    }
    __syncthreads();
    store_tile<T>(tre, tim, TE, TEz, a, nb, pl);
}

// The same spreading without LDS atomics (LDS float atomics run at a small
// fraction of the LDS rate): each thread owns one z-line (x, y) of the bin's
// tile in registers, TE <= SURF_LINE_MAX.  Cells are taken SURF_LINE_CB at a
// time by the whole workgroup: weights, T1 and T2 of every cell of the round
// as above (T2 with its k axis zero-padded by SURF_BIN on the low side and odd
// pitch SURF_LINE_KP, so that a line reads T2[a][y - y0][z - z0] for every z
// without bounds tests), then every line inside a cell's block adds
// sum_a Wx[a][x - x0] T2[a][y - y0][.] to its registers.  Lanes of a wave share
// x rarely and y often, so most T2 reads are broadcasts.
constexpr int SURF_LINE_MAX = 22;                           // tile edge limit (TE^2 <= 512 lines)
constexpr int SURF_LINE_KP = SURF_BIN + SURF_LINE_MAX + 3;  // padded k pitch (odd)

// Reciprocals for fdiv of the line kernel's index splits.
struct LineRecip {
    unsigned p3, U, pU, UU, pU3, ppU, pUU;
};

template <typename T, int P, int LM>
__global__ void __launch_bounds__(512) surface_spread_lines(const SurfArgs a, const LineRecip M)
{
    static_assert(LM <= SURF_LINE_MAX, "line length");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int p = P, p3 = P * P * P, CB = SURF_LINE_CB;
    const int TE = a.TE;
    const int U = a.U, pU = p * U, ppU = p * p * U, pUU = p * U * U, UU = U * U;
    const int CH = a.chunk, cst = 3 + 2 * p3;
    const int tid = threadIdx.x, NT = blockDim.x;
    const int t2p = p * U * SURF_LINE_KP;
    int64_t* ids = reinterpret_cast<int64_t*>(smem_raw);  // [CH]
    T* stage = reinterpret_cast<T*>(ids + CH);           // [CH][3 + 2 p^3]
    T* Ws = stage + (size_t)CH * cst;                    // [CB][3][p][U]
    T* T1 = Ws + CB * 3 * pU;                            // [CB][2][p^2][U]
    T* T2 = T1 + CB * 2 * ppU;                           // [CB][2][p][U][SURF_LINE_KP]

    const int nb = blockIdx.x, pl = a.pl0 + (int)blockIdx.y;
    const int nn = a.n * a.n, e0 = 2 * pl, e1 = e0 + 1;
    const int hw = a.w / 2;
    const int o[3] = {a.bin[3 * nb] * SURF_BIN - hw, a.bin[3 * nb + 1] * SURF_BIN - hw,
                      a.bin[3 * nb + 2] * SURF_BIN - hw};
    const int64_t c0 = a.start[nb], c1 = a.start[nb + 1];
    const int64_t ncell = a.start[a.nbins];
    const T* corner = reinterpret_cast<const T*>(a.pos);
    const T* A = reinterpret_cast<const T*>(a.A);
    const T* Are = A + (size_t)e0 * a.m;
    const T* Aim = A + (size_t)(e1 < nn ? e1 : e0) * a.m;
    const T beta = (T)a.beta, invh = (T)(1.0 / a.h), y0 = (T)a.y0;
    const T W = (T)a.w * (T)0.5, invW = (T)1 / W;
    T nd[P], nwt[P];
#pragma unroll
    for (int an = 0; an < P; ++an) {
        nd[an] = reinterpret_cast<const T*>(a.nodes)[an];
        nwt[an] = reinterpret_cast<const T*>(a.nwts)[an];
    }
    // union start of a staged cell along axis d, relative to the tile (0 ..
    // SURF_BIN for a cell listed in this bin; clamped: see the atomic variant)
    auto start_of = [&](const T* cs, int d) {
        const T u0 = (cs[d] + nd[0] - y0) * invh;
        const int rr = (int)ceil(u0 - W) - o[d];
        return rr < 0 ? 0 : (rr > TE - U ? TE - U : rr);
    };
    // this thread's line: x = tid / TE, y = tid % TE (y fastest)
    const bool owns = tid < TE * TE;
    const int lx = owns ? tid / TE : 0, ly = owns ? tid - (tid / TE) * TE : 0;
    T accr[LM], acci[LM];
#pragma unroll
    for (int z = 0; z < LM; ++z) {
        accr[z] = (T)0;
        acci[z] = (T)0;
    }
    for (int i = tid; i < CB * 2 * t2p; i += NT) T2[i] = (T)0;  // the padding stays zero

    for (int64_t cb = c0; cb < c1; cb += CH) {
        const int nch = (int)(c1 - cb < CH ? c1 - cb : CH);
        __syncthreads();  // the previous chunk is consumed
        for (int i = tid; i < nch; i += NT) ids[i] = a.perm[cb + i] * p3;
        for (int i = tid; i < 3 * nch; i += NT) {
            const int d = i / nch, c = i - d * nch;
            stage[c * cst + d] = corner[d * ncell + cb + c];
        }
        __syncthreads();
        const int tot = nch * p3;
        for (int i0 = tid; i0 < tot; i0 += 4 * NT) {
            T vr[4], vi[4];
            int dst[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * NT;
                const int ii = i < tot ? i : tot - 1;
                const int c = fdiv(ii, M.p3), e = ii - c * p3;
                const int64_t q = ids[c] + e;
                vr[u] = Are[q];
                vi[u] = Aim[q];
                dst[u] = i < tot ? c * cst + 3 + e : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (dst[u] >= 0) {
                    stage[dst[u]] = vr[u];
                    stage[dst[u] + p3] = e1 < nn ? vi[u] : (T)0;
                }
            }
        }
        for (int cr = 0; cr < nch; cr += CB) {
            const int nr = nch - cr < CB ? nch - cr : CB;  // cells of this round
            __syncthreads();  // staged values visible; the previous round's scratch is read
            for (int e = tid; e < nr * 3 * pU; e += NT) {
                const int c = fdiv(e, M.pU3), r3 = e - c * 3 * pU;
                const int d = fdiv(r3, M.pU), r = r3 - d * pU, an = fdiv(r, M.U), i = r - an * U;
                const T* cs = stage + (cr + c) * cst;
                T ndv = nd[0], nwv_ = nwt[0];
#pragma unroll
                for (int k = 1; k < P; ++k) {
                    ndv = an == k ? nd[k] : ndv;
                    nwv_ = an == k ? nwt[k] : nwv_;
                }
                const T u = (cs[d] + ndv - y0) * invh;
                Ws[e] = nwv_ * es_kernel<T>((T)(o[d] + start_of(cs, d) + i) - u, invW, beta);
            }
            __syncthreads();
            for (int e = tid; e < nr * ppU; e += NT) {
                const int c = fdiv(e, M.ppU), r = e - c * ppU, ab = fdiv(r, M.U), k = r - ab * U;
                const T* cs = stage + (cr + c) * cst;
                const T* W3 = Ws + c * 3 * pU;
                T s0 = 0, s1 = 0;
#pragma unroll
                for (int c3 = 0; c3 < P; ++c3) {
                    const T wz = W3[(2 * p + c3) * U + k];
                    s0 += wz * cs[3 + ab * p + c3];
                    s1 += wz * cs[3 + p3 + ab * p + c3];
                }
                T1[c * 2 * ppU + r] = s0;
                T1[c * 2 * ppU + ppU + r] = s1;
            }
            __syncthreads();
            for (int e = tid; e < nr * pUU; e += NT) {
                const int c = fdiv(e, M.pUU), r = e - c * pUU;
                const int an = fdiv(r, M.UU), r2 = r - an * UU, j = fdiv(r2, M.U), k = r2 - j * U;
                const T* W3 = Ws + c * 3 * pU;
                const T* t1 = T1 + c * 2 * ppU;
                T s0 = 0, s1 = 0;
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    const T wy = W3[(p + b) * U + j];
                    s0 += wy * t1[(an * p + b) * U + k];
                    s1 += wy * t1[ppU + (an * p + b) * U + k];
                }
                const int dst = c * 2 * t2p + (an * U + j) * SURF_LINE_KP + SURF_BIN + k;
                T2[dst] = s0;
                T2[t2p + dst] = s1;
            }
            __syncthreads();
            if (owns) {
                for (int c = 0; c < nr; ++c) {
                    const T* cs = stage + (cr + c) * cst;
                    const int ii = lx - start_of(cs, 0), jj = ly - start_of(cs, 1);
                    if (ii >= 0 && ii < U && jj >= 0 && jj < U) {
                        const T* W3 = Ws + c * 3 * pU;
                        T wx[P];
#pragma unroll
                        for (int an = 0; an < P; ++an) wx[an] = W3[an * U + ii];
                        // element z of the line reads T2[.][jj][z - z0] at padded
                        // index SURF_BIN + z - z0 in [0, SURF_BIN + SURF_LINE_MAX)
                        const T* br = T2 + c * 2 * t2p + jj * SURF_LINE_KP + SURF_BIN - start_of(cs, 2);
                        const T* bi = br + t2p;
#pragma unroll
                        for (int z = 0; z < LM; ++z) {
#pragma unroll
                            for (int an = 0; an < P; ++an) {
                                accr[z] += wx[an] * br[an * U * SURF_LINE_KP + z];
                                acci[z] += wx[an] * bi[an * U * SURF_LINE_KP + z];
                            }
                        }
                    }
                }
            }
        }
    }
    // the line into the bin's slot of the tile buffer
    if (owns) {
        typedef typename cx<T>::type C;
        C* dst = reinterpret_cast<C*>(a.tiles) + ((size_t)nb * a.PL + pl) * TE * TE * TE + (size_t)(lx * TE + ly) * TE;
#pragma unroll
        for (int z = 0; z < LM; ++z) {
            if (z < TE) {
                C v;
                v.x = accr[z];
                v.y = acci[z];
                dst[z] = v;
            }
        }
    }
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
    store_tile<T>(tre, tim, TE, TEz, a, nb, pl);
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
        // float: separable (a z sum per (i, j) column, then its x-y weight),
        // fewer VALU operations; double: the product weight per point, which
        // measured faster there
        T sr = 0, si = 0;
        if constexpr (sizeof(T) == 4) {
#pragma unroll 1
            for (int i = 0; i < W2; ++i) {
                T xr = 0, xi = 0;
#pragma unroll
                for (int j = 0; j < W2; ++j) {
                    const int base = ((ix + i) * TE + (iy + j)) * TE + iz;
                    T zr = 0, zi = 0;
#pragma unroll
                    for (int k = 0; k < W2; ++k) {
                        zr += wz[k] * tile[2 * (base + k)];
                        zi += wz[k] * tile[2 * (base + k) + 1];
                    }
                    xr += wy[j] * zr;
                    xi += wy[j] * zi;
                }
                sr += wx[i] * xr;
                si += wx[i] * xi;
            }
        } else {
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

static unsigned recip32(int d) { return d <= 1 ? 0u : (unsigned)(((1ull << 32) + (unsigned long long)d - 1) / d); }

template <typename T, int P>
static hipError_t surf_cells_p(const SurfArgs& a, int waves, hipStream_t st)
{
    const size_t lds = surface_cell_lds(P, a.U, waves, a.chunk, sizeof(T));
    const void* f = reinterpret_cast<const void*>(&surface_spread_cells<T, P>);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((surface_spread_cells<T, P>), dim3((unsigned)a.nbins, (unsigned)(a.pl1 - a.pl0)),
                       dim3(64 * waves), lds, st, a, recip32(P * P * P), recip32(a.U), recip32(P * a.U),
                       recip32(a.U * a.U));
    return hipGetLastError();
}

template <typename T, int P, int LM>
static hipError_t surf_lines_p(const SurfArgs& a, hipStream_t st)
{
    const size_t lds = surface_lines_lds(P, a.U, a.chunk, sizeof(T));
    const void* f = reinterpret_cast<const void*>(&surface_spread_lines<T, P, LM>);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    LineRecip M;
    M.p3 = recip32(P * P * P);
    M.U = recip32(a.U);
    M.pU = recip32(P * a.U);
    M.UU = recip32(a.U * a.U);
    M.pU3 = recip32(3 * P * a.U);
    M.ppU = recip32(P * P * a.U);
    M.pUU = recip32(P * a.U * a.U);
    hipLaunchKernelGGL((surface_spread_lines<T, P, LM>), dim3((unsigned)a.nbins, (unsigned)(a.pl1 - a.pl0)),
                       dim3(512), lds, st, a, M);
    return hipGetLastError();
}

template <typename T>
static hipError_t surf_lines(const SurfArgs& a, hipStream_t st)
{
    if (a.p < 1 || a.p > 4 || a.U < 2 || a.TE != SURF_BIN + a.U || a.TE > SURF_LINE_MAX || a.chunk < 1)
        return hipErrorInvalidValue;
    static_assert(SURF_LINE_KP % 2 == 1 && SURF_LINE_KP >= SURF_BIN + SURF_LINE_MAX, "padded pitch");
    // registers per line: the smallest of 16, 18, 20, 22 slots that holds the tile edge
    const int lm = a.TE <= 16 ? 16 : (a.TE <= 18 ? 18 : (a.TE <= 20 ? 20 : 22));
#define MBO_LINES_P(PP)                                                  \
    switch (lm) {                                                        \
    case 16: return surf_lines_p<T, PP, 16>(a, st);                      \
    case 18: return surf_lines_p<T, PP, 18>(a, st);                      \
    case 20: return surf_lines_p<T, PP, 20>(a, st);                      \
    default: return surf_lines_p<T, PP, 22>(a, st);                      \
    }
    switch (a.p) {
    case 1: MBO_LINES_P(1)
    case 2: MBO_LINES_P(2)
    case 3: MBO_LINES_P(3)
    default: MBO_LINES_P(4)
    }
#undef MBO_LINES_P
}

template <typename T>
static hipError_t surf_cells(const SurfArgs& a, int waves, hipStream_t st)
{
    if (waves == 0) return surf_lines<T>(a, st);
    if (a.p < 1 || a.p > 8 || a.U < 2 || a.TE != SURF_BIN + a.U || waves < 1 || waves > 4 || a.chunk < 1)
        return hipErrorInvalidValue;
    switch (a.p) {
    case 1: return surf_cells_p<T, 1>(a, waves, st);
    case 2: return surf_cells_p<T, 2>(a, waves, st);
    case 3: return surf_cells_p<T, 3>(a, waves, st);
    case 4: return surf_cells_p<T, 4>(a, waves, st);
    case 5: return surf_cells_p<T, 5>(a, waves, st);
    case 6: return surf_cells_p<T, 6>(a, waves, st);
    case 7: return surf_cells_p<T, 7>(a, waves, st);
    default: return surf_cells_p<T, 8>(a, waves, st);
    }
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

hipError_t launch_surface_gather(int prec, const SurfArgs& a, int TE, hipStream_t st)
{
    if (a.pl1 <= a.pl0) return hipSuccess;
    if (TE < 1 || TE > 4 * SURF_BIN || a.Ng < TE + SURF_BIN || a.Ng % SURF_BIN) return hipErrorInvalidValue;
    const int64_t npts = (int64_t)a.Ng * a.Ng * a.Ng;
    const dim3 g((unsigned)((npts + 255) / 256), (unsigned)(a.pl1 - a.pl0));
    if (prec == 0) hipLaunchKernelGGL((surface_gather<double>), g, dim3(256), 0, st, a, TE);
    else hipLaunchKernelGGL((surface_gather<float>), g, dim3(256), 0, st, a, TE);
    return hipGetLastError();
}

hipError_t launch_surface_interp(int prec, const SurfArgs& a, hipStream_t st)
{
    if (a.nbins <= 0 || a.pl1 <= a.pl0) return hipSuccess;
    return prec == 0 ? surf_w<double, false>(a, st) : surf_w<float, false>(a, st);
}

}  // namespace mbo
