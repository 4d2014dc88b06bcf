// HIP kernel templates of the generalized MBO iteration (Osting & Wang,
// arXiv:1711.01365) for gfx950.  Instantiated by the mbo_*.hip translation units.
//
//   row_pass   one workgroup owns whole rows (the contiguous grid axis) of all
//              ceil(n^2/2) packed complex planes of a field: inverse row FFT,
//              per-point projection onto O(n) (Lemma 1.1, Algorithm 1 step 2)
//              with det-sign / fallback / change diagnostics, forward row FFT.
//              Two real entry planes travel as one complex plane z = A_p + i A_q;
//              this is exact because the heat symbol is real and even in k.
//   col_pass   FFT along a strided axis for a tile of TX neighbouring inner
//              indices (coalesced TX-wide segments, staged through LDS when a
//              line fits in one wave).  CM_HEAT fuses forward FFT -> heat symbol
//              exp(-4 pi^2 tau |k|^2) (Section 5.1) and the Lyapunov partial
//              sum_m symbol |Z|^2 (Section 4) -> inverse FFT.
#pragma once

#include <type_traits>

#include "mbo_device.hpp"
#include "mbo_internal.hpp"
#include "mbo_volume.hpp"

namespace mbo {

// ---------------------------------------------------------------------------
// Deterministic workgroup reductions (result valid in thread 0).  blockDim.x is
// a power of two; waves reduce by xor-shuffles in a fixed pattern, then wave
// totals (or, for workgroups smaller than a wave, all values) by an LDS tree.
// ---------------------------------------------------------------------------
struct OpSum {
    template <typename V> __device__ static V apply(V a, V b) { return a + b; }
};
struct OpMax {
    template <typename V> __device__ static V apply(V a, V b) { return a > b ? a : b; }
};

template <typename Op, typename V>
__device__ V block_reduce(V v, V* sh /* >= 64 entries */)
{
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    if (nt >= 64) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = Op::apply(v, (V)__shfl_xor(v, o, 64));
        const int nw = nt >> 6;
        __syncthreads();
        if ((tid & 63) == 0) sh[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            V s = sh[0];
            for (int w = 1; w < nw; ++w) s = Op::apply(s, sh[w]);
            v = s;
        }
        return v;
    }
    __syncthreads();
    sh[tid] = v;
    __syncthreads();
    for (int h = nt >> 1; h > 0; h >>= 1) {
        if (tid < h) sh[tid] = Op::apply(sh[tid], sh[tid + h]);
        __syncthreads();
    }
    return sh[0];
}

// Sum over the 64 lanes of a wave (butterfly order, the same on every lane).
template <typename V>
__device__ __forceinline__ V wave_sum(V v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (V)__shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Row pass.  A workgroup owns rpw rows (contiguous grid lines of length L) of
// every packed plane: rpw * PL "lines".  Phase 1: groups of L/8 threads load
// one line each (a round at a time), inverse-FFT it, and leave it in natural
// order in LDS (line j at lr/li[j * lds_plane + lds_pad(x)]).  For L <= 512 a
// group lies inside one wave and its exchanges need no workgroup barrier.  Phase 2: every
// thread takes points of the rows (one point per thread and pass over the
// rpw*L points) for the projection and its diagnostics.  Phase 3: the groups
// forward-FFT the lines from LDS and store the spectra.  The projection, which
// dominates the arithmetic, thus runs one point per thread on all threads.
// ---------------------------------------------------------------------------
// One line of L complex values moved between global memory (contiguous, from
// zline) and LDS (natural order, lr/li[lds_pad(x)]) by the L/8 threads of its
// group, 16 bytes per access; consecutive threads take consecutive vectors.
template <typename T, int LOG2L, bool TO_LDS>
__device__ __forceinline__ void line_stage(typename cx<T>::type* zline, T* lr, T* li, int t)
{
    constexpr int L = 1 << LOG2L;
    constexpr int Tn = L / 8;
    constexpr int EPV = sizeof(T) == 4 ? 2 : 1;  // complex values per access
    constexpr int VPT = 8 / EPV;                 // accesses per thread
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
    V* zv = reinterpret_cast<V*>(zline);
    const int x0 = t * EPV, px0 = lds_pad(x0);
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
        const int a = lds_pad_at<Tn * EPV>(x0, px0, v);  // element x0 + v * Tn * EPV
        if constexpr (TO_LDS) {
            const V w = zv[v * Tn + t];
            if constexpr (EPV == 2) {
                lr[a] = w.x;
                li[a] = w.y;
                lr[a + 1] = w.z;  // x0 is even: x0 + 1 gets no extra padding
                li[a + 1] = w.w;
            } else {
                lr[a] = w.x;
                li[a] = w.y;
            }
        } else {
            V w;
            if constexpr (EPV == 2) {
                w.x = lr[a];
                w.y = li[a];
                w.z = lr[a + 1];
                w.w = li[a + 1];
            } else {
                w.x = lr[a];
                w.y = li[a];
            }
            zv[v * Tn + t] = w;
        }
    }
}

// Waves per SIMD the row pass is compiled for: float rows of up to 512 points
// and n <= 3 are held to 128 VGPRs, so that two 512-thread workgroups share a
// compute unit.
// The volume-preserving and relaxed-flow instances are not held (the first
// evaluates both candidates of a point, the second carries the projection's
// double path inline).
template <typename T, int n, int LOG2L, int RM = RM_MBO>
constexpr int row_waves_per_simd() { return (RM == RM_MBO && sizeof(T) == 4 && n <= 3 && LOG2L <= 9) ? 4 : 1; }

// RM_MBO: Algorithm 1 (flags RF_PROJECT ...); RM_VOLUME: the volume-preserving
// step of Section 7 in two launches, RF_VP_KEY (Delta E of every point) and,
// after the selection, RF_VP_APPLY (T+ or T- per point); RM_RELAX: the explicit
// reaction step of the relaxed gradient flows GD-1 / GD-3 (RF_RELAX).
template <typename T, int n, int LOG2L, int RM = RM_MBO>
__global__ void __launch_bounds__(512, (row_waves_per_simd<T, n, LOG2L, RM>())) row_pass(const RowArgs a)
{
    constexpr bool VP = RM == RM_VOLUME;
    constexpr bool RELAX = RM == RM_RELAX;
    constexpr int NN = n * n;
    constexpr int PL = (NN + 1) / 2;
    typedef FftShape<LOG2L> F;
    constexpr int L = F::L;
    constexpr int Tn = F::Tn;
    typedef typename cx<T>::type C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red_d[64];

    const int flags = a.flags;
    const int b = blockIdx.y;
    if ((flags & RF_CHECK_STOP) && a.stop_iter[b] < a.iter) return;  // uniform per workgroup

    const int tid = threadIdx.x;
    const int NT = blockDim.x;
    const int G = NT >> (LOG2L - 3);  // line groups
    const int g = tid >> (LOG2L - 3);
    const int t = tid & (Tn - 1);
    const int rpw = a.rpw;
    const int nlines = rpw * PL;
    const int rounds = (nlines + G - 1) / G;
    const int64_t row0 = (int64_t)blockIdx.x * rpw;
    const int64_t npts = a.npts;
    const int lp = a.lds_plane;
    T* lr = reinterpret_cast<T*>(smem_raw);
    T* li = lr + (size_t)nlines * lp;

    // fallback queue of phase 2 (see there); its counter is cleared before the
    // first workgroup barrier
    constexpr bool DEFER = !VP && sizeof(T) == 4 && n >= 3;
    constexpr int QCAP = DEFER ? row_fb_queue_len(LOG2L) : 1;
    constexpr int SCAP = DEFER ? ROW_FB_STASH : 1;
    __shared__ unsigned short fq[QCAP];
    __shared__ float fv[SCAP * NN];
    __shared__ int fq_n;
    // per-workgroup counters (packed counts, max change bits, waves done)
    __shared__ unsigned long long wg_cnt[3];
    if (tid == 0) {
        if (DEFER) fq_n = 0;
        wg_cnt[0] = 0;
        wg_cnt[1] = 0;
        wg_cnt[2] = 0;
    }
    bool lds_synced = false;  // no LDS write since the last workgroup barrier

    // ---- phase 1: lines into LDS (natural order), inverse FFT on the way
    C* Zb = reinterpret_cast<C*>(a.Z) + (size_t)b * PL * npts;
    const bool staged = LOG2L <= 9 && !(flags & RF_LOAD_REAL);
    if constexpr (LOG2L <= 9) {
        if (staged) {
            // each line group stages its own line through LDS (16-byte
            // accesses) and transforms it in place: only wave-level ordering
            Twiddles<T, LOG2L> tw;
            if (flags & RF_INVERSE) load_twiddles<T, LOG2L>(tw, reinterpret_cast<const C*>(a.tw), t);
            const int pt = lds_pad(t);
            for (int rd = 0; rd < rounds; ++rd) {
                const int j = rd * G + g;
                const bool act = j < nlines;
                const int rloc = j / PL, pl = j - (j / PL) * PL;
                T* lrj = lr + (size_t)(act ? j : 0) * lp;
                T* lij = li + (size_t)(act ? j : 0) * lp;
                if (act && row0 + rloc < a.rows)
                    line_stage<T, LOG2L, true>(Zb + (int64_t)pl * npts + (row0 + rloc) * L, lrj, lij, t);
                wave_lds_sync();
                if (flags & RF_INVERSE) {
                    T r[8], im[8];
                    if (act) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            r[e] = lrj[lds_pad_at<Tn>(t, pt, e)];
                            im[e] = lij[lds_pad_at<Tn>(t, pt, e)];
                        }
                    }
                    fft_wave<T, +1, LOG2L>(r, im, lrj, lij, t, tw, act);
                    wave_lds_sync();  // the line's last exchange has been read
                    if (act) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            lrj[lds_pad_at<Tn>(t, pt, e)] = r[e];
                            lij[lds_pad_at<Tn>(t, pt, e)] = im[e];
                        }
                    }
                }
            }
        }
    }
    for (int rd = 0; rd < (staged ? 0 : rounds); ++rd) {
        const int j = rd * G + g;
        const int rloc = j / PL, pl = j - (j / PL) * PL;
        const bool act = j < nlines;
        const bool ld = act && row0 + rloc < a.rows;
        const int64_t x0 = (row0 + rloc) * L + t;
        T r[1][8], im[1][8];
        if (flags & RF_LOAD_REAL) {
            const T* A = reinterpret_cast<const T*>(a.Ain) + field_base(a.foff, b, NN * npts);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t x = x0 + (int64_t)e * Tn;
                r[0][e] = ld ? A[(int64_t)(2 * pl) * npts + x] : (T)0;
                im[0][e] = (ld && 2 * pl + 1 < NN) ? A[(int64_t)(2 * pl + 1) * npts + x] : (T)0;
            }
        } else {
            const C* Z = reinterpret_cast<const C*>(a.Z) + ((size_t)b * PL + pl) * npts;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                C v;
                if (ld) v = Z[x0 + (int64_t)e * Tn];
                else { v.x = 0; v.y = 0; }
                r[0][e] = v.x;
                im[0][e] = v.y;
            }
        }
        T* lrj = lr + (size_t)(act ? j : 0) * lp;
        T* lij = li + (size_t)(act ? j : 0) * lp;
        if (flags & RF_INVERSE) {
            Twiddles<T, LOG2L> tw;
            load_twiddles<T, LOG2L>(tw, reinterpret_cast<const C*>(a.tw), t);
            if constexpr (LOG2L <= 9) {
                fft_wave<T, +1, LOG2L>(r[0], im[0], lrj, lij, t, tw, act);
                wave_lds_sync();  // the line's last exchange has been read
            } else {
                fft_lines<T, +1, 1, LOG2L>(r, im, lrj, lij, 0, 1, 0, t, tw, act);
                __syncthreads();  // the group has read its last exchange
            }
        }
        if (act) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                lrj[lds_pad_at<Tn>(t, lds_pad(t), e)] = r[0][e];
                lij[lds_pad_at<Tn>(t, lds_pad(t), e)] = im[0][e];
            }
        }
    }
    __syncthreads();

    // ---- phase 2: per-point work, one point per thread and pass
    // Float plans with the double fallback (n >= 3) queue the points whose
    // smallest singular value is small (index, and the float V for the warm
    // start) and re-project them in double after the pass loop, when the float
    // state is dead: the double code then neither adds to the registers of the
    // loop nor runs once per wave that holds such a point.
    unsigned long long nflip = 0, nfb = 0, nbad = 0;
    double dmax = 0.0, dacc = 0.0;
    if (flags & (RF_PROJECT | RF_SIGN_INIT | RF_STORE_REAL | RF_DOT | RF_VP_KEY | RF_VP_APPLY | RF_RELAX)) {
        T* Aout = reinterpret_cast<T*>(a.Aout) + field_base(a.foff, b, NN * npts);
        int8_t* sgn = a.sgn + (size_t)b * npts;
        const bool defer = DEFER && (flags & RF_PROJECT) && (flags & RF_FALLBACK);
        // diagnostics and write-back of a projected point
        auto finish = [&](int64_t x, T* lrr, T* lir, const T (&qv)[NN], int ds, int8_t s_old) {
            if (flags & RF_SIGN) {
                nflip += (s_old != (int8_t)ds) ? 1ull : 0ull;
                sgn[x] = (int8_t)ds;
            }
            if (flags & RF_TRACK) {
                // max |A_s - A_{s-1}|, A_{s-1} read from the caller's field
#pragma unroll
                for (int k = 0; k < NN; ++k) {
                    const double dv = fabs((double)qv[k] - (double)Aout[(int64_t)k * npts + x]);
                    dmax = dv > dmax ? dv : dmax;
                }
            }
#pragma unroll
            for (int k = 0; k < NN; ++k) {
                if (k & 1) lir[(k >> 1) * lp] = qv[k];
                else lrr[(k >> 1) * lp] = qv[k];
            }
            if (NN & 1) lir[(NN >> 1) * lp] = (T)0;
        };
        const int npass = (rpw * L + NT - 1) / NT;
#pragma unroll 1
        for (int pp = 0; pp < npass; ++pp) {
            const int idx = pp * NT + tid;
            if (idx >= rpw * L) continue;  // last pass when NT does not divide the points
            const int rloc = idx >> LOG2L;
            const int xc = idx & (L - 1);
            const int64_t row = row0 + rloc;
            if (row >= a.rows) continue;
            const int64_t x = row * L + xc;
            const int jx = lds_pad(xc);
            T* lrr = lr + (size_t)rloc * PL * lp + jx;
            T* lir = li + (size_t)rloc * PL * lp + jx;
            // previous det sign, loaded before the projection hides its latency
            const int8_t s_old = (flags & RF_SIGN) ? sgn[x] : (int8_t)0;
            T av[NN];
#pragma unroll
            for (int k = 0; k < NN; ++k) av[k] = (k & 1) ? lir[(k >> 1) * lp] : lrr[(k >> 1) * lp];
            if (flags & RF_SIGN_INIT) sgn[x] = det_n<T, n>(av) >= (T)0 ? 1 : -1;
            if (flags & RF_DOT) {
                const T* Gd = reinterpret_cast<const T*>(a.Gdot) + field_base(a.foff, b, NN * npts);
#pragma unroll
                for (int k = 0; k < NN; ++k) dacc += (double)Gd[(int64_t)k * npts + x] * (double)av[k];
            }
            if constexpr (VP) {
                // Section 7: both candidates and Delta E (recomputed identically
                // by the two launches); the keying launch stores Delta E, the
                // applying one takes T+ for the selected points and T- elsewhere
                if (flags & (RF_VP_KEY | RF_VP_APPLY)) {
                    T tp[NN], tm[NN], de;
                    const bool fb = vp_point<T, n>(av, tp, tm, de, (flags & RF_FALLBACK) != 0, a.sigma_fb);
                    T* vde = reinterpret_cast<T*>(a.vde) + (size_t)b * npts;
                    if (flags & RF_VP_KEY) vde[x] = de;
                    if (flags & RF_VP_APPLY) {
                        nbad += all_finite<T, NN>(av) ? 0ull : 1ull;
                        nfb += fb ? 1ull : 0ull;
                        const bool in = vp_member(a.vsel[b], vp_key(vde[x]), x);
                        T qv[NN];
#pragma unroll
                        for (int k = 0; k < NN; ++k) qv[k] = in ? tp[k] : tm[k];
                        finish(x, lrr, lir, qv, in ? 1 : -1, s_old);
#pragma unroll
                        for (int k = 0; k < NN; ++k) av[k] = qv[k];
                    }
                }
            }
            if constexpr (RELAX) {
                // dA/dt = Delta A - eps^-2 N(A), reaction step A - c N(A), c = dt / eps^2:
                // GD-1 N(A) = U (Sigma - I) V^t = A - U V^t, GD-3 N(A) = A (A^t A - I)
                if (flags & RF_RELAX) {
                    nbad += all_finite<T, NN>(av) ? 0ull : 1ull;
                    const T c = (T)a.relax_c;
                    T qv[NN];
                    if (a.relax_kind == 1) {
                        int ds;
                        if (project_point_fb<T, n>(av, qv, ds, (flags & RF_FALLBACK) != 0, a.sigma_fb)) ++nfb;
#pragma unroll
                        for (int k = 0; k < NN; ++k) qv[k] = av[k] - c * (av[k] - qv[k]);
                    } else {
                        T m[NN];
#pragma unroll
                        for (int i = 0; i < n; ++i)
#pragma unroll
                            for (int j = 0; j < n; ++j) {
                                T v = 0;
#pragma unroll
                                for (int k = 0; k < n; ++k) v += av[k * n + i] * av[k * n + j];
                                m[i * n + j] = v - (i == j ? (T)1 : (T)0);
                            }
#pragma unroll
                        for (int i = 0; i < n; ++i)
#pragma unroll
                            for (int j = 0; j < n; ++j) {
                                T v = 0;
#pragma unroll
                                for (int k = 0; k < n; ++k) v += av[i * n + k] * m[k * n + j];
                                qv[i * n + j] = av[i * n + j] - c * v;
                            }
                    }
                    finish(x, lrr, lir, qv, 1, s_old);
#pragma unroll
                    for (int k = 0; k < NN; ++k) av[k] = qv[k];
                }
            }
            if (RM == RM_MBO && (flags & RF_PROJECT)) {
                nbad += all_finite<T, NN>(av) ? 0ull : 1ull;
                T qv[NN];
                int ds;
                bool queued = false;
                if constexpr (DEFER) {
                    bool newton = false;
                    if constexpr (n >= 3) newton = polar_newton<float, n>(av, qv, ds, (float)a.sigma_fb);
                    if (newton) {
                    } else if (defer) {
                        float V[n][n];
                        queued = polar_jacobi_f32_fb<n>(av, qv, ds, V, a.sigma_fb);
                        if (queued) {
                            const int s = atomicAdd(&fq_n, 1);
                            fq[s] = (unsigned short)idx;
                            if (s < SCAP) {
#pragma unroll
                                for (int k = 0; k < NN; ++k) fv[s * NN + k] = V[k / n][k % n];
                            }
                        }
                    } else {
                        T smin;
                        project_point<T, n>(av, qv, ds, smin);
                    }
                } else {
                    if (project_point_fb<T, n>(av, qv, ds, (flags & RF_FALLBACK) != 0, a.sigma_fb))
                        ++nfb;
                }
                if (queued) continue;
                finish(x, lrr, lir, qv, ds, s_old);
#pragma unroll
                for (int k = 0; k < NN; ++k) av[k] = qv[k];
            }
            if (flags & RF_STORE_REAL) {
#pragma unroll
                for (int k = 0; k < NN; ++k) Aout[(int64_t)k * npts + x] = av[k];
            }
        }
        if constexpr (DEFER) {
            if (defer) {
                __syncthreads();
                const int nq = fq_n;
                lds_synced = nq == 0;  // uniform: read after the barrier
#pragma unroll 1
                for (int qi = tid; qi < nq; qi += NT) {
                    const int idx = fq[qi];
                    const int rloc = idx >> LOG2L;
                    const int jx = lds_pad(idx & (L - 1));
                    const int64_t x = (row0 + rloc) * L + (idx & (L - 1));
                    T* lrr = lr + (size_t)rloc * PL * lp + jx;
                    T* lir = li + (size_t)rloc * PL * lp + jx;
                    float aq[NN];
                    float V[n][n];
#pragma unroll
                    for (int k = 0; k < NN; ++k) {
                        aq[k] = (k & 1) ? lir[(k >> 1) * lp] : lrr[(k >> 1) * lp];
                        // points beyond the stash start from V = I (a cold start)
                        V[k / n][k % n] = qi < SCAP ? fv[qi * NN + k] : (k / n == k % n ? 1.0f : 0.0f);
                    }
                    int ds;
                    T qv[NN];
                    polar_jacobi_warm<n>(aq, V, qv, ds);
                    ++nfb;
                    finish(x, lrr, lir, qv, ds, (flags & RF_SIGN) ? sgn[x] : (int8_t)0);
                    if (flags & RF_STORE_REAL) {
#pragma unroll
                        for (int k = 0; k < NN; ++k) Aout[(int64_t)k * npts + x] = qv[k];
                    }
                }
            }
        }
    }

    if constexpr (RELAX) {
        if (flags & RF_STORE_Z) {
            // the lines as they stand in LDS (after the inverse transform) back to Z
            __syncthreads();
            for (int rd = 0; rd < rounds; ++rd) {
                const int j = rd * G + g;
                const int rloc = j / PL, pl = j - (j / PL) * PL;
                if (j < nlines && row0 + rloc < a.rows) {
                    const T* lrj = lr + (size_t)j * lp;
                    const T* lij = li + (size_t)j * lp;
                    C* Z = reinterpret_cast<C*>(a.Z) + ((size_t)b * PL + pl) * npts + (row0 + rloc) * L;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        C v;
                        v.x = lrj[lds_pad_at<Tn>(t, lds_pad(t), e)];
                        v.y = lij[lds_pad_at<Tn>(t, lds_pad(t), e)];
                        Z[t + e * Tn] = v;
                    }
                }
            }
        }
    }

    // ---- phase 3: forward FFT of the lines, store the spectra
    if (flags & RF_FORWARD) {
        // twiddles are (re)loaded here rather than kept in registers through
        // the projection
        Twiddles<T, LOG2L> tw;
        load_twiddles<T, LOG2L>(tw, reinterpret_cast<const C*>(a.tw), t);
        if (!lds_synced) __syncthreads();
        for (int rd = 0; rd < rounds; ++rd) {
            const int j = rd * G + g;
            const int rloc = j / PL, pl = j - (j / PL) * PL;
            const bool act = j < nlines;
            const bool st = act && row0 + rloc < a.rows && LOG2L > 9;
            T* lrj = lr + (size_t)(act ? j : 0) * lp;
            T* lij = li + (size_t)(act ? j : 0) * lp;
            T r[1][8], im[1][8];
            if (act) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    r[0][e] = lrj[lds_pad_at<Tn>(t, lds_pad(t), e)];
                    im[0][e] = lij[lds_pad_at<Tn>(t, lds_pad(t), e)];
                }
            }
            if constexpr (LOG2L <= 9) {
                // back to LDS in natural order, then the group stores its line
                fft_wave<T, -1, LOG2L>(r[0], im[0], lrj, lij, t, tw, act);
                wave_lds_sync();
                if (act) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        lrj[lds_pad_at<Tn>(t, lds_pad(t), e)] = r[0][e];
                        lij[lds_pad_at<Tn>(t, lds_pad(t), e)] = im[0][e];
                    }
                }
                wave_lds_sync();
                if (act && row0 + rloc < a.rows)
                    line_stage<T, LOG2L, false>(Zb + (int64_t)pl * npts + (row0 + rloc) * L, lrj, lij, t);
            } else {
                fft_lines<T, -1, 1, LOG2L>(r, im, lrj, lij, 0, 1, 0, t, tw, act);
            }
            if (st) {
                C* Z = reinterpret_cast<C*>(a.Z) + ((size_t)b * PL + pl) * npts;
                const int64_t x0 = (row0 + rloc) * L + t;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    C v;
                    v.x = r[0][e];
                    v.y = im[0][e];
                    Z[x0 + (int64_t)e * Tn] = v;
                }
            }
        }
    }

    if (flags & RF_DOT) {
        dacc = block_reduce<OpSum>(dacc, red_d);
        if (tid == 0) a.dpart[(int64_t)b * gridDim.x + blockIdx.x] = dacc;
    }
    if (flags & (RF_PROJECT | RF_VP_APPLY | RF_RELAX)) {
        // The three counts of a workgroup are below 2^21 each and travel packed;
        // each wave adds its sums to the workgroup's LDS counters, and the last
        // wave to finish (the release/acquire on the done counter orders every
        // other wave's additions before it) adds the totals to the logs.  No
        // workgroup barrier: waves leave as soon as they are done.
        unsigned long long packed = wave_sum(nflip | (nfb << 21) | (nbad << 42));
        unsigned long long dbits = 0;
        if (flags & RF_TRACK) {
            // non-negative doubles order like their bit patterns
            dbits = (unsigned long long)__double_as_longlong(dmax);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long ob = (unsigned long long)__shfl_xor((long long)dbits, o, 64);
                dbits = ob > dbits ? ob : dbits;
            }
        }
        if ((tid & 63) == 0) {
            if (packed) __hip_atomic_fetch_add(&wg_cnt[0], packed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (dbits) __hip_atomic_fetch_max(&wg_cnt[1], dbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const unsigned long long done =
                __hip_atomic_fetch_add(&wg_cnt[2], 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (done == (unsigned long long)(NT >> 6) - 1) {
                const int64_t slot = (int64_t)b * a.K + (a.iter - 1);
                const unsigned long long tot =
                    __hip_atomic_load(&wg_cnt[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const unsigned long long m21 = (1ull << 21) - 1;
                const unsigned long long f = tot & m21, fb = (tot >> 21) & m21, bad = tot >> 42;
                if (f && a.flips) atomicAdd(a.flips + slot, f);
                if (fb && a.fallbacks) atomicAdd(a.fallbacks + slot, fb);
                if (bad && a.nonfinite) atomicAdd(a.nonfinite + slot, bad);
                if ((flags & RF_TRACK) && a.delta_bits) {
                    const unsigned long long mx =
                        __hip_atomic_load(&wg_cnt[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    atomicMax(a.delta_bits + slot, mx);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Strided-axis pass
// ---------------------------------------------------------------------------
template <typename T, int MODE, int LOG2L>
__global__ void __launch_bounds__(512, (sizeof(T) == 4 && LOG2L <= 9 ? 4 : 1)) col_pass(const ColArgs a)
{
    // modes that weight the spectrum (SYM), that multiply it and transform back
    // (APPLY), and that write it back (STORE)
    constexpr bool SYM = MODE == CM_HEAT || MODE == CM_ENERGY || MODE == CM_DTAU || MODE == CM_RESOLVENT ||
                         MODE == CM_DIRICHLET;
    constexpr bool APPLY = MODE == CM_HEAT || MODE == CM_DTAU || MODE == CM_RESOLVENT;
    constexpr bool STORE = MODE != CM_ENERGY && MODE != CM_DIRICHLET;
    constexpr bool LAPLACE = MODE == CM_RESOLVENT || MODE == CM_DIRICHLET;
    typedef typename cx<T>::type C;
    typedef FftShape<LOG2L> F;
    constexpr int Tn = F::Tn;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red_d[64];

    const int b = blockIdx.y;
    if (a.iter > 0 && a.stop_iter) {
        if (a.stop_iter[b] < a.iter) return;
        if (a.delta_bits && a.tol > 0.0 && a.iter >= 2) {
            // the first pass of iteration s stops field b when s-1 changed it by <= tol
            const double dprev =
                __longlong_as_double((long long)a.delta_bits[(int64_t)b * a.K + (a.iter - 2)]);
            if (dprev <= a.tol) {
                if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(a.stop_iter + b, a.iter - 1);
                return;
            }
        }
    }

    const int TX = a.TX;
    const int tid = threadIdx.x;
    const int tx = tid & (TX - 1);
    // XCD-aware tile order: workgroups are dealt round-robin to the eight XCDs,
    // each with its own L2.  Give every XCD a contiguous run of tiles so that the
    // tiles sharing a 128-byte line (TX * sizeof(C) < 128) meet in one L2.
    const int64_t nwgx = gridDim.x;
    const int64_t wg = ((nwgx & 7) || !a.xcd_remap)
                           ? (int64_t)blockIdx.x
                           : (int64_t)(blockIdx.x & 7) * (nwgx >> 3) + (blockIdx.x >> 3);
    const int64_t o = wg / a.tiles;
    const int64_t tile0 = (wg - o * a.tiles) * TX;
    const int64_t S = a.S;
    C* Zt = reinterpret_cast<C*>(a.Z) + (size_t)b * a.field_elems + o * (int64_t)F::L * S + tile0;
    const C* tw_tab = reinterpret_cast<const C*>(a.tw);

    if constexpr (LOG2L <= 9) {
        // Tile of TX lines staged through LDS: coalesced row segments of TX
        // elements in, one line per group of Tn threads (inside one wave), wave
        // level exchanges, coalesced segments out.  Line c at lr/li[c * pitch].
        const int pitch = a.lds_col;
        T* lrb = reinterpret_cast<T*>(smem_raw);
        T* lib = lrb + (size_t)TX * pitch;
        const int c = tid >> (LOG2L - 3);
        const int tt = tid & (Tn - 1);
        const int ptt = lds_pad(tt);
        // staging: thread tid moves element (row k*Tn + r0, column cc) of the
        // tile for k = 0..7 (the workgroup has Tn * TX threads)
        const int r0 = tid >> a.log2TX, cc = tid & (TX - 1);
        C* const zp = Zt + ((int64_t)r0 << a.log2S) + cc;
        const int64_t kstride = (int64_t)Tn << a.log2S;
        const int pr0 = lds_pad(r0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const C v = zp[k * kstride];
            lrb[cc * pitch + lds_pad_at<Tn>(r0, pr0, k)] = v.x;
            lib[cc * pitch + lds_pad_at<Tn>(r0, pr0, k)] = v.y;
        }
        Twiddles<T, LOG2L> tw;
        load_twiddles<T, LOG2L>(tw, tw_tab, tt);
        __syncthreads();
        T* lr = lrb + (size_t)c * pitch;
        T* li = lib + (size_t)c * pitch;
        // symbol values of this thread's 8 modes, loaded before the transform
        T lam[8];
        if constexpr (LAPLACE) {
            // -4 pi^2 |k|^2 = mu_row + mu_inner
            const T muin = reinterpret_cast<const T*>(a.mu_inner)[tile0 + c];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const T mu = reinterpret_cast<const T*>(a.mu_row)[tt + e * Tn] + muin;
                lam[e] = MODE == CM_RESOLVENT ? (T)a.rnorm / ((T)1 - (T)a.rdt * mu) : -mu;
            }
        } else if (SYM) {
            const T* lrow = reinterpret_cast<const T*>(a.lam_row) + b * a.lam_row_stride;
            const T lin = reinterpret_cast<const T*>(a.lam_inner)[b * a.lam_inner_stride + tile0 + c];
            const T muin = MODE == CM_DTAU ? reinterpret_cast<const T*>(a.mu_inner)[tile0 + c] : (T)0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                lam[e] = lrow[tt + e * Tn] * lin;
                if (MODE == CM_DTAU) lam[e] *= reinterpret_cast<const T*>(a.mu_row)[tt + e * Tn] + muin;
            }
        }
        T r[8], im[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            r[e] = lr[lds_pad_at<Tn>(tt, ptt, e)];
            im[e] = li[lds_pad_at<Tn>(tt, ptt, e)];
        }
        if (MODE == CM_INVERSE) fft_wave<T, +1, LOG2L>(r, im, lr, li, tt, tw, true);
        else fft_wave<T, -1, LOG2L>(r, im, lr, li, tt, tw, true);
        if (SYM) {
            double acc = 0.0;
            if (a.epart) {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    acc += (double)lam[e] * ((double)r[e] * (double)r[e] + (double)im[e] * (double)im[e]);
            }
            if (APPLY) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    r[e] *= lam[e];
                    im[e] *= lam[e];
                }
            }
            if (a.epart) {
                const int slot = a.slot >= 0 ? a.slot : a.stop_iter[b];
                double* ep = a.epart + ((int64_t)b * (a.K + 1) + slot) * a.nwg;
                if ((blockDim.x & 63) == 0) {
                    // whole waves: one partial per wave (fixed order, no barrier)
                    acc = wave_sum(acc);
                    if ((tid & 63) == 0) ep[wg * (blockDim.x >> 6) + (tid >> 6)] = acc;
                } else {
                    acc = block_reduce<OpSum>(acc, red_d);
                    if (tid == 0) ep[wg] = acc;
                }
            }
        }
        if (APPLY) fft_wave<T, +1, LOG2L>(r, im, lr, li, tt, tw, true);
        if (STORE) {
            wave_lds_sync();  // the line's last exchange has been read
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                lr[lds_pad_at<Tn>(tt, ptt, e)] = r[e];
                li[lds_pad_at<Tn>(tt, ptt, e)] = im[e];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                C v;
                v.x = lrb[cc * pitch + lds_pad_at<Tn>(r0, pr0, k)];
                v.y = lib[cc * pitch + lds_pad_at<Tn>(r0, pr0, k)];
                zp[k * kstride] = v;
            }
        }
    } else {
        // Long lines (L > 512): each line spans several waves; thread (t, tx)
        // holds x[t + e*L/8] of line tx and the exchanges use workgroup barriers.
        const int t = tid / TX;
        C* Z = Zt + tx;
        T* lr = reinterpret_cast<T*>(smem_raw);
        T* li = lr + (size_t)a.lds_col * TX;
        T lam[8];
        if constexpr (LAPLACE) {
            // -4 pi^2 |k|^2 = mu_row + mu_inner
            const T muin = reinterpret_cast<const T*>(a.mu_inner)[tile0 + tx];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const T mu = reinterpret_cast<const T*>(a.mu_row)[t + e * Tn] + muin;
                lam[e] = MODE == CM_RESOLVENT ? (T)a.rnorm / ((T)1 - (T)a.rdt * mu) : -mu;
            }
        } else if (SYM) {
            const T* lrow = reinterpret_cast<const T*>(a.lam_row) + b * a.lam_row_stride;
            const T lin = reinterpret_cast<const T*>(a.lam_inner)[b * a.lam_inner_stride + tile0 + tx];
            const T muin = MODE == CM_DTAU ? reinterpret_cast<const T*>(a.mu_inner)[tile0 + tx] : (T)0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                lam[e] = lrow[t + e * Tn] * lin;
                if (MODE == CM_DTAU) lam[e] *= reinterpret_cast<const T*>(a.mu_row)[t + e * Tn] + muin;
            }
        }
        T r[1][8], im[1][8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const C v = Z[(int64_t)(t + e * Tn) * S];
            r[0][e] = v.x;
            im[0][e] = v.y;
        }
        Twiddles<T, LOG2L> tw;
        load_twiddles<T, LOG2L>(tw, tw_tab, t);
        if (MODE == CM_INVERSE)
            fft_lines<T, +1, 1, LOG2L>(r, im, lr, li, 0, TX, tx, t, tw);
        else
            fft_lines<T, -1, 1, LOG2L>(r, im, lr, li, 0, TX, tx, t, tw);
        if (SYM) {
            double acc = 0.0;
            if (a.epart) {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    acc += (double)lam[e] * ((double)r[0][e] * (double)r[0][e] +
                                             (double)im[0][e] * (double)im[0][e]);
            }
            if (APPLY) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    r[0][e] *= lam[e];
                    im[0][e] *= lam[e];
                }
            }
            if (a.epart) {
                // the workgroup's sum in its first partial, zeros in the others
                // (one partial per whole wave, as in the short-line path)
                acc = block_reduce<OpSum>(acc, red_d);
                const int slot = a.slot >= 0 ? a.slot : a.stop_iter[b];
                double* ep = a.epart + ((int64_t)b * (a.K + 1) + slot) * a.nwg;
                if ((blockDim.x & 63) == 0) {
                    if ((tid & 63) == 0) ep[wg * (blockDim.x >> 6) + (tid >> 6)] = tid == 0 ? acc : 0.0;
                } else if (tid == 0) {
                    ep[wg] = acc;
                }
            }
        }
        if (APPLY) fft_lines<T, +1, 1, LOG2L>(r, im, lr, li, 0, TX, tx, t, tw);
        if (STORE) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                C v;
                v.x = r[0][e];
                v.y = im[0][e];
                Z[(int64_t)(t + e * Tn) * S] = v;
            }
        }
    }
}

// Launch helpers used by the translation units: one switch over log2(L).
#define MBO_LOG2L_SWITCH(lg, CASE)                                                             \
    switch (lg) {                                                                              \
    case 3: CASE(3); break;                                                                    \
    case 4: CASE(4); break;                                                                    \
    case 5: CASE(5); break;                                                                    \
    case 6: CASE(6); break;                                                                    \
    case 7: CASE(7); break;                                                                    \
    case 8: CASE(8); break;                                                                    \
    case 9: CASE(9); break;                                                                    \
    case 10: CASE(10); break;                                                                  \
    case 11: CASE(11); break;                                                                  \
    default: return hipErrorInvalidValue;                                                      \
    }

}  // namespace mbo
