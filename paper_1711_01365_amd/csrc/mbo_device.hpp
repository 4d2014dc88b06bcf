// Device building blocks for gfx950: radix-8 Stockham FFT stages held in
// registers with LDS exchanges, and the per-point closest-orthogonal-matrix
// projection (closed form for n = 2, one-sided Jacobi for n = 3, 4).
//
// Method: Osting & Wang, arXiv:1711.01365.  The FFT realises the flat-torus
// diffusion step of Section 5.1; the projection is Lemma 1.1 (Algorithm 1,
// step 2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbo {

template <typename T> struct cx;
template <> struct cx<float> { typedef float2 type; };
template <> struct cx<double> { typedef double2 type; };

template <typename T> struct num;
template <> struct num<float> {
    // unit roundoff scale used by the singular-value zero test and the Jacobi
    // stopping rule (columns orthogonal to working precision)
    static constexpr float eps = 1.1920928955078125e-07f;
    static constexpr float jtol2 = 1.4210854715202004e-14f;  // eps^2
    // a sweep whose rotations all had |sin| below this leaves inner products
    // of order sin^2 < eps: the next sweep would not rotate
    static constexpr float sdone = 2.5e-4f;
    // hardware approximations (about 1 ulp): the rotation angle of a Jacobi step
    // need not be correctly rounded, any accurate rotation serves
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
};
template <> struct num<double> {
    static constexpr double eps = 2.220446049250313e-16;
    static constexpr double jtol2 = 1e-30;  // (1e-15)^2
    static constexpr double sdone = 1e-8;
    // hardware estimate refined by two Newton steps y <- y (3 - x y^2) / 2
    static __device__ __forceinline__ double rsq(double x)
    {
        double y = __builtin_amdgcn_rsq(x);
        y = y * (1.5 - 0.5 * x * y * y);
        y = y * (1.5 - 0.5 * x * y * y);
        return y;
    }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
};

// ---------------------------------------------------------------------------
// FFT: small DFTs.  S = -1: forward (exp(-2 pi i jk/R)), S = +1: inverse.
// ---------------------------------------------------------------------------

template <typename T, int S>
__device__ __forceinline__ void mul_si(T& r, T& i)  // (r + i i) * (S i)
{
    T t = r;
    r = (S > 0) ? -i : i;
    i = (S > 0) ? t : -t;
}

template <typename T, int S>
__device__ __forceinline__ void dft2(T* r, T* i)
{
    T tr = r[0] - r[1], ti = i[0] - i[1];
    r[0] += r[1]; i[0] += i[1];
    r[1] = tr; i[1] = ti;
}

template <typename T, int S>
__device__ __forceinline__ void dft4(T* r, T* i)
{
    T t0r = r[0] + r[2], t0i = i[0] + i[2];
    T t1r = r[0] - r[2], t1i = i[0] - i[2];
    T t2r = r[1] + r[3], t2i = i[1] + i[3];
    T t3r = r[1] - r[3], t3i = i[1] - i[3];
    mul_si<T, S>(t3r, t3i);
    r[0] = t0r + t2r; i[0] = t0i + t2i;
    r[2] = t0r - t2r; i[2] = t0i - t2i;
    r[1] = t1r + t3r; i[1] = t1i + t3i;
    r[3] = t1r - t3r; i[3] = t1i - t3i;
}

// Second half of the length-8 DFT: the length-4 DFTs of the even (er, ei)
// and odd (orr, oi) inputs are combined through exp(S 2 pi i k / 8).
template <typename T, int S>
__device__ __forceinline__ void dft8_combine(const T (&er)[4], const T (&ei)[4], T (&orr)[4], T (&oi)[4], T* r, T* i)
{
    const T c = (T)0.70710678118654752440084436210485;
    // odd half times exp(S 2 pi i k / 8), k = 1, 2, 3
    {
        T x = orr[1], y = oi[1];
        orr[1] = c * (x - (T)S * y);
        oi[1] = c * ((T)S * x + y);
    }
    mul_si<T, S>(orr[2], oi[2]);
    {
        T x = orr[3], y = oi[3];
        orr[3] = c * (-x - (T)S * y);
        oi[3] = c * ((T)S * x - y);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r[k] = er[k] + orr[k]; i[k] = ei[k] + oi[k];
        r[k + 4] = er[k] - orr[k]; i[k + 4] = ei[k] - oi[k];
    }
}

template <typename T, int S>
__device__ __forceinline__ void dft8(T* r, T* i)
{
    T er[4] = {r[0], r[2], r[4], r[6]}, ei[4] = {i[0], i[2], i[4], i[6]};
    T orr[4] = {r[1], r[3], r[5], r[7]}, oi[4] = {i[1], i[3], i[5], i[7]};
    dft4<T, S>(er, ei);
    dft4<T, S>(orr, oi);
    dft8_combine<T, S>(er, ei, orr, oi, r, i);
}

// dft8 of inputs 1..6 known to be zero: the two length-4 DFTs reduce to copies
// and sign changes of inputs 0 and 7 (adding or subtracting an exact zero), so
// the result is that of dft8, with fewer operations.
template <typename T, int S>
__device__ __forceinline__ void dft8_in07(T* r, T* i)
{
    const T x0r = r[0], x0i = i[0], x7r = r[7], x7i = i[7];
    T er[4] = {x0r, x0r, x0r, x0r}, ei[4] = {x0i, x0i, x0i, x0i};
    // odd inputs (0, 0, 0, x7): dft4 gives (x7, -S i x7... ) as below
    T t3r = -x7r, t3i = -x7i;
    mul_si<T, S>(t3r, t3i);
    T orr[4] = {x7r, t3r, -x7r, -t3r}, oi[4] = {x7i, t3i, -x7i, -t3i};
    dft8_combine<T, S>(er, ei, orr, oi, r, i);
}

// dft8 of which only outputs 0 and 7 are needed: the operations of dft8 that
// lead to them, in the same order (the same values); outputs 1..6 are left
// unset.
template <typename T, int S>
__device__ __forceinline__ void dft8_out07(T* r, T* i)
{
    const T c = (T)0.70710678118654752440084436210485;
    // even inputs 0, 2, 4, 6: outputs 0 and 3 of their dft4
    const T e0r = r[0] + r[4], e0i = i[0] + i[4];
    const T e1r = r[0] - r[4], e1i = i[0] - i[4];
    const T e2r = r[2] + r[6], e2i = i[2] + i[6];
    T e3r = r[2] - r[6], e3i = i[2] - i[6];
    mul_si<T, S>(e3r, e3i);
    const T er0 = e0r + e2r, ei0 = e0i + e2i;
    const T er3 = e1r - e3r, ei3 = e1i - e3i;
    // odd inputs 1, 3, 5, 7
    const T o0r = r[1] + r[5], o0i = i[1] + i[5];
    const T o1r = r[1] - r[5], o1i = i[1] - i[5];
    const T o2r = r[3] + r[7], o2i = i[3] + i[7];
    T o3r = r[3] - r[7], o3i = i[3] - i[7];
    mul_si<T, S>(o3r, o3i);
    const T or0 = o0r + o2r, oi0 = o0i + o2i;
    const T x = o1r - o3r, y = o1i - o3i;
    const T or3 = c * (-x - (T)S * y);
    const T oi3 = c * ((T)S * x - y);
    r[0] = er0 + or0; i[0] = ei0 + oi0;
    r[7] = er3 - or3; i[7] = ei3 - oi3;
}

template <typename T, int R, int S>
__device__ __forceinline__ void dft(T* r, T* i)
{
    if constexpr (R == 8) dft8<T, S>(r, i);
    else if constexpr (R == 4) dft4<T, S>(r, i);
    else dft2<T, S>(r, i);
}

// Twiddle table entries hold exp(-2 pi i m / L); the inverse uses the conjugate.
template <typename T, int S>
__device__ __forceinline__ void twiddle(T& r, T& i, const typename cx<T>::type w)
{
    T wr = w.x, wi = (S < 0) ? w.y : -w.y;
    T nr = r * wr - i * wi;
    T ni = r * wi + i * wr;
    r = nr;
    i = ni;
}

// LDS index with one pad slot per eight elements (spreads the strided stage
// writes over all banks).
__device__ __forceinline__ int lds_pad(int j) { return j + (j >> 3); }

// lds_pad(j0 + m * STEP) = lds_pad(j0) + m * (STEP + STEP / 8) when STEP is a
// multiple of 8: the offset is a compile-time constant the compiler folds into
// the LDS instruction, so a thread keeps one address instead of one per element.
template <int STEP>
__device__ __forceinline__ int lds_pad_at(int j0, int pad_j0, int m)
{
    if constexpr (STEP % 8 == 0) return pad_j0 + m * (STEP + STEP / 8);
    else return lds_pad(j0 + m * STEP);
}

// ---------------------------------------------------------------------------
// Length-L Stockham FFT, L = 2^LOG2L in [8, 2048], fixed at compile time.
//
// Register layout: the thread with index t of Tn = L/8 cooperating threads
// holds x[t + e*Tn], e < 8, before and after the transform.  Stage 0 has span
// p = 1 and radix R0 = L / 8^N8 (2, 4 or, when LOG2L is a multiple of 3, 8);
// every later stage is radix 8.  A stage of radix R and span p computes, for
// each butterfly i (thread t owns i = t + b*Tn, b < 8/R), the length-R DFT of
// x[i + j*L/R] * W_L^{j*k*L/(p*R)}, k = i mod p, j < R, and its output q
// belongs at index (i - k)*R + k + q*p.  For the last stage that index is
// t + q*Tn, so the result ends in natural order in the registers; earlier
// stages exchange through LDS.  Only radix-8 stages with p > 1 need twiddles
// (seven per thread and stage); they are loaded once per kernel.
// ---------------------------------------------------------------------------
template <int LOG2L>
struct FftShape {
    static constexpr int L = 1 << LOG2L;
    static constexpr int Tn = L >> 3;
    static constexpr int N8 = LOG2L / 3;
    static constexpr int R0 = 1 << (LOG2L - 3 * N8);  // 1: no short first stage
    static constexpr int NST = N8 + (R0 > 1 ? 1 : 0);
    static constexpr int NTW = NST - 1;                // stages with twiddles
    static constexpr int radix(int s) { return (s == 0 && R0 > 1) ? R0 : 8; }
    static constexpr int log2span(int s)
    {
        return s == 0 ? 0 : (R0 > 1 ? (LOG2L - 3 * N8) + 3 * (s - 1) : 3 * s);
    }
};

template <typename T, int LOG2L>
struct Twiddles {
    typename cx<T>::type w[FftShape<LOG2L>::NTW > 0 ? FftShape<LOG2L>::NTW : 1][7];
};

// table[m] = exp(-2 pi i m / L); stage s >= 1 needs W_L^{j k L/(8p)}, j = 1..7.
template <typename T, int LOG2L>
__device__ __forceinline__ void load_twiddles(Twiddles<T, LOG2L>& tw,
                                              const typename cx<T>::type* __restrict__ table, int t)
{
    typedef FftShape<LOG2L> F;
#pragma unroll
    for (int s = 1; s < F::NST; ++s) {
        const int lp = F::log2span(s);
        const int k = t & ((1 << lp) - 1);
        const int shift = LOG2L - 3 - lp;
#pragma unroll
        for (int j = 1; j < 8; ++j) tw.w[s - 1][j - 1] = table[(j * k) << shift];
    }
}

// The twiddle table itself as the source of a transform's twiddles: each
// stage loads its seven values just before it (cache or LDS hits), so only one
// stage's twiddles take registers at a time.
template <typename T, int LOG2L>
struct TwiddleTable {
    const typename cx<T>::type* table;
};

template <typename T, int LOG2L, int STAGE>
__device__ __forceinline__ void stage_twiddles(const Twiddles<T, LOG2L>& tw, int, typename cx<T>::type (&w)[7])
{
#pragma unroll
    for (int j = 0; j < 7; ++j) w[j] = tw.w[STAGE - 1][j];
}

template <typename T, int LOG2L, int STAGE>
__device__ __forceinline__ void stage_twiddles(const TwiddleTable<T, LOG2L>& tw, int t, typename cx<T>::type (&w)[7])
{
    typedef FftShape<LOG2L> F;
    const int lp = F::log2span(STAGE);
    const int k = t & ((1 << lp) - 1);
    const int shift = LOG2L - 3 - lp;
#pragma unroll
    for (int j = 1; j < 8; ++j) w[j - 1] = tw.table[(j * k) << shift];
}

// Butterflies of a span-1 stage of radix R: butterfly b uses registers b + j*(8/R).
template <typename T, int R, int S>
__device__ __forceinline__ void stage_span1(T (&r)[8], T (&im)[8])
{
    constexpr int B = 8 / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        T ur[R], ui[R];
#pragma unroll
        for (int j = 0; j < R; ++j) { ur[j] = r[b + j * B]; ui[j] = im[b + j * B]; }
        dft<T, R, S>(ur, ui);
#pragma unroll
        for (int q = 0; q < R; ++q) { r[b + q * B] = ur[q]; im[b + q * B] = ui[q]; }
    }
}

// Radix-8 stage with twiddles (one butterfly per thread).
template <typename T, int S>
__device__ __forceinline__ void stage_tw8(T (&r)[8], T (&im)[8], const typename cx<T>::type (&w)[7])
{
#pragma unroll
    for (int j = 1; j < 8; ++j) twiddle<T, S>(r[j], im[j], w[j - 1]);
    dft8<T, S>(r, im);
}

// LDS element index of position j of a line, by layout: LIX_PAD pads one slot
// per eight; LIX_XOR keeps the line's L slots and swaps bits 1-3 of j with the
// XOR of bits 4-6 (a permutation of each run of 16), which spreads the
// exchanges of a radix-8 stage of a 64- or 128-point line over the banks when
// the line's elements are 8 bytes apart or more (interleaved complex, or a
// column of a padded plane); LIX_PLAIN leaves j as it is.
enum { LIX_PLAIN = 0, LIX_PAD = 1, LIX_XOR = 2 };

template <int LIX>
__device__ __forceinline__ int line_index(int j)
{
    if constexpr (LIX == LIX_PAD) return lds_pad(j);
    else if constexpr (LIX == LIX_XOR) return j ^ (((j >> 4) & 7) << 1);
    else return j;
}

template <typename T, int S, int NP, int LOG2L, int STAGE, int PADJ = LIX_PAD, typename TW = Twiddles<T, LOG2L>>
__device__ __forceinline__ void fft_stages(T (&r)[NP][8], T (&im)[NP][8], T* lr, T* li, int lplane,
                                           int lmul, int ladd, int t, const TW& tw, bool act)
{
    typedef FftShape<LOG2L> F;
    if constexpr (STAGE < F::NST) {
        constexpr int R = F::radix(STAGE);
        constexpr int lp = F::log2span(STAGE);
        constexpr int p = 1 << lp;
        if constexpr (STAGE == 0) {
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) stage_span1<T, R, S>(r[pl], im[pl]);
        } else {
            typename cx<T>::type w[7];
            stage_twiddles<T, LOG2L, STAGE>(tw, t, w);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) stage_tw8<T, S>(r[pl], im[pl], w);
        }
        if constexpr (STAGE != F::NST - 1) {
            __syncthreads();  // earlier readers of the LDS lines are done
            if (!act) {
            } else if constexpr (STAGE == 0) {
                constexpr int B = 8 / R;
#pragma unroll
                for (int pl = 0; pl < NP; ++pl)
#pragma unroll
                    for (int b = 0; b < B; ++b)
#pragma unroll
                        for (int q = 0; q < R; ++q) {
                            const int a = pl * lplane + line_index<PADJ>((t + b * F::Tn) * R + q) * lmul + ladd;
                            lr[a] = r[pl][b + q * B];
                            li[a] = im[pl][b + q * B];
                        }
            } else {
                const int k = t & (p - 1);
                const int base = ((t - k) << 3) + k;
#pragma unroll
                for (int pl = 0; pl < NP; ++pl)
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int a = pl * lplane + line_index<PADJ>(base + q * p) * lmul + ladd;
                        lr[a] = r[pl][q];
                        li[a] = im[pl][q];
                    }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int pl = 0; pl < NP; ++pl)
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int a = pl * lplane + line_index<PADJ>(t + e * F::Tn) * lmul + ladd;
                        r[pl][e] = lr[a];
                        im[pl][e] = li[a];
                    }
            }
            fft_stages<T, S, NP, LOG2L, STAGE + 1, PADJ, TW>(r, im, lr, li, lplane, lmul, ladd, t, tw, act);
        }
    }
}

// Orders LDS accesses among the lanes of one wave: a wave issues its LDS
// operations in program order, so a fence at wavefront scope (which keeps the
// compiler from moving LDS accesses across it) is all the exchange needs.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Pruning of a line transform (band-limited lines, half-width c < L/8):
// FFT_IN07, the inputs x[t + e L/8] with 1 <= e <= 6 are zero (radix-8 first
// stage only); FFT_OUT07, only the outputs x[t + e L/8] with e = 0 or 7 are
// used (the others are left unset).
enum { FFT_FULL = 0, FFT_IN07 = 1, FFT_OUT07 = 2 };

// The same transform for a line whose L/8 threads lie inside one wave
// (L <= 512): exchanges need no workgroup barrier.  LDS element j of the line is
// at lr/li[lds_pad(j)].  Threads with act = false touch no LDS.
template <typename T, int S, int LOG2L, int STAGE = 0, int PR = FFT_FULL>
__device__ __forceinline__ void fft_wave(T (&r)[8], T (&im)[8], T* lr, T* li, int t,
                                         const Twiddles<T, LOG2L>& tw, bool act)
{
    typedef FftShape<LOG2L> F;
    static_assert(LOG2L <= 9, "a line must fit in one wave");
    static_assert(!(PR & FFT_IN07) || F::radix(0) == 8, "input pruning needs a radix-8 first stage");
    if constexpr (STAGE < F::NST) {
        constexpr int R = F::radix(STAGE);
        constexpr int p = 1 << F::log2span(STAGE);
        if constexpr (STAGE == 0 && (PR & FFT_IN07)) dft8_in07<T, S>(r, im);
        else if constexpr (STAGE == 0) stage_span1<T, R, S>(r, im);
        else if constexpr (STAGE == F::NST - 1 && (PR & FFT_OUT07)) {
#pragma unroll
            for (int j = 1; j < 8; ++j) twiddle<T, S>(r[j], im[j], tw.w[STAGE - 1][j - 1]);
            dft8_out07<T, S>(r, im);
        } else stage_tw8<T, S>(r, im, tw.w[STAGE - 1]);
        if constexpr (STAGE != F::NST - 1) {
            wave_lds_sync();  // earlier reads of the line are done
            if (act) {
                if constexpr (STAGE == 0) {
                    // element (t + b*Tn)*R + q; R divides 8, so q never carries
                    // into the padding term
                    constexpr int B = 8 / R;
                    const int j0 = t * R, pj0 = lds_pad(j0);
#pragma unroll
                    for (int b = 0; b < B; ++b)
#pragma unroll
                        for (int q = 0; q < R; ++q) {
                            const int a = lds_pad_at<F::Tn * R>(j0, pj0, b) + q;
                            lr[a] = r[b + q * B];
                            li[a] = im[b + q * B];
                        }
                } else {
                    const int k = t & (p - 1);
                    const int base = ((t - k) << 3) + k;
                    const int pbase = lds_pad(base);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int a = lds_pad_at<p>(base, pbase, q);
                        lr[a] = r[q];
                        li[a] = im[q];
                    }
                }
            }
            wave_lds_sync();
            if (act) {
                const int pt = lds_pad(t);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int a = lds_pad_at<F::Tn>(t, pt, e);
                    r[e] = lr[a];
                    im[e] = li[a];
                }
            }
            fft_wave<T, S, LOG2L, STAGE + 1, PR>(r, im, lr, li, t, tw, act);
        }
    }
}

// In-place FFT of NP lines (S = -1 forward, +1 inverse, unscaled).  LDS element
// j of line pl is at lr/li[pl*lplane + line_index<PADJ>(j)*lmul + ladd].  Every thread of the workgroup must call it (it contains
// barriers); threads with act = false only take part in the barriers and touch
// no LDS.
template <typename T, int S, int NP, int LOG2L, int PADJ = LIX_PAD, typename TW = Twiddles<T, LOG2L>>
__device__ __forceinline__ void fft_lines(T (&r)[NP][8], T (&im)[NP][8], T* lr, T* li, int lplane,
                                          int lmul, int ladd, int t, const TW& tw, bool act = true)
{
    fft_stages<T, S, NP, LOG2L, 0, PADJ, TW>(r, im, lr, li, lplane, lmul, ladd, t, tw, act);
}

// ---------------------------------------------------------------------------
// Projection onto O(n) (Lemma 1.1): Q = U V^t of the SVD A = U Sigma V^t.
// Matrices are row-major in registers, a[i*n + j] = A_ij.
// ---------------------------------------------------------------------------

template <typename T, int n>
__device__ __forceinline__ T det_n(const T* m)
{
    if constexpr (n == 1) {
        return m[0];
    } else if constexpr (n == 2) {
        return m[0] * m[3] - m[1] * m[2];
    } else if constexpr (n == 3) {
        return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
               m[2] * (m[3] * m[7] - m[4] * m[6]);
    } else {
        // Laplace expansion along rows 0-1 (2x2 minors against rows 2-3)
        const T a01 = m[0] * m[5] - m[1] * m[4], a02 = m[0] * m[6] - m[2] * m[4];
        const T a03 = m[0] * m[7] - m[3] * m[4], a12 = m[1] * m[6] - m[2] * m[5];
        const T a13 = m[1] * m[7] - m[3] * m[5], a23 = m[2] * m[7] - m[3] * m[6];
        const T b01 = m[8] * m[13] - m[9] * m[12], b02 = m[8] * m[14] - m[10] * m[12];
        const T b03 = m[8] * m[15] - m[11] * m[12], b12 = m[9] * m[14] - m[10] * m[13];
        const T b13 = m[9] * m[15] - m[11] * m[13], b23 = m[10] * m[15] - m[11] * m[14];
        return a01 * b23 - a02 * b13 + a03 * b12 + a12 * b03 - a13 * b02 + a23 * b01;
    }
}

// Largest |entry| as a power of two 2^ex (ex = 0 for a zero or non-finite
// matrix): scaling by 2^-ex is exact and keeps every square representable.
template <typename T, int n>
__device__ __forceinline__ int scale_exponent(const T* a)
{
    T amax = 0;
#pragma unroll
    for (int i = 0; i < n * n; ++i) {
        const T v = a[i] < (T)0 ? -a[i] : a[i];
        amax = v > amax ? v : amax;
    }
    int ex = 0;
    if (amax > (T)0 && amax - amax == (T)0) (void)frexp(amax, &ex);
    return ex;
}

// n = 2 closed form.  The closest rotation [[c,-s],[s,c]] maximises
// c (a00 + a11) + s (a10 - a01); the closest reflection [[c,s],[s,-c]] maximises
// c (a00 - a11) + s (a01 + a10).  Lemma 1.1 keeps the sign of det A, with the
// rotation taken when det A = 0.  Also returns sigma_min for the fallback test.
// The matrix is first scaled by a power of two (exact; for matrices of
// moderate magnitude, whose products are normal numbers either way, the result
// is unchanged), so that no square or product under- or overflows whatever the
// magnitude.
template <typename T>
__device__ __forceinline__ void polar2(const T* a_in, T* q, int& dsign, T& smin)
{
    const int ex = scale_exponent<T, 2>(a_in);
    T a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = ldexp(a_in[k], -ex);
    const T det = a[0] * a[3] - a[1] * a[2];
    const bool rot = det >= (T)0;
    const T p = rot ? a[0] + a[3] : a[0] - a[3];
    const T s = rot ? a[2] - a[1] : a[1] + a[2];
    const T rr = p * p + s * s;
    if (rr == (T)0) {  // only A = 0 reaches this: take the identity
        q[0] = 1; q[1] = 0; q[2] = 0; q[3] = 1;
        dsign = 1;
        smin = 0;
        return;
    }
    const T inv = num<T>::rsq(rr);
    const T c = p * inv, sn = s * inv;
    q[0] = c;
    q[1] = rot ? -sn : sn;
    q[2] = sn;
    q[3] = rot ? c : -c;
    dsign = rot ? 1 : -1;
    const T f2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3];
    const T ad = det < (T)0 ? -det : det;
    const T lo = f2 - 2 * ad;
    const T smax = (T)0.5 * (num<T>::sqrt_(f2 + 2 * ad) + num<T>::sqrt_(lo > (T)0 ? lo : (T)0));
    smin = ldexp(smax > (T)0 ? ad * num<T>::rcp(smax) : (T)0, ex);
}

// One-sided (Hestenes) Jacobi: rotate pairs of columns of W = A until they are
// mutually orthogonal (to working precision), accumulating the rotations in V;
// then sigma_j = |w_j|, U = W Sigma^{-1} and Q = U V^t.
//
// The rotation of a pair (p, r) with a = |w_p|^2, b = |w_r|^2, g = 2 w_p.w_r
// zeroes their inner product: with h = b - a and k = |h| / sqrt(h^2 + g^2)
// (= cos 2phi), c = sqrt((1 + k)/2) and s = sgn(h) g / (2 c sqrt(h^2 + g^2)), so
// that c^2 + s^2 = 1 holds identically; only two reciprocal square roots are
// needed.  It is applied unconditionally with (c, s) = (1, 0) when the pair is
// already orthogonal, which keeps the wave free of divergent branches.  A lane
// stops after a sweep without rotations, or after a sweep whose rotations all
// had |s| < sdone (the inner products left are then of order s^2, below the
// tolerance, so the confirming sweep is skipped).
template <typename T, int n>
__device__ __forceinline__ void jacobi_sweeps(T (&W)[n][n], T (&V)[n][n])
{
    constexpr T sdone = num<T>::sdone;
#pragma unroll 1
    for (int sweep = 0; sweep < 30; ++sweep) {
        bool rotated = false;
        T smax = 0;
#pragma unroll
        for (int p = 0; p < n - 1; ++p) {
#pragma unroll
            for (int r = p + 1; r < n; ++r) {
                T al = 0, be = 0, ga = 0;
#pragma unroll
                for (int i = 0; i < n; ++i) {
                    al += W[i][p] * W[i][p];
                    be += W[i][r] * W[i][r];
                    ga += W[i][p] * W[i][r];
                }
                const bool rot = ga * ga > num<T>::jtol2 * (al * be);
                rotated = rotated || rot;
                const T h = be - al;
                const T g = ga + ga;
                const T rinv = num<T>::rsq(h * h + g * g);
                const T k = (h < (T)0 ? -h : h) * rinv;
                const T hk = (T)0.5 + (T)0.5 * k;
                const T qq = num<T>::rsq(hk);
                const T c = rot ? hk * qq : (T)1;
                const T sn = rot ? (h >= (T)0 ? g : -g) * rinv * (T)0.5 * qq : (T)0;
                const T asn = sn < (T)0 ? -sn : sn;
                smax = asn > smax ? asn : smax;
#pragma unroll
                for (int i = 0; i < n; ++i) {
                    const T wp = W[i][p], wr = W[i][r];
                    W[i][p] = c * wp - sn * wr;
                    W[i][r] = sn * wp + c * wr;
                    const T vp = V[i][p], vr = V[i][r];
                    V[i][p] = c * vp - sn * vr;
                    V[i][r] = sn * vp + c * vr;
                }
            }
        }
        if (!rotated || smax < sdone) break;
    }
}

// Q = U V^t from the orthogonalised columns W = U Sigma (scaled by 2^-ex).  On
// return W holds U (completed for zero singular values) unless the matrix is
// zero; sig (nullable) receives the singular values of the unscaled input.
template <typename T, int n, typename Tq = T>
__device__ __forceinline__ void jacobi_finish(T (&W)[n][n], const T (&V)[n][n], int ex, Tq* q, int& dsign, T& smin,
                                              T* sig = nullptr)
{
    T ss[n], sg[n];
    T smax = 0;
    smin = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) {
        T v = 0;
#pragma unroll
        for (int i = 0; i < n; ++i) v += W[i][j] * W[i][j];
        ss[j] = v;
        sg[j] = num<T>::sqrt_(v);
        smax = sg[j] > smax ? sg[j] : smax;
        smin = (j == 0 || sg[j] < smin) ? sg[j] : smin;
    }
    smin = ldexp(smin, ex);  // singular values of the unscaled input
    if (sig) {
#pragma unroll
        for (int j = 0; j < n; ++j) sig[j] = ldexp(sg[j], ex);
    }
    if (!(smax > (T)0)) {  // zero matrix (or NaN): identity
#pragma unroll
        for (int i = 0; i < n * n; ++i) q[i] = (i % (n + 1) == 0) ? (Tq)1 : (Tq)0;
        dsign = 1;
        return;
    }
    const T thr = (T)n * num<T>::eps * smax;
    bool filled[n];
    bool anyzero = false;
#pragma unroll
    for (int j = 0; j < n; ++j) {
        filled[j] = sg[j] > thr;
        anyzero = anyzero || !filled[j];
        const T inv = filled[j] ? num<T>::rsq(ss[j]) : (T)0;
#pragma unroll
        for (int i = 0; i < n; ++i) W[i][j] *= inv;  // W becomes U
    }
    if constexpr (n == 3 || n == 4) {
        if (!anyzero) {
            // The column of the smallest singular value from the others: the
            // unit vector orthogonal to them (cross product; for n = 4 the
            // generalised one), signed like w_min.  Dividing w_min by its small
            // norm would carry an error of about eps sigma_max / sigma_min into
            // U even where the polar factor is well conditioned
            // (sigma_{n-1} + sigma_n large); the completion does not.
            // (columns picked by selects, not by a run-time index: an indexed
            // register array would be placed in scratch memory)
            int jm = 0;
            T sm = sg[0];
#pragma unroll
            for (int j = 1; j < n; ++j) {
                jm = sg[j] < sm ? j : jm;
                sm = sg[j] < sm ? sg[j] : sm;
            }
            T cv[n], wm[n];
#pragma unroll
            for (int i = 0; i < n; ++i) {
                wm[i] = W[i][0];
#pragma unroll
                for (int j = 1; j < n; ++j) wm[i] = jm == j ? W[i][j] : wm[i];
            }
            if constexpr (n == 3) {
                T ua[3], ub[3];  // the two other columns, in increasing order
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ua[i] = jm == 0 ? W[i][1] : W[i][0];
                    ub[i] = jm == 2 ? W[i][1] : W[i][2];
                }
                cv[0] = ua[1] * ub[2] - ua[2] * ub[1];
                cv[1] = ua[2] * ub[0] - ua[0] * ub[2];
                cv[2] = ua[0] * ub[1] - ua[1] * ub[0];
            } else {
                T u0[4], u1[4], u2[4];  // the three other columns, in increasing order
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    u0[i] = jm == 0 ? W[i][1] : W[i][0];
                    u1[i] = jm <= 1 ? W[i][2] : W[i][1];
                    u2[i] = jm <= 2 ? W[i][3] : W[i][2];
                }
                // cv_i = (-1)^i det of the 3x3 rows other than i of [u0 u1 u2]
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int r[3], m = 0;
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
                        if (rr != i) r[m++] = rr;
                    const T d = u0[r[0]] * (u1[r[1]] * u2[r[2]] - u1[r[2]] * u2[r[1]]) -
                                u0[r[1]] * (u1[r[0]] * u2[r[2]] - u1[r[2]] * u2[r[0]]) +
                                u0[r[2]] * (u1[r[0]] * u2[r[1]] - u1[r[1]] * u2[r[0]]);
                    cv[i] = (i & 1) ? -d : d;
                }
            }
            T cn = 0, dt = 0;
#pragma unroll
            for (int i = 0; i < n; ++i) {
                cn += cv[i] * cv[i];
                dt += cv[i] * wm[i];
            }
            if (cn > (T)0) {
                const T inv = (dt < (T)0 ? (T)-1 : (T)1) * num<T>::rsq(cn);
#pragma unroll
                for (int i = 0; i < n; ++i)
#pragma unroll
                    for (int j = 0; j < n; ++j) W[i][j] = jm == j ? cv[i] * inv : W[i][j];
            }
        }
    }
    int lastz = -1;
    if (anyzero) {
        // Singular input: complete U by Gram-Schmidt of the unit vector with the
        // largest residual against the columns already present.
#pragma unroll
        for (int j = 0; j < n; ++j) {
            if (filled[j]) continue;
            T best[n];
            T bestn = (T)-1;
#pragma unroll
            for (int e = 0; e < n; ++e) {
                T rv[n];
#pragma unroll
                for (int i = 0; i < n; ++i) rv[i] = (i == e) ? (T)1 : (T)0;
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    if (!filled[k]) continue;
                    const T dot = W[e][k];
#pragma unroll
                    for (int i = 0; i < n; ++i) rv[i] -= dot * W[i][k];
                }
                T nn = 0;
#pragma unroll
                for (int i = 0; i < n; ++i) nn += rv[i] * rv[i];
                if (nn > bestn) {
                    bestn = nn;
#pragma unroll
                    for (int i = 0; i < n; ++i) best[i] = rv[i];
                }
            }
            const T inv = num<T>::rsq(bestn);
#pragma unroll
            for (int i = 0; i < n; ++i) W[i][j] = best[i] * inv;
            filled[j] = true;
            lastz = j;
        }
    }
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int k = 0; k < n; ++k) {
            T v = 0;
#pragma unroll
            for (int j = 0; j < n; ++j) v += W[i][j] * V[k][j];
            q[i * n + k] = (Tq)v;
        }
    Tq dq = det_n<Tq, n>(q);
    if (lastz >= 0 && dq < (T)0) {
        // the completed direction's sign is free: choose det Q = +1
#pragma unroll
        for (int j = 0; j < n; ++j) {
            if (j != lastz) continue;
#pragma unroll
            for (int i = 0; i < n; ++i) W[i][j] = -W[i][j];
        }
#pragma unroll
        for (int i = 0; i < n; ++i)
#pragma unroll
            for (int k = 0; k < n; ++k) {
                T v = 0;
#pragma unroll
                for (int j = 0; j < n; ++j) v += W[i][j] * V[k][j];
                q[i * n + k] = (Tq)v;
            }
        dq = -dq;
    }
    dsign = dq >= (Tq)0 ? 1 : -1;
}


template <typename T, int n>
__device__ __forceinline__ void polar_jacobi(const T* a_in, T* q, int& dsign, T& smin)
{
    const int ex = scale_exponent<T, n>(a_in);
    T W[n][n], V[n][n];
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            W[i][j] = ldexp(a_in[i * n + j], -ex);
            V[i][j] = (i == j) ? (T)1 : (T)0;
        }
    jacobi_sweeps<T, n>(W, V);
    jacobi_finish<T, n>(W, V, ex, q, dsign, smin);
}

// The same in double, warm-started from the right singular vectors V0 of a
// float run on the same matrix, for a result that is rounded to float: V0 is
// re-orthonormalised in double (modified Gram-Schmidt), W = A V0 is then nearly
// column-orthogonal, and the sweeps (rotations of order float rounding) run to
// the double stopping rule: the points that come here may have an
// ill-conditioned polar factor (2 / (sigma_{n-1} + sigma_n) up to ~1e7), which
// would carry a looser stop into the float result.  A is read as float (its
// entries widen exactly, so the products are those of a double copy and the
// float exponent is the double one) and Q is rounded to float as it is formed;
// the sign of det Q is taken from the rounded Q (orthogonal: |det| = 1 up to
// rounding).  Both save the registers of a double copy.
template <int n>
__device__ __forceinline__ void polar_jacobi_warm(const float* a_in, const float (&V0)[n][n], float* q, int& dsign)
{
    const int ex = scale_exponent<float, n>(a_in);
    double V[n][n], W[n][n];
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) V[i][j] = (double)V0[i][j];
#pragma unroll
    for (int j = 0; j < n; ++j) {
#pragma unroll
        for (int k = 0; k < j; ++k) {
            double d = 0;
#pragma unroll
            for (int i = 0; i < n; ++i) d += V[i][k] * V[i][j];
#pragma unroll
            for (int i = 0; i < n; ++i) V[i][j] -= d * V[i][k];
        }
        double nn = 0;
#pragma unroll
        for (int i = 0; i < n; ++i) nn += V[i][j] * V[i][j];
        const double inv = num<double>::rsq(nn);
#pragma unroll
        for (int i = 0; i < n; ++i) V[i][j] *= inv;
    }
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            double v = 0;
#pragma unroll
            for (int k = 0; k < n; ++k) v += (double)a_in[i * n + k] * V[k][j];
            W[i][j] = ldexp(v, -ex);
        }
    jacobi_sweeps<double, n>(W, V);
    double smin;
    jacobi_finish<double, n, float>(W, V, ex, q, dsign, smin);
}

// Closest orthogonal matrix of a (n*n values).  Returns sgn det Q and the
// smallest singular value of a (used by the double-precision fallback test).
template <typename T, int n>
__device__ __forceinline__ void project_point(const T* a, T* q, int& dsign, T& smin)
{
    if constexpr (n == 1) {
        const bool pos = a[0] >= (T)0;  // sgn(0) = +1
        q[0] = pos ? (T)1 : (T)-1;
        dsign = pos ? 1 : -1;
        smin = a[0] < (T)0 ? -a[0] : a[0];
    } else if constexpr (n == 2) {
        polar2<T>(a, q, dsign, smin);
    } else {
        polar_jacobi<T, n>(a, q, dsign, smin);
    }
}

// Vector-Jacobian product of the projection at a (n >= 2): with a = U Sigma V^t
// and Q = U V^t, a perturbation da moves Q by U X V^t, X skew with
// X_ij = (F_ij - F_ji) / (sigma_i + sigma_j), F = U^t da V.  The cotangent g of
// Q therefore pulls back to ga = U K V^t, K_ij = (M_ij - M_ji) / (sigma_i +
// sigma_j), M = U^t g V (K_ii = 0; a pair with sigma_i + sigma_j = 0 gives 0).
// Returns the smallest singular value of a.
template <typename T, int n>
__device__ __forceinline__ T polar_vjp(const T* a, const T* g, T* ga)
{
    const int ex = scale_exponent<T, n>(a);
    T W[n][n], V[n][n], sig[n], q[n * n];
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            W[i][j] = ldexp(a[i * n + j], -ex);
            V[i][j] = (i == j) ? (T)1 : (T)0;
        }
    jacobi_sweeps<T, n>(W, V);
    int ds;
    T smin;
    jacobi_finish<T, n>(W, V, ex, q, ds, smin, sig);
    T smax = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) smax = sig[j] > smax ? sig[j] : smax;
    if (!(smax > (T)0)) {  // zero matrix: no pair has a positive denominator
#pragma unroll
        for (int k = 0; k < n * n; ++k) ga[k] = 0;
        return smin;
    }
    T GV[n][n], K[n][n];
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            T v = 0;
#pragma unroll
            for (int l = 0; l < n; ++l) v += g[i * n + l] * V[l][j];
            GV[i][j] = v;
        }
    T M[n][n];
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            T v = 0;
#pragma unroll
            for (int k = 0; k < n; ++k) v += W[k][i] * GV[k][j];
            M[i][j] = v;
        }
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            const T den = sig[i] + sig[j];
            K[i][j] = (i == j || !(den > (T)0)) ? (T)0 : (M[i][j] - M[j][i]) / den;
        }
    // ga = U K V^t
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            T uk = 0;
#pragma unroll
            for (int k = 0; k < n; ++k) uk += W[i][k] * K[k][j];
            GV[i][j] = uk;
        }
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            T v = 0;
#pragma unroll
            for (int k = 0; k < n; ++k) v += GV[i][k] * V[j][k];
            ga[i * n + j] = v;
        }
    return smin;
}

// Cofactor matrix of a row-major 3x3 matrix (cof(X) = det(X) X^{-T}).
template <typename T>
__device__ __forceinline__ void cofactor3(const T* x, T* c)
{
    c[0] = x[4] * x[8] - x[5] * x[7];
    c[1] = x[5] * x[6] - x[3] * x[8];
    c[2] = x[3] * x[7] - x[4] * x[6];
    c[3] = x[2] * x[7] - x[1] * x[8];
    c[4] = x[0] * x[8] - x[2] * x[6];
    c[5] = x[1] * x[6] - x[0] * x[7];
    c[6] = x[1] * x[5] - x[2] * x[4];
    c[7] = x[2] * x[3] - x[0] * x[5];
    c[8] = x[0] * x[4] - x[1] * x[3];
}

// Cofactor matrix of a row-major 4x4 matrix, from the 2x2 minors of rows 0-1
// (s) and rows 2-3 (t): a cofactor of row 0 or 1 expands its 3x3 minor along
// the other of the two rows against t, one of row 2 or 3 along the other of
// those rows against s.
template <typename T>
__device__ __forceinline__ void cofactor4(const T* x, T* c)
{
    const T* a = x;
    const T* b = x + 4;
    const T* e = x + 8;
    const T* d = x + 12;
    const T s01 = a[0] * b[1] - a[1] * b[0], s02 = a[0] * b[2] - a[2] * b[0], s03 = a[0] * b[3] - a[3] * b[0];
    const T s12 = a[1] * b[2] - a[2] * b[1], s13 = a[1] * b[3] - a[3] * b[1], s23 = a[2] * b[3] - a[3] * b[2];
    const T t01 = e[0] * d[1] - e[1] * d[0], t02 = e[0] * d[2] - e[2] * d[0], t03 = e[0] * d[3] - e[3] * d[0];
    const T t12 = e[1] * d[2] - e[2] * d[1], t13 = e[1] * d[3] - e[3] * d[1], t23 = e[2] * d[3] - e[3] * d[2];
    // minors of rows {1,2,3} (row 0's cofactors) and {0,2,3} (row 1's)
    c[0] = b[1] * t23 - b[2] * t13 + b[3] * t12;
    c[1] = -(b[0] * t23 - b[2] * t03 + b[3] * t02);
    c[2] = b[0] * t13 - b[1] * t03 + b[3] * t01;
    c[3] = -(b[0] * t12 - b[1] * t02 + b[2] * t01);
    c[4] = -(a[1] * t23 - a[2] * t13 + a[3] * t12);
    c[5] = a[0] * t23 - a[2] * t03 + a[3] * t02;
    c[6] = -(a[0] * t13 - a[1] * t03 + a[3] * t01);
    c[7] = a[0] * t12 - a[1] * t02 + a[2] * t01;
    // minors of rows {0,1,3} (row 2's) and {0,1,2} (row 3's)
    c[8] = d[1] * s23 - d[2] * s13 + d[3] * s12;
    c[9] = -(d[0] * s23 - d[2] * s03 + d[3] * s02);
    c[10] = d[0] * s13 - d[1] * s03 + d[3] * s01;
    c[11] = -(d[0] * s12 - d[1] * s02 + d[2] * s01);
    c[12] = -(e[1] * s23 - e[2] * s13 + e[3] * s12);
    c[13] = e[0] * s23 - e[2] * s03 + e[3] * s02;
    c[14] = -(e[0] * s13 - e[1] * s03 + e[3] * s01);
    c[15] = e[0] * s12 - e[1] * s02 + e[2] * s01;
}

template <typename T, int n>
__device__ __forceinline__ void cofactor_n(const T* x, T* c)
{
    static_assert(n == 3 || n == 4, "cofactors of 3x3 and 4x4 matrices");
    if constexpr (n == 3) cofactor3(x, c);
    else cofactor4(x, c);
}

// Constants of the Newton polar iteration by precision: the unit roundoff u,
// the smallest squared cofactor norm accepted (the first step's products must
// stay normal), and the bounds on |X|_F^2 - 3 that end the scaled phase and
// start the last step (newton3_near_done).
template <typename T> struct newton3_consts;
template <> struct newton3_consts<float> {
    static constexpr float u = 5.9604644775390625e-08f;  // 2^-24
    static constexpr float cf2_min = 1e-36f;
    static constexpr float unscaled = 2e-2f, last = 1.2e-3f;
};
template <> struct newton3_consts<double> {
    static constexpr double u = 1.1102230246251565e-16;  // 2^-53
    static constexpr double cf2_min = 1e-280;
    static constexpr double unscaled = 2e-2, last = 1e-7;
};

// Stopping test of the Newton polar iteration from xf2 = |X|_F^2 at the start
// of a step after the first (n x n).  A step maps each singular value s to
// (z s + 1/(z s)) / 2 >= 1, so from then on xf2 - n = sum (s_i^2 - 1) has no
// negative term and bounds every s_i - 1 by half its value.  Scaling stops
// once that is below unscaled / 2 (quadratic convergence takes over), and the
// step is the last once it is below last / 2: the step then leaves an error of
// about (last / 2)^2 / 2 (float: 1.8e-7, below the FP32 bar by far and about
// the rounding of the result; double: 1.3e-15).  A rounding of xf2 below the
// bound only ends the iteration where it has converged to that rounding.
template <typename T, int n = 3>
__device__ __forceinline__ void newton3_near_done(T xf2, bool& scaled, bool& last)
{
    const T e = xf2 - (T)n;
    if (e < newton3_consts<T>::unscaled) scaled = false;
    last = e < newton3_consts<T>::last;
}

// Whether the n x n matrix a (n = 3, 4; cofactors C, det, squared cofactor
// norm cf2) certainly has sigma_min > thr.
template <typename T, int n = 3>
__device__ __forceinline__ bool newton3_certain(const T* a, const T* C, T det, T cf2, T thr)
{
    // 1/|A^{-1}|_F = |det| / |cof A|_F <= sigma_min, so |det| > thr |cof|_F
    // proves sigma_min > thr, provided the computed det and cofactors are
    // accurate enough.  n = 3: a cofactor (a 2x2 minor) carries an error of at
    // most 2u|A|_F^2 and det at most 4u|A|_F^3 + 3u|A|_F|cof|_F.  n = 4: a
    // cofactor (a 3x3 minor from 2x2 minors) at most 8u|A|_F^3, so 32u|A|_F^3
    // over the matrix, and det at most 32u|A|_F^4 + 4u|A|_F|cof|_F.  The test
    // is made with that margin (doubled).  Without it a numerically
    // rank-deficient matrix, whose cofactors are mostly rounding, could pass.
    // Strict: det = 0 with a zero cofactor matrix fails, and so does a matrix
    // whose squared cofactor norm is not a normal number with room (the first
    // step's products would underflow; Jacobi rescales by a power of two), one
    // whose cofactors overflow (then thr |cof|_F is infinite), and NaN.
    T af2 = 0;
#pragma unroll
    for (int k = 0; k < n * n; ++k) af2 += a[k] * a[k];
    const T an = num<T>::sqrt_(af2), cn = num<T>::sqrt_(cf2);
    const T u = newton3_consts<T>::u;
    T margin;
    if constexpr (n == 3) margin = (T)2 * u * (thr * ((T)6 * af2 + cn) + an * ((T)4 * af2 + (T)3 * cn));
    else margin = (T)2 * u * (thr * ((T)32 * an * af2 + cn) + an * ((T)32 * an * af2 + (T)4 * cn));
    const T adet = det < (T)0 ? -det : det;
    return (cf2 >= newton3_consts<T>::cf2_min) && (adet > thr * cn + margin);
}

// Closest orthogonal matrix of an n x n matrix (n = 3, 4) by the scaled
// Newton iteration for the polar decomposition, X <- (zeta X + X^{-T} / zeta)
// / 2 (Higham, 1986), X^{-T} = cof(X) / det(X), with Frobenius-norm scaling
// zeta = (|X^{-1}|_F / |X|_F)^{1/2} until the singular values are near 1 and
// unscaled steps after it (newton3_near_done).  Each step maps every singular
// value s to (zeta s + 1/(zeta s)) / 2 and keeps U, V and the sign of det, so
// the limit is U V^t; convergence is quadratic.  Returns false (q unset)
// unless newton3_certain proves sigma_min > thr (it fails when sigma_min may
// be at most about sqrt(n) thr, when A is singular or numerically of lower
// rank); such points go to the Jacobi route.
template <typename T, int n>
__device__ __forceinline__ bool polar_newton(const T* a, T* q, int& dsign, T thr)
{
    constexpr int NN = n * n;
    T X[NN], C[NN];
#pragma unroll
    for (int k = 0; k < NN; ++k) X[k] = a[k];
    cofactor_n<T, n>(X, C);
    T det = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) det += X[j] * C[j];
    T cf2 = 0;
#pragma unroll
    for (int k = 0; k < NN; ++k) cf2 += C[k] * C[k];
    if (!newton3_certain<T, n>(X, C, det, cf2, thr)) return false;
    dsign = det >= (T)0 ? 1 : -1;
    bool scaled = true;
#pragma unroll 1
    for (int it = 0; it < 16; ++it) {
        if (it > 0) {
            cofactor_n<T, n>(X, C);
            det = 0;
#pragma unroll
            for (int j = 0; j < n; ++j) det += X[j] * C[j];
            cf2 = 0;
#pragma unroll
            for (int k = 0; k < NN; ++k) cf2 += C[k] * C[k];
        }
        T xf2 = 0;
#pragma unroll
        for (int k = 0; k < NN; ++k) xf2 += X[k] * X[k];
        bool last = false;
        if (it > 0) newton3_near_done<T, n>(xf2, scaled, last);
        const T idet = (T)1 / det;
        // zeta^2 = |C/det|_F / |X|_F
        const T zeta = scaled ? num<T>::sqrt_(num<T>::sqrt_(cf2) * (idet < (T)0 ? -idet : idet) * num<T>::rsq(xf2))
                              : (T)1;
        const T cx = (T)0.5 * zeta, cc = (T)0.5 * idet / zeta;
#pragma unroll
        for (int k = 0; k < NN; ++k) X[k] = cx * X[k] + cc * C[k];
        if (last) break;
    }
#pragma unroll
    for (int k = 0; k < NN; ++k) q[k] = X[k];
    return true;
}

template <typename T>
__device__ __forceinline__ bool polar_newton3(const T* a, T* q, int& dsign, T thr)
{
    return polar_newton<T, 3>(a, q, dsign, thr);
}

// Double plans take the Newton route for n = 3, 4 points whose smallest
// singular value is certainly above this (Jacobi below it).
constexpr double kNewtonMinSigmaF64 = 1e-3;

// Float Jacobi of a point of a plan with the double fallback: when the smallest
// singular value is below sigma_fb it stops before forming Q and returns true,
// leaving in V the right singular vectors that warm-start the double run;
// otherwise it returns false with the float result in q and dsign.
template <int n>
__device__ __forceinline__ bool polar_jacobi_f32_fb(const float* a, float* q, int& dsign,
                                                    float (&V)[n][n], double sigma_fb)
{
    const int ex = scale_exponent<float, n>(a);
    float W[n][n];
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            W[i][j] = ldexp(a[i * n + j], -ex);
            V[i][j] = (i == j) ? 1.0f : 0.0f;
        }
    jacobi_sweeps<float, n>(W, V);
    float s2 = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) {
        float v = 0;
#pragma unroll
        for (int i = 0; i < n; ++i) v += W[i][j] * W[i][j];
        s2 = (j == 0 || v < s2) ? v : s2;
    }
    if ((double)ldexp(num<float>::sqrt_(s2), ex) < sigma_fb) return true;
    float smin;
    jacobi_finish<float, n>(W, V, ex, q, dsign, smin);
    return false;
}

// Projection of a point in the plan's precision T, with the double-precision
// fallback of float plans: when fallback is set and the float-computed smallest
// singular value is below sigma_fb, the point is projected again in double from
// the same float values (n = 2 by the closed form, n >= 3 by Jacobi
// warm-started from the float run's V).  Returns true when it fell back.
template <typename T, int n>
__device__ __forceinline__ bool project_point_fb(const T* a, T* q, int& dsign, bool fallback,
                                                 double sigma_fb)
{
    constexpr int NN = n * n;
    if constexpr (sizeof(T) == 4 && n >= 3) {
        // well-conditioned points (sigma_min >= sigma_fb): Newton, no fallback
        if (polar_newton<float, n>(a, q, dsign, (float)sigma_fb)) return false;
    }
    if constexpr (sizeof(T) == 8 && n >= 3) {
        if (polar_newton<double, n>(a, q, dsign, kNewtonMinSigmaF64)) return false;
    }
    if constexpr (sizeof(T) == 4 && n >= 3) {
        if (fallback) {
            float V[n][n];
            if (!polar_jacobi_f32_fb<n>(a, q, dsign, V, sigma_fb)) return false;
            polar_jacobi_warm<n>(a, V, q, dsign);
            return true;
        }
    }
    T smin;
    project_point<T, n>(a, q, dsign, smin);
    if constexpr (sizeof(T) == 4 && n == 2) {
        if (fallback && (double)smin < sigma_fb) {
            double ad[4], qd[4], smd;
#pragma unroll
            for (int k = 0; k < 4; ++k) ad[k] = (double)a[k];
            polar2<double>(ad, qd, dsign, smd);
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = (T)qd[k];
            return true;
        }
    }
    return false;
}

// True when every one of the m values is finite.
template <typename T, int m>
__device__ __forceinline__ bool all_finite(const T* a)
{
    bool ok = true;
#pragma unroll
    for (int i = 0; i < m; ++i) ok = ok && (a[i] - a[i] == (T)0);
    return ok;
}

}  // namespace mbo
