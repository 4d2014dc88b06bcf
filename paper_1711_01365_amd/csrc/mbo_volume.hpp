// Device building blocks of the volume-preserving MBO step (Section 7 of
// Osting & Wang, arXiv:1711.01365): the two candidates T+ / T- of a point
// (Lemma 7.1 with Lemma 1.1), the increment Delta E = <T+ - T-, A>_F that ranks
// the points, an order-preserving integer key of Delta E for the radix
// selection, and the membership test of a finished selection.
#pragma once

#include "mbo_device.hpp"
#include "mbo_internal.hpp"

namespace mbo {

// Unsigned key with key(u) < key(v) exactly when u < v as numbers; -0 and +0
// share the key of +0 (they compare equal).  NaN sorts above +Inf or below -Inf
// by its sign bit.
__device__ __forceinline__ unsigned long long vp_key(float v)
{
    unsigned u = __float_as_uint(v);
    if ((u << 1) == 0u) u = 0u;
    return (u & 0x80000000u) ? (unsigned long long)(~u) : (unsigned long long)(u | 0x80000000u);
}

__device__ __forceinline__ unsigned long long vp_key(double v)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    if ((u << 1) == 0ull) u = 0ull;
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// True when point idx (key of its Delta E) is among the n_plus selected points
// of a field whose selection has finished.
__device__ __forceinline__ bool vp_member(const VpSel& s, unsigned long long key, int64_t idx)
{
    switch (s.mode) {
    case VS_ALL: return true;
    case VS_TIES_ALL: return key >= s.kstar;
    case VS_TIES_PART: return key > s.kstar || (key == s.kstar && idx <= s.istar);
    default: return false;  // VS_NONE
    }
}

// T+ (closest point of SO(n)), T- (closest point of SO^-(n)) and Delta E of one
// matrix a in precision T.
//   n = 1: T+ = 1, T- = -1, Delta E = 2a.
//   n = 2: the closest rotation [[c,-s],[s,c]] maximises c (a00 + a11) +
//     s (a10 - a01), the closest reflection [[c,s],[s,-c]] maximises
//     c (a00 - a11) + s (a01 + a10); with r+ and r- those maxima, Delta E =
//     r+ - r- = 4 det(a) / (r+ + r-) (the form without cancellation).  A zero
//     maximiser direction (r = 0: every candidate is equally close) takes c = 1.
//   n >= 3: one-sided Jacobi gives a = U Sigma V^t and Q = U V^t; with j the
//     first column of the smallest singular value, Q' = Q - 2 u_j v_j^t =
//     U D V^t reverses that direction (Lemma 7.1).  The one of Q, Q' with
//     det +1 is T+, and Delta E = 2 sgn(det Q) sigma_min.
template <typename T, int n>
__device__ __forceinline__ T vp_candidates(const T* a_in, T* tp, T* tm)
{
    const T* a = a_in;
    if constexpr (n == 1) {
        tp[0] = (T)1;
        tm[0] = (T)-1;
        return a[0] + a[0];
    } else if constexpr (n == 2) {
        // scaled by a power of two first (exact), as in polar2: no square or
        // product under- or overflows; Delta E scales back by the same power
        const int ex = scale_exponent<T, 2>(a_in);
        T a[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = ldexp(a_in[k], -ex);
        const T p1 = a[0] + a[3], s1 = a[2] - a[1];
        const T p2 = a[0] - a[3], s2 = a[1] + a[2];
        const T q1 = p1 * p1 + s1 * s1, q2 = p2 * p2 + s2 * s2;
        const T i1 = q1 > (T)0 ? num<T>::rsq(q1) : (T)0;
        const T i2 = q2 > (T)0 ? num<T>::rsq(q2) : (T)0;
        const T c1 = q1 > (T)0 ? p1 * i1 : (T)1, n1 = s1 * i1;
        const T c2 = q2 > (T)0 ? p2 * i2 : (T)1, n2 = s2 * i2;
        tp[0] = c1; tp[1] = -n1; tp[2] = n1; tp[3] = c1;
        tm[0] = c2; tm[1] = n2; tm[2] = n2; tm[3] = -c2;
        const T r = q1 * i1 + q2 * i2;  // r+ + r-
        const T det = a[0] * a[3] - a[1] * a[2];
        return r > (T)0 ? ldexp((T)4 * det / r, ex) : (T)0;
    } else {
        const int ex = scale_exponent<T, n>(a);
        T W[n][n], V[n][n];
#pragma unroll
        for (int i = 0; i < n; ++i)
#pragma unroll
            for (int j = 0; j < n; ++j) {
                W[i][j] = ldexp(a[i * n + j], -ex);
                V[i][j] = (i == j) ? (T)1 : (T)0;
            }
        jacobi_sweeps<T, n>(W, V);
        T q[n * n], sig[n], smin;
        int ds;
        jacobi_finish<T, n>(W, V, ex, q, ds, smin, sig);
        // W holds U (the zero matrix leaves W = 0 and V = I: then U = I too,
        // with Q = I); pick the column of the smallest singular value
        T u[n], v[n];
        int jm = 0;
        bool zero = !(sig[0] > (T)0);
#pragma unroll
        for (int j = 1; j < n; ++j) {
            jm = sig[j] < sig[jm] ? j : jm;
            zero = zero && !(sig[j] > (T)0);
        }
#pragma unroll
        for (int i = 0; i < n; ++i) {
            u[i] = zero ? (i == 0 ? (T)1 : (T)0) : W[i][0];
            v[i] = V[i][0];
#pragma unroll
            for (int j = 1; j < n; ++j) {
                u[i] = (jm == j && !zero) ? W[i][j] : u[i];
                v[i] = jm == j ? V[i][j] : v[i];
            }
        }
#pragma unroll
        for (int i = 0; i < n; ++i)
#pragma unroll
            for (int k = 0; k < n; ++k) {
                const T r = q[i * n + k] - (T)2 * u[i] * v[k];
                tp[i * n + k] = ds > 0 ? q[i * n + k] : r;
                tm[i * n + k] = ds > 0 ? r : q[i * n + k];
            }
        return ds > 0 ? smin + smin : -(smin + smin);
    }
}

// The same in the plan's precision T, with the double-precision fallback of
// float plans: when fallback is set and the float-computed smallest singular
// value (|Delta E| / 2) is below sigma_fb, the point is evaluated again in double
// from the same float values and rounded.  Returns true when it fell back.
template <typename T, int n>
__device__ __forceinline__ bool vp_point(const T* a, T* tp, T* tm, T& de, bool fallback, double sigma_fb)
{
    de = vp_candidates<T, n>(a, tp, tm);
    if constexpr (sizeof(T) == 4 && n >= 2) {
        const T half = (de < (T)0 ? -de : de) * (T)0.5;
        if (fallback && (double)half < sigma_fb) {
            double ad[n * n], pd[n * n], md[n * n];
#pragma unroll
            for (int k = 0; k < n * n; ++k) ad[k] = (double)a[k];
            const double dd = vp_candidates<double, n>(ad, pd, md);
#pragma unroll
            for (int k = 0; k < n * n; ++k) {
                tp[k] = (T)pd[k];
                tm[k] = (T)md[k];
            }
            de = (T)dd;
            return true;
        }
    }
    return false;
}

}  // namespace mbo
