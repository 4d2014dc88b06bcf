// Band-limited passes of Algorithm 1 on the 2-D flat torus for gfx950: the
// diffusion step of Section 5.1 (FFT, multiply by exp(-4 pi^2 tau |k|^2),
// inverse FFT) and the projection of Lemma 1.1, in two kernels per iteration.
//
// Kept modes.  The heat symbol is a product over the axes of
// exp(-4 pi^2 tau k^2); along an axis of length N the host keeps |k| <= c,
// with c the smallest half-width whose discarded symbol mass
// sum_{k outside the kept box} exp(-4 pi^2 tau |k|^2) is at most eta.  A value
// of the diffused field then moves by at most eta * max|A| when those modes
// are dropped (|A^(k)| <= N^d max|A| for every mode), far below the rounding of
// the transforms themselves (eta = 1e-12 for float plans, 1e-20 for double
// plans).  The row pass therefore stores, for every row, only the row spectrum
// at kx = 0..c and kx = N-c..N-1, in W slots per row (slot w holds kx = w for
// w <= c and kx = N - W + w for w >= W - c; the slots between hold zeros), and
// the column pass transforms only those W columns.  With c >= N/2 nothing is
// dropped and W = N.
//
//   row_fast   one workgroup owns 512 points (512/L whole rows) or, for rows of
//              1024 and 2048 points, one row: the line groups of its packed
//              planes load their kept modes straight into the FFT register
//              layout (lane t holds x[t + e L/8]), inverse-FFT (inside one wave
//              for L <= 512, with workgroup exchanges and in rounds of lines
//              beyond) and leave the lines in LDS; 512 threads, one to four
//              points each, project (Lemma 1.1) with the det-sign,
//              fallback, non-finite and change diagnostics; the line groups
//              forward-FFT and store the kept modes.  Float plans with n = 3
//              run the Newton polar iteration on every point that is certainly
//              well conditioned (1/|A^{-1}|_F > sigma_fb) and queue the others
//              for the first wave done with its own points, which projects
//              them by Jacobi (and in double when sigma_min < sigma_fb) at
//              raised priority.
//   heat_fast  a tile of TX stored columns of one packed plane: thread (t, cc)
//              loads rows t + e L/8 of column cc (TX-wide coalesced segments),
//              forward FFT along the column with workgroup exchanges, Lyapunov
//              partial sum_k symbol |Z|^2 (Section 4), symbol multiply, inverse
//              FFT, store in place.
#pragma once

#include "mbo_kernels.hpp"

namespace mbo {

// Stored slot of row mode kx, or -1 when the mode is not kept.
__device__ __forceinline__ int band_slot(int kx, int L, int c, int W)
{
    if (kx <= c) return kx;
    if (kx >= L - c) return W - (L - kx);
    return -1;
}

// ---------------------------------------------------------------------------
// Float n = 3 Newton polar iteration (Higham, 1986), split so that the
// workgroup can decide which points it runs before iterating: the steps of
// polar_newton3 with hardware reciprocals.
// ---------------------------------------------------------------------------
struct Newton3 {
    float X[9], C[9];
    float det, cf2;
};

// True when the float test of newton3_certain proves sigma_min > thr;
// otherwise the point goes to the Jacobi route.
__device__ __forceinline__ bool newton3_init(const float* a, Newton3& s, float thr)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) s.X[k] = a[k];
    cofactor3(s.X, s.C);
    s.det = s.X[0] * s.C[0] + s.X[1] * s.C[1] + s.X[2] * s.C[2];
    s.cf2 = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) s.cf2 += s.C[k] * s.C[k];
    return newton3_certain(s.X, s.C, s.det, s.cf2, thr);
}

__device__ __forceinline__ void newton3_run(Newton3& s, float* q, int& dsign)
{
    dsign = s.det >= 0.f ? 1 : -1;
    bool scaled = true;
#pragma unroll 1
    for (int it = 0; it < 16; ++it) {
        if (it > 0) {
            cofactor3(s.X, s.C);
            s.det = s.X[0] * s.C[0] + s.X[1] * s.C[1] + s.X[2] * s.C[2];
            s.cf2 = 0.f;
#pragma unroll
            for (int k = 0; k < 9; ++k) s.cf2 += s.C[k] * s.C[k];
        }
        float xf2 = 0.f;
#pragma unroll
        for (int k = 0; k < 9; ++k) xf2 += s.X[k] * s.X[k];
        // the stopping test of polar_newton3 (newton3_near_done)
        bool last = false;
        if (it > 0) newton3_near_done(xf2, scaled, last);
        // hardware reciprocal (about 1 ulp): the iteration corrects its own
        // rounding, and a relative error of one ulp in the step's two scalar
        // factors stays below the float rounding of the result
        const float idet = num<float>::rcp(s.det);
        const float zeta = scaled ? num<float>::sqrt_(num<float>::sqrt_(s.cf2) * (idet < 0.f ? -idet : idet) *
                                                      num<float>::rsq(xf2))
                                  : 1.0f;
        const float cx = 0.5f * zeta, cc = 0.5f * idet * num<float>::rcp(zeta);
#pragma unroll
        for (int k = 0; k < 9; ++k) s.X[k] = cx * s.X[k] + cc * s.C[k];
        if (last) break;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) q[k] = s.X[k];
}

// ---------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------

// Shape of a row-pass workgroup: 512 points (512/L rows) for L <= 512, one row
// of L points otherwise; 512 projection threads (PPT points each); the line
// groups of L/8 threads run in ROUNDS rounds of G lines over NT threads.
template <typename T, int n, int LOG2L>
struct RowFastShape {
    static constexpr int L = 1 << LOG2L;
    static constexpr int Tn = L / 8;
    static constexpr int NN = n * n;
    static constexpr int PL = (NN + 1) / 2;
    static constexpr int RPW = L >= 512 ? 1 : 512 / L;
    static constexpr int P = RPW * L;
    static constexpr int PPT = P / 512;
    static constexpr int LINES = RPW * PL;
    static constexpr bool WAVE_LINE = LOG2L <= 9;
    static constexpr bool HELPER = sizeof(T) == 4 && n == 3;
    // float n = 4: points below sigma_fb are queued and re-projected in double
    // after the pass's loop (the double Jacobi inside the loop would spill)
    static constexpr bool DEFER4 = sizeof(T) == 4 && n == 4;
    // long rows: at most 768 threads for float n = 3 (twelve waves, a budget of
    // 168 registers for the queued points' double Jacobi), else 1024
    static constexpr int NTMAX = HELPER ? 768 : 1024;
    static constexpr int NT_LINES = LINES * Tn < NTMAX / Tn * Tn ? LINES * Tn : NTMAX / Tn * Tn;
    static constexpr int NT = WAVE_LINE ? 512 : (NT_LINES > 512 ? NT_LINES : 512);
    static constexpr int G = NT / Tn;  // lines per round
    static constexpr int ROUNDS = (LINES + G - 1) / G;
    static constexpr int THREADS = NT;
    static constexpr int LP = L + L / 8;  // padded LDS line
    static constexpr size_t LDS_LINES = (size_t)LINES * LP * 2 * sizeof(T);
    // the twiddle table staged in LDS, where it fits beside the lines and the
    // static arrays (the queue, at most 4 KiB; 12 KiB are reserved): one load
    // per thread instead of 7 per radix-8 stage
    static constexpr size_t TW_BYTES = (size_t)L * 2 * sizeof(T);
    static constexpr bool TW_LDS = LDS_LINES + TW_BYTES + 12288 <= 163840;
    static constexpr size_t LDS = LDS_LINES + (TW_LDS ? TW_BYTES : 0);
    // waves per SIMD the instance is compiled for: two 512-point workgroups
    // (eight waves each, two per SIMD) per CU for short rows, one long-row
    // workgroup.  The register budget this leaves (128) holds the queued
    // points' double Jacobi without spilling: any scratch use would delay the
    // launch of the workgroups, and a ninth wave per workgroup would leave
    // room for only one of them per CU at that budget.
    static constexpr int WAVES = WAVE_LINE ? 4 : (THREADS + 255) / 256;
};

template <typename T, int n, int LOG2L, bool PM>
__global__ void __launch_bounds__((RowFastShape<T, n, LOG2L>::THREADS), (RowFastShape<T, n, LOG2L>::WAVES))
    row_fast(const FastRowArgs a)
{
    typedef RowFastShape<T, n, LOG2L> S;
    constexpr int NN = S::NN, PL = S::PL, L = S::L, Tn = S::Tn, RPW = S::RPW, LP = S::LP;
    constexpr int G = S::G, ROUNDS = S::ROUNDS, NT = S::NT, PPT = S::PPT;
    constexpr bool HELPER = S::HELPER;
    typedef typename cx<T>::type C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lr = reinterpret_cast<T*>(smem_raw);
    T* li = lr + (size_t)S::LINES * LP;
    __shared__ unsigned short fq[(HELPER || S::DEFER4) ? S::P : 1];
    __shared__ int fq_n, fq_claim;
    // rows of at most 512 points (every wave holds points): the last wave's
    // Newton points, handed to the other waves when it runs the queue
    constexpr bool SPLIT = HELPER && S::THREADS == 512 && S::PPT == 1;
    __shared__ int hq[SPLIT ? 64 : 1];
    __shared__ int hq_n, hq_claim;
    __shared__ unsigned long long wg_cnt[2];

    const int flags = a.flags;
    const int b = blockIdx.y;
    const int tid = threadIdx.x;
    if (tid == 0) {
        fq_n = 0;
        fq_claim = 0;
        hq_n = 0;
        hq_claim = 0;
        wg_cnt[0] = 0;
        wg_cnt[1] = 0;
    }
    const int64_t npts = a.npts;
    const int W = a.W, c = a.band;
    // PM: spectra stored plane by plane (a.plane_major, the 3-D layout).
    constexpr bool pm = PM;
    // Plane by plane, a workgroup's loads and stores of one mode cover RPW
    // consecutive rows, part of a cache line: the eight XCDs (own L2 each) then
    // take contiguous runs of row groups, so that the groups sharing a line
    // run on one XCD.
    const int64_t nwgx = gridDim.x;
    const int64_t row0 = RPW * (((nwgx & 7) || !pm) ? (int64_t)blockIdx.x
                                                    : (int64_t)(blockIdx.x & 7) * (nwgx >> 3) + (blockIdx.x >> 3));
    C* Zb = reinterpret_cast<C*>(a.Z) + (size_t)b * PL * a.rows * W;

    // Every global load that does not depend on another is issued first (the
    // kept modes of the first round of lines, the twiddles, the previous det
    // signs, the stop mark): at the start of a launch each round trip to memory
    // is a cold miss, and none of them waits for another.
    const int g = tid / Tn, t = tid - (tid / Tn) * Tn;
    const int pt = lds_pad(t);
    const bool fft_thread = tid < NT;
    Twiddles<T, LOG2L> tw;
    T r[1][8], im[1][8];
    // Line j of a round is row rl, packed plane pl of the workgroup (LDS line
    // rl*PL + pl).  Spectra are stored row by row (Z[plane][row][w]) or, for
    // the 3-D plane pass, plane by plane (Z[plane][w][row]): there the lines
    // of one plane go to neighbouring groups, so that a wave's stores of one
    // mode cover consecutive rows.
    auto line_of = [&](int j, int& rl, int& pl) {
        if (pm) {
            rl = j % RPW;
            pl = j / RPW;
        } else {
            rl = j / PL;
            pl = j - (j / PL) * PL;
        }
    };
    auto zat = [&](int pl, int64_t row, int w) -> size_t {
        return pm ? ((size_t)pl * W + w) * a.rows + row : ((size_t)pl * a.rows + row) * W + w;
    };
    auto load_line = [&](int j) {
        int rl, pl;
        line_of(j, rl, pl);
        const bool live = j < S::LINES && row0 + rl < a.rows;
        const int64_t row = live ? row0 + rl : 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int w = band_slot(t + e * Tn, L, c, W);
            C v;
            if (live && w >= 0) v = Zb[zat(pl, row, w)];
            else { v.x = 0; v.y = 0; }
            r[0][e] = v.x;
            im[0][e] = v.y;
        }
    };
    if ((flags & RF_INVERSE) && fft_thread) load_line(g);
    const C* twg = reinterpret_cast<const C*>(a.tw);
    C* twl = reinterpret_cast<C*>(smem_raw + S::LDS_LINES);
    if constexpr (S::TW_LDS) {
        if (flags & (RF_INVERSE | RF_FORWARD)) {
            for (int m = tid; m < L; m += S::THREADS) twl[m] = twg[m];
            __syncthreads();
        }
    }
    if (fft_thread && (flags & RF_INVERSE)) load_twiddles<T, LOG2L>(tw, S::TW_LDS ? twl : twg, t);
    int8_t* sgn = a.sgn + (size_t)b * npts;
    // previous det signs of the thread's points, a byte each (a register, not
    // an array: the projection loops index it at run time)
    unsigned s_old = 0;
#pragma unroll
    for (int pp = 0; pp < PPT; ++pp) {
        const int idx = pp * 512 + tid;
        const bool live = tid < 512 && row0 + (idx >> LOG2L) < a.rows;
        const int8_t so = (live && (flags & RF_SIGN)) ? sgn[(row0 + (idx >> LOG2L)) * L + (idx & (L - 1))] : (int8_t)0;
        s_old |= (unsigned)(uint8_t)so << (8 * pp);
    }
    const int stop = (flags & RF_CHECK_STOP) ? a.stop_iter[b] : a.iter;

    // ---- phase 1: inverse FFT of each line, natural order into LDS
    if (flags & RF_INVERSE) {
#pragma unroll 1
        for (int rd = 0; rd < ROUNDS; ++rd) {
            const int j = rd * G + g;
            const bool act = fft_thread && j < S::LINES;
            if (rd > 0 && fft_thread) load_line(j);
            int rl, pl;
            line_of(j, rl, pl);
            const int lj = act ? rl * PL + pl : 0;
            T* lrj = lr + (size_t)lj * LP;
            T* lij = li + (size_t)lj * LP;
            if constexpr (S::WAVE_LINE) {
                if (act) {
                    // with c < L/8 only the loads e = 0, 7 hold kept modes (float, n <= 3:
                    // the double and n = 4 instances have no registers to spare for a
                    // second copy of the transform)
                    if constexpr (sizeof(T) == 4 && n <= 3 && FftShape<LOG2L>::R0 == 1 && FftShape<LOG2L>::NST > 1) {
                        if (c < Tn) fft_wave<T, +1, LOG2L, 0, FFT_IN07>(r[0], im[0], lrj, lij, t, tw, true);
                        else fft_wave<T, +1, LOG2L>(r[0], im[0], lrj, lij, t, tw, true);
                    } else {
                        fft_wave<T, +1, LOG2L>(r[0], im[0], lrj, lij, t, tw, true);
                    }
                    wave_lds_sync();  // the line's last exchange has been read
                }
            } else {
                fft_lines<T, +1, 1, LOG2L>(r, im, lrj, lij, 0, 1, 0, t, tw, act);
                __syncthreads();  // the line's last exchange has been read
            }
            if (act) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    lrj[lds_pad_at<Tn>(t, pt, e)] = r[0][e];
                    lij[lds_pad_at<Tn>(t, pt, e)] = im[0][e];
                }
            }
        }
    }
    // a field that already stopped is left alone (uniform per workgroup; the
    // loads above only read)
    if (stop < a.iter) return;

    // ---- phase 2: PPT points per projection thread
    T* Aout = reinterpret_cast<T*>(a.Aout) + field_base(a.foff, b, NN * npts);
    unsigned long long nflip = 0, nfb = 0, nbad = 0;
    double dmax = 0.0;
    const bool fallback = (flags & RF_FALLBACK) != 0;
    auto point_of = [&](int idx, int64_t& xp, T*& lrq, T*& liq) {
        const int rq = idx >> LOG2L, xq = idx & (L - 1);
        xp = (row0 + rq) * L + xq;
        lrq = lr + (size_t)rq * PL * LP + lds_pad(xq);
        liq = li + (size_t)rq * PL * LP + lds_pad(xq);
        return row0 + rq < a.rows;
    };

    // diagnostics and write-back of a projected point (LDS slot at lrq/liq)
    auto finish = [&](int64_t xp, T* lrq, T* liq, const T (&qv)[NN], int ds, int8_t so) {
        if (flags & RF_SIGN) {
            nflip += (so != (int8_t)ds) ? 1ull : 0ull;
            sgn[xp] = (int8_t)ds;
        }
        if (flags & RF_TRACK) {
#pragma unroll
            for (int k = 0; k < NN; ++k) {
                const double dv = fabs((double)qv[k] - (double)Aout[(int64_t)k * npts + xp]);
                dmax = dv > dmax ? dv : dmax;
            }
        }
        if (flags & RF_STORE_REAL) {
#pragma unroll
            for (int k = 0; k < NN; ++k) Aout[(int64_t)k * npts + xp] = qv[k];
        }
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            if (k & 1) liq[(k >> 1) * LP] = qv[k];
            else lrq[(k >> 1) * LP] = qv[k];
        }
        if (NN & 1) liq[(NN >> 1) * LP] = (T)0;
    };
    auto load_point = [&](const T* lrq, const T* liq, T (&av)[NN]) {
#pragma unroll
        for (int k = 0; k < NN; ++k) av[k] = (k & 1) ? liq[(k >> 1) * LP] : lrq[(k >> 1) * LP];
    };

    if (flags & RF_LOAD_REAL) {
        // forward transform of a real field: the points' entries from A
        const T* A = reinterpret_cast<const T*>(a.Ain) + field_base(a.foff, b, NN * npts);
#pragma unroll 1
        for (int pp = 0; pp < PPT; ++pp) {
            int64_t xp;
            T *lrq, *liq;
            if (tid < 512 && point_of(pp * 512 + tid, xp, lrq, liq)) {
                T av[NN];
#pragma unroll
                for (int k = 0; k < NN; ++k) av[k] = A[(int64_t)k * npts + xp];
                if (flags & RF_SIGN_INIT) sgn[xp] = det_n<T, n>(av) >= (T)0 ? 1 : -1;
#pragma unroll
                for (int k = 0; k < NN; ++k) {
                    if (k & 1) liq[(k >> 1) * LP] = av[k];
                    else lrq[(k >> 1) * LP] = av[k];
                }
                if (NN & 1) liq[(NN >> 1) * LP] = (T)0;
            }
        }
    }
    __syncthreads();

    if (flags & RF_PROJECT) {
        if constexpr (HELPER) {
            // which points are certainly well conditioned: the Newton
            // iteration; the others are queued
            Newton3 ns;       // kept from the test when each thread has one point
            unsigned ok = 0;  // bit pp: point pp runs Newton
#pragma unroll 1
            for (int pp = 0; pp < PPT; ++pp) {
                int64_t xp;
                T *lrq, *liq;
                if (tid < 512 && point_of(pp * 512 + tid, xp, lrq, liq)) {
                    T av[NN];
                    load_point(lrq, liq, av);
                    nbad += all_finite<T, NN>(av) ? 0ull : 1ull;
                    if (newton3_init(av, ns, (float)a.sigma_fb)) {
                        ok |= 1u << pp;
                        // the last wave's Newton points, with their previous
                        // det sign, for the other waves to take over when it
                        // becomes the queue's wave
                        if (SPLIT && tid >= 512 - 64)
                            hq[atomicAdd(&hq_n, 1)] = (pp * 512 + tid) | ((int)(uint8_t)(s_old >> (8 * pp)) << 16);
                    } else {
                        fq[atomicAdd(&fq_n, 1)] = (unsigned short)(pp * 512 + tid);
                    }
                }
            }
            __syncthreads();
            // Queued points: Jacobi in float, and in double (warm-started from
            // the float right singular vectors) when sigma_min < sigma_fb, at
            // raised priority, one point per lane of the wave that runs them.
            auto run_queue = [&]() {
                __builtin_amdgcn_s_setprio(3);
                const int nq = fq_n;
                const int lane = tid & 63;
#pragma unroll 1
                for (int qi = lane; qi < nq; qi += 64) {
                    int64_t xp;
                    T *lrq, *liq;
                    (void)point_of(fq[qi], xp, lrq, liq);
                    float aq[NN], qv[NN];
                    load_point(lrq, liq, aq);
                    int ds;
                    if (fallback) {
                        float V[n][n];
                        if (polar_jacobi_f32_fb<n>(aq, qv, ds, V, a.sigma_fb)) {
                            polar_jacobi_warm<n>(aq, V, qv, ds);
                            ++nfb;
                        }
                    } else {
                        float smin;
                        polar_jacobi<float, n>(aq, qv, ds, smin);
                    }
                    finish(xp, lrq, liq, qv, ds, (flags & RF_SIGN) ? sgn[xp] : (int8_t)0);
                }
                __builtin_amdgcn_s_setprio(0);
            };
            // With every wave holding points (rows of at most 512 points) and a
            // non-empty queue, the last wave starts on the queue at once and
            // the first wave done with its own points takes the last wave's
            // Newton points: the queue's serial Jacobi chain then overlaps the
            // other waves' Newton iterations instead of following them.
            const bool split = SPLIT && fq_n > 0;
            const bool qwave = split && tid >= 512 - 64;
            if (tid < 512 && !qwave) {
#pragma unroll 1
                for (int pp = 0; pp < PPT; ++pp) {
                    if (!(ok >> pp & 1u)) continue;
                    int64_t xp;
                    T *lrq, *liq;
                    (void)point_of(pp * 512 + tid, xp, lrq, liq);
                    if constexpr (PPT > 1) {
                        T av[NN];
                        load_point(lrq, liq, av);
                        (void)newton3_init(av, ns, (float)a.sigma_fb);
                    }
                    T qv[NN];
                    int ds;
                    newton3_run(ns, qv, ds);
                    finish(xp, lrq, liq, qv, ds, (int8_t)(s_old >> (8 * pp)));
                }
            }
            if (split) {
                if (qwave) {
                    run_queue();
                } else {
                    // the last wave's Newton points, one per lane of the first
                    // wave(s) to get here (hq_n is final since the barrier)
#pragma unroll 1
                    for (;;) {
                        const int i = atomicAdd(&hq_claim, 1);
                        if (i >= hq_n) break;
                        const int e = hq[i];
                        int64_t xp;
                        T *lrq, *liq;
                        (void)point_of(e & 0xffff, xp, lrq, liq);
                        T av[NN];
                        load_point(lrq, liq, av);
                        Newton3 hs;
                        (void)newton3_init(av, hs, (float)a.sigma_fb);
                        T qv[NN];
                        int ds;
                        newton3_run(hs, qv, ds);
                        finish(xp, lrq, liq, qv, ds, (int8_t)(e >> 16));
                    }
                }
            } else {
                // The queued points go to the first wave done with its own
                // points (threads beyond the 512 projection threads, for long
                // rows, have none).  A wave of its own would cost the registers
                // that let two workgroups share a CU.
                int claim = 0;
                if ((tid & 63) == 0) claim = atomicAdd(&fq_claim, 1);
                claim = __shfl(claim, 0, 64);
                if (claim == 0) run_queue();
            }
        } else {
#pragma unroll 1
            for (int pp = 0; pp < PPT; ++pp) {
                int64_t xp;
                T *lrq, *liq;
                if (tid < 512 && point_of(pp * 512 + tid, xp, lrq, liq)) {
                    T av[NN], qv[NN];
                    load_point(lrq, liq, av);
                    nbad += all_finite<T, NN>(av) ? 0ull : 1ull;
                    int ds;
                    if constexpr (S::DEFER4) {
                        if (polar_newton<float, n>(av, qv, ds, (float)a.sigma_fb)) {
                            // well conditioned: Newton, no fallback
                        } else if (fallback) {
                            float V[n][n];
                            if (polar_jacobi_f32_fb<n>(av, qv, ds, V, a.sigma_fb)) {
                                fq[atomicAdd(&fq_n, 1)] = (unsigned short)(pp * 512 + tid);
                                continue;
                            }
                        } else {
                            T smin;
                            project_point<T, n>(av, qv, ds, smin);
                        }
                    } else {
                        if (project_point_fb<T, n>(av, qv, ds, fallback, a.sigma_fb)) ++nfb;
                    }
                    finish(xp, lrq, liq, qv, ds, (int8_t)(s_old >> (8 * pp)));
                }
            }
            if constexpr (S::DEFER4) {
                // the queued points: float Jacobi again for its V, then the
                // double Jacobi warm-started from it
                if (fallback) {
                    __syncthreads();
                    const int nq = fq_n;
#pragma unroll 1
                    for (int qi = tid; qi < nq; qi += S::THREADS) {
                        int64_t xp;
                        T *lrq, *liq;
                        (void)point_of(fq[qi], xp, lrq, liq);
                        float aq[NN], qv[NN];
                        load_point(lrq, liq, aq);
                        float V[n][n];
                        int ds;
                        (void)polar_jacobi_f32_fb<n>(aq, qv, ds, V, a.sigma_fb);
                        polar_jacobi_warm<n>(aq, V, qv, ds);
                        ++nfb;
                        finish(xp, lrq, liq, qv, ds, (flags & RF_SIGN) ? sgn[xp] : (int8_t)0);
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- phase 3: forward FFT of the lines, store the kept modes
    if (flags & RF_FORWARD) {
        // the twiddles again (from LDS or cache), into a fresh variable: the
        // values of phase 1 kept alive across the projection would raise its
        // register peak above what the kernel's occupancy allows
        Twiddles<T, LOG2L> tw3;
        if (fft_thread) load_twiddles<T, LOG2L>(tw3, S::TW_LDS ? twl : twg, t);
#pragma unroll 1
        for (int rd = 0; rd < ROUNDS; ++rd) {
            const int j = rd * G + g;
            const bool act = fft_thread && j < S::LINES;
            int rl, pl;
            line_of(j, rl, pl);
            const int lj = act ? rl * PL + pl : 0;
            T* lrj = lr + (size_t)lj * LP;
            T* lij = li + (size_t)lj * LP;
            T r3[1][8], im3[1][8];  // fresh, as tw3
            if (act) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    r3[0][e] = lrj[lds_pad_at<Tn>(t, pt, e)];
                    im3[0][e] = lij[lds_pad_at<Tn>(t, pt, e)];
                }
            }
            if constexpr (S::WAVE_LINE) {
                if (act) {
                    wave_lds_sync();  // every lane has read its elements before the exchanges
                    // with c < L/8 only the modes e = 0, 7 are stored
                    if constexpr (sizeof(T) == 4 && n <= 3 && FftShape<LOG2L>::NST > 1) {
                        if (c < Tn) fft_wave<T, -1, LOG2L, 0, FFT_OUT07>(r3[0], im3[0], lrj, lij, t, tw3, true);
                        else fft_wave<T, -1, LOG2L>(r3[0], im3[0], lrj, lij, t, tw3, true);
                    } else {
                        fft_wave<T, -1, LOG2L>(r3[0], im3[0], lrj, lij, t, tw3, true);
                    }
                }
            } else {
                fft_lines<T, -1, 1, LOG2L>(r3, im3, lrj, lij, 0, 1, 0, t, tw3, act);
            }
            if (act && row0 + rl < a.rows) {
                const int64_t row = row0 + rl;
                // slots w < W - c take mode w (zero when w > c); slots w >= W - c
                // take mode L - W + w
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int kx = t + e * Tn;
                    C v;
                    v.x = r3[0][e];
                    v.y = im3[0][e];
                    if (kx < W - c) {
                        if (kx > c) { v.x = 0; v.y = 0; }
                        Zb[zat(pl, row, kx)] = v;
                    } else if (kx >= L - c) {
                        Zb[zat(pl, row, W - L + kx)] = v;
                    }
                }
            }
        }
    }

    if (flags & (RF_PROJECT | RF_TRACK)) {
        // counts of the workgroup: packed 21 bits each (at most 2048 per workgroup)
        unsigned long long packed = wave_sum(nflip | (nfb << 21) | (nbad << 42));
        unsigned long long dbits = (unsigned long long)__double_as_longlong(dmax);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long ob = (unsigned long long)__shfl_xor((long long)dbits, o, 64);
            dbits = ob > dbits ? ob : dbits;
        }
        if ((tid & 63) == 0) {
            if (packed) atomicAdd(&wg_cnt[0], packed);
            if (dbits) atomicMax(&wg_cnt[1], dbits);
        }
        __syncthreads();
        if (tid == 0) {
            // the workgroup's packed counts into its own slot (summed per
            // iteration after the loop: no same-address atomics from every
            // workgroup at the end of the pass); the largest change by atomic max
            if (a.cnt_part)
                a.cnt_part[((int64_t)b * a.K + (a.iter - 1)) * gridDim.x + blockIdx.x] = wg_cnt[0];
            if ((flags & RF_TRACK) && a.delta_bits && wg_cnt[1])
                atomicMax(a.delta_bits + (int64_t)b * a.K + (a.iter - 1), wg_cnt[1]);
        }
    }
}

// ---------------------------------------------------------------------------
// Column pass over the stored columns
// ---------------------------------------------------------------------------

// Dynamic LDS of a heat_fast workgroup: the TX padded lines, then the twiddle
// table when it fits.
template <typename T, int LOG2L, int TX>
struct HeatFastShape {
    static constexpr int L = 1 << LOG2L;
    static constexpr size_t LINES = (size_t)TX * (L + L / 8) * 2 * sizeof(T);
    static constexpr size_t TW_BYTES = (size_t)L * 2 * sizeof(T);
    static constexpr bool TW_LDS = LINES + TW_BYTES <= 159744;
    static constexpr size_t LDS = LINES + (TW_LDS ? TW_BYTES : 0);
};

template <typename T, int LOG2L, int TX>
__global__ void __launch_bounds__(TX * (1 << LOG2L) / 8) heat_fast(const FastColArgs a)
{
    typedef typename cx<T>::type C;
    typedef FftShape<LOG2L> F;
    constexpr int L = F::L, Tn = F::Tn;
    constexpr int LP = L + L / 8;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lr = reinterpret_cast<T*>(smem_raw);
    T* li = lr + (size_t)TX * LP;

    const int b = blockIdx.y;
    const int tid = threadIdx.x;
    const int cc = tid % TX, t = tid / TX;
    // XCD-aware order: the eight XCDs (own L2 each) get contiguous runs of tiles
    const int64_t nwgx = gridDim.x;
    const int64_t wg = ((nwgx & 7) || !a.xcd_remap) ? (int64_t)blockIdx.x
                                                    : (int64_t)(blockIdx.x & 7) * (nwgx >> 3) + (blockIdx.x >> 3);
    const int64_t o = wg / a.tiles;
    const int col = (int)(wg - o * a.tiles) * TX + cc;
    C* Zc = reinterpret_cast<C*>(a.Z) + (size_t)b * a.field_elems + o * (int64_t)L * a.W + col;
    // every independent global load first (column data, symbol, twiddles, the
    // stop marks): at the start of a launch each round trip is a cold miss
    T r[1][8], im[1][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const C v = Zc[(int64_t)(t + e * Tn) * a.W];
        r[0][e] = v.x;
        im[0][e] = v.y;
    }
    const T* lrow = reinterpret_cast<const T*>(a.lam_row) + b * a.lam_row_stride;
    const T lcol = reinterpret_cast<const T*>(a.lam_col)[b * a.lam_col_stride + col];
    T lam[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) lam[e] = lrow[t + e * Tn];
    // the twiddle table staged in LDS after the tile's lines where it fits:
    // 8/TX loads per thread instead of 7 per radix-8 stage
    const C* twg = reinterpret_cast<const C*>(a.tw);
    C* twl = reinterpret_cast<C*>(li + (size_t)TX * LP);
    if constexpr (HeatFastShape<T, LOG2L, TX>::TW_LDS) {
#pragma unroll
        for (int m = tid; m < L; m += TX * Tn) twl[m] = twg[m];
        __syncthreads();
    }
    Twiddles<T, LOG2L> tw;
    load_twiddles<T, LOG2L>(tw, HeatFastShape<T, LOG2L, TX>::TW_LDS ? twl : twg, t);
    const bool marks = a.iter > 0 && a.stop_iter;
    const int stop = marks ? a.stop_iter[b] : a.iter;
    const bool check_tol = marks && a.delta_bits && a.tol > 0.0 && a.iter >= 2;
    const unsigned long long dbits = check_tol ? a.delta_bits[(int64_t)b * a.K + (a.iter - 2)] : 0ull;
    if (marks) {
        if (stop < a.iter) return;  // uniform per workgroup
        // the first pass of iteration s stops field b when s-1 changed it by <= tol
        if (check_tol && __longlong_as_double((long long)dbits) <= a.tol) {
            if (blockIdx.x == 0 && tid == 0) atomicMin(a.stop_iter + b, a.iter - 1);
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) lam[e] *= lcol;
    fft_lines<T, -1, 1, LOG2L>(r, im, lr, li, 0, TX, cc, t, tw);
    if (a.epart) {
        // this thread's eight terms in the plan's precision, the wave's sum in double
        T acc = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) acc += lam[e] * (r[0][e] * r[0][e] + im[0][e] * im[0][e]);
        const double s = wave_sum((double)acc);
        const int slot = a.slot >= 0 ? a.slot : a.stop_iter[b];
        if ((tid & 63) == 0)
            a.epart[((int64_t)b * (a.K + 1) + slot) * a.nwg + wg * (blockDim.x >> 6) + (tid >> 6)] = s;
    }
    if (!a.apply) return;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        r[0][e] *= lam[e];
        im[0][e] *= lam[e];
    }
    fft_lines<T, +1, 1, LOG2L>(r, im, lr, li, 0, TX, cc, t, tw);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        C v;
        v.x = r[0][e];
        v.y = im[0][e];
        Zc[(int64_t)(t + e * Tn) * a.W] = v;
    }
}

// ---------------------------------------------------------------------------
// Plane pass of the 3-D iteration (float): the heat step along y and z
// ---------------------------------------------------------------------------

// One workgroup per (field, packed plane, stored x mode w): the N0 x N1 plane of
// that mode, contiguous in Z[plane][w][z][y] as the row pass stores it for
// 3-D, is loaded once, transformed along y and then z in LDS, its Lyapunov
// partial taken, multiplied by lambda_z(kz) lambda_y(ky) lambda_x(w),
// transformed back along z and y, and stored in place: the whole diffusion
// between two row passes in one read and one write of the spectra.  Each
// thread holds two lines of eight values.  The plane sits in LDS as complex
// pairs (real and imaginary part side by side: one address per element) in
// rows of odd pitch, so that the z lines spread over the banks; the exchanges
// inside a line use the XOR-permuted positions of line_index<LIX_XOR>.
template <typename T, int LOG2Y, int LOG2Z>
struct PlaneFastShape {
    static constexpr int NY = 1 << LOG2Y, NZ = 1 << LOG2Z;
    static constexpr int TY = NY / 8, TZ = NZ / 8;
    static constexpr int THREADS = NY * NZ / 16;
    static constexpr int PZ = NY + 1;  // row pitch in complex elements
    // the plane, then the y and z twiddle tables
    static constexpr size_t LDS = ((size_t)NZ * PZ + NY + NZ) * 2 * sizeof(T);
};

template <typename T, int LOG2Y, int LOG2Z>
__global__ void __launch_bounds__((PlaneFastShape<T, LOG2Y, LOG2Z>::THREADS)) plane_fast(const FastColArgs a)
{
    typedef PlaneFastShape<T, LOG2Y, LOG2Z> S;
    typedef typename cx<T>::type C;
    constexpr int NY = S::NY, NZ = S::NZ, TY = S::TY, TZ = S::TZ, PZ = S::PZ;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lc = reinterpret_cast<T*>(smem_raw);  // element o: lc[2 o] (real), lc[2 o + 1] (imaginary)

    const int b = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t wg = blockIdx.x;  // packed plane * W + stored mode
    const int w = (int)(wg % a.W);
    C* Zp = reinterpret_cast<C*>(a.Z) + (size_t)b * a.field_elems + (size_t)wg * NZ * NY;
    // y lines: group gy takes z = gy and gy + NZ/2, lane ty elements y = ty + e TY
    const int gy = tid / TY, ty = tid - gy * TY;
    T r[2][8], im[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const C v = Zp[(gy + h * (NZ / 2)) * NY + ty + e * TY];
            r[h][e] = v.x;
            im[h][e] = v.y;
        }
    // z lines: group gz takes ky = gz and gz + NY/2, lane tz elements kz = tz + e TZ
    const int gz = tid / TZ, tz = tid - gz * TZ;
    const T* lz = reinterpret_cast<const T*>(a.lam_row) + b * a.lam_row_stride;
    const T* ly = reinterpret_cast<const T*>(a.lam_y) + b * a.lam_y_stride;
    const T lx = reinterpret_cast<const T*>(a.lam_col)[b * a.lam_col_stride + w];
    // twiddles are read stage by stage from copies of the tables in LDS (the
    // copies of global reads would be merged across the kernel and kept in
    // registers, more than the 1024-thread instance's 128 hold), and the symbol
    // where it is used
    C* twl = reinterpret_cast<C*>(lc + 2 * (size_t)NZ * PZ);
    for (int m = tid; m < NY + NZ; m += S::THREADS)
        twl[m] = m < NY ? reinterpret_cast<const C*>(a.tw_y)[m] : reinterpret_cast<const C*>(a.tw)[m - NY];
    __syncthreads();
    const TwiddleTable<T, LOG2Y> twy{twl};
    const TwiddleTable<T, LOG2Z> twz{twl + NY};
    const bool marks = a.iter > 0 && a.stop_iter;
    const int stop = marks ? a.stop_iter[b] : a.iter;
    const bool check_tol = marks && a.delta_bits && a.tol > 0.0 && a.iter >= 2;
    const unsigned long long dbits = check_tol ? a.delta_bits[(int64_t)b * a.K + (a.iter - 2)] : 0ull;
    if (marks) {
        if (stop < a.iter) return;  // uniform per workgroup
        // the first pass of iteration s stops field b when s-1 changed it by <= tol
        if (check_tol && __longlong_as_double((long long)dbits) <= a.tol) {
            if (blockIdx.x == 0 && tid == 0) atomicMin(a.stop_iter + b, a.iter - 1);
            return;
        }
    }
    // A lane index the compiler takes as a new value: the index arithmetic of
    // one transform is then not kept in registers for the transform back.
    auto fresh = [](int v) {
        asm volatile("" : "+v"(v));
        return v;
    };
    // y line h of the group: element y at 2 ((gy + h NZ/2) PZ + y); z line h:
    // element z at 2 (z PZ + gz + h NY/2)
    const int yl = 2 * gy * PZ, yp = 2 * (NZ / 2) * PZ;
    const int zl = 2 * gz, zp = 2 * (NY / 2);

    // forward along y (rows z of the plane), the result to LDS
    fft_lines<T, -1, 2, LOG2Y, LIX_XOR>(r, im, lc, lc + 1, yp, 2, yl, fresh(ty), twy);
    __syncthreads();  // the rows' last exchanges have been read
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int o = yl + h * yp + 2 * (ty + e * TY);
            lc[o] = r[h][e];
            lc[o + 1] = im[h][e];
        }
    __syncthreads();
    // forward along z (columns ky)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int o = zl + h * zp + 2 * PZ * (tz + e * TZ);
            r[h][e] = lc[o];
            im[h][e] = lc[o + 1];
        }
    fft_lines<T, -1, 2, LOG2Z, LIX_XOR>(r, im, lc, lc + 1, zp, 2 * PZ, zl, fresh(tz), twz);
    T lzv[8], lyv[2];
#pragma unroll
    for (int e = 0; e < 8; ++e) lzv[e] = lz[tz + e * TZ] * lx;
#pragma unroll
    for (int h = 0; h < 2; ++h) lyv[h] = ly[gz + h * (NY / 2)];
    if (a.epart) {
        // this thread's terms in float, the wave's sum in double
        T acc = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 8; ++e) acc += (lzv[e] * lyv[h]) * (r[h][e] * r[h][e] + im[h][e] * im[h][e]);
        const double sum = wave_sum((double)acc);
        const int slot = a.slot >= 0 ? a.slot : a.stop_iter[b];
        if ((tid & 63) == 0)
            a.epart[((int64_t)b * (a.K + 1) + slot) * a.nwg + wg * (blockDim.x >> 6) + (tid >> 6)] = sum;
    }
    if (!a.apply) return;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const T lm = lzv[e] * lyv[h];
            r[h][e] *= lm;
            im[h][e] *= lm;
        }
    // back along z, then y
    fft_lines<T, +1, 2, LOG2Z, LIX_XOR>(r, im, lc, lc + 1, zp, 2 * PZ, zl, fresh(tz), twz);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int o = zl + h * zp + 2 * PZ * (tz + e * TZ);
            lc[o] = r[h][e];
            lc[o + 1] = im[h][e];
        }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int o = yl + h * yp + 2 * (ty + e * TY);
            r[h][e] = lc[o];
            im[h][e] = lc[o + 1];
        }
    fft_lines<T, +1, 2, LOG2Y, LIX_XOR>(r, im, lc, lc + 1, yp, 2, yl, fresh(ty), twy);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            C v;
            v.x = r[h][e];
            v.y = im[h][e];
            Zp[(gy + h * (NZ / 2)) * NY + ty + e * TY] = v;
        }
}

}  // namespace mbo
