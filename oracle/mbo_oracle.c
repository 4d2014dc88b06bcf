/*
 * FP64 CPU oracle for the generalized MBO diffusion generated motion for
 * orthogonal matrix-valued fields on flat tori (Osting & Wang, arXiv:1711.01365:
 * Algorithm 1, Lemma 1.1, Section 4, Section 5.1; the volume-preserving
 * variant of Section 7: Lemmas 7.1, 7.2; the relaxed gradient flows GD-1 and
 * GD-3 of Section 1 with their energies; surface diffusion on a sphere by the
 * closest point method of Section 5.2, Theorem 5.2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or helper with the
 * HIP implementation; it is written to be read against the paper, not to be
 * fast.
 *
 * Conventions (all arrays row-major, last grid axis fastest):
 *   grid      d axes (d = 1, 2 or 3), N[a] points on axis a, x_a = j / N[a]
 *             on the unit-period torus (Section 5.1 identifies opposite edges
 *             of a unit square; the offset of the square is irrelevant here).
 *   field     "entry-planar": A[i][j][p] = entry (i,j) of the n x n matrix at
 *             grid point p, i.e. n*n real planes of prod(N) doubles each.
 *   DFT       forward  X(m) = sum_x x(p) exp(-2 pi i sum_a m_a j_a / N_a),
 *             inverse  uses exp(+...), no scaling inside the transforms.
 *
 * Readings of points the paper leaves open (each is restated where it is used):
 *   - the heat multiplier is the exact Fourier symbol of e^{tau Delta} on the
 *     unit torus, exp(-4 pi^2 tau |k|^2), with k_a = m_a for m_a < N_a/2 and
 *     m_a - N_a otherwise (so the Nyquist index counts as -N_a/2);
 *   - the closest orthogonal matrix of a singular input is not unique; a
 *     singular value <= n * eps * sigma_max is treated as zero and the missing
 *     left singular directions are completed so that det Q = +1 (the matrix
 *     analogue of sgn(0) = +1 in thresholding); the zero matrix maps to I;
 *   - the Lyapunov functional is evaluated with quadrature weight 1/prod(N):
 *     E(A) = (1/tau) * (1/prod(N)) * sum_p [ n - <A(p), (e^{tau Delta}A)(p)>_F ].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define ORC_PI 3.14159265358979323846264338328
#define ORC_TWO_PI (2.0 * ORC_PI)

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */

static int64_t orc_npoints(int d, const int64_t* N)
{
    int64_t p = 1;
    for (int a = 0; a < d; ++a) p *= N[a];
    return p;
}

static int orc_is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }

/* Pairwise (cascade) summation; error grows like log(len) instead of len. */
static double orc_pairwise_sum(const double* v, int64_t len)
{
    if (len <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < len; ++i) s += v[i];
        return s;
    }
    int64_t h = len / 2;
    return orc_pairwise_sum(v, h) + orc_pairwise_sum(v + h, len - h);
}

/* Determinant of an n x n row-major matrix (n <= 4) by Gaussian elimination
 * with partial pivoting. */
static double orc_det(int n, const double* m)
{
    double a[16];
    memcpy(a, m, sizeof(double) * n * n);
    double det = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * n + c]) > fabs(a[piv * n + c])) piv = r;
        if (a[piv * n + c] == 0.0) return 0.0;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = a[c * n + k]; a[c * n + k] = a[piv * n + k]; a[piv * n + k] = t;
            }
            det = -det;
        }
        det *= a[c * n + c];
        for (int r = c + 1; r < n; ++r) {
            double f = a[r * n + c] / a[c * n + c];
            for (int k = c; k < n; ++k) a[r * n + k] -= f * a[c * n + k];
        }
    }
    return det;
}

/* sgn with sgn(0) = +1 (the MBO threshold keeps the boundary value). */
static int orc_sgn(double v) { return v >= 0.0 ? 1 : -1; }

/* ------------------------------------------------------------------------ */
/* Discrete Fourier transforms                                               */
/* ------------------------------------------------------------------------ */

/* Naive d-dimensional DFT straight from its definition, O(P^2) for P points.
 * The phase is reduced exactly in integers per axis before the cos/sin call.
 * sign = -1 forward, +1 inverse (unscaled).  Any N (not only powers of two). */
int orc_dft_naive(int d, const int64_t* N, const double* xr, const double* xi,
                  double* yr, double* yi, int sign)
{
    if (d < 1 || d > 3 || (sign != 1 && sign != -1)) return -1;
    int64_t P = orc_npoints(d, N);
    int64_t Nn[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) Nn[3 - d + a] = N[a];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t m = 0; m < P; ++m) {
        int64_t m2 = m % Nn[2], m1 = (m / Nn[2]) % Nn[1], m0 = m / (Nn[2] * Nn[1]);
        double sr = 0.0, si = 0.0;
        for (int64_t x = 0; x < P; ++x) {
            int64_t x2 = x % Nn[2], x1 = (x / Nn[2]) % Nn[1], x0 = x / (Nn[2] * Nn[1]);
            double ph = (double)((m0 * x0) % Nn[0]) / (double)Nn[0] +
                        (double)((m1 * x1) % Nn[1]) / (double)Nn[1] +
                        (double)((m2 * x2) % Nn[2]) / (double)Nn[2];
            double c = cos(ORC_TWO_PI * ph), s = sign * sin(ORC_TWO_PI * ph);
            sr += xr[x] * c - xi[x] * s;
            si += xr[x] * s + xi[x] * c;
        }
        yr[m] = sr;
        yi[m] = si;
    }
    return 0;
}

/* In-place iterative radix-2 Cooley-Tukey transform of one line of length L
 * (power of two) with element stride `st`.  Twiddles exp(sign 2 pi i k / L)
 * come from tables of cos/sin(2 pi k / L) evaluated directly for each k (no
 * recurrence).  sign = -1 forward, +1 inverse (unscaled). */
static void orc_fft_line(double* re, double* im, int64_t L, int64_t st, int sign,
                         const double* ct, const double* snt)
{
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < L; ++i) {
        int64_t bit = L >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i * st]; re[i * st] = re[j * st]; re[j * st] = t;
            t = im[i * st]; im[i * st] = im[j * st]; im[j * st] = t;
        }
    }
    /* butterflies: sub-transforms of length len are merged pairwise */
    for (int64_t len = 2; len <= L; len <<= 1) {
        int64_t half = len >> 1, step = L / len;
        for (int64_t b = 0; b < L; b += len) {
            for (int64_t k = 0; k < half; ++k) {
                double wr = ct[k * step], wi = sign * snt[k * step];
                int64_t u = (b + k) * st, v = (b + k + half) * st;
                double tr = re[v] * wr - im[v] * wi;
                double ti = re[v] * wi + im[v] * wr;
                re[v] = re[u] - tr; im[v] = im[u] - ti;
                re[u] += tr;        im[u] += ti;
            }
        }
    }
}

/* d-dimensional FFT (row-column: the 1-D transform along every axis in turn),
 * in place, unscaled.  Requires every N[a] to be a power of two. */
int orc_fft(int d, const int64_t* N, double* re, double* im, int sign)
{
    if (d < 1 || d > 3 || (sign != 1 && sign != -1)) return -1;
    for (int a = 0; a < d; ++a) if (!orc_is_pow2(N[a])) return -2;
    int64_t P = orc_npoints(d, N);
    for (int a = 0; a < d; ++a) {
        int64_t L = N[a];
        int64_t st = 1;
        for (int b = a + 1; b < d; ++b) st *= N[b];
        double* ct = (double*)malloc(sizeof(double) * (size_t)L);
        double* snt = (double*)malloc(sizeof(double) * (size_t)L);
        for (int64_t k = 0; k < L; ++k) {
            ct[k] = cos(ORC_TWO_PI * (double)k / (double)L);
            snt[k] = sin(ORC_TWO_PI * (double)k / (double)L);
        }
        int64_t lines = P / L;
#pragma omp parallel for schedule(static)
        for (int64_t ln = 0; ln < lines; ++ln) {
            int64_t outer = ln / st, inner = ln % st;
            int64_t base = outer * L * st + inner;
            orc_fft_line(re + base, im + base, L, st, sign, ct, snt);
        }
        free(ct);
        free(snt);
    }
    return 0;
}

/* The heat symbol of Section 5.1 on the unit torus for the multi-index m:
 * exp(-4 pi^2 tau sum_a k_a^2), with the wrap-around k_a = m_a or m_a - N_a. */
static double orc_heat_symbol(int d, const int64_t* N, int64_t flat, double tau)
{
    double ksq = 0.0;
    for (int a = d - 1; a >= 0; --a) {
        int64_t m = flat % N[a];
        flat /= N[a];
        int64_t k = (2 * m < N[a]) ? m : m - N[a];
        ksq += (double)k * (double)k;
    }
    return exp(-4.0 * ORC_PI * ORC_PI * tau * ksq);
}

/* Transform of one complex plane, by the FFT or by the naive DFT. */
static void orc_transform(int d, const int64_t* N, double* re, double* im, int sign,
                          int use_naive, double* tr, double* ti)
{
    if (use_naive) {
        int64_t P = orc_npoints(d, N);
        orc_dft_naive(d, N, re, im, tr, ti, sign);
        memcpy(re, tr, sizeof(double) * (size_t)P);
        memcpy(im, ti, sizeof(double) * (size_t)P);
    } else {
        orc_fft(d, N, re, im, sign);
    }
}

/* Diffusion step of Algorithm 1 on the flat torus (Section 5.1): every real
 * plane is transformed, multiplied by the heat symbol and transformed back,
 * out = F^{-1}( symbol * F(in) ).  `nplanes` planes of prod(N) values.
 * max_imag (nullable) receives max |Im| left after the inverse transform. */
static int orc_apply_symbol(int d, const int64_t* N, int64_t nplanes, double tau, const double* in,
                            double* out, int use_naive, double* max_imag, int dtau);

int orc_heat(int d, const int64_t* N, int64_t nplanes, double tau, const double* in,
             double* out, int use_naive, double* max_imag)
{
    return orc_apply_symbol(d, N, nplanes, tau, in, out, use_naive, max_imag, 0);
}

/* Derivative of the diffusion step with respect to tau (used by the adjoint):
 * d/dtau e^{tau Delta} = Delta e^{tau Delta}, whose Fourier symbol is
 * -4 pi^2 |k|^2 exp(-4 pi^2 tau |k|^2).  Same conventions as orc_heat. */
int orc_heat_dtau(int d, const int64_t* N, int64_t nplanes, double tau, const double* in,
                  double* out)
{
    return orc_apply_symbol(d, N, nplanes, tau, in, out, 0, NULL, 1);
}

/* -4 pi^2 |k|^2 for the multi-index m (same wrap-around as the heat symbol). */
static double orc_laplace_symbol(int d, const int64_t* N, int64_t flat)
{
    double ksq = 0.0;
    for (int a = d - 1; a >= 0; --a) {
        int64_t m = flat % N[a];
        flat /= N[a];
        int64_t k = (2 * m < N[a]) ? m : m - N[a];
        ksq += (double)k * (double)k;
    }
    return -4.0 * ORC_PI * ORC_PI * ksq;
}

static int orc_apply_symbol(int d, const int64_t* N, int64_t nplanes, double tau, const double* in,
                            double* out, int use_naive, double* max_imag, int dtau)
{
    if (d < 1 || d > 3 || nplanes < 1 || !(tau >= 0.0)) return -1;
    if (!use_naive)
        for (int a = 0; a < d; ++a) if (!orc_is_pow2(N[a])) return -2;
    int64_t P = orc_npoints(d, N);
    double* re = (double*)malloc(sizeof(double) * (size_t)P);
    double* im = (double*)malloc(sizeof(double) * (size_t)P);
    double* tr = (double*)malloc(sizeof(double) * (size_t)P);
    double* ti = (double*)malloc(sizeof(double) * (size_t)P);
    double mi = 0.0;
    for (int64_t pl = 0; pl < nplanes; ++pl) {
        memcpy(re, in + pl * P, sizeof(double) * (size_t)P);
        memset(im, 0, sizeof(double) * (size_t)P);
        orc_transform(d, N, re, im, -1, use_naive, tr, ti);
        for (int64_t m = 0; m < P; ++m) {
            double g = orc_heat_symbol(d, N, m, tau);
            if (dtau) g *= orc_laplace_symbol(d, N, m);
            re[m] *= g;
            im[m] *= g;
        }
        orc_transform(d, N, re, im, +1, use_naive, tr, ti);
        for (int64_t p = 0; p < P; ++p) {
            out[pl * P + p] = re[p] / (double)P;
            double a = fabs(im[p] / (double)P);
            if (a > mi) mi = a;
        }
    }
    free(re); free(im); free(tr); free(ti);
    if (max_imag) *max_imag = mi;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Projection step: closest orthogonal matrix (Lemma 1.1)                    */
/* ------------------------------------------------------------------------ */

/* One-sided (Hestenes) Jacobi SVD of the n x n row-major matrix a:
 * orthogonalise the columns of W = A by plane rotations, accumulating them in
 * V, so that W = U Sigma with sigma_j = ||w_j||.  Then Q = U V^t, the minimiser
 * of ||B - A||_F over orthogonal B (Lemma 1.1).  Returns the sweep count. */
static int orc_project_point_usv(int n, const double* a, double* q, double* sig, double* Uo,
                                 double* Vo);

static int orc_project_point(int n, const double* a, double* q, double* sig)
{
    return orc_project_point_usv(n, a, q, sig, NULL, NULL);
}

/* The same, also returning (nullable) the factors U and V of Q = U V^t, row
 * major, with U completed as described for singular input; A = U diag(sig) V^t. */
static int orc_project_point_usv(int n, const double* a, double* q, double* sig, double* Uo,
                                 double* Vo)
{
    if (n == 1) {
        q[0] = (double)orc_sgn(a[0]);
        if (sig) sig[0] = fabs(a[0]);
        if (Uo) Uo[0] = q[0];
        if (Vo) Vo[0] = 1.0;
        return 0;
    }
    double W[16], V[16];
    memcpy(W, a, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;

    int sweep = 0;
    for (; sweep < 30; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p) {
            for (int r = p + 1; r < n; ++r) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < n; ++i) {
                    al += W[i * n + p] * W[i * n + p];
                    be += W[i * n + r] * W[i * n + r];
                    ga += W[i * n + p] * W[i * n + r];
                }
                if (fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int i = 0; i < n; ++i) {
                    double wp = W[i * n + p], wr = W[i * n + r];
                    W[i * n + p] = c * wp - s * wr;
                    W[i * n + r] = s * wp + c * wr;
                    double vp = V[i * n + p], vr = V[i * n + r];
                    V[i * n + p] = c * vp - s * vr;
                    V[i * n + r] = s * vp + c * vr;
                }
                rotated = 1;
            }
        }
        if (!rotated) { ++sweep; break; }
    }

    double sg[4], smax = 0.0;
    for (int j = 0; j < n; ++j) {
        double s2 = 0.0;
        for (int i = 0; i < n; ++i) s2 += W[i * n + j] * W[i * n + j];
        sg[j] = sqrt(s2);
        if (sg[j] > smax) smax = sg[j];
        if (sig) sig[j] = sg[j];
    }
    if (smax == 0.0) { /* A = 0: every orthogonal matrix is equally close; take I */
        for (int i = 0; i < n * n; ++i) q[i] = 0.0;
        for (int i = 0; i < n; ++i) q[i * n + i] = 1.0;
        if (Uo) memcpy(Uo, q, sizeof(double) * n * n);
        if (Vo) memcpy(Vo, q, sizeof(double) * n * n);
        return sweep;
    }
    /* U: normalised columns; columns with a (numerically) zero singular value
     * are completed by Gram-Schmidt against the unit vectors. */
    double U[16];
    int zero[4], last_zero = -1;
    for (int j = 0; j < n; ++j) {
        zero[j] = sg[j] <= (double)n * DBL_EPSILON * smax;
        if (!zero[j]) for (int i = 0; i < n; ++i) U[i * n + j] = W[i * n + j] / sg[j];
    }
    for (int j = 0; j < n; ++j) {
        if (!zero[j]) continue;
        double best[4], bestn = -1.0;
        for (int e = 0; e < n; ++e) {
            double r[4];
            for (int i = 0; i < n; ++i) r[i] = (i == e) ? 1.0 : 0.0;
            for (int k = 0; k < n; ++k) {
                if (zero[k] && k >= j) continue; /* not filled yet */
                double dot = 0.0;
                for (int i = 0; i < n; ++i) dot += U[i * n + k] * r[i];
                for (int i = 0; i < n; ++i) r[i] -= dot * U[i * n + k];
            }
            double rn = 0.0;
            for (int i = 0; i < n; ++i) rn += r[i] * r[i];
            if (rn > bestn) { bestn = rn; memcpy(best, r, sizeof(double) * n); }
        }
        bestn = sqrt(bestn);
        for (int i = 0; i < n; ++i) U[i * n + j] = best[i] / bestn;
        last_zero = j;
    }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += U[i * n + j] * V[k * n + j];
            q[i * n + k] = s;
        }
    if (last_zero >= 0 && orc_det(n, q) < 0.0) {
        /* the completed direction's sign is free: pick the one with det Q = +1 */
        for (int i = 0; i < n; ++i) U[i * n + last_zero] = -U[i * n + last_zero];
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += U[i * n + j] * V[k * n + j];
                q[i * n + k] = s;
            }
    }
    if (Uo) memcpy(Uo, U, sizeof(double) * n * n);
    if (Vo) memcpy(Vo, V, sizeof(double) * n * n);
    return sweep;
}

/* Pointwise projection of an entry-planar field (Algorithm 1, step 2).
 * detsign (nullable): sign of det Q per point (+1 / -1).
 * sigma   (nullable): singular values, sigma[j * npts + p], unsorted.
 * sweeps  (nullable): Jacobi sweeps used per point. */
int orc_project(int64_t npts, int n, const double* A, double* Q, int8_t* detsign,
                double* sigma, int32_t* sweeps)
{
    if (npts < 0 || n < 1 || n > 4) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        double a[16], q[16], sg[4];
        for (int e = 0; e < n * n; ++e) a[e] = A[e * npts + p];
        int sw = orc_project_point(n, a, q, sg);
        for (int e = 0; e < n * n; ++e) Q[e * npts + p] = q[e];
        if (detsign) detsign[p] = (int8_t)orc_sgn(orc_det(n, q));
        if (sigma) for (int j = 0; j < n; ++j) sigma[j * npts + p] = sg[j];
        if (sweeps) sweeps[p] = sw;
    }
    return 0;
}

/* sgn(det A(p)) per point of a general (not necessarily orthogonal) field. */
int orc_det_sign(int64_t npts, int n, const double* A, int8_t* detsign)
{
    if (npts < 0 || n < 1 || n > 4) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        double a[16];
        for (int e = 0; e < n * n; ++e) a[e] = A[e * npts + p];
        detsign[p] = (int8_t)orc_sgn(orc_det(n, a));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Lyapunov functional (Section 4, eq. (Lyapunov))                           */
/* ------------------------------------------------------------------------ */

/* E(A) = (1/tau) (1/P) sum_p [ n - <A(p), HA(p)>_F ], with HA given. */
static double orc_energy_given(int64_t P, int n, double tau, const double* A, const double* HA)
{
    double* e = (double*)malloc(sizeof(double) * (size_t)P);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        double s = 0.0;
        for (int k = 0; k < n * n; ++k) s += A[k * P + p] * HA[k * P + p];
        e[p] = (double)n - s;
    }
    double tot = orc_pairwise_sum(e, P);
    free(e);
    return tot / ((double)P * tau);
}

int orc_energy(int d, const int64_t* N, int n, double tau, const double* A, int use_naive,
               double* E)
{
    if (n < 1 || n > 4 || !(tau > 0.0)) return -1;
    int64_t P = orc_npoints(d, N);
    double* HA = (double*)malloc(sizeof(double) * (size_t)(P * n * n));
    int rc = orc_heat(d, N, (int64_t)n * n, tau, A, HA, use_naive, NULL);
    if (rc == 0) *E = orc_energy_given(P, n, tau, A, HA);
    free(HA);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: A_s = P(e^{tau Delta} A_{s-1}), s = 1..K                     */
/* ------------------------------------------------------------------------ */

/* A (in/out) holds A_0 on entry and the last iterate on return.  Logs (all
 * nullable): energy[s] = E(A_s) for s = 0..iters, flips[s-1] = number of points
 * whose det sign differs between A_s and A_{s-1}, delta[s-1] = max |A_s -
 * A_{s-1}| over all entries, max_imag = largest |Im| after any inverse
 * transform.  With tol > 0 the loop stops after the first s with delta <= tol;
 * *iters receives the number of iterations performed. */
int orc_iterate(int d, const int64_t* N, int n, double tau, double* A, int K, double tol,
                int* iters, double* energy, int64_t* flips, double* delta, double* max_imag,
                int use_naive)
{
    if (n < 1 || n > 4 || !(tau > 0.0) || K < 0) return -1;
    int64_t P = orc_npoints(d, N);
    int64_t nn = (int64_t)n * n;
    double* At = (double*)malloc(sizeof(double) * (size_t)(P * nn));
    double* An = (double*)malloc(sizeof(double) * (size_t)(P * nn));
    int8_t* sp = (int8_t*)malloc((size_t)P);
    int8_t* sn = (int8_t*)malloc((size_t)P);
    double mi_all = 0.0, mi = 0.0;
    int rc = 0, done = 0;
    orc_det_sign(P, n, A, sp);
    for (int s = 1; s <= K; ++s) {
        rc = orc_heat(d, N, nn, tau, A, At, use_naive, &mi);           /* diffusion step */
        if (rc) break;
        if (mi > mi_all) mi_all = mi;
        if (energy) energy[s - 1] = orc_energy_given(P, n, tau, A, At); /* E(A_{s-1}) */
        orc_project(P, n, At, An, sn, NULL, NULL);                      /* projection step */
        int64_t fl = 0;
        double dl = 0.0;
        for (int64_t p = 0; p < P; ++p) fl += (sn[p] != sp[p]);
        for (int64_t k = 0; k < P * nn; ++k) {
            double v = fabs(An[k] - A[k]);
            if (v > dl) dl = v;
        }
        if (flips) flips[s - 1] = fl;
        if (delta) delta[s - 1] = dl;
        memcpy(A, An, sizeof(double) * (size_t)(P * nn));
        memcpy(sp, sn, (size_t)P);
        done = s;
        if (tol > 0.0 && dl <= tol) break;
    }
    if (rc == 0 && energy) {
        rc = orc_heat(d, N, nn, tau, A, At, use_naive, &mi);
        if (mi > mi_all) mi_all = mi;
        energy[done] = orc_energy_given(P, n, tau, A, At);
    }
    if (iters) *iters = done;
    if (max_imag) *max_imag = mi_all;
    free(At); free(An); free(sp); free(sn);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of K unrolled steps of Algorithm 1                                */
/* ------------------------------------------------------------------------ */

/* Vector-Jacobian product of the projection step (Lemma 1.1: Q = U V^t for
 * A = U Sigma V^t).  A perturbation dA moves the orthogonal polar factor by
 * dQ = U X V^t with X skew, X_ij = (F_ij - F_ji) / (sigma_i + sigma_j) and
 * F = U^t dA V.  Hence for a cotangent G of Q the cotangent of A is
 *     G_A = U K V^t,  K_ij = (M_ij - M_ji) / (sigma_i + sigma_j),  M = U^t G V,
 * (K_ii = 0).  n = 1 (sign thresholding) has zero derivative away from 0.  A
 * pair with sigma_i + sigma_j = 0 (rank <= n - 2, where Q is not a function of
 * A) contributes 0. */
int orc_project_vjp(int64_t npts, int n, const double* A, const double* G, double* GA)
{
    if (npts < 0 || n < 1 || n > 4) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        double a[16], g[16], q[16], sg[4], U[16], V[16], M[16], Kx[16], T1[16];
        for (int e = 0; e < n * n; ++e) {
            a[e] = A[e * npts + p];
            g[e] = G[e * npts + p];
        }
        if (n == 1) {
            GA[p] = 0.0;
            continue;
        }
        orc_project_point_usv(n, a, q, sg, U, V);
        for (int i = 0; i < n; ++i)          /* M = U^t G V */
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k)
                    for (int l = 0; l < n; ++l) s += U[k * n + i] * g[k * n + l] * V[l * n + j];
                M[i * n + j] = s;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double den = sg[i] + sg[j];
                Kx[i * n + j] = (i == j || den == 0.0) ? 0.0 : (M[i * n + j] - M[j * n + i]) / den;
            }
        for (int i = 0; i < n; ++i)          /* T1 = U K */
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += U[i * n + k] * Kx[k * n + j];
                T1[i * n + j] = s;
            }
        for (int i = 0; i < n; ++i)          /* G_A = T1 V^t */
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += T1[i * n + k] * V[j * n + k];
                GA[(i * n + j) * npts + p] = s;
            }
    }
    return 0;
}

/* Loss L = (1/2) sum_p ||A_K(p) - T(p)||_F^2 of K steps of Algorithm 1 from A_0
 * and its gradients by the chain rule taken backwards:
 *     Gbar_K = A_K - T;  for s = K..1:
 *         Gtil_s = VJP of the projection at Atil_s = e^{tau Delta} A_{s-1},
 *         dL/dtau += <Gtil_s, Delta e^{tau Delta} A_{s-1}>,
 *         Gbar_{s-1} = e^{tau Delta} Gtil_s   (the heat operator is self-adjoint);
 *     dL/dA_0 = Gbar_0.
 * All iterates are kept.  flips (nullable, [K]) logs the det sign changes of
 * the forward run, as orc_iterate does. */
int orc_unroll_grad(int d, const int64_t* N, int n, double tau, const double* A0, const double* T,
                    int K, double* loss, double* gA0, double* gtau, int64_t* flips)
{
    if (n < 1 || n > 4 || !(tau > 0.0) || K < 0) return -1;
    int64_t P = orc_npoints(d, N);
    int64_t nn = (int64_t)n * n, F = P * nn;
    double* As = (double*)malloc(sizeof(double) * (size_t)(F * (K + 1)));
    double* At = (double*)malloc(sizeof(double) * (size_t)F);
    double* Gb = (double*)malloc(sizeof(double) * (size_t)F);
    double* Gt = (double*)malloc(sizeof(double) * (size_t)F);
    double* Dt = (double*)malloc(sizeof(double) * (size_t)F);
    int8_t* sp = (int8_t*)malloc((size_t)P);
    int8_t* sn = (int8_t*)malloc((size_t)P);
    int rc = 0;
    memcpy(As, A0, sizeof(double) * (size_t)F);
    orc_det_sign(P, n, As, sp);
    for (int s = 1; s <= K && rc == 0; ++s) {
        rc = orc_heat(d, N, nn, tau, As + (s - 1) * F, At, 0, NULL);
        if (rc) break;
        orc_project(P, n, At, As + s * F, sn, NULL, NULL);
        int64_t fl = 0;
        for (int64_t p = 0; p < P; ++p) fl += (sn[p] != sp[p]);
        if (flips) flips[s - 1] = fl;
        memcpy(sp, sn, (size_t)P);
    }
    double gt = 0.0;
    if (rc == 0) {
        const double* AK = As + (int64_t)K * F;
        for (int64_t k = 0; k < F; ++k) {
            Gb[k] = AK[k] - T[k];
            Dt[k] = 0.5 * Gb[k] * Gb[k];
        }
        *loss = orc_pairwise_sum(Dt, F);
        for (int s = K; s >= 1 && rc == 0; --s) {
            const double* Aprev = As + (int64_t)(s - 1) * F;
            rc = orc_heat(d, N, nn, tau, Aprev, At, 0, NULL);
            if (rc) break;
            orc_project_vjp(P, n, At, Gb, Gt);
            rc = orc_heat_dtau(d, N, nn, tau, Aprev, Dt);
            if (rc) break;
            for (int64_t k = 0; k < F; ++k) Dt[k] *= Gt[k];
            gt += orc_pairwise_sum(Dt, F);
            rc = orc_heat(d, N, nn, tau, Gt, Gb, 0, NULL);
        }
    }
    if (rc == 0) {
        memcpy(gA0, Gb, sizeof(double) * (size_t)F);
        *gtau = gt;
    }
    free(As); free(At); free(Gb); free(Gt); free(Dt); free(sp); free(sn);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Volume-preserving MBO (Section 7)                                         */
/* ------------------------------------------------------------------------ */

/* T^+(A), T^-(A) and Delta E = <T^+(A) - T^-(A), A>_F of one matrix.
 * With A = U Sigma V^t, U V^t is the closest orthogonal matrix (Lemma 1.1) and
 * U D_n V^t, which reverses the direction of the smallest singular value, the
 * closest one of the opposite determinant (Lemma 7.1).  T^+ is whichever of the
 * two has determinant +1 (the closest point of SO(n)) and T^- the other (the
 * closest point of SO^-(n)); for det A > 0 this is U V^t and U D_n V^t, for
 * det A < 0 the reverse, as Section 7 defines them.  The Jacobi singular values
 * are unsorted: D_n acts on the first column holding the smallest one (when
 * that value is repeated, T^- is not unique and this picks one minimiser). */
static double orc_vp_point(int n, const double* a, double* tp, double* tm)
{
    double q[16], r[16], sig[4], U[16], V[16];
    orc_project_point_usv(n, a, q, sig, U, V);
    int jm = 0;
    for (int j = 1; j < n; ++j)
        if (sig[j] < sig[jm]) jm = j;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) r[i * n + k] = q[i * n + k] - 2.0 * U[i * n + jm] * V[k * n + jm];
    const int q_plus = orc_det(n, q) >= 0.0;
    memcpy(tp, q_plus ? q : r, sizeof(double) * n * n);
    memcpy(tm, q_plus ? r : q, sizeof(double) * n * n);
    double de = 0.0;
    for (int e = 0; e < n * n; ++e) de += (tp[e] - tm[e]) * a[e];
    return de;
}

typedef struct {
    double de;
    int64_t idx;
} orc_rank_t;

/* Descending Delta E; equal values in ascending point index. */
static int orc_rank_cmp(const void* x, const void* y)
{
    const orc_rank_t* u = (const orc_rank_t*)x;
    const orc_rank_t* v = (const orc_rank_t*)y;
    if (u->de > v->de) return -1;
    if (u->de < v->de) return 1;
    return (u->idx > v->idx) - (u->idx < v->idx);
}

/* The flat-torus selection rule at the end of Section 7: sort Delta E in
 * descending order and take the first n_plus points; equal values are taken
 * in ascending point index (the paper leaves ties open).  sel[p] = 1 for the
 * selected points, 0 elsewhere.  Returns -1 on bad arguments, -2 when a value
 * is not finite. */
int orc_volume_select(int64_t npts, const double* dE, int64_t n_plus, int8_t* sel)
{
    if (npts < 0 || n_plus < 0 || n_plus > npts) return -1;
    for (int64_t p = 0; p < npts; ++p)
        if (!isfinite(dE[p])) return -2;
    orc_rank_t* rk = (orc_rank_t*)malloc(sizeof(orc_rank_t) * (size_t)(npts + 1));
    for (int64_t p = 0; p < npts; ++p) {
        rk[p].de = dE[p];
        rk[p].idx = p;
    }
    qsort(rk, (size_t)npts, sizeof(orc_rank_t), orc_rank_cmp);
    memset(sel, 0, (size_t)npts);
    for (int64_t r = 0; r < n_plus; ++r) sel[rk[r].idx] = 1;
    free(rk);
    return 0;
}

/* Volume-constrained projection of an entry-planar field A (the reassignment of
 * Lemma 7.2 on a uniform grid): the n_plus points selected by the rule above
 * receive T^+, all others T^-, so that exactly n_plus points end in SO(n).
 * dE and selected are nullable.  Returns -1 on bad arguments, -2 when a Delta E
 * is not finite. */
int orc_volume_project(int64_t npts, int n, const double* A, int64_t n_plus, double* B, double* dE,
                       int8_t* selected)
{
    if (npts < 0 || n < 1 || n > 4 || n_plus < 0 || n_plus > npts) return -1;
    const int64_t nn = (int64_t)n * n;
    double* tp = (double*)malloc(sizeof(double) * (size_t)(npts * nn + 1));
    double* tm = (double*)malloc(sizeof(double) * (size_t)(npts * nn + 1));
    double* de = (double*)malloc(sizeof(double) * (size_t)(npts + 1));
    int8_t* sel = (int8_t*)malloc((size_t)npts + 1);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        double a[16];
        for (int e = 0; e < nn; ++e) a[e] = A[e * npts + p];
        de[p] = orc_vp_point(n, a, tp + p * nn, tm + p * nn);
    }
    int rc = orc_volume_select(npts, de, n_plus, sel);
    if (rc == 0) {
        for (int64_t p = 0; p < npts; ++p) {
            const double* t = sel[p] ? tp + p * nn : tm + p * nn;
            for (int e = 0; e < nn; ++e) B[e * npts + p] = t[e];
        }
        if (dE) memcpy(dE, de, sizeof(double) * (size_t)npts);
        if (selected) memcpy(selected, sel, (size_t)npts);
    }
    free(tp); free(tm); free(de); free(sel);
    return rc;
}

/* Volume-preserving MBO: Algorithm 1 with step 2 replaced by the projection
 * above, for K iterations in place on A.  n_plus < 0 takes the number of points
 * of A_0 with det >= 0 (the volume of its SO(n) region).  Logs (nullable):
 * energy[s] = E(A_s) for s = 0..K, n_pos[s] = #{p : det A_s(p) >= 0}.  The
 * n_plus used is returned in *n_plus_used (nullable). */
int orc_iterate_volume(int d, const int64_t* N, int n, double tau, double* A, int K, int64_t n_plus,
                       double* energy, int64_t* n_pos, int64_t* n_plus_used)
{
    if (n < 1 || n > 4 || !(tau > 0.0) || K < 0) return -1;
    int64_t P = orc_npoints(d, N);
    int64_t nn = (int64_t)n * n;
    double* At = (double*)malloc(sizeof(double) * (size_t)(P * nn));
    int8_t* sg = (int8_t*)malloc((size_t)P);
    int rc = 0;
    orc_det_sign(P, n, A, sg);
    int64_t c0 = 0;
    for (int64_t p = 0; p < P; ++p) c0 += sg[p] > 0;
    if (n_pos) n_pos[0] = c0;
    if (n_plus < 0) n_plus = c0;
    if (n_plus > P) rc = -1;
    for (int s = 1; s <= K && rc == 0; ++s) {
        rc = orc_heat(d, N, nn, tau, A, At, 0, NULL);                   /* diffusion step */
        if (rc) break;
        if (energy) energy[s - 1] = orc_energy_given(P, n, tau, A, At); /* E(A_{s-1}) */
        rc = orc_volume_project(P, n, At, n_plus, A, NULL, NULL);      /* Lemma 7.2 step */
        if (rc) break;
        if (n_pos) {
            orc_det_sign(P, n, A, sg);
            int64_t c = 0;
            for (int64_t p = 0; p < P; ++p) c += sg[p] > 0;
            n_pos[s] = c;
        }
    }
    if (rc == 0 && energy) {
        rc = orc_heat(d, N, nn, tau, A, At, 0, NULL);
        energy[K] = orc_energy_given(P, n, tau, A, At);
    }
    if (n_plus_used) *n_plus_used = n_plus;
    free(At); free(sg);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Relaxed gradient flows (eqs. GD-1 and GD-3)                               */
/* ------------------------------------------------------------------------ */

/* The reaction term of one matrix: kind 1 (GD-1) U (Sigma - I) V^t, which by
 * Lemma 1.1 is A - U V^t; kind 3 (GD-3) A (A^t A - I). */
static void orc_relax_reaction(int n, int kind, const double* a, double* r)
{
    if (kind == 1) {
        double q[16], sig[4];
        orc_project_point(n, a, q, sig);
        for (int e = 0; e < n * n; ++e) r[e] = a[e] - q[e];
    } else {
        double m[16];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += a[k * n + i] * a[k * n + j];
                m[i * n + j] = s - (i == j ? 1.0 : 0.0);
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += a[i * n + k] * m[k * n + j];
                r[i * n + j] = s;
            }
    }
}

/* K steps of the semi-implicit scheme for dA/dt = Delta A - eps^-2 N(A) (GD-1
 * or GD-3), in place: an implicit-Euler diffusion step B = (I - dt Delta)^{-1} A
 * (Fourier symbol 1 / (1 + 4 pi^2 dt |k|^2)) followed by an explicit reaction
 * step A = B - (dt / eps^2) N(B).  (The paper states the flows, not a scheme;
 * the IMEX Euler step A <- (I - dt Delta)^{-1} (A - dt eps^-2 N(A)) gives the
 * same sequence shifted by one reaction step.)  eps = +inf drops the
 * reaction. */
int orc_relaxed_flow(int d, const int64_t* N, int n, int kind, double eps, double dt, double* A, int K)
{
    if (n < 1 || n > 4 || (kind != 1 && kind != 3) || !(eps > 0.0) || !(dt > 0.0) || K < 0) return -1;
    if (d < 1 || d > 3) return -1;
    for (int a = 0; a < d; ++a)
        if (!orc_is_pow2(N[a])) return -2;
    const int64_t P = orc_npoints(d, N);
    const int64_t nn = (int64_t)n * n;
    const double c = isinf(eps) ? 0.0 : dt / (eps * eps);
    double* re = (double*)malloc(sizeof(double) * (size_t)P);
    double* im = (double*)malloc(sizeof(double) * (size_t)P);
    double* B = (double*)malloc(sizeof(double) * (size_t)(P * nn));
    for (int s = 0; s < K; ++s) {
        for (int64_t pl = 0; pl < nn; ++pl) { /* diffusion step */
            memcpy(re, A + pl * P, sizeof(double) * (size_t)P);
            memset(im, 0, sizeof(double) * (size_t)P);
            orc_fft(d, N, re, im, -1);
            for (int64_t m = 0; m < P; ++m) {
                const double g = 1.0 / (1.0 - dt * orc_laplace_symbol(d, N, m));
                re[m] *= g;
                im[m] *= g;
            }
            orc_fft(d, N, re, im, +1);
            for (int64_t p = 0; p < P; ++p) B[pl * P + p] = re[p] / (double)P;
        }
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < P; ++p) { /* reaction step */
            double b[16], r[16];
            for (int e = 0; e < nn; ++e) b[e] = B[e * P + p];
            orc_relax_reaction(n, kind, b, r);
            for (int e = 0; e < nn; ++e) A[e * P + p] = b[e] - c * r[e];
        }
    }
    free(re); free(im); free(B);
    return 0;
}

/* The relaxed energies E_{1,eps} (kind 1) and E_{2,eps} (kind 3) on the unit
 * torus: (1/2) int |grad A|_F^2, by Parseval (1/2) sum over entry planes and
 * modes of 4 pi^2 |k|^2 |F(A)(k) / P|^2, plus the mean over points of the
 * penalty, (1/(2 eps^2)) dist^2(O_n, A) = (1/(2 eps^2)) sum (sigma_i - 1)^2
 * (Lemma 1.1, computed as |A - U V^t|_F^2) or (1/(4 eps^2)) |A^t A - I|_F^2. */
int orc_relaxed_energy(int d, const int64_t* N, int n, int kind, double eps, const double* A, double* E)
{
    if (n < 1 || n > 4 || (kind != 1 && kind != 3) || !(eps > 0.0)) return -1;
    if (d < 1 || d > 3) return -1;
    for (int a = 0; a < d; ++a)
        if (!orc_is_pow2(N[a])) return -2;
    const int64_t P = orc_npoints(d, N);
    const int64_t nn = (int64_t)n * n;
    double* re = (double*)malloc(sizeof(double) * (size_t)P);
    double* im = (double*)malloc(sizeof(double) * (size_t)P);
    double* t = (double*)malloc(sizeof(double) * (size_t)P);
    double dir = 0.0;
    for (int64_t pl = 0; pl < nn; ++pl) {
        memcpy(re, A + pl * P, sizeof(double) * (size_t)P);
        memset(im, 0, sizeof(double) * (size_t)P);
        orc_fft(d, N, re, im, -1);
        for (int64_t m = 0; m < P; ++m)
            t[m] = -orc_laplace_symbol(d, N, m) * (re[m] * re[m] + im[m] * im[m]);
        dir += orc_pairwise_sum(t, P);
    }
    dir *= 0.5 / ((double)P * (double)P);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        double a[16], r[16];
        for (int e = 0; e < nn; ++e) a[e] = A[e * P + p];
        double s = 0.0;
        if (kind == 1) {
            orc_relax_reaction(n, 1, a, r); /* A - U V^t */
            for (int e = 0; e < nn; ++e) s += r[e] * r[e];
            t[p] = 0.5 * s;
        } else {
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double m = 0.0;
                    for (int k = 0; k < n; ++k) m += a[k * n + i] * a[k * n + j];
                    m -= (i == j ? 1.0 : 0.0);
                    s += m * m;
                }
            t[p] = 0.25 * s;
        }
    }
    const double pen = isinf(eps) ? 0.0 : orc_pairwise_sum(t, P) / ((double)P * eps * eps);
    *E = dir + pen;
    free(re); free(im); free(t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Surface diffusion on a sphere by the closest point method (Section 5.2)   */
/* ------------------------------------------------------------------------ */

/* T(x) = (2x / sqrt(pi)) exp(-x^2) + erfc(x) of Theorem 5.2: the heat-kernel
 * mass outside a ball of radius 2 x sqrt(tau). */
double orc_band_T(double x) { return 2.0 * x / sqrt(ORC_PI) * exp(-x * x) + erfc(x); }

/* The band width w_b with T(w_b / (2 sqrt(tau))) = eps (T decreases from 1 at
 * 0), by bisection. */
double orc_band_width(double tau, double eps)
{
    double lo = 0.0, hi = 40.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (orc_band_T(mid) > eps) lo = mid;
        else hi = mid;
    }
    return 2.0 * sqrt(tau) * 0.5 * (lo + hi);
}

/* p-point rule on [0, 1] at the Chebyshev points (the zeros of T_p) with the
 * weights that integrate every polynomial of degree < p exactly (Fejer's first
 * rule), nodes in ascending order. */
void orc_cheb_rule(int p, double* x, double* w)
{
    for (int k = 0; k < p; ++k) {
        const double th = ORC_PI * (2.0 * (p - 1 - k) + 1.0) / (2.0 * p); /* ascending cos */
        double s = 0.0;
        for (int j = 1; j <= p / 2; ++j) s += cos(2.0 * j * th) / (4.0 * j * j - 1.0);
        x[k] = 0.5 * (1.0 + cos(th));
        w[k] = 0.5 * (2.0 / p) * (1.0 - 2.0 * s);
    }
}

/* The closest-point sample set of a sphere of radius R centred at the origin
 * (Algorithm 2, step 1): grid points x_g = dx (i, j, k) with | |x_g| - R | < w_b,
 * in lexicographic (i, j, k) order; in each cell x_g + [0, dx]^3 the p^3
 * points of the rule above (lexicographic, first coordinate slowest), their
 * weights dx^3 w_a w_b w_c, and their closest points R x / |x| on the sphere
 * ((R, 0, 0) for x = 0).  With xq == NULL only counts: *count receives the
 * number of sample points (p^3 per band cell) and *cells the band cells. */
int orc_sphere_band(double R, double dx, int p, double wb, int64_t* count, int64_t* cells, double* xq,
                    double* xc, double* wq)
{
    if (!(R > 0.0) || !(dx > 0.0) || p < 1 || p > 8 || !(wb > 0.0)) return -1;
    double nx[8], nw[8];
    orc_cheb_rule(p, nx, nw);
    const int64_t lim = (int64_t)ceil((R + wb) / dx) + 1;
    int64_t c = 0, q = 0;
    for (int64_t i = -lim; i <= lim; ++i)
        for (int64_t j = -lim; j <= lim; ++j)
            for (int64_t k = -lim; k <= lim; ++k) {
                const double gx = dx * (double)i, gy = dx * (double)j, gz = dx * (double)k;
                const double d = fabs(sqrt(gx * gx + gy * gy + gz * gz) - R);
                if (!(d < wb)) continue;
                ++c;
                for (int a = 0; a < p; ++a)
                    for (int b = 0; b < p; ++b)
                        for (int e = 0; e < p; ++e) {
                            if (xq) {
                                const double x = gx + dx * nx[a], y = gy + dx * nx[b], z = gz + dx * nx[e];
                                const double r = sqrt(x * x + y * y + z * z);
                                xq[q] = x;
                                xq[*count + q] = y;
                                xq[2 * *count + q] = z;
                                xc[q] = r > 0.0 ? R * x / r : R;
                                xc[*count + q] = r > 0.0 ? R * y / r : 0.0;
                                xc[2 * *count + q] = r > 0.0 ? R * z / r : 0.0;
                                wq[q] = dx * dx * dx * nw[a] * nw[b] * nw[e];
                            }
                            ++q;
                        }
            }
    if (!xq) {
        *count = q;
        if (cells) *cells = c;
    }
    return 0;
}

/* Surfaces of revolution about the x axis (Section 6.3): a meridian
 * (X(s), rho(s)), s in [s0, s1], rho >= 0, rotated about the x axis.
 *   kind 0: the sphere of radius R, X = -R cos(pi s), rho = R sin(pi s), s in [0, 1];
 *   kind 1: the peanut, X = 3 t - t^3, rho = (1/2) sqrt((1 + X^2)(4 - X^2)),
 *           t in [-1, 1], with 4 - X^2 = (1 - t^2)^2 (4 - t^2) so that rho is
 *           a smooth function of t. */
static void orc_meridian(int kind, double R, double s, double* X, double* rho)
{
    if (kind == 0) {
        *X = -R * cos(ORC_PI * s);
        *rho = R * sin(ORC_PI * s);
    } else {
        const double x = 3.0 * s - s * s * s;
        *X = x;
        *rho = 0.5 * (1.0 - s * s) * sqrt((1.0 + x * x) * (4.0 - s * s));
    }
}

/* First and second derivatives of the meridian in its parameter. */
static void orc_meridian_d(int kind, double R, double s, double* X1, double* X2, double* r1, double* r2)
{
    if (kind == 0) {
        *X1 = R * ORC_PI * sin(ORC_PI * s);
        *X2 = R * ORC_PI * ORC_PI * cos(ORC_PI * s);
        *r1 = R * ORC_PI * cos(ORC_PI * s);
        *r2 = -R * ORC_PI * ORC_PI * sin(ORC_PI * s);
    } else {
        /* rho = a sqrt(h) / 2, a = 1 - t^2, h = u v, u = 1 + X^2, v = 4 - t^2 */
        const double t = s, X = 3.0 * t - t * t * t, Xp = 3.0 - 3.0 * t * t, Xpp = -6.0 * t;
        const double u = 1.0 + X * X, up = 2.0 * X * Xp, upp = 2.0 * (Xp * Xp + X * Xpp);
        const double v = 4.0 - t * t, vp = -2.0 * t, vpp = -2.0;
        const double h = u * v, hp = up * v + u * vp, hpp = upp * v + 2.0 * up * vp + u * vpp;
        const double a = 1.0 - t * t, ap = -2.0 * t, app = -2.0;
        const double sh = sqrt(h);
        *X1 = Xp;
        *X2 = Xpp;
        *r1 = 0.5 * (ap * sh + a * hp / (2.0 * sh));
        *r2 = 0.5 * (app * sh + ap * hp / sh + a * (hpp / (2.0 * sh) - hp * hp / (4.0 * h * sh)));
    }
}

static void orc_meridian_range(int kind, double* s0, double* s1)
{
    *s0 = kind == 0 ? 0.0 : -1.0;
    *s1 = 1.0;
}

/* Closest point on the surface of revolution to p = (x, y, z): the closest
 * point (X(s), rho(s)) of the meridian to (x, r), r = |(y, z)|, rotated into the
 * half plane of p ((y, z) = (r, 0) taken when r = 0, where it is not unique).
 * The meridian is scanned at 8193 parameter values, and the best one refined
 * by golden-section search between its neighbours.  Returns the distance. */
double orc_revolution_cp(int kind, double R, double x, double y, double z, double* c)
{
    const double r = sqrt(y * y + z * z);
    double s0, s1;
    orc_meridian_range(kind, &s0, &s1);
    const int N = 8192;
    int best = 0;
    double bd = INFINITY;
    for (int k = 0; k <= N; ++k) {
        double X, rho;
        orc_meridian(kind, R, s0 + (s1 - s0) * k / N, &X, &rho);
        const double d = (X - x) * (X - x) + (rho - r) * (rho - r);
        if (d < bd) {
            bd = d;
            best = k;
        }
    }
    double a = s0 + (s1 - s0) * (best > 0 ? best - 1 : 0) / N;
    double b = s0 + (s1 - s0) * (best < N ? best + 1 : N) / N;
    const double g = 0.5 * (sqrt(5.0) - 1.0);
    for (int it = 0; it < 200 && b - a > 1e-16; ++it) {
        const double u = b - g * (b - a), v = a + g * (b - a);
        double Xu, ru, Xv, rv;
        orc_meridian(kind, R, u, &Xu, &ru);
        orc_meridian(kind, R, v, &Xv, &rv);
        const double du = (Xu - x) * (Xu - x) + (ru - r) * (ru - r);
        const double dv = (Xv - x) * (Xv - x) + (rv - r) * (rv - r);
        if (du <= dv) b = v;
        else a = u;
    }
    /* Newton on the derivative of the squared distance polishes the golden-
     * section bracket (whose width is limited by the flat minimum to about the
     * square root of the rounding) to full precision */
    double t = 0.5 * (a + b);
    for (int it = 0; it < 4; ++it) {
        double X, rho, X1, X2, r1, r2;
        orc_meridian(kind, R, t, &X, &rho);
        orc_meridian_d(kind, R, t, &X1, &X2, &r1, &r2);
        const double g = (X - x) * X1 + (rho - r) * r1;
        const double H = X1 * X1 + (X - x) * X2 + r1 * r1 + (rho - r) * r2;
        if (!(H > 0.0)) break;
        const double tn = t - g / H;
        if (!(tn >= a - 1e-6 && tn <= b + 1e-6) || tn < s0 || tn > s1) break;
        t = tn;
    }
    double X, rho;
    orc_meridian(kind, R, t, &X, &rho);
    c[0] = X;
    c[1] = r > 0.0 ? rho * y / r : rho;
    c[2] = r > 0.0 ? rho * z / r : 0.0;
    return sqrt((c[0] - x) * (c[0] - x) + (c[1] - y) * (c[1] - y) + (c[2] - z) * (c[2] - z));
}

/* The closest-point sample set of a surface of revolution (as orc_sphere_band,
 * with the distance and closest points of orc_revolution_cp): grid points
 * x_g = dx (i, j, k) within w_b of the surface over the box that holds the
 * surface grown by w_b, lexicographic; p^3 Chebyshev points per cell. */
int orc_revolution_band(int kind, double R, double dx, int p, double wb, int64_t* count, int64_t* cells,
                        double* xq, double* xc, double* wq)
{
    if (kind < 0 || kind > 1 || !(R > 0.0) || !(dx > 0.0) || p < 1 || p > 8 || !(wb > 0.0)) return -1;
    double nx[8], nw[8];
    orc_cheb_rule(p, nx, nw);
    const double xext = kind == 0 ? R : 2.0, rext = kind == 0 ? R : 1.25;
    const int64_t lx = (int64_t)ceil((xext + wb) / dx) + 1, lr = (int64_t)ceil((rext + wb) / dx) + 1;
    int64_t c = 0, q = 0;
    for (int64_t i = -lx; i <= lx; ++i)
        for (int64_t j = -lr; j <= lr; ++j)
            for (int64_t k = -lr; k <= lr; ++k) {
                const double gx = dx * (double)i, gy = dx * (double)j, gz = dx * (double)k;
                double cc[3];
                if (!(orc_revolution_cp(kind, R, gx, gy, gz, cc) < wb)) continue;
                ++c;
                for (int a = 0; a < p; ++a)
                    for (int b = 0; b < p; ++b)
                        for (int e = 0; e < p; ++e) {
                            if (xq) {
                                const double x = gx + dx * nx[a], y = gy + dx * nx[b], z = gz + dx * nx[e];
                                xq[q] = x;
                                xq[*count + q] = y;
                                xq[2 * *count + q] = z;
                                orc_revolution_cp(kind, R, x, y, z, cc);
                                xc[q] = cc[0];
                                xc[*count + q] = cc[1];
                                xc[2 * *count + q] = cc[2];
                                wq[q] = dx * dx * dx * nw[a] * nw[b] * nw[e];
                            }
                            ++q;
                        }
            }
    if (!xq) {
        *count = q;
        if (cells) *cells = c;
    }
    return 0;
}

/* One step of surface diffusion by the closest point method (eqs.
 * surface_diffusion_extended, freeSpace): the field A (entry-planar [n*n][m],
 * its value at sample q being A(x_q^c), i.e. already the constant extension
 * to x_q) is convolved with the free-space heat kernel
 * G_tau(x) = (4 pi tau)^{-3/2} exp(-|x|^2 / (4 tau)) by the quadrature of the
 * band, and the result is taken at the closest points:
 *   out(c) = sum_q w_q G_tau(x_c^c - x_q) A(q).
 * Direct sums, O(m^2). */
int orc_surface_diffuse(int64_t m, const double* xq, const double* xc, const double* wq, int n, double tau,
                        const double* A, double* out)
{
    if (m < 0 || n < 1 || n > 4 || !(tau > 0.0)) return -1;
    const int nn = n * n;
    const double norm = pow(4.0 * ORC_PI * tau, -1.5);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < m; ++c) {
        double acc[16] = {0.0};
        const double cx = xc[c], cy = xc[m + c], cz = xc[2 * m + c];
        for (int64_t q = 0; q < m; ++q) {
            const double dx = cx - xq[q], dy = cy - xq[m + q], dz = cz - xq[2 * m + q];
            const double g = wq[q] * exp(-(dx * dx + dy * dy + dz * dz) / (4.0 * tau));
            for (int e = 0; e < nn; ++e) acc[e] += g * A[e * m + q];
        }
        for (int e = 0; e < nn; ++e) out[e * m + c] = norm * acc[e];
    }
    return 0;
}

/* The same convolution taken at nt arbitrary target points xt ([3][nt]):
 *   out(t) = sum_q w_q G_tau(x_t - x_q) A(q),   out entry-planar [n*n][nt].
 * At xt = the closest points this is orc_surface_diffuse restricted to the
 * chosen targets (large bands, sampled outputs).  O(m nt). */
int orc_heat_at(int64_t m, const double* xq, const double* wq, int n, double tau, const double* A, int64_t nt,
                const double* xt, double* out)
{
    if (m < 0 || nt < 0 || n < 1 || n > 4 || !(tau > 0.0)) return -1;
    const int nn = n * n;
    const double norm = pow(4.0 * ORC_PI * tau, -1.5);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; ++t) {
        double acc[16] = {0.0};
        const double cx = xt[t], cy = xt[nt + t], cz = xt[2 * nt + t];
        for (int64_t q = 0; q < m; ++q) {
            const double dx = cx - xq[q], dy = cy - xq[m + q], dz = cz - xq[2 * m + q];
            const double g = wq[q] * exp(-(dx * dx + dy * dy + dz * dz) / (4.0 * tau));
            for (int e = 0; e < nn; ++e) acc[e] += g * A[e * m + q];
        }
        for (int e = 0; e < nn; ++e) out[e * nt + t] = norm * acc[e];
    }
    return 0;
}

/* The MBO iteration on the sphere (Algorithm 1 with the diffusion step above):
 * K steps of A <- P(S_tau A), P the pointwise projection of Lemma 1.1.
 * flips (nullable, [K]) counts the samples whose det sign changed. */
int orc_surface_iterate(int64_t m, const double* xq, const double* xc, const double* wq, int n, double tau,
                        double* A, int K, int64_t* flips)
{
    if (m < 0 || n < 1 || n > 4 || !(tau > 0.0) || K < 0) return -1;
    const int64_t nn = (int64_t)n * n;
    double* T = (double*)malloc(sizeof(double) * (size_t)(m * nn + 1));
    int8_t* sp = (int8_t*)malloc((size_t)m + 1);
    int8_t* sn = (int8_t*)malloc((size_t)m + 1);
    orc_det_sign(m, n, A, sp);
    int rc = 0;
    for (int s = 0; s < K && rc == 0; ++s) {
        rc = orc_surface_diffuse(m, xq, xc, wq, n, tau, A, T);
        if (rc) break;
        orc_project(m, n, T, A, sn, NULL, NULL);
        int64_t f = 0;
        for (int64_t i = 0; i < m; ++i) f += sn[i] != sp[i];
        if (flips) flips[s] = f;
        memcpy(sp, sn, (size_t)m);
    }
    free(T); free(sp); free(sn);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Volume-preserving MBO on a surface (Section 7, Algorithm 3)               */
/* ------------------------------------------------------------------------ */

/* Algorithm 3: sort Delta E in descending order (equal values in ascending
 * sample index, as on the flat torus), then take the samples in that order,
 * adding their volume weights W, while the sum is below V.  sel[q] = 1 for the
 * taken samples: V <= 0 takes none, V above the total takes all.  The weights
 * are integers (the sample's quadrature weight in units of 2^-30 dx^3), so the
 * cut does not depend on the order of summation.  Returns -1 on bad
 * arguments, -2 when a value is not finite. */
int orc_weighted_select(int64_t m, const double* dE, const int64_t* W, int64_t V, int8_t* sel)
{
    if (m < 0) return -1;
    for (int64_t q = 0; q < m; ++q) {
        if (!isfinite(dE[q])) return -2;
        if (W[q] < 0) return -1;
    }
    orc_rank_t* rk = (orc_rank_t*)malloc(sizeof(orc_rank_t) * (size_t)(m + 1));
    for (int64_t q = 0; q < m; ++q) {
        rk[q].de = dE[q];
        rk[q].idx = q;
    }
    qsort(rk, (size_t)m, sizeof(orc_rank_t), orc_rank_cmp);
    memset(sel, 0, (size_t)m);
    int64_t acc = 0;
    for (int64_t r = 0; r < m && acc < V; ++r) {
        sel[rk[r].idx] = 1;
        acc += W[rk[r].idx];
    }
    free(rk);
    return 0;
}

/* Volume-preserving MBO on the sphere: K steps of diffusion (the direct band
 * quadrature above) followed by the reassignment of Lemma 7.2 with the
 * selection of Algorithm 3: T+ on the selected samples, T- elsewhere.
 * V (nullable): the volume to keep in SO(n), in weight units; NULL takes the
 * weight of the samples of A with det >= 0.  V_used (nullable) receives it.
 * flips (nullable, [K]) counts the samples whose det sign changed. */
int orc_surface_iterate_volume(int64_t m, const double* xq, const double* xc, const double* wq,
                               const int64_t* W, int n, double tau, double* A, int K, const int64_t* V,
                               int64_t* V_used, int64_t* flips)
{
    if (m < 0 || n < 1 || n > 4 || !(tau > 0.0) || K < 0) return -1;
    const int64_t nn = (int64_t)n * n;
    int8_t* sp = (int8_t*)malloc((size_t)m + 1);
    int8_t* sel = (int8_t*)malloc((size_t)m + 1);
    double* T = (double*)malloc(sizeof(double) * (size_t)(m * nn + 1));
    double* tp = (double*)malloc(sizeof(double) * (size_t)(m * nn + 1));
    double* tm = (double*)malloc(sizeof(double) * (size_t)(m * nn + 1));
    double* de = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    orc_det_sign(m, n, A, sp);
    int64_t vol = 0;
    if (V) {
        vol = *V;
    } else {
        for (int64_t q = 0; q < m; ++q) vol += sp[q] > 0 ? W[q] : 0;
    }
    if (V_used) *V_used = vol;
    int rc = 0;
    for (int s = 0; s < K && rc == 0; ++s) {
        rc = orc_surface_diffuse(m, xq, xc, wq, n, tau, A, T);
        if (rc) break;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < m; ++q) {
            double a[16];
            for (int e = 0; e < nn; ++e) a[e] = T[e * m + q];
            de[q] = orc_vp_point(n, a, tp + q * nn, tm + q * nn);
        }
        rc = orc_weighted_select(m, de, W, vol, sel);
        if (rc) break;
        int64_t f = 0;
        for (int64_t q = 0; q < m; ++q) {
            const double* t = sel[q] ? tp + q * nn : tm + q * nn;
            for (int e = 0; e < nn; ++e) A[e * m + q] = t[e];
            const int8_t sn = sel[q] ? 1 : -1;
            f += sn != sp[q];
            sp[q] = sn;
        }
        if (flips) flips[s] = f;
    }
    free(sp); free(sel); free(T); free(tp); free(tm); free(de);
    return rc;
}

/* Number of threads the OpenMP loops above use (1 without OpenMP), and its
 * setter for the loops that follow (timing on a chosen number of threads). */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_num_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
#else
int orc_num_threads(void) { return 1; }
void orc_set_num_threads(int t) { (void)t; }
#endif
