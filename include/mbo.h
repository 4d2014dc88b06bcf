/*
 * mbo.h -- C ABI of libmbo: the generalized MBO diffusion generated motion for
 * orthogonal matrix-valued fields on flat tori, on AMD Instinct MI355X (gfx950).
 *
 * Method: B. Osting and D. Wang, "A generalized MBO diffusion generated motion
 * for orthogonal matrix-valued fields", arXiv:1711.01365.  Algorithm 1 alternates
 *   (1) a diffusion step: every entry of the n x n field A is evolved by the heat
 *       equation for time tau; on the flat torus (Section 5.1) this is a forward
 *       FFT, a multiplication by the heat symbol exp(-4 pi^2 |k|^2 tau), and an
 *       inverse FFT;
 *   (2) a projection step: each point is replaced by its closest orthogonal
 *       matrix U V^t (Lemma 1.1), where U Sigma V^t is its SVD.
 * The Lyapunov functional of Section 4 (eq. (Lyapunov)),
 *       E(A) = (1/tau) * integral over the torus of [ n - <A, e^{tau Delta} A>_F ],
 * does not increase along the iterates (Proposition 4.3).
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every entry point
 * ---------------------------------------------------------------------------
 * Domain      the unit-period torus [0,1)^d, d = 2 or 3, sampled at N[a] points
 *             per axis (x = j / N[a]); each N[a] is a power of two in [8, 2048].
 *             Axis 0 is the slowest-varying one.
 * Field       DEVICE memory, "entry-planar", row-major:
 *                 A[b][i][j][p]  =  entry (i, j) of the matrix at grid point p
 *             of field b (b < batch, i, j < n, p < prod(N), last axis fastest).
 *             Element type is double for MBO_F64 and float otherwise.  Buffers
 *             must be 16-byte aligned.  A torch tensor of shape
 *             (batch, n, n, *N) in C order has exactly this layout.
 * Heat symbol exp(-4 pi^2 tau sum_a k_a^2) with k_a = m_a for m_a < N[a]/2 and
 *             m_a - N[a] otherwise (Nyquist counts as -N[a]/2), the exact Fourier
 *             multiplier of e^{tau Delta} on the unit torus.
 * Energy      E(A) = (1/tau) * (1/prod(N)) * sum_p [ n - <A(p), (e^{tau Delta}A)(p)>_F ]
 *             (quadrature weight 1/prod(N) for the integral).
 * Projection  closest orthogonal matrix of Lemma 1.1.  When the input is singular
 *             the minimiser is not unique: a singular value <= n*eps*sigma_max
 *             (eps of the working precision) counts as zero and the minimiser
 *             with det = +1 is returned; the zero matrix maps to the identity.
 *             n = 1 is sign thresholding with sgn(0) = +1 (Remark 1.2).
 * Ownership   the caller owns every field buffer; the plan owns its workspace,
 *             tables and graphs and frees them in mbo_plan_destroy.  No call
 *             keeps a caller pointer after it returns (a captured iteration graph
 *             is keyed by the field pointer and re-captured when it changes).
 * Streams     all device work is enqueued on the plan's HIP stream.  Calls that
 *             return host values (mbo_energy, the logs of mbo_iterate)
 *             synchronise that stream before returning.  A plan must not be used
 *             by two host threads at once.
 * Errors      every entry point returns an mbo_status; nothing is thrown and
 *             nothing aborts.  On error the outputs are unspecified and
 *             mbo_last_error() describes the failure.
 * Precision   MBO_F64: all arithmetic in double.
 *             MBO_F32: diffusion and projection in float.
 *             MBO_F32_F64FALLBACK: as MBO_F32, but a point whose float-computed
 *             smallest singular value of the diffused matrix is below
 *             sigma_fallback is re-projected in double from the float values.
 * ---------------------------------------------------------------------------
 */
#ifndef MBO_H
#define MBO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbo_plan_s* mbo_plan_t;

typedef enum {
    MBO_OK = 0,
    MBO_ERR_INVALID_ARG = 1,  /* null pointer, d not in {2,3}, n not in [1,4],
                                 tau not finite and > 0, batch < 1, bad precision */
    MBO_ERR_UNSUPPORTED = 2,  /* some N[a] not a power of two in [8, 2048], or a
                                 row (last axis) whose packed planes do not fit
                                 in LDS: in MBO_F64, a last axis of 2048 with
                                 n >= 3 */
    MBO_ERR_ALLOC = 3,        /* device allocation failed */
    MBO_ERR_HIP = 4,          /* a HIP runtime call failed (see mbo_last_error) */
    MBO_ERR_NONFINITE = 5,    /* NaN or Inf met in the input of a projection */
    MBO_ERR_SCRATCH = 6       /* mbo_step_static: the field's working memory
                                 exceeds MBO_STEP_STATIC_MAX_BYTES */
} mbo_status;

typedef enum {
    MBO_F64 = 0,
    MBO_F32 = 1,
    MBO_F32_F64FALLBACK = 2
} mbo_precision;

/* Kernels that mbo_iterate runs (Algorithm 1 with the diffusion of Section 5.1).
 * MBO_PATH_BANDED (the default) keeps, in 2-D, only the row modes |kx| <= c of
 * every row spectrum between the two passes of an iteration: c is the smallest
 * half-width for which the heat symbol summed over every dropped mode,
 * sum exp(-4 pi^2 tau |k|^2), is at most eta = 1e-12 (float plans) or 1e-20
 * (MBO_F64).  Since every Fourier coefficient of a field is at most
 * prod(N) max|A| in modulus, dropping those modes moves each diffused value by
 * at most eta max|A|, far below the rounding of the transforms.  A plan whose
 * tau and grid leave nothing to drop runs the same kernels with every mode kept.
 * MBO_PATH_FULL runs the same kernels with every mode kept; MBO_PATH_GENERIC the
 * general kernels (any d, any row length), which the other calls always use.
 * The band-limited kernels serve d = 2 with a first axis of at least 64 points
 * (every last axis a plan accepts); other shapes run the general kernels. */
typedef enum {
    MBO_PATH_GENERIC = 0,
    MBO_PATH_FULL = 1,
    MBO_PATH_BANDED = 2
} mbo_path;

/* Create a plan for `batch` fields of n x n matrices on the grid N[0..d-1].
 * tau: diffusion time of one step (Algorithm 1, step 1).
 * sigma_fallback: threshold of MBO_F32_F64FALLBACK (ignored otherwise); a value
 *   <= 0 selects the default 1e-3.
 * hip_stream: a hipStream_t (NULL = the default stream) on which all work runs;
 *   the device is the current HIP device at this call.
 * On success *out receives the plan. */
mbo_status mbo_plan(mbo_plan_t* out, int d, const int64_t* N, int n, int64_t batch,
                    double tau, mbo_precision prec, double sigma_fallback, void* hip_stream);

/* Free a plan and everything it owns (NULL is accepted). */
mbo_status mbo_plan_destroy(mbo_plan_t plan);

/* Change the diffusion time; the heat-symbol tables are rebuilt. */
mbo_status mbo_plan_set_tau(mbo_plan_t plan, double tau);

/* Choose the kernels of mbo_iterate (see mbo_path; a batched plan applies the
 * choice to every field class).  Synchronises the plan's stream; a captured
 * iteration graph is rebuilt on the next mbo_iterate.  MBO_ERR_INVALID_ARG for an
 * unknown path. */
mbo_status mbo_plan_set_path(mbo_plan_t plan, mbo_path path);

/* The kernels mbo_iterate runs for `field` (0 <= field < count, or < batch for
 * a plain plan): *path (MBO_PATH_GENERIC when the shape has no band-limited
 * kernels), the kept half-width *band_half_width along the last axis and the
 * modes *stored_modes kept per row between the passes (the axis length when
 * every mode is kept).  All outputs nullable. */
mbo_status mbo_plan_path(mbo_plan_t plan, int field, int* path, int* band_half_width, int* stored_modes);

/* Change the stream subsequent calls are enqueued on. */
mbo_status mbo_plan_set_stream(mbo_plan_t plan, void* hip_stream);

/* Kernel timing (a diagnostic, off by default).  When enabled, mbo_iterate
 * launches its kernels directly on the plan's stream instead of through the
 * captured graph, each row pass (inverse row FFT, projection, forward row FFT)
 * and heat pass (strided-axis FFT, heat symbol, inverse) with HIP start/stop
 * events recorded by its own dispatch. */
mbo_status mbo_plan_set_timing(mbo_plan_t plan, int enable);

/* Average durations, in microseconds, of the row passes and heat passes of the
 * last mbo_iterate call made with timing enabled, and the number of iterations
 * averaged over (all nullable). */
mbo_status mbo_last_timing(mbo_plan_t plan, double* row_us, double* heat_us, int* launches);

/* Diffusion step (Algorithm 1 step 1, Section 5.1):
 *   A_out = e^{tau Delta} A_in, entry by entry, for every field of the batch.
 * A_out may alias A_in.  Asynchronous. */
mbo_status mbo_diffuse(mbo_plan_t plan, const void* A_in, void* A_out);

/* Projection step (Algorithm 1 step 2, Lemma 1.1): A_out(p) = U(p) V(p)^t.
 * det_sign (nullable, device, int8 [batch][prod(N)]) receives sgn det A_out(p),
 * which equals sgn det A_in(p) for nonsingular input.  A_out may alias A_in.
 * Returns MBO_ERR_NONFINITE (after synchronising) if any input value is NaN/Inf. */
mbo_status mbo_project(mbo_plan_t plan, const void* A_in, void* A_out, int8_t* det_sign);

/* Counts of the last mbo_project call on this plan (all fields): points
 * re-projected in double (MBO_F32_F64FALLBACK: float-computed smallest singular
 * value below sigma_fallback) and points whose input held NaN/Inf.  Nullable
 * outputs. */
mbo_status mbo_last_project_counts(mbo_plan_t plan, int64_t* fallbacks, int64_t* nonfinite);

/* Algorithm 1: A_s = P(e^{tau Delta} A_{s-1}) for s = 1..max_iter, in place on A
 * (device, holds A_0 on entry and the last iterate on return).  A_0 need not be
 * orthogonal: the first step diffuses whatever is given.
 * tol > 0: field b stops after the first s with max|A_s - A_{s-1}| <= tol
 *   (the change is then tracked every iteration, which costs one extra read and
 *   write of the field per iteration); tol <= 0 runs all max_iter iterations.
 * Host-side logs, all nullable, laid out [batch][...]:
 *   iters_done  [batch]              iterations performed per field;
 *   energy      [batch][max_iter+1]  E(A_s) for s = 0..iters_done (rest unset);
 *   flips       [batch][max_iter]    points whose det sign differs between A_s
 *                                    and A_{s-1} (A_0: sgn det with sgn(0) = +1);
 *   delta       [batch][max_iter]    max|A_s - A_{s-1}| (only when tol > 0,
 *                                    otherwise filled with -1);
 *   fallbacks   [batch][max_iter]    points re-projected in double (fallback mode).
 * The iteration runs as one captured HIP graph (re-used while A, max_iter and the
 * requested logs stay the same); the logs are copied back once, at the end,
 * which synchronises the stream.  max_iter = 0 only evaluates E(A_0). */
mbo_status mbo_iterate(mbo_plan_t plan, void* A, int max_iter, double tol, int* iters_done,
                       double* energy, int64_t* flips, double* delta, int64_t* fallbacks);

/* Lyapunov functional E(A) of each field of the batch (Section 4,
 * eq. (Lyapunov)), evaluated through Parseval in Fourier space:
 *   E = (1/tau) (n - prod(N)^{-2} sum_m symbol(m) sum_ij |FFT(A_ij)(m)|^2).
 * E: host, [batch].  Synchronises the stream. */
mbo_status mbo_energy(mbo_plan_t plan, const void* A, double* E);

/* ---------------------------------------------------------------------------
 * Relaxed gradient flows (Section 1), the comparison PDEs of the MBO method:
 *   GD-1  dA/dt = Delta A - eps^-2 U (Sigma - I) V^t   (E_{1,eps}, penalty
 *         dist^2(O_n, A) / (2 eps^2); U (Sigma - I) V^t = A - U V^t by Lemma 1.1)
 *   GD-3  dA/dt = Delta A - eps^-2 A (A^t A - I)        (E_{2,eps}, penalty
 *         |A^t A - I|_F^2 / (4 eps^2); the same flow as GD-2)
 * The paper states the flows, not a scheme.  One step here is an implicit-Euler
 * diffusion step B = (I - dt Delta)^{-1} A (Fourier symbol 1 / (1 + 4 pi^2 dt
 * |k|^2)) followed by an explicit reaction step A = B - (dt / eps^2) N(B): first
 * order in dt, energy-decreasing for small dt / eps^2.  eps = +inf drops the
 * reaction (pure implicit heat steps).  GD-1 at a singular point uses the
 * projection's convention (det +1 minimiser).  The plan's tau is not used.
 * Batched plans return MBO_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------- */
typedef enum { MBO_GD1 = 1, MBO_GD3 = 3 } mbo_flow;

/* `steps` steps of the flow `kind` (an mbo_flow) in place on A (device, plan
 * layout).  dt > 0 finite, eps > 0.  Runs as one captured HIP graph (re-used
 * while A, steps, kind, eps and dt stay the same); synchronises and returns
 * MBO_ERR_NONFINITE if a NaN/Inf was met. */
mbo_status mbo_relaxed_flow(mbo_plan_t plan, void* A, int steps, int kind, double eps, double dt);

/* E_{1,eps} (kind MBO_GD1) or E_{2,eps} (MBO_GD3) of each field on the unit
 * torus: (1/2) int |grad A|_F^2 (from the spectrum, Parseval) plus the mean
 * over grid points of the penalty.  E: host [batch].  Synchronises. */
mbo_status mbo_relaxed_energy(mbo_plan_t plan, const void* A, int kind, double eps, double* E);

/* ---------------------------------------------------------------------------
 * Surface diffusion on a closed surface, the sphere of radius R centred at the
 * origin, by the closest point method (Section 5.2): the diffusion step of
 * Algorithm 1 on the surface is the free-space heat convolution of the field
 * extended constant along normals, evaluated at the closest points,
 *     (S_tau A)(c_j) = sum_q w_q G_tau(c_j - x_q) A(c(x_q)),
 *     G_tau(r) = (4 pi tau)^{-3/2} exp(-|r|^2 / (4 tau)),
 * over quadrature points x_q that fill a band of half width w_b around the
 * surface (Theorem 5.2: w_b solves T(w_b / (2 sqrt tau)) = eps with
 * T(x) = 2 x e^{-x^2} / sqrt(pi) + erfc(x)).  The band is the union of the
 * grid cells [dx i, dx (i+1)) x ... whose corner dx (i, j, k) lies within w_b
 * of the sphere; each cell holds p^3 points, the tensor product of p Chebyshev
 * points (zeros of T_p mapped to [0, 1]) with the Fejer weights, times dx^3.
 * Samples are in canonical order: cells lexicographic in (i, j, k), then the
 * points of a cell lexicographic in their Chebyshev indices.  Every sample q is
 * both a quadrature point x_q and, through its closest point c_q = R x_q / |x_q|,
 * a target: fields live at the samples, entry-planar [n*n][m] (entry (i, j) of
 * sample q at (i n + j) m + q), in the surface's precision.
 *
 * The sum is not formed directly: the samples are spread onto a periodic
 * Cartesian grid (a power of two per axis, at most 512) with the
 * "exponential of semicircle" kernel, the grid is transformed by the FFT of a
 * 3-D plan, multiplied by the heat symbol divided by the kernel's transform,
 * transformed back and interpolated at the closest points, with a gridding
 * tolerance of max(eps / 10, 1e-11) (float surfaces: max(eps / 10, 1e-7)).
 * The result then matches the sum to within about eps times the largest |A|
 * entry (float surfaces: max(eps, 4e-6) times it).
 * ------------------------------------------------------------------------- */
typedef struct mbo_surface_s* mbo_surface_t;

/* Build the sample set (host, FP64) and the device state of the sphere of
 * radius R > 0 for band cells of size dx > 0, p in [1, 8] Chebyshev points per
 * cell axis, diffusion time tau > 0, band tolerance eps in (0, 0.5), matrices
 * of size n in [1, 4] and precision prec (MBO_F32_F64FALLBACK: float surface
 * whose projection falls back to double near singular points).  hip_stream
 * (hipStream_t, nullable) carries every later call.  MBO_ERR_UNSUPPORTED when
 * the grid would need more than 512 points per axis (tau too small for the
 * radius), when the lattice to scan has more than 1501 points per half axis
 * ((R + w_b) / dx too large) or when the band holds 2^31 samples or more.  On
 * error *out is NULL and mbo_surface_last_error(NULL) explains. */
mbo_status mbo_surface_sphere(mbo_surface_t* out, double R, double dx, int p, double tau, double eps, int n,
                              mbo_precision prec, void* hip_stream);

/* The same for the peanut of Section 6.3: the meridian X(t) = 3t - t^3,
 * rho(t) = sqrt((1 + X^2)(4 - X^2)) / 2, t in [-1, 1], rotated about the x axis
 * (tips at x = +-2, waist radius 1, largest radius 1.25).  Closest points are
 * the closest points of the meridian to (x, |(y, z)|) turned into the half plane
 * of the point ((y, z) = (rho, 0) on the axis, where they are not unique);
 * the band, cells, weights, diffusion and steps are as for the sphere. */
mbo_status mbo_surface_peanut(mbo_surface_t* out, double dx, int p, double tau, double eps, int n,
                              mbo_precision prec, void* hip_stream);

/* Free the surface (synchronises its stream).  NULL is a no-op. */
mbo_status mbo_surface_destroy(mbo_surface_t s);

/* Sample count m, band cell count, grid points per axis, band half width w_b
 * (each output nullable). */
mbo_status mbo_surface_info(mbo_surface_t s, int64_t* samples, int64_t* cells, int* grid, double* band_width);

/* Copy the sample set to host buffers (each nullable): quadrature points xq
 * [3][m], closest points xc [3][m], weights w [m], FP64, canonical order. */
mbo_status mbo_surface_points(mbo_surface_t s, double* xq, double* xc, double* w);

/* A_out = S_tau A_in (device buffers [n*n][m], which must not alias).
 * Asynchronous on the surface's stream; no NaN check. */
mbo_status mbo_surface_diffuse(mbo_surface_t s, const void* A_in, void* A_out);

/* K steps of Algorithm 1 on the surface in place on A (device [n*n][m]):
 * A <- P(S_tau A), P the projection of Lemma 1.1 per sample.  flips (host,
 * nullable, [K]): per step, the samples whose det sign changed.  Synchronises;
 * MBO_ERR_NONFINITE when a NaN/Inf was met. */
mbo_status mbo_surface_iterate(mbo_surface_t s, void* A, int K, int64_t* flips);

/* Volume-preserving MBO on the surface (Section 7, Algorithm 3).  Each sample
 * carries an integer volume weight W_q: its quadrature weight in units of
 * 2^-30 dx^3, rounded, so that sums of weights are exact and the selection does
 * not depend on the order of summation.  After the diffusion, Delta E =
 * 2 sgn(det) sigma_min per sample (as on the flat torus); the samples are taken
 * in descending Delta E (equal values in ascending sample index) while the
 * weight taken is below V; the taken samples receive T+ (closest point of
 * SO(n)), all others T- (Lemma 7.2).  V <= 0 takes none, V above the total
 * weight takes all.  MBO_F32_F64FALLBACK surfaces re-evaluate a sample in
 * double when its float sigma_min is below 1e-3. */

/* The weights W_q, host int64 [m], canonical order. */
mbo_status mbo_surface_volume_weights(mbo_surface_t s, int64_t* W);

/* Selection alone: selected[q] = 1 for the samples Algorithm 3 takes for the
 * values dE (device [m], the surface's element type, finite) and the volume V
 * (weight units), 0 elsewhere (device uint8 [m]).  Synchronises. */
mbo_status mbo_surface_volume_select(mbo_surface_t s, const void* dE, int64_t V, uint8_t* selected);

/* K volume-preserving steps in place on A (device [n*n][m]).  V: host, the
 * volume to keep in SO(n) in weight units, or NULL for the weight of the
 * samples of A with det >= 0; V_used (host, nullable) receives it.  flips
 * (host, nullable, [K]): per step, the samples whose det sign changed.
 * Synchronises; MBO_ERR_NONFINITE when a NaN/Inf was met. */
mbo_status mbo_surface_iterate_volume(mbo_surface_t s, void* A, int K, const int64_t* V, int64_t* V_used,
                                      int64_t* flips);

/* Description of the last error on this surface (or of the last failed
 * mbo_surface_sphere call when s is NULL). */
const char* mbo_surface_last_error(mbo_surface_t s);

/* Index of an SO(2)-valued field (Section 6.1), a diagnostic of the flat-torus
 * examples: for each field of an n = 2 plan on a 2-D grid, the winding of the
 * first column (A_00, A_10) of the matrices -- the vector field the paper draws;
 * a rotation and a reflection with the same angle share it -- along the loops
 * that wrap once around the torus:
 *   w_x[b][j]  along axis 0 (x) at column j, the class [gamma]_{1,0};  host [batch][N1];
 *   w_y[b][i]  along axis 1 (y) at row i,    the class [gamma]_{0,1};  host [batch][N0].
 * Each is (1/2 pi) times the sum, over consecutive samples with the last joined
 * to the first, of the angle from one first column to the next in (-pi, pi]:
 * an integer (to rounding) when neighbouring samples differ by less than pi.
 * Either output may be NULL.  Other plans return MBO_ERR_UNSUPPORTED.
 * Allocates a small device buffer per call; synchronises. */
mbo_status mbo_so2_index(mbo_plan_t plan, const void* A, double* w_x, double* w_y);

/* ---------------------------------------------------------------------------
 * Volume-preserving MBO (Section 7).  Step 2 of Algorithm 1 is replaced by a
 * reassignment that keeps the number of grid points in SO(n) fixed (the volume
 * of the SO(n) region on the uniform grid).  For the diffused matrix A~ at a
 * point, with A~ = U Sigma V^t:
 *   T+(A~)  the closest point of SO(n), T-(A~) the closest point of SO^-(n):
 *           U V^t and U D_n V^t (Lemma 1.1, Lemma 7.1), D_n reversing the
 *           direction of the smallest singular value; which of the two has
 *           det +1 decides which is T+;
 *   Delta E = <T+ - T-, A~>_F = 2 sgn(det A~) sigma_min(A~).
 * The n_plus points of a field with the largest Delta E receive T+, all others
 * T- (Lemma 7.2, with the flat-torus rule of taking the first n_plus values in
 * descending order).  Equal values are taken in ascending point index (flat
 * index p of the entry-planar layout); the paper leaves ties open.  When the
 * smallest singular value is repeated, T- is not unique and one minimiser is
 * returned.  MBO_F32_F64FALLBACK re-evaluates a point in double when its float
 * sigma_min (|Delta E| / 2) is below sigma_fallback.
 * Batched plans return MBO_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------- */

/* Selection alone: selected[b][p] = 1 for the n_plus[b] points of field b with
 * the largest dE[b][p] (ties in ascending p), 0 elsewhere.
 * dE: device, [batch][prod(N)] in the plan's element type, finite values (NaN
 * orders by its sign bit); n_plus: host [batch], each in [0, prod(N)]
 * (MBO_ERR_INVALID_ARG otherwise); selected: device uint8 [batch][prod(N)].
 * Asynchronous. */
mbo_status mbo_volume_select(mbo_plan_t plan, const void* dE, const int64_t* n_plus, uint8_t* selected);

/* The volume-constrained step 2 on a given field (no diffusion):
 * A_out = T+(A_in) on the n_plus[b] selected points of field b, T-(A_in)
 * elsewhere.  dE (nullable, device, [batch][prod(N)], plan element type)
 * receives Delta E.  A_out may alias A_in.  n_plus: host [batch], each in
 * [0, prod(N)].  Synchronises; MBO_ERR_NONFINITE if any input is NaN/Inf. */
mbo_status mbo_project_volume(mbo_plan_t plan, const void* A_in, void* A_out, const int64_t* n_plus,
                              void* dE);

/* Volume-preserving MBO: A_s = V(e^{tau Delta} A_{s-1}), s = 1..max_iter, in
 * place on A, V the step above.  n_plus: host [batch] points to keep in SO(n),
 * or NULL for the number of points of A_0 with det >= 0.  Host logs, nullable:
 *   n_plus_used [batch]               the n_plus of each field;
 *   energy      [batch][max_iter+1]   E(A_s), s = 0..max_iter (Proposition 7.3:
 *                                     non-increasing once A_0 has n_plus points
 *                                     with det > 0);
 *   flips       [batch][max_iter]     points whose det sign changed;
 *   fallbacks   [batch][max_iter]     points evaluated in double.
 * Runs as one captured HIP graph (re-used while A, max_iter, the energy request
 * and whether n_plus is given stay the same); synchronises at the end. */
mbo_status mbo_iterate_volume(mbo_plan_t plan, void* A, int max_iter, const int64_t* n_plus,
                              int64_t* n_plus_used, double* energy, int64_t* flips, int64_t* fallbacks);

/* ---------------------------------------------------------------------------
 * Batched plans of mixed fields.  Many independent fields, each with its own
 * grid, matrix size n and tau, iterated together: fields of equal (d, N, n)
 * share one set of kernels and launches (a class), each field keeping its own
 * heat symbol; mbo_iterate captures every class's iterations into one HIP
 * graph.  The caller's field buffer is the concatenation of the fields in
 * descriptor order, field f entry-planar [n_f][n_f][prod N_f] and starting at
 * element sum_{g<f} n_g^2 prod(N_g).  mbo_iterate, mbo_energy, mbo_diffuse and
 * mbo_project (det_sign must be NULL) accept a batched plan; their per-field
 * outputs and logs are in descriptor order ([count][...]).  mbo_plan_set_tau,
 * mbo_plan_set_timing (enable), mbo_project_vjp and mbo_diffuse_dtau return
 * MBO_ERR_UNSUPPORTED for it.
 * ------------------------------------------------------------------------- */
typedef struct mbo_field_desc {
    int d;          /* 2 or 3 */
    int64_t N[3];   /* grid, axis 0 slowest; N[d..2] ignored */
    int n;          /* matrix size, 1..4 */
    double tau;     /* diffusion time of one step of this field */
} mbo_field_desc;

/* Create a batched plan for `count` fields (the shape rules of mbo_plan apply to
 * each descriptor).  autotune != 0 times candidate launch shapes of every class
 * on the device (tiles of lines per strided-pass workgroup, the XCD-aware tile
 * order, rows and threads per row-pass workgroup) on a pseudo-random field and keeps the
 * fastest; 0 keeps the fixed rules.  The choice changes neither the transforms
 * nor the projection of any point, only the summation order of the energy. */
mbo_status mbo_plan_batched(mbo_plan_t* out, int count, const mbo_field_desc* descs, mbo_precision prec,
                            double sigma_fallback, int autotune, void* hip_stream);

/* Run the autotuner described above on an existing plan (plain or batched):
 * candidate launch shapes are timed on a pseudo-random field in the plan's own
 * workspace and the fastest kept.  Synchronises the plan's stream; a captured
 * iteration graph is rebuilt on the next mbo_iterate. */
mbo_status mbo_plan_autotune(mbo_plan_t plan);

/* Launch shape used for `field` (0 <= field < count, or < batch for a plain
 * plan): rows per row-pass workgroup and its thread count, lines per heat-pass
 * workgroup, and whether heat-pass tiles are dealt to the XCDs in contiguous
 * runs (all nullable). */
mbo_status mbo_plan_tuning(mbo_plan_t plan, int field, int* rows_per_group, int* row_threads,
                           int* heat_lines_per_group, int* xcd_order);

/* ---------------------------------------------------------------------------
 * Adjoint building blocks.  The paper stops at the forward iteration; these
 * calls differentiate it.  With L a scalar function of A_K = P(H A_{K-1}) ...,
 * H = e^{tau Delta}, the chain rule runs backwards over s = K..1:
 *     Gtil_s = mbo_project_vjp(H A_{s-1}, Gbar_s)
 *     dL/dtau += <Gtil_s, d/dtau H A_{s-1}>       (mbo_diffuse_dtau with G, dot)
 *     Gbar_{s-1} = H Gtil_s                        (mbo_diffuse: H is self-adjoint)
 * and dL/dA_0 = Gbar_0.
 * ------------------------------------------------------------------------- */

/* Vector-Jacobian product of the projection step (Lemma 1.1): for every point,
 * with A_tilde = U Sigma V^t (so that the projection is Q = U V^t) and the
 * cotangent G_Q of Q,
 *     G_A = U K V^t,   K_ij = (M_ij - M_ji) / (sigma_i + sigma_j),   M = U^t G_Q V,
 * K_ii = 0; a pair with sigma_i + sigma_j = 0 (rank <= n-2, where the projection
 * is not a function of A_tilde) contributes 0.  n = 1 gives G_A = 0 (sign
 * thresholding is locally constant).  Float plans with the double fallback
 * evaluate points whose smallest singular value is below sigma_fallback in
 * double.  All three fields are device buffers in the plan's layout; G_A may
 * alias G_Q but not A_tilde.  Returns MBO_ERR_NONFINITE (after synchronising) if
 * A_tilde holds NaN/Inf. */
mbo_status mbo_project_vjp(mbo_plan_t plan, const void* A_tilde, const void* G_Q, void* G_A);

/* Derivative of the diffusion step (Section 5.1) with respect to tau:
 *     out = d/dtau e^{tau Delta} A = Delta e^{tau Delta} A,
 * Fourier symbol -4 pi^2 |k|^2 exp(-4 pi^2 tau |k|^2), entry by entry.
 * out (device, nullable) receives the field; if G (device) and dot (host,
 * [batch]) are both given, dot[b] = sum over grid points and entries of
 * G_b * (d/dtau e^{tau Delta} A_b), accumulated in double, and the call
 * synchronises the stream.  At least one of out and (G, dot) must be given.
 * out may alias A. */
mbo_status mbo_diffuse_dtau(mbo_plan_t plan, const void* A, void* out, const void* G, double* dot);

/* One step of Algorithm 1 without logs: A_next = P(e^{tau Delta} A_prev), with
 * the plan's precision and fallback, bit for bit the iterate mbo_iterate
 * produces from A_prev.  Asynchronous (no synchronisation, no NaN check: a
 * non-finite input propagates).  Device buffers; A_next must not alias A_prev.
 * Used to recompute iterates between checkpoints of the adjoint. */
mbo_status mbo_step(mbo_plan_t plan, const void* A_prev, void* A_next);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one step of
 * Algorithm 1, A_next = P(e^{tau Delta} A_prev), of ONE field on the 2-D grid
 * N0 x N1 with n x n entries, with no plan.  Results are those of mbo_step on a
 * plan (1, {N0, N1}, n, tau, prec, sigma_fallback) with the default path and no
 * autotuning: the same band-limited kernels, launch shapes and tables.
 *   Arguments  N0, N1: powers of two in [8, 2048], N0 >= 64 (the band-limited
 *              kernels' range; MBO_ERR_UNSUPPORTED otherwise); n in [1, 4];
 *              prec, tau, sigma_fallback as for mbo_plan; A_prev (read) and
 *              A_next (written): device fields [n][n][N0][N1] of the precision's
 *              element type, caller-owned, A_next not aliasing A_prev;
 *              hip_stream: the stream all work is enqueued on (NULL = default).
 *   Memory     calls no allocator.  The working memory (the kept row spectra of
 *              the ceil(n^2/2) packed planes, twiddles, heat-symbol factors)
 *              lives in one fixed device array of MBO_STEP_STATIC_MAX_BYTES per
 *              GPU, held from the library's first use on that GPU until the
 *              process ends; a field that needs more is refused with
 *              MBO_ERR_SCRATCH (mbo_last_error(NULL) gives the sizes).  In
 *              float with n = 3 and tau = 2e-4, 512 x 512 needs about 2.5 MiB
 *              and 2048 x 2048 about 10 MiB; with every row mode kept the
 *              spectra take 8 ceil(n^2/2) N0 N1 bytes (16 in double).
 *   Sharing    every call on a GPU uses that GPU's one array: calls that overlap
 *              on one GPU (on two streams, or from two host threads without
 *              ordering) race.  Nothing is carried between calls: each call
 *              rebuilds its tables, and the forward pass writes every stored
 *              slot, so nothing needs clearing.
 *   Set-up     the first call on a device resolves the array's address
 *              (hipGetSymbolAddress) with that device current; make that first
 *              call outside graph capture.
 *   Errors     asynchronous like mbo_step: no synchronisation, no NaN check.
 *              Argument errors are returned before anything is enqueued;
 *              mbo_last_error(NULL) describes them. */
#define MBO_STEP_STATIC_MAX_BYTES 67108864 /* 64 MiB */
mbo_status mbo_step_static(int64_t N0, int64_t N1, int n, mbo_precision prec, double tau, double sigma_fallback,
                           const void* A_prev, void* A_next, void* hip_stream);

/* Backward step of the adjoint (the chain rule through one step of
 * Algorithm 1), asynchronous: with A~ = e^{tau Delta} A_prev and on entry G =
 * Gbar_s, the cotangent of A_s = P(A~),
 *     G~      = mbo_project_vjp(A~, Gbar_s)
 *     dtau[b] += <G~_b, d/dtau e^{tau Delta} A_prev_b>   (device, [batch], double;
 *                                                        skipped when NULL)
 *     G      <- e^{tau Delta} G~  (= Gbar_{s-1}; the heat operator is self-adjoint).
 * Plan-owned workspaces of two fields are allocated on the first call.  No
 * NaN check (a non-finite input propagates).  G must not alias A_prev. */
mbo_status mbo_step_vjp(mbo_plan_t plan, const void* A_prev, void* G, double* dtau);

/* Human-readable name of a status code (static storage). */
const char* mbo_status_string(mbo_status s);

/* Description of the last error on this plan (or, when plan is NULL, of the
 * last failed plan-less call on this thread: mbo_plan, mbo_plan_batched or
 * mbo_step_static).  Valid until the next call on the same plan. */
const char* mbo_last_error(mbo_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* MBO_H */
