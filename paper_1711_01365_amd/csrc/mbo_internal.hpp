// Internal interface between the host runtime (mbo_api.cpp) and the HIP
// kernels (mbo_kernels.hpp and the mbo_*.hip units).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbo {

// Runtime flags of the row pass.
enum RowFlags : int {
    RF_LOAD_REAL = 1 << 0,   // read the real field A instead of the spectra Z
    RF_INVERSE = 1 << 1,     // inverse row FFT after loading spectra
    RF_PROJECT = 1 << 2,     // per-point projection (Algorithm 1, step 2)
    RF_FORWARD = 1 << 3,     // forward row FFT, then store the spectra Z
    RF_STORE_REAL = 1 << 4,  // store the (projected) real values into A / A_out
    RF_TRACK = 1 << 5,       // read the previous iterate from A: max |change|
    RF_SIGN = 1 << 6,        // compare det signs with sgn[] (flips) and update it
    RF_SIGN_INIT = 1 << 7,   // write sgn det of the loaded real field into sgn[]
    RF_FALLBACK = 1 << 8,    // float plan: re-project small-sigma points in double
    RF_CHECK_STOP = 1 << 9,  // return when this field already stopped
    RF_DOT = 1 << 10,        // per-workgroup partials of <G, values after the inverse FFT>
    RF_VP_KEY = 1 << 11,     // volume-preserving step: Delta E of the loaded values into vde[]
    RF_VP_APPLY = 1 << 12,   // volume-preserving step: T+ / T- as the selection vsel[] says
    RF_RELAX = 1 << 13,      // relaxed flow: explicit reaction step of GD-1 / GD-3
    RF_STORE_Z = 1 << 14,    // store the lines back to Z as they are (no forward FFT)
};

// Instances of the row pass: Algorithm 1, the volume-preserving step, the
// reaction step of the relaxed gradient flows.
enum RowMode : int { RM_MBO = 0, RM_VOLUME = 1, RM_RELAX = 2 };

// Selection of the n_plus points with the largest Delta E of a field (the
// volume-preserving step), found by a radix search over order-preserving keys
// of Delta E: the key kstar of the n_plus-th largest value, and among the
// points whose key equals kstar, those up to index istar.
enum VpMode : int {
    VS_SEARCH = 0,     // digits of kstar still being found
    VS_NONE = 1,       // n_plus = 0
    VS_ALL = 2,        // n_plus = all points
    VS_TIES_ALL = 3,   // selected: key >= kstar
    VS_TIES_PART = 4,  // selected: key > kstar, or key == kstar and index <= istar
};
struct VpSel {
    unsigned long long kstar;  // while searching: the digits found so far
    long long need;            // points still to select among those matching kstar's digits
    long long ties;            // points whose key matches kstar's digits found so far
    long long istar;
    int mode;
    int pad;
};

struct RowArgs {
    int L, log2L;            // row length (last grid axis) and its log2
    int rpw;                 // rows per workgroup
    int lds_plane;           // LDS elements per line (lds_pad(L - 1) + 1)
    int64_t rows;            // rows per field plane = npts / L
    int64_t npts;            // grid points per field
    const void* tw;          // twiddles exp(-2 pi i m / L), m < L
    void* Z;                 // spectra [batch][PL][npts] complex
    const void* Ain;         // real field read by RF_LOAD_REAL [batch][n*n][npts]
    void* Aout;              // real field written by RF_STORE_REAL / read by RF_TRACK
    int8_t* sgn;             // det signs [batch][npts]
    unsigned long long* flips;       // [batch][K] per-iteration counters
    unsigned long long* fallbacks;   // [batch][K]
    unsigned long long* nonfinite;   // [batch][K]
    unsigned long long* delta_bits;  // [batch][K] max |A_s - A_{s-1}| (double bits)
    int* stop_iter;          // [batch]
    int iter;                // 1-based iteration index (log slot iter-1)
    int K;                   // log stride
    int flags;
    double sigma_fb;         // fallback threshold
    const void* Gdot;        // RF_DOT: real field G [batch][n*n][npts]
    double* dpart;           // RF_DOT: partials [batch][gridDim.x]
    const int64_t* foff;     // nullable: element offset of field b in Ain / Aout / Gdot
                             // (default b * n*n * npts)
    void* vde;               // RF_VP_KEY / RF_VP_APPLY: Delta E per point [batch][npts]
    const VpSel* vsel;       // RF_VP_APPLY: finished selection of each field [batch]
    int relax_kind;          // RF_RELAX: 1 = GD-1, 3 = GD-3
    double relax_c;          // RF_RELAX: dt / eps^2
};

// Element offset of field b of a real-field buffer.
__host__ __device__ inline int64_t field_base(const int64_t* foff, int b, int64_t field_elems)
{
    return foff ? foff[b] : (int64_t)b * field_elems;
}

// Double-precision re-projection queue of the float row pass for n >= 3: one
// 16-bit index per point of the workgroup's rows (the host keeps it within max(1024, L) points)
// and the float right singular vectors of the first ROW_FB_STASH queued points.
constexpr int ROW_FB_STASH = 32;
constexpr int row_fb_queue_len(int log2L) { return (1 << log2L) > 1024 ? (1 << log2L) : 1024; }
// Static LDS the queue adds to a row-pass workgroup, in bytes.
constexpr size_t row_fb_lds(int esz, int n, int log2L)
{
    return (esz == 4 && n >= 3) ? (size_t)row_fb_queue_len(log2L) * 2 + (size_t)ROW_FB_STASH * n * n * 4 + 16
                                : 0;
}

// Modes of the strided-axis pass.
// CM_RESOLVENT multiplies by rnorm / (1 + 4 pi^2 rdt |k|^2) (the implicit
// diffusion step of the relaxed flows); CM_DIRICHLET only sums
// 4 pi^2 |k|^2 |Z|^2 into the energy partials.
enum ColMode : int {
    CM_FORWARD = 0, CM_INVERSE = 1, CM_HEAT = 2, CM_ENERGY = 3, CM_DTAU = 4, CM_RESOLVENT = 5,
    CM_DIRICHLET = 6
};

struct ColArgs {
    int L, log2L;            // transform length along the axis
    int TX;                  // inner indices per workgroup (a power of two)
    int log2TX;
    int log2S;               // log2 of S (S is a power of two)
    int lds_col;             // LDS words per line (>= lds_pad(L - 1) + 1)
    int64_t S;               // element stride along the axis (= inner extent)
    int64_t tiles;           // S / TX
    int64_t field_elems;     // complex elements per field (PL * npts)
    const void* tw;
    void* Z;
    const void* lam_row;     // heat symbol factor of this axis [L] (incl. 1/L)
    const void* lam_inner;   // product of the factors of the faster axes [S]
    int64_t lam_row_stride;   // per-field tables: offset between fields (0: shared)
    int64_t lam_inner_stride;
    int xcd_remap;           // deal tiles to XCDs in contiguous runs
    const void* mu_row;      // CM_DTAU: -4 pi^2 k^2 of this axis [L]
    const void* mu_inner;    // CM_DTAU: -4 pi^2 |k|^2 summed over the faster axes [S]
    double* epart;           // energy partials [batch][K+1][nwg]
    int nwg;                 // energy partials per field and iterate
    int slot;                // energy slot (iteration - 1); -1: use stop_iter
    int iter;                // 1-based iteration (CM_HEAT inside mbo_iterate), 0 otherwise
    int K;
    int* stop_iter;          // nullable
    const unsigned long long* delta_bits;  // nullable
    double tol;
    double rdt;              // CM_RESOLVENT: the step dt
    double rnorm;            // CM_RESOLVENT: 1 / prod(N) (the inverse transforms are unscaled)
};

struct ProjArgs {
    int64_t npts;
    const void* A;
    void* Q;
    int8_t* dsign;           // nullable
    unsigned long long* nonfinite;
    unsigned long long* fallbacks;
    int fallback;
    double sigma_fb;
    const int64_t* foff;     // nullable: element offset of field b in A and Q
};

// Vector-Jacobian product of the projection, one point per thread.
struct VjpArgs {
    int64_t npts;
    const void* A;           // point of the projection (the diffused field)
    const void* G;           // cotangent of the projected field
    void* GA;                // cotangent of A
    unsigned long long* nonfinite;
    int fallback;
    double sigma_fb;
};

struct ReduceArgs {
    const double* epart;     // [batch][K+1][nwg]
    int nwg;
    int K;
    int batch;
    int n;
    int64_t npts;
    double tau;
    const double* taus;      // nullable: per-field tau [batch]
    const int* stop_iter;    // nullable: all slots 0..K
    double* energy;          // [batch][K+1]
};

// prec: 0 = double, 1 = float.  log2L: log2 of the transform length.  With
// prepare = true a launcher only raises the kernel's dynamic-LDS limit.
// ev0 / ev1 (optional): events recorded by the dispatch itself at the kernel's
// start and end (AMD's extended launch), for kernel timing.
hipError_t launch_row(int prec, int n, int log2L, const RowArgs& a, dim3 grid, dim3 block,
                      size_t lds, hipStream_t st, bool prepare = false, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
hipError_t launch_col(int prec, int mode, int log2L, const ColArgs& a, dim3 grid, dim3 block,
                      size_t lds, hipStream_t st, bool prepare = false, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
hipError_t launch_project(int prec, int n, const ProjArgs& a, int batch, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v,
                           hipStream_t st);
hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t st);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);
hipError_t launch_vjp(int prec, int n, const VjpArgs& a, int batch, hipStream_t st);
// count values uniform in [-1, 1) from a counter-based hash of (seed, index)
hipError_t launch_fill_uniform(int prec, void* p, int64_t count, uint64_t seed, hipStream_t st);
// out[b] = (accumulate ? out[b] : 0) + sum of part[b * m .. b * m + m - 1] in a fixed order
// Index of the first-column field of a 2-D n = 2 field along every loop of
// one axis: out[b][l], l < (axis == 0 ? N1 : N0)
hipError_t launch_so2_index(int prec, const void* A, int64_t N0, int64_t N1, int batch, int axis, double* out,
                            hipStream_t st);
hipError_t launch_sum_rows(const double* part, int64_t m, int batch, double* out, hipStream_t st,
                           bool accumulate = false);

// Radix selection of the volume-preserving step over the Delta E values dE
// (plan precision) of each field; keys are taken SEL_BITS bits at a time from
// the top, the histograms of a pass built per chunk of SEL_CHUNK points.
constexpr int SEL_CHUNK = 4096;
constexpr int SEL_PER = SEL_CHUNK / 256;  // points per thread of a 256-thread workgroup
constexpr int SEL_BITS = 11;
struct SelArgs {
    const void* dE;          // [batch][npts]
    int64_t npts;
    const int64_t* nplus;    // [batch] points to select per field
    VpSel* st;               // [batch]
    unsigned* hist;          // [batch][1 << SEL_BITS], zero between passes
    unsigned* tcnt;          // [batch][chunks] points per chunk whose key is kstar
    int64_t chunks;          // ceil(npts / SEL_CHUNK)
    unsigned* done;          // [batch] workgroups of the tie count finished, zero between uses
    uint8_t* mask;           // launch_sel_mark: 1 = selected [batch][npts]
};
hipError_t launch_select(int prec, const SelArgs& a, int batch, hipStream_t st);
hipError_t launch_sel_mark(int prec, const SelArgs& a, int batch, hipStream_t st);
// out[b] = number of points p with sgn[b][p] > 0 (out is overwritten)
hipError_t launch_count_pos(const int8_t* sgn, int64_t npts, int batch, long long* out,
                            hipStream_t st);
// Row pass of the volume-preserving step (flags RF_VP_KEY / RF_VP_APPLY)
hipError_t launch_row_vp(int prec, int n, int log2L, const RowArgs& a, dim3 grid, dim3 block,
                         size_t lds, hipStream_t st, bool prepare = false);

// Surface diffusion by the closest point method: the spreading / interpolation
// of the samples onto / from a periodic Cartesian grid (the complex planes Z of
// a 3-D plan, PL planes, Ng^3 points, axis 0 slowest) with the "exponential of
// semicircle" kernel psi(z) = exp(beta (sqrt(1 - (z / W)^2) - 1)), |z| < W = w / 2
// grid units.  Work is split in bins of SURF_BIN^3 grid points; the workgroup of
// a (bin, plane) accumulates into, or reads from, an LDS tile of the grid
// around its bin.
//   Cell spreading: the samples of a band cell are the tensor product of p
//   nodes per axis with separable weights; the cell is listed in the bin of its
//   first sample and spread as a whole (U grid points per axis cover the
//   stencils of all its samples; tile edge TE = SURF_BIN + U).
//   Sample spreading / interpolation: one sample at a time (tile edge
//   SURF_BIN + w).
constexpr int SURF_BIN = 8;
struct SurfArgs {
    int64_t m;               // samples
    int n, PL;               // matrix size, packed complex planes
    int Ng;                  // grid points per axis
    int w;                   // kernel width in grid points
    double beta;             // kernel shape
    double y0, h;            // grid: y_g = y0 + g h
    const void* pos;         // samples: [3][m] positions sorted by bin; cells: [3][cells] corners sorted by bin
    const void* wts;         // sample spreading: [m] weights sorted by bin (nullable: 1)
    const int64_t* perm;     // sorted index -> sample (cell) index of the canonical order
    const int64_t* start;    // [bins + 1] first sorted index of each listed bin
    const int* bin;          // [bins][3] bin coordinates
    int nbins;
    int p, U, TE;            // cells: nodes per axis, union stencil width, tile edge
    int chunk;               // cells: cells staged in LDS at a time
    const void* nodes;       // cells: [p] node offsets dx n_a (ascending)
    const void* nwts;        // cells: [p] per-axis weight factors dx w_a
    const void* A;           // spread: entry-planar [n*n][m] field
    void* out;               // interpolate: entry-planar [n*n][m] field
    void* Z;                 // grid: [PL][Ng^3] complex
    int pl0, pl1;            // planes of this launch (one workgroup row per plane)
    void* tiles;             // spreading: [bins][PL][TE^3] complex, each workgroup's tile
    const int* binmap;       // [(Ng / SURF_BIN)^3] listed index of each bin, -1 when empty
};
hipError_t launch_surface_spread(int prec, const SurfArgs& a, hipStream_t st);
// waves = 0: the line-owner variant without atomics (p <= 4, TE <= 22), else
// the cell-per-wave variant with that many waves per workgroup
hipError_t launch_surface_spread_cells(int prec, const SurfArgs& a, int waves, hipStream_t st);
hipError_t launch_surface_interp(int prec, const SurfArgs& a, hipStream_t st);
// Z = sum of the spreading tiles over every grid point (tile edge TE; the
// tiles of bin b start at grid point SURF_BIN b - w / 2 per axis, wrapping).
// Needs Ng >= TE + SURF_BIN.
hipError_t launch_surface_gather(int prec, const SurfArgs& a, int TE, hipStream_t st);
// LDS bytes of the sample kernels' tile (one complex plane) for kernel width w
inline size_t surface_tile_bytes(int w, size_t esz)
{
    const size_t te = (size_t)(SURF_BIN + w);
    return te * te * te * 2 * esz;
}
// LDS of the cell kernel: tile (re and im, z pitch TE | 1), the staged cells
// of a chunk (corner and the values of one complex plane: 3 + 2 p^3 each, and
// an int64 first-sample index) and a scratch per wave (weights 3 p U, partial
// sums 2 p^2 U and 2 p U^2)
__host__ __device__ inline size_t surface_cell_scratch(int p, int U)
{
    return (size_t)(3 * p * U + 2 * p * p * U + 2 * p * U * U);
}
// LDS of the line-owner variant: chunk ids and staged cells, and per cell of a
// round the weights, T1 and the padded T2 (k pitch SURF_BIN + 22 + 3)
constexpr int SURF_LINE_CB = 4;  // cells contracted per round of workgroup barriers
inline size_t surface_lines_lds(int p, int U, int chunk, size_t esz)
{
    return (size_t)chunk * 8 +
           ((size_t)chunk * (3 + 2 * p * p * p) +
            (size_t)SURF_LINE_CB * (3 * p * U + 2 * p * p * U + 2 * p * U * (SURF_BIN + 22 + 3))) * esz;
}
inline size_t surface_cell_lds(int p, int U, int waves, int chunk, size_t esz)
{
    const size_t te = (size_t)(SURF_BIN + U);
    return (2 * te * te * (te | 1) + (size_t)chunk * (3 + 2 * p * p * p) +
            (size_t)waves * surface_cell_scratch(p, U)) * esz + (size_t)chunk * 8;
}

// Volume-preserving MBO on a surface: the weighted selection of Algorithm 3
// (samples in descending Delta E order, ties by ascending index, taken while
// their integer volume weights sum below V) and the reassignment of Lemma 7.2.
constexpr int WSEL_CHUNK = 4096;  // samples per workgroup of the tie scan
struct WSelState {
    unsigned long long prefix;  // digits of kstar found so far
    unsigned long long kstar;   // key of the last sample taken
    long long vrem;             // weight still needed among the keys matching prefix
    long long istar;            // the last sample taken among those with key kstar
    int mode;                   // VpMode: VS_SEARCH until the tie scan ends, VS_NONE, VS_ALL, VS_TIES_PART
    int pad;
};
struct SurfVolArgs {
    int64_t m;                 // samples
    const void* D;             // diffused field, entry-planar [n*n][m] (plan precision)
    void* A;                   // reassigned field, entry-planar [n*n][m]
    void* de;                  // [m] Delta E
    const int64_t* W;          // [m] volume weights
    WSelState* sel;
    unsigned long long* hist;  // [256] weights per digit (zero between passes)
    long long* csum;           // [chunks] tie weight per chunk
    int8_t* sgn;               // [m] nullable: +1 where T+ was taken, -1 elsewhere
    uint8_t* selected;         // [m] selection mask (mark only)
    unsigned long long* nonfinite;
    int fallback;
    double sigma_fb;
};
hipError_t launch_surf_vp_key(int prec, int n, const SurfVolArgs& a, hipStream_t st);
hipError_t launch_wsel(int prec, const SurfVolArgs& a, long long V, long long total, hipStream_t st);
hipError_t launch_wsel_mark(int prec, const SurfVolArgs& a, hipStream_t st);
hipError_t launch_surf_vp_apply(int prec, int n, const SurfVolArgs& a, hipStream_t st);

// per-translation-unit launchers behind launch_row / launch_col
hipError_t launch_row_f32(int n, int log2L, const RowArgs& a, dim3 g, dim3 b, size_t lds,
                          hipStream_t st, bool prepare, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_row_f64(int n, int log2L, const RowArgs& a, dim3 g, dim3 b, size_t lds,
                          hipStream_t st, bool prepare, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_col_f32(int mode, int log2L, const ColArgs& a, dim3 g, dim3 b, size_t lds,
                          hipStream_t st, bool prepare, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_col_f64(int mode, int log2L, const ColArgs& a, dim3 g, dim3 b, size_t lds,
                          hipStream_t st, bool prepare, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_row_vp_f32(int n, int log2L, const RowArgs& a, dim3 g, dim3 b, size_t lds,
                             hipStream_t st, bool prepare);
hipError_t launch_row_relax_f32(int n, int log2L, const RowArgs& a, dim3 g, dim3 b, size_t lds,
                                hipStream_t st, bool prepare);
hipError_t launch_row_relax_f64(int n, int log2L, const RowArgs& a, dim3 g, dim3 b, size_t lds,
                                hipStream_t st, bool prepare);
// Row pass of the relaxed flows (flag RF_RELAX)
hipError_t launch_row_relax(int prec, int n, int log2L, const RowArgs& a, dim3 grid, dim3 block,
                            size_t lds, hipStream_t st, bool prepare = false);
// Per-workgroup sums of the pointwise penalty of E_{1,eps} (kind 1:
// |A - U V^t|^2 / 2) or E_{2,eps} (kind 3: |A^t A - I|^2 / 4), without the
// 1 / eps^2: part[b][blocks], blocks = ceil(npts / 256)
hipError_t launch_penalty(int prec, int n, const void* A, int64_t npts, int batch, int kind, double* part,
                          hipStream_t st);
hipError_t launch_row_vp_f64(int n, int log2L, const RowArgs& a, dim3 g, dim3 b, size_t lds,
                             hipStream_t st, bool prepare);


// Band-limited passes of the 2-D iteration (mbo_fast.hpp): the row spectra
// keep only the modes kx <= band and kx >= L - band, W slots per row.
struct FastRowArgs {
    int L;                   // row length (last grid axis)
    int band;                // kept half-width c along the row axis
    int W;                   // stored modes per row
    int64_t rows;            // rows per field plane
    int64_t npts;            // points per field
    const void* tw;          // twiddles exp(-2 pi i m / L)
    void* Z;                 // kept row spectra [batch][PL][rows][W] complex, or
                             // [batch][PL][W][rows] when plane_major
    int plane_major;         // 3-D: spectra stored plane by plane for the plane pass
    const void* Ain;         // RF_LOAD_REAL: real field [batch][n*n][npts]
    void* Aout;              // RF_STORE_REAL / RF_TRACK: real field
    int8_t* sgn;             // det signs [batch][npts]
    unsigned long long* delta_bits;  // [batch][K] max |A_s - A_{s-1}| (double bits)
    int* stop_iter;          // [batch]
    int iter, K, flags;
    double sigma_fb;
    const int64_t* foff;     // nullable field offsets of the real fields
    unsigned long long* cnt_part;  // nullable: packed flips | fallbacks << 21 | non-finite << 42
                                   // per workgroup [batch][K][gridDim.x]
};

struct FastColArgs {
    int L;                   // column length (grid axis 0)
    int W;                   // stored columns per plane (row stride of the layout)
    int64_t tiles;           // W / TX
    int64_t field_elems;     // PL * L * W complex elements per field
    const void* tw;          // twiddles exp(-2 pi i m / L)
    void* Z;
    const void* lam_row;     // [L] exp(-4 pi^2 tau ky^2) / L
    const void* lam_col;     // [W] exp(-4 pi^2 tau kx^2) / N1 of the stored column (0 in unused slots)
    int64_t lam_row_stride;  // per-field tables (0: shared)
    int64_t lam_col_stride;
    int xcd_remap;
    double* epart;           // energy partials [batch][K+1][nwg]
    int nwg;
    int slot;                // energy slot; -1: stop_iter[b]
    int iter, K;
    int* stop_iter;          // nullable
    const unsigned long long* delta_bits;  // nullable
    double tol;
    int apply;               // 1: multiply and transform back (heat step); 0: energy only
    // the 3-D plane pass (L = N0 is the z axis): the y axis, its twiddles and
    // heat factor [Ny] exp(-4 pi^2 tau ky^2) / Ny
    int Ny;
    const void* tw_y;
    const void* lam_y;
    int64_t lam_y_stride;
};

hipError_t launch_row_fast(int prec, int n, int log2L, const FastRowArgs& a, dim3 grid, hipStream_t st,
                           bool prepare = false, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_heat_fast(int prec, int log2L, int TX, const FastColArgs& a, dim3 grid, hipStream_t st,
                            bool prepare = false, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// the 3-D plane pass (float): one workgroup per (packed plane, stored x mode)
hipError_t launch_plane_fast(int log2Y, int log2Z, const FastColArgs& a, dim3 grid, hipStream_t st,
                             bool prepare = false, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
int plane_fast_threads(int log2Y, int log2Z);
size_t plane_fast_lds_bytes(int log2Y, int log2Z);
// flips / fallbacks / non-finite of every iteration and field from the row
// pass's per-workgroup packed counts [batch][K][nwg]
hipError_t launch_sum_counts(const unsigned long long* part, int nwg, int K, int batch, unsigned long long* flips,
                             unsigned long long* fallbacks, unsigned long long* nonfinite, hipStream_t st);
// Layout of the band-limited passes of a 2-D grid N0 x N1 with n x n entries in
// precision pk (1 float, 0 double) for the diffusion times taus[0..ntau): kept
// half-width, stored modes per row (every mode when banded is false or nothing
// would be dropped), heat tile width (tune_tx, or the default rule when 0).
// false when the band-limited kernels do not serve the shape.
bool fast_layout(int64_t N0, int64_t N1, int n, int pk, const double* taus, int64_t ntau, bool banded,
                 size_t lds_max, int tune_tx, int* band_c, int* band_W, int* heat_tx);
// message of a failed plan-less call, returned by mbo_last_error(NULL) (fixed
// buffer: allocates nothing)
void report_static_error(const char* fmt, ...);
// dynamic LDS bytes and rows of a row_fast workgroup
size_t row_fast_lds_bytes(int prec, int n, int log2L);
int row_fast_rows_per_group(int log2L);

}  // namespace mbo
