// Host runtime and C ABI of libmbo (declared in include/mbo.h).
//
// The plan owns: the packed spectra workspace Z (ceil(n^2/2) complex planes per
// field), per-point det signs, twiddle tables per axis length, the heat-symbol
// tables, the device logs of mbo_iterate, and one cached HIP graph of the whole
// iteration.  All device work goes to the plan's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "mbo.h"
#include "mbo_internal.hpp"

using namespace mbo;

namespace {

thread_local std::string g_plan_error;  // failures of mbo_plan (no plan to hold them)
// failures of mbo_step_static, in a fixed buffer (that call allocates nothing)
thread_local char g_static_error[256];
thread_local bool g_static_failed = false;  // the last plan-less failure was mbo_step_static's

int ilog2(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }

// The integer a C caller passed for an enum parameter.  Read as bytes: a value
// outside the enumerators may arrive, and reading it as the enum type would be
// undefined in C++ before it can be rejected.
template <typename E>
int raw_enum(const E& e)
{
    int v = 0;
    static_assert(sizeof(E) == sizeof(int), "enums of the ABI are int-sized");
    std::memcpy(&v, &e, sizeof v);
    return v;
}

bool valid_precision(const mbo_precision& prec)
{
    const int v = raw_enum(prec);
    return v == MBO_F64 || v == MBO_F32 || v == MBO_F32_F64FALLBACK;
}

int lds_len(int L) { return (L - 1) + ((L - 1) >> 3) + 1; }  // lds_pad(L-1) + 1

struct ColCfg {
    int L = 0, TX = 1, pitch = 0;
    int64_t S = 0, outer = 0;
    dim3 grid, block;
    size_t lds = 0;
    int axis = 0;
};

}  // namespace

namespace mbo {

void report_static_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_static_error, sizeof g_static_error, fmt, ap);
    va_end(ap);
    g_static_failed = true;
}

}  // namespace mbo

struct mbo_plan_s {
    int device = 0;
    int d = 2;
    int64_t N[3] = {1, 1, 1};
    int n = 1;
    int64_t batch = 1;
    double tau = 0.0;
    mbo_precision prec = MBO_F64;
    double sigma_fb = 1e-3;
    int pk = 0;      // 0 = double kernels, 1 = float kernels
    size_t esz = 8;  // bytes per real
    int PL = 1;
    int64_t npts = 1;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    // a batched plan: side streams (default priority) its field classes run on
    // concurrently, and the events of the fork and of each class's end
    std::vector<hipStream_t> side;
    std::vector<int> side_of;       // stream of each member class
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;  // per side stream
    size_t lds_max = 65536;

    void* Z = nullptr;
    int8_t* sgn = nullptr;
    void* tw[3] = {nullptr, nullptr, nullptr};
    void* lam_row = nullptr;    // heat axis (axis 0) factor [N0]
    void* lam_inner = nullptr;  // product over the faster axes [npts / N0]
    void* mu_row = nullptr;     // -4 pi^2 k^2 of axis 0 [N0]
    void* mu_inner = nullptr;   // -4 pi^2 |k|^2 over the faster axes [npts / N0]
    double* dpart = nullptr;    // dot-product partials [batch][row workgroups]
    double* dsum = nullptr;     // [batch]
    void* ws_a = nullptr;       // adjoint step workspaces, one field each (lazy)
    void* ws_g = nullptr;
    unsigned long long* counters = nullptr;  // project: [0] nonfinite, [1] fallbacks

    // per-field diffusion times (fields of a batched plan): tables per field
    bool per_field_tau = false;
    std::vector<double> taus;     // [batch]
    double* taus_dev = nullptr;   // [batch]
    // field offsets (elements) in the caller's buffer, when not b * n*n * npts
    int64_t* foff_dev = nullptr;  // [batch]

    // launch configuration (tune_*: overrides chosen by the autotuner, 0 = rule)
    dim3 row_grid, row_block;
    size_t row_lds = 0;
    int row_rpw = 1;
    ColCfg heat, ypass;
    int tune_rpw = 0, tune_tx_heat = 0, tune_tx_y = 0;
    int tune_row_groups = 0;  // row workgroup sized by line groups instead of points
    int xcd_remap = 1;
    bool tuned = false;

    // a batched plan of mixed fields is a group of member plans, one per
    // (d, N, n) class; field f is field f_index[f] of member f_member[f] and
    // starts at element f_off[f] of the caller's buffer
    bool group = false;
    std::vector<mbo_plan_s*> members;
    std::vector<int> f_member, f_index;
    std::vector<int64_t> f_off;

    // logs of mbo_iterate, capacity log_K
    int log_K = -1;
    double* epart = nullptr;
    double* energy = nullptr;
    unsigned long long* flips = nullptr;
    unsigned long long* fallbacks = nullptr;
    unsigned long long* nonfinite = nullptr;
    unsigned long long* delta_bits = nullptr;
    int* stop_iter = nullptr;

    // optional kernel timing: events around every row / heat pass of mbo_iterate
    bool timing = false;
    std::vector<hipEvent_t> ev;   // [4 * K]: row start, row end, heat start, heat end
    int ev_K = 0;
    double t_row_us = 0.0, t_col_us = 0.0;
    int t_launches = 0;

    // band-limited passes of mbo_iterate (2-D, rows of at most 512 points,
    // columns of at least 64): path chosen by the caller (mbo_plan_set_path),
    // whether this plan runs them, the kept half-width along the rows and the
    // stored modes per row, the heat tile width, the symbol of the stored
    // columns [nt][W]
    int path = MBO_PATH_BANDED;
    bool fast = false;
    int band_c = 0, band_W = 0;
    int fast_tx = 0, tune_fast_tx = 0;
    void* lam_col = nullptr;
    void* lam_y = nullptr;      // 3-D band-limited plane pass: axis-1 factor [N1] (per field with own tau)
    unsigned long long* cnt_part = nullptr;
    // counts of the last mbo_project: double re-projections, non-finite inputs
    int64_t last_fb = 0, last_bad = 0;  // row-pass counts per workgroup [batch][log_K][workgroups]

    // cached iteration graph
    hipGraphExec_t gexec = nullptr;
    void* g_A = nullptr;
    int g_K = -1;
    int g_key = -1;
    double g_tol = 0.0;

    // volume-preserving step (allocated on first use): Delta E per point, the
    // selection state, its histograms and tie counts, points to select
    void* vde = nullptr;          // [batch][npts], plan precision
    VpSel* vsel = nullptr;        // [batch]
    unsigned* vhist = nullptr;    // [batch][1 << SEL_BITS]
    unsigned* vtcnt = nullptr;    // [batch][chunks]
    long long* vnplus = nullptr;  // [batch]
    unsigned* vdone = nullptr;    // [batch] finished-workgroup counters of the tie count
    // relaxed flows: cached graph of mbo_relaxed_flow, penalty partials
    hipGraphExec_t rexec = nullptr;
    void* rg_A = nullptr;
    int rg_K = -1, rg_kind = 0;
    double rg_c = 0.0, rg_dt = 0.0;
    double* pen = nullptr;       // [batch][ceil(npts / 256)]
    double* pen_sum = nullptr;   // [batch]
    hipGraphExec_t vexec = nullptr;  // cached graph of mbo_iterate_volume
    void* vg_A = nullptr;
    int vg_K = -1;
    int vg_key = -1;

    std::string err;
};

namespace {

mbo_status fail(mbo_plan_t p, mbo_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (p) p->err = buf;
    else g_plan_error = buf;
    return s;
}

#define HIP_TRY(plan, expr)                                                                   \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(plan, e_ == hipErrorOutOfMemory ? MBO_ERR_ALLOC : MBO_ERR_HIP,         \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                        \
    } while (0)

template <typename T>
void free_dev(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void drop_graph(mbo_plan_t p)
{
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->g_A = nullptr;
    p->g_K = -1;
    p->g_key = -1;
    if (p->vexec) (void)hipGraphExecDestroy(p->vexec);
    p->vexec = nullptr;
    if (p->rexec) (void)hipGraphExecDestroy(p->rexec);
    p->rexec = nullptr;
    p->rg_A = nullptr;
    p->rg_K = -1;
    p->vg_A = nullptr;
    p->vg_K = -1;
    p->vg_key = -1;
}

void destroy(mbo_plan_t p)
{
    if (!p) return;
    for (mbo_plan_t m : p->members) destroy(m);
    p->members.clear();
    (void)hipSetDevice(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    drop_graph(p);
    free_dev(p->Z);
    free_dev(p->sgn);
    void* seen[3] = {nullptr, nullptr, nullptr};
    for (int a = 0; a < 3; ++a) {
        bool dup = false;
        for (int b = 0; b < a; ++b) dup = dup || (seen[b] == p->tw[a]);
        seen[a] = p->tw[a];
        if (!dup && p->tw[a]) (void)hipFree(p->tw[a]);
        p->tw[a] = nullptr;
    }
    free_dev(p->lam_row);
    free_dev(p->lam_inner);
    free_dev(p->lam_col);
    free_dev(p->lam_y);
    free_dev(p->mu_row);
    free_dev(p->mu_inner);
    free_dev(p->dpart);
    free_dev(p->dsum);
    free_dev(p->ws_a);
    free_dev(p->ws_g);
    free_dev(p->taus_dev);
    free_dev(p->foff_dev);
    free_dev(p->counters);
    free_dev(p->epart);
    free_dev(p->energy);
    free_dev(p->flips);
    free_dev(p->fallbacks);
    free_dev(p->nonfinite);
    free_dev(p->delta_bits);
    free_dev(p->stop_iter);
    free_dev(p->vde);
    free_dev(p->vsel);
    free_dev(p->vhist);
    free_dev(p->vtcnt);
    free_dev(p->vnplus);
    free_dev(p->vdone);
    free_dev(p->pen);
    free_dev(p->pen_sum);
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    for (hipStream_t q : p->side) (void)hipStreamDestroy(q);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    for (hipEvent_t e : p->ev_join) (void)hipEventDestroy(e);
    delete p;
}

// Copy an FP64 host table to the device in the plan's precision.
mbo_status upload(mbo_plan_t p, void* dst, const std::vector<double>& h)
{
    if (p->pk == 0) {
        HIP_TRY(p, hipMemcpy(dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(h.size());
        for (size_t i = 0; i < h.size(); ++i) f[i] = (float)h[i];
        HIP_TRY(p, hipMemcpy(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    return MBO_OK;
}

// Heat-symbol factor of one axis: exp(-4 pi^2 tau k^2) / N, k the wrapped
// frequency (m < N/2 ? m : m - N).  The 1/N folds the inverse-DFT scaling in.
std::vector<double> axis_symbol(int64_t N, double tau)
{
    std::vector<double> v((size_t)N);
    const double pi = 3.14159265358979323846;
    for (int64_t m = 0; m < N; ++m) {
        const double k = (2 * m < N) ? (double)m : (double)(m - N);
        v[(size_t)m] = std::exp(-4.0 * pi * pi * tau * k * k) / (double)N;
    }
    return v;
}

// Heat-symbol tables of the plan: one pair (axis 0, product over the faster
// axes), or one pair per field when the fields have their own tau.
mbo_status build_symbol_tables(mbo_plan_t p)
{
    const int64_t inner_n = p->npts / p->N[0];
    const int64_t nt = p->per_field_tau ? p->batch : 1;
    std::vector<double> row, inner;
    row.reserve((size_t)(nt * p->N[0]));
    inner.reserve((size_t)(nt * inner_n));
    for (int64_t b = 0; b < nt; ++b) {
        const double tau = p->per_field_tau ? p->taus[(size_t)b] : p->tau;
        std::vector<double> r = axis_symbol(p->N[0], tau);
        row.insert(row.end(), r.begin(), r.end());
        if (p->d == 2) {
            std::vector<double> i2 = axis_symbol(p->N[1], tau);
            inner.insert(inner.end(), i2.begin(), i2.end());
        } else {
            std::vector<double> ly = axis_symbol(p->N[1], tau), lx = axis_symbol(p->N[2], tau);
            for (int64_t y = 0; y < p->N[1]; ++y)
                for (int64_t x = 0; x < p->N[2]; ++x) inner.push_back(ly[(size_t)y] * lx[(size_t)x]);
        }
    }
    mbo_status s = upload(p, p->lam_row, row);
    if (s != MBO_OK) return s;
    return upload(p, p->lam_inner, inner);
}

// -4 pi^2 k^2 per index of an axis (same wrap-around as axis_symbol).
std::vector<double> axis_laplace(int64_t N)
{
    std::vector<double> v((size_t)N);
    const double pi = 3.14159265358979323846;
    for (int64_t m = 0; m < N; ++m) {
        const double k = (2 * m < N) ? (double)m : (double)(m - N);
        v[(size_t)m] = -4.0 * pi * pi * k * k;
    }
    return v;
}

// Tables of the tau-derivative multiplier: -4 pi^2 |k|^2 = row + inner term.
mbo_status build_laplace_tables(mbo_plan_t p)
{
    std::vector<double> row = axis_laplace(p->N[0]);
    const int64_t inner_n = p->npts / p->N[0];
    std::vector<double> inner((size_t)inner_n);
    if (p->d == 2) {
        inner = axis_laplace(p->N[1]);
    } else {
        std::vector<double> ly = axis_laplace(p->N[1]), lx = axis_laplace(p->N[2]);
        for (int64_t y = 0; y < p->N[1]; ++y)
            for (int64_t x = 0; x < p->N[2]; ++x) inner[(size_t)(y * p->N[2] + x)] = ly[(size_t)y] + lx[(size_t)x];
    }
    mbo_status s = upload(p, p->mu_row, row);
    if (s != MBO_OK) return s;
    return upload(p, p->mu_inner, inner);
}

// Kept half-width of the row axis for the band-limited passes (2-D).  The
// heat symbol is exp(-4 pi^2 tau ky^2) exp(-4 pi^2 tau kx^2); dropping the
// modes with |kx| > c changes a diffused value by at most
// max|A| * S_y(tau) * sum_{|kx| > c} exp(-4 pi^2 tau kx^2), S_y the sum of the
// column axis's factor over all its modes (|A^(k)| <= N0 N1 max|A|).  c is the
// smallest half-width that keeps this below eta; c = N1/2 keeps every mode.
// The tail sum is accumulated from the top (the dropped modes are the
// smallest terms), so it only grows as c decreases.
double axis_weight(int64_t N, double tau)
{
    const double pi = 3.14159265358979323846;
    double s = 0.0;
    for (int64_t m = 0; m < N; ++m) {
        const double k = (2 * m < N) ? (double)m : (double)(m - N);
        s += std::exp(-4.0 * pi * pi * tau * k * k);
    }
    return s;
}

// sy: the other axes' factors summed over all their modes (their product in 3-D)
int band_halfwidth_w(double sy, int64_t N1, double tau, double eta)
{
    const double pi = 3.14159265358979323846;
    const int64_t h = N1 / 2;
    double tail = 0.0;  // sum over |kx| > c
    int64_t c = h;
    while (c > 0) {
        // |kx| = c occurs twice, except the Nyquist mode N1/2 (once)
        const double k = (double)c;
        const double t = tail + (c == h ? 1.0 : 2.0) * std::exp(-4.0 * pi * pi * tau * k * k);
        if (sy * t > eta) break;
        tail = t;
        --c;
    }
    return (int)c;
}

int band_halfwidth(int64_t N0, int64_t N1, double tau, double eta)
{
    return band_halfwidth_w(axis_weight(N0, tau), N1, tau, eta);
}

}  // namespace

namespace mbo {

bool fast_layout(int64_t N0, int64_t N1, int n, int pk, const double* taus, int64_t ntau, bool banded,
                 size_t lds_max, int tune_tx, int* band_c, int* band_W, int* heat_tx)
{
    if (N1 < 8 || N1 > 2048 || N0 < 64 || N0 > 2048) return false;
    // the row pass keeps a workgroup's lines (512 points, or one row) in LDS
    // beside its static arrays (the helper wave's queue and matrices, at most
    // 12 KiB)
    if (row_fast_lds_bytes(pk, n, ilog2((int)N1)) + 12288 > lds_max) return false;
    int c = (int)(N1 / 2), W = (int)N1;
    if (banded) {
        const double eta = pk == 1 ? 1e-12 : 1e-20;
        int cmax = 0;
        for (int64_t i = 0; i < ntau; ++i) {
            const int ci = band_halfwidth(N0, N1, taus[i], eta);
            cmax = ci > cmax ? ci : cmax;
        }
        const int Wb = ((2 * cmax + 1) + 15) / 16 * 16;
        if (Wb < N1) {
            c = cmax;
            W = Wb;
        }
    }
    // heat tile: TX columns of 2^k with 64..1024 threads and TX | W
    const int Tn = (int)(N0 / 8);
    int tx = tune_tx ? tune_tx : 2;
    while (tx * Tn < 64) tx *= 2;
    while (tx > 1 && (tx * Tn > 1024 || W % tx)) tx /= 2;
    if (tx * Tn < 64 || tx * Tn > 1024 || W % tx) return false;
    *band_c = c;
    *band_W = W;
    *heat_tx = tx;
    return true;
}

}  // namespace mbo

namespace {

// 3-D band-limited path (float plans): the row pass over the x rows and one
// plane pass per (packed plane, stored x mode) holding the whole y-z plane in
// LDS, so y and z planes of 64 or 128 points.  The kept x half-width bounds the
// dropped symbol mass by eta with the y and z axes' summed factors.
void config_fast3(mbo_plan_t p)
{
    const int64_t N0 = p->N[0], N1 = p->N[1], N2 = p->N[2];
    if (p->pk != 1) return;
    if ((N0 != 64 && N0 != 128) || (N1 != 64 && N1 != 128) || N2 < 8 || N2 > 2048) return;
    if (row_fast_lds_bytes(p->pk, p->n, ilog2((int)N2)) + 12288 > p->lds_max) return;
    if (plane_fast_lds_bytes(ilog2((int)N1), ilog2((int)N0)) > p->lds_max) return;
    int c = (int)(N2 / 2), W = (int)N2;
    if (p->path == MBO_PATH_BANDED) {
        const double* taus = p->per_field_tau ? p->taus.data() : &p->tau;
        const int64_t ntau = p->per_field_tau ? (int64_t)p->taus.size() : 1;
        int cmax = 0;
        for (int64_t i = 0; i < ntau; ++i) {
            const double sy = axis_weight(N0, taus[i]) * axis_weight(N1, taus[i]);
            const int ci = band_halfwidth_w(sy, N2, taus[i], 1e-12);
            cmax = ci > cmax ? ci : cmax;
        }
        // the plane-major layout needs no alignment of W: a plane pass per
        // kept mode, nothing for slots between the two halves of the band
        const int Wb = 2 * cmax + 1;
        if (Wb < N2) {
            c = cmax;
            W = Wb;
        }
    }
    p->band_c = c;
    p->band_W = W;
    p->fast_tx = 1;
    p->fast = true;
}

// Whether mbo_iterate runs the band-limited passes, and their layout: kept
// half-width c and stored modes W per row (a multiple of 16, at least 2c + 1;
// W = N1 when nothing would be saved), the heat tile width.
void config_fast(mbo_plan_t p)
{
    p->fast = false;
    p->band_c = (int)(p->N[p->d - 1] / 2);
    p->band_W = (int)p->N[p->d - 1];
    if (p->path == MBO_PATH_GENERIC) return;
    if (p->d == 3) {
        config_fast3(p);
        return;
    }
    const double* taus = p->per_field_tau ? p->taus.data() : &p->tau;
    const int64_t ntau = p->per_field_tau ? (int64_t)p->taus.size() : 1;
    int c, W, tx;
    if (!fast_layout(p->N[0], p->N[1], p->n, p->pk, taus, ntau, p->path == MBO_PATH_BANDED, p->lds_max,
                     p->tune_fast_tx, &c, &W, &tx))
        return;
    p->band_c = c;
    p->band_W = W;
    p->fast_tx = tx;
    p->fast = true;
}

// Symbol of the stored columns of the band-limited layout, per field when the
// fields have their own tau: slot w holds kx = w (w <= c) or kx = w - W
// (w >= W - c), exp(-4 pi^2 tau kx^2) / N1; 0 in the unused slots.
mbo_status build_fast_tables(mbo_plan_t p)
{
    free_dev(p->lam_col);
    free_dev(p->lam_y);
    if (!p->fast) return MBO_OK;
    const int W = p->band_W, c = p->band_c;
    const int64_t N1 = p->N[p->d - 1];
    const int64_t nt = p->per_field_tau ? p->batch : 1;
    const double pi = 3.14159265358979323846;
    std::vector<double> v;
    v.reserve((size_t)(nt * W));
    for (int64_t b = 0; b < nt; ++b) {
        const double tau = p->per_field_tau ? p->taus[(size_t)b] : p->tau;
        for (int w = 0; w < W; ++w) {
            double k;
            if (W == N1) k = (2 * w < N1) ? (double)w : (double)(w - N1);
            else if (w <= c) k = (double)w;
            else if (w >= W - c) k = (double)(w - W);
            else {
                v.push_back(0.0);
                continue;
            }
            v.push_back(std::exp(-4.0 * pi * pi * tau * k * k) / (double)N1);
        }
    }
    HIP_TRY(p, hipMalloc(&p->lam_col, v.size() * p->esz));
    const mbo_status s = upload(p, p->lam_col, v);
    if (s != MBO_OK || p->d != 3) return s;
    // 3-D: the y factor, exp(-4 pi^2 tau ky^2) / N1 of the plane pass
    std::vector<double> y;
    for (int64_t b = 0; b < nt; ++b) {
        std::vector<double> f = axis_symbol(p->N[1], p->per_field_tau ? p->taus[(size_t)b] : p->tau);
        y.insert(y.end(), f.begin(), f.end());
    }
    HIP_TRY(p, hipMalloc(&p->lam_y, y.size() * p->esz));
    return upload(p, p->lam_y, y);
}

// Twiddles exp(-2 pi i m / L), m < L, interleaved (re, im).
std::vector<double> twiddles(int64_t L)
{
    std::vector<double> v(2 * (size_t)L);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t m = 0; m < L; ++m) {
        v[2 * (size_t)m] = std::cos(two_pi * (double)m / (double)L);
        v[2 * (size_t)m + 1] = -std::sin(two_pi * (double)m / (double)L);
    }
    return v;
}

// Strided pass along `axis` (0 = slowest): transform length L = N[axis], stride
// S = product of the faster axes, `outer` independent blocks per field.
mbo_status config_col(mbo_plan_t p, ColCfg& c, int axis)
{
    c.axis = axis;
    c.L = (int)p->N[axis];
    c.S = 1;
    for (int a = axis + 1; a < p->d; ++a) c.S *= p->N[a];
    c.outer = (int64_t)p->PL * (p->npts / (c.L * c.S));
    const int T = c.L / 8;
    int TX = 1;
    if (c.L <= 512) {
        // lines inside one wave: a tile of TX lines is staged through LDS with a
        // line pitch of 8 (mod 64) words, so the coalesced staging is free of
        // bank conflicts; up to 512 threads per workgroup
        // rule: workgroups of at most 256 threads (a tile per four waves keeps
        // enough workgroups to balance the CUs); the autotuner may widen it
        const int cap = axis == 0 ? p->tune_tx_heat : p->tune_tx_y;
        const int tmax = cap ? 512 : 256;
        while (TX * 2 <= c.S && T * TX * 2 <= tmax && (cap == 0 || TX * 2 <= cap)) TX *= 2;
        // LDS is read and written 32 lanes at a time over 32 banks; the staging
        // of a tile puts lanes (line cc < TX, row r0 < 32/TX) at cc * pitch + r0,
        // all in distinct banks when pitch = 32/TX (mod 32)
        auto pitch_for = [&](int tx) {
            int pt = lds_len(c.L);
            const int want = tx > 1 ? 32 / tx : 0;
            if (want) pt += ((want - pt % 32) + 32) % 32;
            return pt;
        };
        c.pitch = pitch_for(TX);
        while (TX > 1 && (size_t)c.pitch * 2 * p->esz * TX > p->lds_max) {
            TX /= 2;
            c.pitch = pitch_for(TX);
        }
        const size_t per_line = (size_t)c.pitch * 2 * p->esz;
        if (per_line * TX > p->lds_max)
            return fail(p, MBO_ERR_UNSUPPORTED, "axis of length %d needs more LDS than available", c.L);
        c.lds = per_line * TX;
    } else {
        c.pitch = lds_len(c.L);
        const int cap = axis == 0 ? p->tune_tx_heat : p->tune_tx_y;
        while (TX < 16 && TX * 2 <= c.S && T * TX * 2 <= 512 && (cap == 0 || TX * 2 <= cap)) TX *= 2;
        const size_t per_col = (size_t)c.pitch * 2 * p->esz;
        while (TX > 1 && per_col * TX > p->lds_max) TX /= 2;
        if (per_col * TX > p->lds_max)
            return fail(p, MBO_ERR_UNSUPPORTED, "axis of length %d needs more LDS than available", c.L);
        c.lds = per_col * TX;
    }
    c.TX = TX;
    c.block = dim3((unsigned)(T * TX));
    c.grid = dim3((unsigned)(c.outer * (c.S / TX)), (unsigned)p->batch);
    return MBO_OK;
}

// Row pass: a workgroup owns rpw whole rows (at least 256 points) of every
// packed plane; NT = min(512, rpw * L) threads, one point per thread and pass in
// the projection phase, groups of L/8 threads per line in the FFT phases.
mbo_status config_row(mbo_plan_t p)
{
    const int L = (int)p->N[p->d - 1];
    const int64_t rows = p->npts / L;
    int rpw = 1;
    if (p->tune_rpw > 0)
        while (rpw * 2 <= p->tune_rpw && rpw * 2 <= rows) rpw *= 2;
    else
        while (rpw * L < 256 && rpw * 2 <= rows) rpw *= 2;
    const size_t per_row = (size_t)p->PL * lds_len(L) * 2 * p->esz;
    const size_t budget = p->lds_max - row_fb_lds((int)p->esz, p->n, ilog2(L));
    while (rpw > 1 && per_row * rpw > budget) rpw /= 2;
    if (per_row * rpw > budget)
        return fail(p, MBO_ERR_UNSUPPORTED,
                    "rows of length %d with %d packed planes need %zu bytes of LDS (max %zu)", L,
                    p->PL, per_row, budget);
    if (rpw * L > row_fb_queue_len(ilog2(L)))
        return fail(p, MBO_ERR_UNSUPPORTED, "row workgroup of %d points exceeds its queue", rpw * L);
    // threads: one per point up to 512 (rule), or one L/8-thread group per line
    // of the workgroup (the transform phases then keep every wave busy and the
    // projection takes several passes)
    int nt = rpw * L < 512 ? rpw * L : 512;
    if (p->tune_row_groups) {
        const int per_line = L / 8 < 64 ? 64 : L / 8;
        const int lines = rpw * p->PL;
        int g = lines * (L / 8);
        g = (g + 63) / 64 * 64;
        if (g < per_line) g = per_line;
        nt = g < 512 ? g : 512;
    }
    nt = (nt + 63) / 64 * 64;  // whole waves (the kernel's reductions assume them)
    p->row_rpw = rpw;
    p->row_block = dim3((unsigned)nt);
    p->row_grid = dim3((unsigned)((rows + rpw - 1) / rpw), (unsigned)p->batch);
    p->row_lds = per_row * rpw;
    return MBO_OK;
}

RowArgs row_args(mbo_plan_t p)
{
    RowArgs a;
    std::memset(&a, 0, sizeof a);
    const int L = (int)p->N[p->d - 1];
    a.L = L;
    a.log2L = ilog2(L);
    a.rpw = p->row_rpw;
    a.lds_plane = lds_len(L);
    a.rows = p->npts / L;
    a.npts = p->npts;
    a.tw = p->tw[p->d - 1];
    a.Z = p->Z;
    a.sgn = p->sgn;
    a.sigma_fb = p->sigma_fb;
    a.K = 1;
    a.foff = p->foff_dev;
    return a;
}

ColArgs col_args(mbo_plan_t p, const ColCfg& c)
{
    ColArgs a;
    std::memset(&a, 0, sizeof a);
    a.L = c.L;
    a.log2L = ilog2(c.L);
    a.TX = c.TX;
    a.log2TX = ilog2(c.TX);
    a.log2S = ilog2(c.S);
    a.lds_col = c.pitch;
    a.S = c.S;
    a.tiles = c.S / c.TX;
    a.field_elems = (int64_t)p->PL * p->npts;
    a.tw = p->tw[c.axis];
    a.Z = p->Z;
    a.lam_row = p->lam_row;
    a.lam_inner = p->lam_inner;
    a.mu_row = p->mu_row;
    a.mu_inner = p->mu_inner;
    a.lam_row_stride = p->per_field_tau ? p->N[0] : 0;
    a.lam_inner_stride = p->per_field_tau ? p->npts / p->N[0] : 0;
    a.xcd_remap = p->xcd_remap;
    // energy partials per field and iterate: one per whole wave (one per
    // workgroup when the workgroup is not a whole number of waves)
    a.nwg = (int)(c.outer * (c.S / c.TX)) * ((c.block.x % 64) ? 1 : (int)(c.block.x / 64));
    a.slot = 0;
    return a;
}

hipError_t run_row(mbo_plan_t p, const RowArgs& a, hipStream_t st, hipEvent_t ev0 = nullptr,
                   hipEvent_t ev1 = nullptr)
{
    return launch_row(p->pk, p->n, a.log2L, a, p->row_grid, p->row_block, p->row_lds, st, false, ev0, ev1);
}

hipError_t run_col(mbo_plan_t p, const ColCfg& c, int mode, const ColArgs& a, hipStream_t st,
                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    return launch_col(p->pk, mode, a.log2L, a, c.grid, c.block, c.lds, st, false, ev0, ev1);
}

// Raise the dynamic-LDS limit of every kernel instance this plan launches to
// the device maximum.  Advisory: the launch configuration never asks for more
// than the device's sharedMemPerBlock, so a refusal is not an error.
void prepare_plan_kernels(mbo_plan_t p)
{
    RowArgs r = row_args(p);
    (void)launch_row(p->pk, p->n, r.log2L, r, p->row_grid, p->row_block, p->lds_max, nullptr, true);
    for (int m = CM_FORWARD; m <= CM_ENERGY; ++m) {
        ColArgs h = col_args(p, p->heat);
        (void)launch_col(p->pk, m, h.log2L, h, p->heat.grid, p->heat.block, p->lds_max, nullptr, true);
        if (p->d == 3) {
            ColArgs y = col_args(p, p->ypass);
            (void)launch_col(p->pk, m, y.log2L, y, p->ypass.grid, p->ypass.block, p->lds_max, nullptr, true);
        }
    }
    (void)hipGetLastError();
}

// Dynamic-LDS limits of the band-limited kernels of this plan (every tile width
// the autotuner may pick).  Advisory, as above.
void prepare_fast_kernels(mbo_plan_t p)
{
    if (!p->fast) return;
    FastRowArgs r;
    std::memset(&r, 0, sizeof r);
    (void)launch_row_fast(p->pk, p->n, ilog2((int)p->N[p->d - 1]), r, dim3(1), nullptr, true);
    FastColArgs h;
    std::memset(&h, 0, sizeof h);
    if (p->d == 3) {
        (void)launch_plane_fast(ilog2((int)p->N[1]), ilog2((int)p->N[0]), h, dim3(1), nullptr, true);
    } else {
        for (int tx = 1; tx <= 16; tx *= 2)
            (void)launch_heat_fast(p->pk, ilog2((int)p->N[0]), tx, h, dim3(1), nullptr, true);
    }
    (void)hipGetLastError();
}

// Energy partials per field and iterate: one per wave of the heat pass.
int energy_partials(mbo_plan_t p)
{
    const unsigned bx = p->heat.block.x;
    return (int)(p->heat.grid.x * ((bx % 64) ? 1 : bx / 64));  // = col_args(p, p->heat).nwg
}

// Workgroups of the band-limited row pass per field (512 points, or one row
// of 1024 or 2048 points, each).
int fast_row_groups(mbo_plan_t p)
{
    const int64_t L = p->N[p->d - 1];
    const int64_t rows = p->npts / L;
    const int rpw = row_fast_rows_per_group(ilog2((int)L));
    return (int)((rows + rpw - 1) / rpw);
}

// Grid of the band-limited heat pass and its energy partials per field and
// iterate (one per wave).
dim3 fast_heat_grid(mbo_plan_t p)
{
    return dim3((unsigned)((int64_t)p->PL * (p->band_W / p->fast_tx)), (unsigned)p->batch);
}

int fast_energy_partials(mbo_plan_t p)
{
    if (!p->fast) return 0;
    const int nt = p->d == 3 ? plane_fast_threads(ilog2((int)p->N[1]), ilog2((int)p->N[0]))
                             : p->fast_tx * (int)(p->N[0] / 8);
    return (int)fast_heat_grid(p).x * (nt / 64);
}

// Free the device logs; the next ensure_logs reallocates them (their energy
// partials are sized by the heat pass's workgroup count).
void drop_logs(mbo_plan_t p)
{
    drop_graph(p);
    free_dev(p->epart);
    free_dev(p->energy);
    free_dev(p->flips);
    free_dev(p->fallbacks);
    free_dev(p->nonfinite);
    free_dev(p->delta_bits);
    free_dev(p->stop_iter);
    free_dev(p->cnt_part);
    p->log_K = -1;
}

mbo_status ensure_logs(mbo_plan_t p, int K)
{
    if (K <= p->log_K) return MBO_OK;
    drop_logs(p);
    const size_t slots = (size_t)p->batch * (size_t)(K + 1);
    // room for the partials of either heat pass (the band-limited one when
    // mbo_iterate runs it, the generic one for the other calls)
    const int nwg = std::max(energy_partials(p), fast_energy_partials(p));
    HIP_TRY(p, hipMalloc((void**)&p->epart, slots * (size_t)nwg * sizeof(double)));
    HIP_TRY(p, hipMalloc((void**)&p->energy, slots * sizeof(double)));
    const size_t cslots = (size_t)p->batch * (size_t)(K > 0 ? K : 1);
    HIP_TRY(p, hipMalloc((void**)&p->flips, cslots * sizeof(unsigned long long)));
    HIP_TRY(p, hipMalloc((void**)&p->fallbacks, cslots * sizeof(unsigned long long)));
    HIP_TRY(p, hipMalloc((void**)&p->nonfinite, cslots * sizeof(unsigned long long)));
    HIP_TRY(p, hipMalloc((void**)&p->delta_bits, cslots * sizeof(unsigned long long)));
    HIP_TRY(p, hipMalloc((void**)&p->stop_iter, (size_t)p->batch * sizeof(int)));
    if (p->fast)
        HIP_TRY(p, hipMalloc((void**)&p->cnt_part, cslots * (size_t)fast_row_groups(p) * sizeof(unsigned long long)));
    p->log_K = K;
    return MBO_OK;
}

// Forward transforms of a real field into Z: rows, then (3-D, with_mid) the
// middle axis.
hipError_t enqueue_forward(mbo_plan_t p, const void* A, int extra_flags, bool with_mid, hipStream_t st)
{
    RowArgs r = row_args(p);
    r.Ain = A;
    r.flags = RF_LOAD_REAL | RF_FORWARD | extra_flags;
    hipError_t e = run_row(p, r, st);
    if (e != hipSuccess) return e;
    if (p->d == 3 && with_mid) {
        ColArgs y = col_args(p, p->ypass);
        e = run_col(p, p->ypass, CM_FORWARD, y, st);
    }
    return e;
}

// E(A_final) into energy slot stop_iter[b] (Z holds the row spectra of the last
// iterate, A_0 for K = 0), then every energy of the run from its partials.
hipError_t enqueue_final_energy(mbo_plan_t p, int K, hipStream_t st)
{
    hipError_t e;
    if (p->d == 3) {
        ColArgs y = col_args(p, p->ypass);
        if ((e = run_col(p, p->ypass, CM_FORWARD, y, st)) != hipSuccess) return e;
    }
    ColArgs h = col_args(p, p->heat);
    h.K = K;
    h.slot = -1;
    h.stop_iter = p->stop_iter;
    h.epart = p->epart;
    if ((e = run_col(p, p->heat, CM_ENERGY, h, st)) != hipSuccess) return e;
    ReduceArgs ra;
    ra.epart = p->epart;
    ra.nwg = energy_partials(p);
    ra.K = K;
    ra.batch = (int)p->batch;
    ra.n = p->n;
    ra.npts = p->npts;
    ra.tau = p->tau;
    ra.taus = p->taus_dev;
    ra.stop_iter = p->stop_iter;
    ra.energy = p->energy;
    return launch_reduce(ra, st);
}

FastRowArgs fast_row_args(mbo_plan_t p)
{
    FastRowArgs a;
    std::memset(&a, 0, sizeof a);
    a.L = (int)p->N[p->d - 1];
    a.band = p->band_c;
    a.W = p->band_W;
    a.rows = p->npts / p->N[p->d - 1];
    a.npts = p->npts;
    a.tw = p->tw[p->d - 1];
    a.plane_major = p->d == 3;
    a.Z = p->Z;
    a.sgn = p->sgn;
    a.sigma_fb = p->sigma_fb;
    a.K = 1;
    a.foff = p->foff_dev;
    return a;
}

FastColArgs fast_col_args(mbo_plan_t p)
{
    FastColArgs a;
    std::memset(&a, 0, sizeof a);
    a.L = (int)p->N[0];
    a.W = p->band_W;
    a.tiles = p->band_W / p->fast_tx;
    a.field_elems = (int64_t)p->PL * (p->npts / p->N[p->d - 1]) * p->band_W;
    a.tw = p->tw[0];
    if (p->d == 3) {
        a.Ny = (int)p->N[1];
        a.tw_y = p->tw[1];
        a.lam_y = p->lam_y;
        a.lam_y_stride = p->per_field_tau ? p->N[1] : 0;
    }
    a.Z = p->Z;
    a.lam_row = p->lam_row;
    a.lam_col = p->lam_col;
    a.lam_row_stride = p->per_field_tau ? p->N[0] : 0;
    a.lam_col_stride = p->per_field_tau ? p->band_W : 0;
    a.xcd_remap = p->xcd_remap;
    a.nwg = fast_energy_partials(p);
    a.apply = 1;
    return a;
}

hipError_t run_row_fast(mbo_plan_t p, const FastRowArgs& a, hipStream_t st, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr)
{
    const dim3 g((unsigned)fast_row_groups(p), (unsigned)p->batch);
    return launch_row_fast(p->pk, p->n, ilog2((int)p->N[p->d - 1]), a, g, st, false, ev0, ev1);
}

hipError_t run_heat_fast(mbo_plan_t p, const FastColArgs& a, hipStream_t st, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr)
{
    if (p->d == 3)
        return launch_plane_fast(ilog2((int)p->N[1]), ilog2((int)p->N[0]), a, fast_heat_grid(p), st, false, ev0, ev1);
    return launch_heat_fast(p->pk, ilog2((int)p->N[0]), p->fast_tx, a, fast_heat_grid(p), st, false, ev0, ev1);
}

// mbo_iterate through the band-limited passes: the row pass of A_0 (forward
// row FFT, det signs), then per iteration the heat pass over the stored columns
// and the row pass (inverse row FFT, projection, forward row FFT).
hipError_t enqueue_iterate_fast(mbo_plan_t p, void* A, int K, double tol, bool want_energy, hipStream_t st)
{
    const bool track = tol > 0.0;
    const bool fallback = p->prec == MBO_F32_F64FALLBACK;
    const int64_t cs = (int64_t)p->batch * (K > 0 ? K : 1);
    hipError_t e;
    if ((e = launch_fill_u64(p->flips, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->fallbacks, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->nonfinite, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->delta_bits, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_i32(p->stop_iter, p->batch, K, st)) != hipSuccess) return e;
    FastRowArgs r0 = fast_row_args(p);
    r0.Ain = A;
    r0.flags = RF_LOAD_REAL | RF_FORWARD | RF_SIGN_INIT;
    if ((e = run_row_fast(p, r0, st)) != hipSuccess) return e;
    for (int s = 1; s <= K; ++s) {
        FastColArgs h = fast_col_args(p);
        h.iter = s;
        h.K = K;
        h.stop_iter = track ? p->stop_iter : nullptr;
        h.delta_bits = track ? p->delta_bits : nullptr;
        h.tol = tol;
        h.slot = s - 1;
        h.epart = want_energy ? p->epart : nullptr;
        hipEvent_t hs = p->timing ? p->ev[4 * (s - 1) + 2] : nullptr;
        hipEvent_t he = p->timing ? p->ev[4 * (s - 1) + 3] : nullptr;
        if ((e = run_heat_fast(p, h, st, hs, he)) != hipSuccess) return e;
        FastRowArgs r = fast_row_args(p);
        r.Aout = A;
        r.iter = s;
        r.K = K;
        r.delta_bits = p->delta_bits;
        r.cnt_part = p->cnt_part;
        r.flags = RF_INVERSE | RF_PROJECT | RF_SIGN;
        if (track) {
            // only a tolerance can stop a field before the last iteration
            r.stop_iter = p->stop_iter;
            r.flags |= RF_CHECK_STOP;
        }
        if (s < K || want_energy) r.flags |= RF_FORWARD;
        if (s == K || track) r.flags |= RF_STORE_REAL;
        if (track) r.flags |= RF_TRACK;
        if (fallback) r.flags |= RF_FALLBACK;
        hipEvent_t rs = p->timing ? p->ev[4 * (s - 1)] : nullptr;
        hipEvent_t re = p->timing ? p->ev[4 * (s - 1) + 1] : nullptr;
        if ((e = run_row_fast(p, r, st, rs, re)) != hipSuccess) return e;
    }
    if ((e = launch_sum_counts(p->cnt_part, fast_row_groups(p), K, (int)p->batch, p->flips, p->fallbacks,
                               p->nonfinite, st)) != hipSuccess)
        return e;
    if (!want_energy) return hipSuccess;
    // E(A_final) into slot stop_iter[b], then every energy from its partials
    FastColArgs h = fast_col_args(p);
    h.K = K;
    h.slot = -1;
    h.stop_iter = p->stop_iter;
    h.epart = p->epart;
    h.apply = 0;
    if ((e = run_heat_fast(p, h, st)) != hipSuccess) return e;
    ReduceArgs ra;
    ra.epart = p->epart;
    ra.nwg = fast_energy_partials(p);
    ra.K = K;
    ra.batch = (int)p->batch;
    ra.n = p->n;
    ra.npts = p->npts;
    ra.tau = p->tau;
    ra.taus = p->taus_dev;
    ra.stop_iter = p->stop_iter;
    ra.energy = p->energy;
    return launch_reduce(ra, st);
}

// Enqueue the whole of mbo_iterate on stream st (captured into a graph by the caller).
hipError_t enqueue_iterate(mbo_plan_t p, void* A, int K, double tol, bool want_energy, hipStream_t st)
{
    if (p->fast) return enqueue_iterate_fast(p, A, K, tol, want_energy, st);
    const bool track = tol > 0.0;
    const bool fallback = p->prec == MBO_F32_F64FALLBACK;
    const int64_t cs = (int64_t)p->batch * (K > 0 ? K : 1);
    hipError_t e;
    if ((e = launch_fill_u64(p->flips, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->fallbacks, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->nonfinite, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->delta_bits, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_i32(p->stop_iter, p->batch, K, st)) != hipSuccess) return e;

    // A_0: forward row FFT (and det signs for the flip count of iteration 1);
    // in 3-D each iteration starts with the middle-axis forward pass itself.
    if ((e = enqueue_forward(p, A, RF_SIGN_INIT, false, st)) != hipSuccess) return e;

    for (int s = 1; s <= K; ++s) {
        ColArgs h = col_args(p, p->heat);
        h.iter = s;
        h.K = K;
        h.stop_iter = p->stop_iter;
        h.delta_bits = track ? p->delta_bits : nullptr;
        h.tol = tol;
        h.slot = s - 1;
        h.epart = want_energy ? p->epart : nullptr;
        if (p->d == 3) {
            // the first pass of the iteration takes the stop decision
            ColArgs y = col_args(p, p->ypass);
            y.iter = s;
            y.K = K;
            y.stop_iter = p->stop_iter;
            y.delta_bits = track ? p->delta_bits : nullptr;
            y.tol = tol;
            if ((e = run_col(p, p->ypass, CM_FORWARD, y, st)) != hipSuccess)
                return e;
            h.delta_bits = nullptr;
        }
        hipEvent_t hs = p->timing ? p->ev[4 * (s - 1) + 2] : nullptr;
        hipEvent_t he = p->timing ? p->ev[4 * (s - 1) + 3] : nullptr;
        if ((e = run_col(p, p->heat, CM_HEAT, h, st, hs, he)) != hipSuccess) return e;
        if (p->d == 3) {
            ColArgs y = col_args(p, p->ypass);
            y.iter = s;
            y.K = K;
            y.stop_iter = p->stop_iter;
            if ((e = run_col(p, p->ypass, CM_INVERSE, y, st)) != hipSuccess) return e;
        }
        RowArgs r = row_args(p);
        r.Aout = A;
        r.iter = s;
        r.K = K;
        r.flips = p->flips;
        r.fallbacks = p->fallbacks;
        r.nonfinite = p->nonfinite;
        r.delta_bits = p->delta_bits;
        r.stop_iter = p->stop_iter;
        r.flags = RF_INVERSE | RF_PROJECT | RF_SIGN | RF_CHECK_STOP;
        if (s < K || want_energy) r.flags |= RF_FORWARD;
        if (s == K || track) r.flags |= RF_STORE_REAL;
        if (track) r.flags |= RF_TRACK;
        if (fallback) r.flags |= RF_FALLBACK;
        hipEvent_t rs = p->timing ? p->ev[4 * (s - 1)] : nullptr;
        hipEvent_t re = p->timing ? p->ev[4 * (s - 1) + 1] : nullptr;
        if ((e = run_row(p, r, st, rs, re)) != hipSuccess) return e;
    }
    if (want_energy) return enqueue_final_energy(p, K, st);
    return hipSuccess;
}

// ---- volume-preserving step (Section 7) -----------------------------------

int64_t sel_chunks(mbo_plan_t p) { return (p->npts + SEL_CHUNK - 1) / SEL_CHUNK; }

// Workspace of the volume-preserving step, allocated on first use.  The
// histograms start at zero; every selection leaves them at zero.
mbo_status ensure_volume(mbo_plan_t p)
{
    if (p->vnplus) return MBO_OK;  // allocated last
    const size_t B = (size_t)p->batch;
    if (!p->vde) HIP_TRY(p, hipMalloc(&p->vde, B * (size_t)p->npts * p->esz));
    if (!p->vsel) HIP_TRY(p, hipMalloc((void**)&p->vsel, B * sizeof(VpSel)));
    if (!p->vhist) HIP_TRY(p, hipMalloc((void**)&p->vhist, B * ((size_t)1 << SEL_BITS) * sizeof(unsigned)));
    if (!p->vtcnt) HIP_TRY(p, hipMalloc((void**)&p->vtcnt, B * (size_t)sel_chunks(p) * sizeof(unsigned)));
    if (!p->vdone) HIP_TRY(p, hipMalloc((void**)&p->vdone, B * sizeof(unsigned long long)));
    HIP_TRY(p, launch_fill_u64(reinterpret_cast<unsigned long long*>(p->vhist),
                               (int64_t)B * ((1 << SEL_BITS) / 2), 0ull, p->stream));
    HIP_TRY(p, launch_fill_u64(reinterpret_cast<unsigned long long*>(p->vdone), (int64_t)B, 0ull, p->stream));
    RowArgs r = row_args(p);
    (void)launch_row_vp(p->pk, p->n, r.log2L, r, p->row_grid, p->row_block, p->lds_max, nullptr, true);
    (void)hipGetLastError();
    HIP_TRY(p, hipMalloc((void**)&p->vnplus, B * sizeof(long long)));
    return MBO_OK;
}

SelArgs sel_args(mbo_plan_t p, const void* dE)
{
    SelArgs a;
    std::memset(&a, 0, sizeof a);
    a.dE = dE;
    a.npts = p->npts;
    a.nplus = reinterpret_cast<const int64_t*>(p->vnplus);
    a.st = p->vsel;
    a.hist = p->vhist;
    a.tcnt = p->vtcnt;
    a.chunks = sel_chunks(p);
    a.done = p->vdone;
    return a;
}

hipError_t run_row_vp(mbo_plan_t p, const RowArgs& a, hipStream_t st)
{
    return launch_row_vp(p->pk, p->n, a.log2L, a, p->row_grid, p->row_block, p->row_lds, st);
}

// Points to select per field, from the host, checked against [0, npts].
mbo_status upload_nplus(mbo_plan_t p, const int64_t* n_plus)
{
    for (int64_t b = 0; b < p->batch; ++b)
        if (n_plus[b] < 0 || n_plus[b] > p->npts)
            return fail(p, MBO_ERR_INVALID_ARG, "n_plus[%lld] = %lld is outside [0, %lld]", (long long)b,
                        (long long)n_plus[b], (long long)p->npts);
    HIP_TRY(p, hipMemcpyAsync(p->vnplus, n_plus, (size_t)p->batch * sizeof(long long),
                              hipMemcpyHostToDevice, p->stream));
    return MBO_OK;
}

// The volume-preserving step on the real values the row pass loads or the
// inverse row transform yields (load_flags): Delta E into vde, the selection,
// then T+ / T- with the extra flags of the applying launch (apply).
hipError_t enqueue_volume_step(mbo_plan_t p, int load_flags, const void* Ain, void* vde, RowArgs apply,
                               hipStream_t st)
{
    const int fb = p->prec == MBO_F32_F64FALLBACK ? RF_FALLBACK : 0;
    RowArgs r = row_args(p);
    r.Ain = Ain;
    r.vde = vde;
    r.flags = load_flags | RF_VP_KEY | fb;
    hipError_t e = run_row_vp(p, r, st);
    if (e != hipSuccess) return e;
    if ((e = launch_select(p->pk, sel_args(p, vde), (int)p->batch, st)) != hipSuccess) return e;
    apply.Ain = Ain;
    apply.vde = vde;
    apply.vsel = p->vsel;
    apply.flags |= load_flags | RF_VP_APPLY | fb;
    return run_row_vp(p, apply, st);
}

// Enqueue the whole of mbo_iterate_volume on stream st.  from_a0: the points to
// select are the points of A_0 with det >= 0 (else vnplus holds them).
hipError_t enqueue_iterate_volume(mbo_plan_t p, void* A, int K, bool from_a0, bool want_energy, hipStream_t st)
{
    const int64_t cs = (int64_t)p->batch * (K > 0 ? K : 1);
    hipError_t e;
    if ((e = launch_fill_u64(p->flips, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->fallbacks, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->nonfinite, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_i32(p->stop_iter, p->batch, K, st)) != hipSuccess) return e;
    if ((e = enqueue_forward(p, A, RF_SIGN_INIT, false, st)) != hipSuccess) return e;
    if (from_a0 && (e = launch_count_pos(p->sgn, p->npts, (int)p->batch, p->vnplus, st)) != hipSuccess)
        return e;
    for (int s = 1; s <= K; ++s) {
        if (p->d == 3) {
            ColArgs y = col_args(p, p->ypass);
            if ((e = run_col(p, p->ypass, CM_FORWARD, y, st)) != hipSuccess) return e;
        }
        ColArgs h = col_args(p, p->heat);
        h.iter = s;
        h.K = K;
        h.stop_iter = p->stop_iter;
        h.slot = s - 1;
        h.epart = want_energy ? p->epart : nullptr;
        if ((e = run_col(p, p->heat, CM_HEAT, h, st)) != hipSuccess) return e;
        if (p->d == 3) {
            ColArgs y = col_args(p, p->ypass);
            if ((e = run_col(p, p->ypass, CM_INVERSE, y, st)) != hipSuccess) return e;
        }
        RowArgs r = row_args(p);
        r.Aout = A;
        r.iter = s;
        r.K = K;
        r.flips = p->flips;
        r.fallbacks = p->fallbacks;
        r.nonfinite = p->nonfinite;
        r.flags = RF_SIGN;
        if (s < K || want_energy) r.flags |= RF_FORWARD;
        if (s == K) r.flags |= RF_STORE_REAL;
        if ((e = enqueue_volume_step(p, RF_INVERSE, nullptr, p->vde, r, st)) != hipSuccess) return e;
    }
    if (want_energy) return enqueue_final_energy(p, K, st);
    return hipSuccess;
}

// ---- relaxed gradient flows (GD-1, GD-3) -------------------------------------

hipError_t run_row_relax(mbo_plan_t p, const RowArgs& a, hipStream_t st)
{
    return launch_row_relax(p->pk, p->n, a.log2L, a, p->row_grid, p->row_block, p->row_lds, st);
}

// K steps of B = (I - dt Delta)^{-1} A, A = B - c N(B) in place on A.
hipError_t enqueue_relaxed_flow(mbo_plan_t p, void* A, int K, int kind, double c, double dt, hipStream_t st)
{
    const int64_t cs = (int64_t)p->batch * (K > 0 ? K : 1);
    hipError_t e;
    if ((e = launch_fill_u64(p->fallbacks, cs, 0ull, st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(p->nonfinite, cs, 0ull, st)) != hipSuccess) return e;
    if (K == 0) return hipSuccess;
    if ((e = enqueue_forward(p, A, 0, false, st)) != hipSuccess) return e;
    const int fb = p->prec == MBO_F32_F64FALLBACK ? RF_FALLBACK : 0;
    for (int s = 1; s <= K; ++s) {
        if (p->d == 3) {
            ColArgs y = col_args(p, p->ypass);
            if ((e = run_col(p, p->ypass, CM_FORWARD, y, st)) != hipSuccess) return e;
        }
        ColArgs h = col_args(p, p->heat);
        h.rdt = dt;
        h.rnorm = 1.0 / (double)p->npts;
        if ((e = run_col(p, p->heat, CM_RESOLVENT, h, st)) != hipSuccess) return e;
        if (p->d == 3) {
            ColArgs y = col_args(p, p->ypass);
            if ((e = run_col(p, p->ypass, CM_INVERSE, y, st)) != hipSuccess) return e;
        }
        RowArgs r = row_args(p);
        r.Aout = A;
        r.iter = s;
        r.K = K;
        r.fallbacks = p->fallbacks;
        r.nonfinite = p->nonfinite;
        r.relax_kind = kind;
        r.relax_c = c;
        r.flags = RF_INVERSE | RF_RELAX | fb | (s < K ? RF_FORWARD : 0) | (s == K ? RF_STORE_REAL : 0);
        if ((e = run_row_relax(p, r, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

mbo_status check_relax_args(mbo_plan_t p, int kind, double eps)
{
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (kind != MBO_GD1 && kind != MBO_GD3) return fail(p, MBO_ERR_INVALID_ARG, "kind must be MBO_GD1 or MBO_GD3");
    if (!(eps > 0.0)) return fail(p, MBO_ERR_INVALID_ARG, "eps must be > 0 (+inf drops the penalty)");
    return MBO_OK;
}

// Shape checks shared by mbo_plan and mbo_plan_batched.
mbo_status check_shape(int d, const int64_t* N, int n, double tau)
{
    if (d != 2 && d != 3) return fail(nullptr, MBO_ERR_INVALID_ARG, "d must be 2 or 3 (got %d)", d);
    if (n < 1 || n > 4) return fail(nullptr, MBO_ERR_INVALID_ARG, "n must be in [1,4] (got %d)", n);
    if (!(tau > 0.0) || !std::isfinite(tau))
        return fail(nullptr, MBO_ERR_INVALID_ARG, "tau must be finite and > 0");
    for (int a = 0; a < d; ++a)
        if (!is_pow2(N[a]) || N[a] < 8 || N[a] > 2048)
            return fail(nullptr, MBO_ERR_UNSUPPORTED,
                        "N[%d] = %lld: each axis must be a power of two in [8, 2048]", a,
                        (long long)N[a]);
    return MBO_OK;
}

void set_shape(mbo_plan_t p, int d, const int64_t* N, int n, int64_t batch, double tau, mbo_precision prec,
               double sigma_fallback, void* hip_stream)
{
    p->d = d;
    for (int a = 0; a < d; ++a) p->N[a] = N[a];
    p->n = n;
    p->batch = batch;
    p->tau = tau;
    p->prec = prec;
    p->sigma_fb = sigma_fallback > 0.0 ? sigma_fallback : 1e-3;
    p->pk = prec == MBO_F64 ? 0 : 1;
    p->esz = prec == MBO_F64 ? 8 : 4;
    p->PL = (n * n + 1) / 2;
    p->npts = 1;
    for (int a = 0; a < d; ++a) p->npts *= N[a];
    p->stream = (hipStream_t)hip_stream;
}

// Device set-up of a plan whose shape fields are filled in: launch
// configuration, workspace, tables and (batched members) the per-field tau and
// offset arrays.  On failure p->err holds the message and the caller destroys p.
mbo_status plan_init(mbo_plan_t p, const int64_t* foff_host)
{
    HIP_TRY(p, hipGetDevice(&p->device));
    hipDeviceProp_t prop;
    HIP_TRY(p, hipGetDeviceProperties(&prop, p->device));
    // leave room for the kernels' static LDS (reduction scratch)
    p->lds_max = prop.sharedMemPerBlock > 4096 ? (size_t)prop.sharedMemPerBlock - 2048 : 65536;
    HIP_TRY(p, hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));

    mbo_status s;
    if ((s = config_row(p)) != MBO_OK) return s;
    if ((s = config_col(p, p->heat, 0)) != MBO_OK) return s;
    if (p->d == 3 && (s = config_col(p, p->ypass, 1)) != MBO_OK) return s;
    prepare_plan_kernels(p);

    const int64_t batch = p->batch;
    const size_t zbytes = (size_t)batch * p->PL * (size_t)p->npts * 2 * p->esz;
    HIP_TRY(p, hipMalloc(&p->Z, zbytes));
    HIP_TRY(p, hipMalloc((void**)&p->sgn, (size_t)batch * (size_t)p->npts));
    HIP_TRY(p, hipMalloc((void**)&p->counters, 4 * sizeof(unsigned long long)));
    for (int a = 0; a < p->d; ++a) {
        for (int b = 0; b < a; ++b)
            if (p->N[b] == p->N[a]) p->tw[a] = p->tw[b];
        if (p->tw[a]) continue;
        HIP_TRY(p, hipMalloc(&p->tw[a], (size_t)p->N[a] * 2 * p->esz));
        if ((s = upload(p, p->tw[a], twiddles(p->N[a]))) != MBO_OK) return s;
    }
    const size_t nt = p->per_field_tau ? (size_t)batch : 1;
    HIP_TRY(p, hipMalloc(&p->lam_row, nt * (size_t)p->N[0] * p->esz));
    HIP_TRY(p, hipMalloc(&p->lam_inner, nt * (size_t)(p->npts / p->N[0]) * p->esz));
    if ((s = build_symbol_tables(p)) != MBO_OK) return s;
    config_fast(p);
    if ((s = build_fast_tables(p)) != MBO_OK) return s;
    prepare_fast_kernels(p);
    HIP_TRY(p, hipMalloc(&p->mu_row, (size_t)p->N[0] * p->esz));
    HIP_TRY(p, hipMalloc(&p->mu_inner, (size_t)(p->npts / p->N[0]) * p->esz));
    if ((s = build_laplace_tables(p)) != MBO_OK) return s;
    // dot partials: one per row workgroup, sized for any rows-per-workgroup choice
    HIP_TRY(p, hipMalloc((void**)&p->dpart,
                         (size_t)batch * (size_t)(p->npts / p->N[p->d - 1]) * sizeof(double)));
    HIP_TRY(p, hipMalloc((void**)&p->dsum, (size_t)batch * sizeof(double)));
    if (p->per_field_tau) {
        HIP_TRY(p, hipMalloc((void**)&p->taus_dev, (size_t)batch * sizeof(double)));
        HIP_TRY(p, hipMemcpy(p->taus_dev, p->taus.data(), (size_t)batch * sizeof(double),
                             hipMemcpyHostToDevice));
    }
    if (foff_host) {
        HIP_TRY(p, hipMalloc((void**)&p->foff_dev, (size_t)batch * sizeof(int64_t)));
        HIP_TRY(p, hipMemcpy(p->foff_dev, foff_host, (size_t)batch * sizeof(int64_t),
                             hipMemcpyHostToDevice));
    }
    return MBO_OK;
}

// Copy the iteration logs of plan p back (on stream st, synchronising) and
// store them for field row map[b] (or b) of the caller's arrays; counts the
// projections that met NaN/Inf into *bad.  Also evaluates kernel timing.
mbo_status read_logs(mbo_plan_t p, int K, double tol, hipStream_t st, int* iters_done, double* energy,
                     int64_t* flips, double* delta, int64_t* fallbacks, const std::vector<int>* map,
                     unsigned long long* bad)
{
    const size_t B = (size_t)p->batch;
    const size_t cs = B * (size_t)(K > 0 ? K : 1);
    std::vector<int> stp(B);
    std::vector<unsigned long long> hf(cs), hfb(cs), hbad(cs), hd(cs);
    std::vector<double> he(B * (size_t)(K + 1));
    HIP_TRY(p, hipMemcpyAsync(stp.data(), p->stop_iter, B * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(p, hipMemcpyAsync(hf.data(), p->flips, cs * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(p, hipMemcpyAsync(hfb.data(), p->fallbacks, cs * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(p, hipMemcpyAsync(hbad.data(), p->nonfinite, cs * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(p, hipMemcpyAsync(hd.data(), p->delta_bits, cs * 8, hipMemcpyDeviceToHost, st));
    if (energy)
        HIP_TRY(p, hipMemcpyAsync(he.data(), p->energy, he.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(p, hipStreamSynchronize(st));

    if (p->timing && K > 0) {
        // average over the iterations every field ran (stopped fields skip kernels)
        int ran = K;
        for (size_t b = 0; b < B; ++b) ran = stp[b] < ran ? stp[b] : ran;
        double tr = 0.0, tc = 0.0;
        for (int k = 0; k < ran; ++k) {
            float ms_r = 0.f, ms_c = 0.f;
            HIP_TRY(p, hipEventElapsedTime(&ms_r, p->ev[4 * k], p->ev[4 * k + 1]));
            HIP_TRY(p, hipEventElapsedTime(&ms_c, p->ev[4 * k + 2], p->ev[4 * k + 3]));
            tr += ms_r;
            tc += ms_c;
        }
        p->t_launches = ran;
        p->t_row_us = ran ? 1000.0 * tr / ran : 0.0;
        p->t_col_us = ran ? 1000.0 * tc / ran : 0.0;
    }

    for (size_t b = 0; b < B; ++b) {
        const int done = stp[b];
        const size_t f = map ? (size_t)(*map)[b] : b;
        if (iters_done) iters_done[f] = done;
        for (int k = 0; k < K; ++k) {
            const size_t i = b * (size_t)K + (size_t)k;
            const size_t o = f * (size_t)K + (size_t)k;
            const bool ran = k < done;
            if (flips) flips[o] = ran ? (int64_t)hf[i] : 0;
            if (fallbacks) fallbacks[o] = ran ? (int64_t)hfb[i] : 0;
            if (delta) {
                double dv;
                std::memcpy(&dv, &hd[i], sizeof dv);
                delta[o] = (ran && tol > 0.0) ? dv : -1.0;
            }
            if (ran) *bad += hbad[i];
        }
        if (energy)
            for (int k = 0; k <= K; ++k) {
                const size_t i = b * (size_t)(K + 1) + (size_t)k;
                energy[f * (size_t)(K + 1) + (size_t)k] = k <= done ? he[i] : std::nan("");
            }
    }
    return MBO_OK;
}

// ---------------------------------------------------------------------------
// Autotuner of a plan's launch shapes.  Coordinate search, each choice timed
// on the device over `reps` iterations of a pseudo-random field (direct
// launches between two events): heat-pass tile width (lines per workgroup)
// and the XCD-aware tile order on/off, the middle-axis tile width (3-D), then
// the rows per row-pass workgroup.  The transforms and the projection do the
// same arithmetic per line and per point for every choice; only the launch
// shape, and with it the order of the energy partial sums, changes.
// ---------------------------------------------------------------------------
// Time per iteration of `reps` iterations from the same uniform field: the
// least of three runs after a warm-up iteration (single runs of a few hundred
// microseconds vary by several percent, enough to flip the choice between two
// shapes whose iterations differ by less).
mbo_status time_iterations(mbo_plan_t p, void* A, int reps, hipEvent_t e0, hipEvent_t e1, double* us)
{
    const int64_t count = p->batch * (int64_t)p->n * p->n * p->npts;
    HIP_TRY(p, launch_fill_uniform(p->pk, A, count, 0x5eedull, p->stream));
    HIP_TRY(p, enqueue_iterate(p, A, 1, 0.0, false, p->stream));  // warm-up
    double best = 0.0;
    for (int run = 0; run < 3; ++run) {
        HIP_TRY(p, launch_fill_uniform(p->pk, A, count, 0x5eedull, p->stream));
        HIP_TRY(p, hipEventRecord(e0, p->stream));
        HIP_TRY(p, enqueue_iterate(p, A, reps, 0.0, false, p->stream));
        HIP_TRY(p, hipEventRecord(e1, p->stream));
        HIP_TRY(p, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(p, hipEventElapsedTime(&ms, e0, e1));
        const double t = 1000.0 * ms / reps;
        if (run == 0 || t < best) best = t;
    }
    *us = best;
    return MBO_OK;
}

// Launch shapes of the general kernels (strided-pass tile widths, the XCD
// order when tune_xcd, rows and threads of the row pass), each kept when the
// timed iteration on the general path gets faster; `best` is the time at the
// shapes in place.
mbo_status tune_general(mbo_plan_t p, void* A, int reps, hipEvent_t e0, hipEvent_t e1, double best, bool tune_xcd)
{
    mbo_status s;
    double t = 0.0;
    // strided passes: tile width, from one line up to what the rule allows
    for (int axis = 0; axis < (p->d == 3 ? 2 : 1); ++axis) {
        ColCfg& c = axis == 0 ? p->heat : p->ypass;
        int& cap = axis == 0 ? p->tune_tx_heat : p->tune_tx_y;
        const int tx_rule = c.TX;
        cap = 1 << 20;  // widest tile the LDS and 512 threads allow
        if ((s = config_col(p, c, axis)) != MBO_OK) return s;
        const int tx_max = c.TX;
        int best_tx = tx_rule;
        for (int tx = 1; tx <= tx_max; tx *= 2) {
            if (tx == tx_rule) continue;  // timed above
            cap = tx;
            if ((s = config_col(p, c, axis)) != MBO_OK) return s;
            if ((s = time_iterations(p, A, reps, e0, e1, &t)) != MBO_OK) return s;
            if (t < best) {
                best = t;
                best_tx = tx;
            }
        }
        cap = best_tx;
        if ((s = config_col(p, c, axis)) != MBO_OK) return s;
        if (axis == 0 && tune_xcd) {
            p->xcd_remap = 0;
            if ((s = time_iterations(p, A, reps, e0, e1, &t)) != MBO_OK) return s;
            if (t < best) best = t;
            else p->xcd_remap = 1;
        }
    }
    // rows per row-pass workgroup, threads per point or per line group
    const int L = (int)p->N[p->d - 1];
    const int rpw0 = p->row_rpw;
    int best_rpw = rpw0, best_groups = 0;
    for (int groups = 0; groups < 2; ++groups)
        for (int rpw = 1; rpw * L <= 2048 && rpw <= p->npts / L; rpw *= 2) {
            if (rpw == rpw0 && groups == 0) continue;  // timed above
            p->tune_rpw = rpw;
            p->tune_row_groups = groups;
            if (config_row(p) != MBO_OK) break;  // beyond the LDS or queue limits
            if ((s = time_iterations(p, A, reps, e0, e1, &t)) != MBO_OK) return s;
            if (t < best) {
                best = t;
                best_rpw = rpw;
                best_groups = groups;
            }
        }
    p->tune_rpw = best_rpw;
    p->tune_row_groups = best_groups;
    return config_row(p);
}

mbo_status autotune_plan(mbo_plan_t p)
{
    const int reps = 6;
    mbo_status s = ensure_logs(p, reps);
    if (s != MBO_OK) return s;
    void* A = nullptr;
    HIP_TRY(p, hipMalloc(&A, (size_t)(p->batch * p->n * p->n * p->npts) * p->esz));
    int64_t* foff = p->foff_dev;  // the scratch field has the default layout
    p->foff_dev = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    auto done = [&](mbo_status st) {
        p->foff_dev = foff;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(A);
        drop_logs(p);  // the heat pass's workgroup count may have changed
        return st;
    };
    if (he != hipSuccess) return done(fail(p, MBO_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(he)));
    double best = 0.0, t = 0.0;
    if ((s = time_iterations(p, A, reps, e0, e1, &best)) != MBO_OK) return done(s);
    if (!p->fast) {
        if ((s = tune_general(p, A, reps, e0, e1, best, true)) != MBO_OK) return done(s);
        p->err.clear();
        p->tuned = true;
        return done(MBO_OK);
    }
    if (p->d == 2) {
        // band-limited passes: the heat tile width and the XCD-aware tile order
        // (the 3-D passes have no launch shape to choose)
        int best_tx = p->fast_tx;
        for (int tx = 1; tx <= 16; tx *= 2) {
            if (tx == best_tx) continue;
            p->tune_fast_tx = tx;
            config_fast(p);
            if (!p->fast || p->fast_tx != tx) continue;  // not a valid width here
            drop_logs(p);
            if ((s = ensure_logs(p, reps)) != MBO_OK) return done(s);
            if ((s = time_iterations(p, A, reps, e0, e1, &t)) != MBO_OK) return done(s);
            if (t < best) {
                best = t;
                best_tx = tx;
            }
        }
        p->tune_fast_tx = best_tx;
        config_fast(p);
        drop_logs(p);
        if ((s = ensure_logs(p, reps)) != MBO_OK) return done(s);
        p->xcd_remap = 0;
        if ((s = time_iterations(p, A, reps, e0, e1, &t)) != MBO_OK) return done(s);
        if (t < best) best = t;
        else p->xcd_remap = 1;
    }
    // The general kernels serve the plan's other calls (the volume-preserving
    // iteration, relaxed flows, the adjoint, energies): their shapes are timed
    // on the general path, keeping the XCD order the band-limited passes chose.
    p->fast = false;
    drop_logs(p);
    s = ensure_logs(p, reps);
    double bg = 0.0;
    if (s == MBO_OK) s = time_iterations(p, A, reps, e0, e1, &bg);
    if (s == MBO_OK) s = tune_general(p, A, reps, e0, e1, bg, false);
    p->fast = true;
    if (s != MBO_OK) return done(s);
    p->err.clear();
    p->tuned = true;
    return done(MBO_OK);
}

// Lyapunov energy of every field of plan p into E_dev-backed host array E
// (entry map[b] or b); synchronises p's stream.
mbo_status energy_into(mbo_plan_t p, const void* A, double* E, const std::vector<int>* map)
{
    mbo_status s = ensure_logs(p, 0);
    if (s != MBO_OK) return s;
    HIP_TRY(p, enqueue_forward(p, A, 0, true, p->stream));
    ColArgs h = col_args(p, p->heat);
    h.K = 0;
    h.slot = 0;
    h.epart = p->epart;
    HIP_TRY(p, run_col(p, p->heat, CM_ENERGY, h, p->stream));
    ReduceArgs ra;
    ra.epart = p->epart;
    ra.nwg = energy_partials(p);
    ra.K = 0;
    ra.batch = (int)p->batch;
    ra.n = p->n;
    ra.npts = p->npts;
    ra.tau = p->tau;
    ra.taus = p->taus_dev;
    ra.stop_iter = nullptr;
    ra.energy = p->energy;
    HIP_TRY(p, launch_reduce(ra, p->stream));
    std::vector<double> h_e((size_t)p->batch);
    HIP_TRY(p, hipMemcpyAsync(h_e.data(), p->energy, (size_t)p->batch * sizeof(double), hipMemcpyDeviceToHost,
                              p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    for (size_t b = 0; b < h_e.size(); ++b) E[map ? (size_t)(*map)[b] : b] = h_e[b];
    return MBO_OK;
}

// Side streams of a batched plan: as many as the device runs queues at once
// (four), each class dealt to the least loaded one, largest classes first
// (estimated work: fields x points x n^2 x log2 of the points).
mbo_status setup_side_streams(mbo_plan_t g)
{
    const int ns = std::min<int>(4, (int)g->members.size());
    for (int i = 0; i < ns; ++i) {
        hipStream_t q = nullptr;
        HIP_TRY(g, hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        g->side.push_back(q);
        hipEvent_t e = nullptr;
        HIP_TRY(g, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        g->ev_join.push_back(e);
    }
    HIP_TRY(g, hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
    std::vector<std::pair<double, int>> work;
    for (size_t m = 0; m < g->members.size(); ++m) {
        const mbo_plan_t c = g->members[m];
        work.emplace_back((double)c->batch * (double)c->npts * c->n * c->n * std::log2((double)c->npts), (int)m);
    }
    std::sort(work.begin(), work.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
        return a.first > b.first;
    });
    std::vector<double> load((size_t)ns, 0.0);
    g->side_of.assign(g->members.size(), 0);
    for (const auto& w : work) {
        const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        g->side_of[(size_t)w.second] = q;
        load[(size_t)q] += w.first;
    }
    return MBO_OK;
}

std::vector<int> member_fields(mbo_plan_t g, int mi)
{
    std::vector<int> map;
    for (size_t f = 0; f < g->f_member.size(); ++f)
        if (g->f_member[f] == mi) map.push_back((int)f);
    return map;
}

// out = e^{tau Delta} in (one diffusion step), enqueued on st.
hipError_t enqueue_diffuse(mbo_plan_t p, const void* in, void* out, hipStream_t st)
{
    hipError_t e = enqueue_forward(p, in, 0, true, st);
    if (e != hipSuccess) return e;
    ColArgs h = col_args(p, p->heat);
    if ((e = run_col(p, p->heat, CM_HEAT, h, st)) != hipSuccess) return e;
    if (p->d == 3) {
        ColArgs y = col_args(p, p->ypass);
        if ((e = run_col(p, p->ypass, CM_INVERSE, y, st)) != hipSuccess) return e;
    }
    RowArgs r = row_args(p);
    r.Aout = out;
    r.flags = RF_INVERSE | RF_STORE_REAL;
    return run_row(p, r, st);
}

// dot[b] += <G_b, d/dtau e^{tau Delta} A_b> (device accumulator), enqueued on st.
hipError_t enqueue_dtau_dot(mbo_plan_t p, const void* A, const void* G, double* dot, hipStream_t st)
{
    hipError_t e = enqueue_forward(p, A, 0, true, st);
    if (e != hipSuccess) return e;
    ColArgs h = col_args(p, p->heat);
    if ((e = run_col(p, p->heat, CM_DTAU, h, st)) != hipSuccess) return e;
    if (p->d == 3) {
        ColArgs y = col_args(p, p->ypass);
        if ((e = run_col(p, p->ypass, CM_INVERSE, y, st)) != hipSuccess) return e;
    }
    RowArgs r = row_args(p);
    r.flags = RF_INVERSE | RF_DOT;
    r.Gdot = G;
    r.dpart = p->dpart;
    if ((e = run_row(p, r, st)) != hipSuccess) return e;
    return launch_sum_rows(p->dpart, (int64_t)p->row_grid.x, (int)p->batch, dot, st, true);
}

bool use_graphs()
{
    const char* v = std::getenv("MBO_NO_GRAPH");
    return !(v && v[0] == '1');
}


// ---- surface diffusion on a sphere (closest point method) -------------------

// T(x) of the band-width estimate: the heat-kernel mass outside the ball of
// radius 2 x sqrt(tau) (Theorem 5.2).
double band_tail(double x) { return 2.0 * x / std::sqrt(3.14159265358979323846) * std::exp(-x * x) + std::erfc(x); }

// w_b with T(w_b / (2 sqrt(tau))) = eps (T falls from 1 at 0), by bisection.
double band_width_of(double tau, double eps)
{
    double lo = 0.0, hi = 40.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        (band_tail(mid) > eps ? lo : hi) = mid;
    }
    return std::sqrt(tau) * (lo + hi);
}

// p Chebyshev points on [0, 1] (zeros of T_p, ascending) and the weights that
// integrate polynomials of degree < p exactly (Fejer's first rule).
void chebyshev_rule(int p, double* x, double* w)
{
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < p; ++k) {
        const double th = pi * (2.0 * (p - 1 - k) + 1.0) / (2.0 * p);
        double s = 0.0;
        for (int j = 1; j <= p / 2; ++j) s += std::cos(2.0 * j * th) / (4.0 * j * j - 1.0);
        x[k] = 0.5 * (1.0 + std::cos(th));
        w[k] = (1.0 - 2.0 * s) / p;
    }
}

// Gauss-Legendre rule on [-1, 1] by Newton's method on P_q.
// The peanut of Section 6.3: the meridian X(t) = 3t - t^3,
// rho(t) = sqrt((1 + X^2)(4 - X^2)) / 2 = (1 - t^2) sqrt((1 + X^2)(4 - t^2)) / 2,
// t in [-1, 1] (the second form is smooth at the tips), rotated about the x
// axis.  The closest point of p = (x, y, z) is the closest point (X(t), rho(t))
// of the meridian to (x, |(y, z)|), turned into the half plane of p.
void peanut_eval(double t, double& X, double& r)
{
    X = 3.0 * t - t * t * t;
    r = 0.5 * (1.0 - t * t) * std::sqrt((1.0 + X * X) * (4.0 - t * t));
}

// d/dt and d^2/dt^2 of X and rho
void peanut_deriv(double t, double& X1, double& X2, double& r1, double& r2)
{
    const double X = 3.0 * t - t * t * t, Xp = 3.0 - 3.0 * t * t, Xpp = -6.0 * t;
    const double u = 1.0 + X * X, up = 2.0 * X * Xp, upp = 2.0 * (Xp * Xp + X * Xpp);
    const double v = 4.0 - t * t, vp = -2.0 * t;
    const double h = u * v, hp = up * v + u * vp, hpp = upp * v + 2.0 * up * vp - 2.0 * u;
    const double a = 1.0 - t * t, ap = -2.0 * t;
    const double sh = std::sqrt(h);
    X1 = Xp;
    X2 = Xpp;
    r1 = 0.5 * (ap * sh + a * hp / (2.0 * sh));
    r2 = 0.5 * (-2.0 * sh + ap * hp / sh + a * (hpp / (2.0 * sh) - hp * hp / (4.0 * h * sh)));
}

double peanut_d2(double t, double x, double rr)
{
    double X, r;
    peanut_eval(t, X, r);
    return (X - x) * (X - x) + (r - rr) * (r - rr);
}

// Minimise the squared meridian distance over [a, b]: golden section, then
// Newton on its derivative (the flat minimum limits the golden bracket to about
// the square root of the rounding).  Returns the minimiser.
double peanut_refine(double x, double rr, double a, double b)
{
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int it = 0; it < 120 && b - a > 1e-15; ++it) {
        const double u = b - g * (b - a), v = a + g * (b - a);
        if (peanut_d2(u, x, rr) <= peanut_d2(v, x, rr)) b = v;
        else a = u;
    }
    double t = 0.5 * (a + b);
    for (int it = 0; it < 4; ++it) {
        double X, r, X1, X2, r1, r2;
        peanut_eval(t, X, r);
        peanut_deriv(t, X1, X2, r1, r2);
        const double gr = (X - x) * X1 + (r - rr) * r1;
        const double H = X1 * X1 + (X - x) * X2 + r1 * r1 + (r - rr) * r2;
        if (!(H > 0.0)) break;
        const double tn = t - gr / H;
        if (!(tn >= a - 1e-6 && tn <= b + 1e-6) || tn < -1.0 || tn > 1.0) break;
        t = tn;
    }
    return t;
}

// Closest point of (x, y, z) on the peanut: the meridian distance scanned at
// 257 parameters, its two best local minima refined, the better one turned into
// the half plane of the point.  Returns the distance.
double peanut_cp(double x, double y, double z, double c[3])
{
    const int N = 256;
    const double rr = std::sqrt(y * y + z * z);
    double d[N + 1];
    for (int k = 0; k <= N; ++k) d[k] = peanut_d2(-1.0 + 2.0 * k / N, x, rr);
    int b1 = -1, b2 = -1;
    for (int k = 0; k <= N; ++k) {
        const bool lmin = (k == 0 || d[k] <= d[k - 1]) && (k == N || d[k] <= d[k + 1]);
        if (!lmin) continue;
        if (b1 < 0 || d[k] < d[b1]) {
            b2 = b1;
            b1 = k;
        } else if (b2 < 0 || d[k] < d[b2]) {
            b2 = k;
        }
    }
    double best = 0.0, bd = INFINITY;
    for (int i = 0; i < 2; ++i) {
        const int k = i == 0 ? b1 : b2;
        if (k < 0) continue;
        const double t = peanut_refine(x, rr, -1.0 + 2.0 * std::max(k - 1, 0) / N, -1.0 + 2.0 * std::min(k + 1, N) / N);
        const double dd = peanut_d2(t, x, rr);
        if (dd < bd) {
            bd = dd;
            best = t;
        }
    }
    double X, r;
    peanut_eval(best, X, r);
    c[0] = X;
    c[1] = rr > 0.0 ? r * y / rr : r;
    c[2] = rr > 0.0 ? r * z / rr : 0.0;
    return std::sqrt((c[0] - x) * (c[0] - x) + (c[1] - y) * (c[1] - y) + (c[2] - z) * (c[2] - z));
}

// Run f(i) for i in [0, count) on the host's cores (at most 16 threads).
template <typename F>
void parallel_for(int64_t count, F f)
{
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt == 0 ? 1 : (nt > 16 ? 16 : nt);
    if (count < 64 || nt == 1) {
        for (int64_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nt; ++w)
        th.emplace_back([&, w]() {
            for (int64_t i = w; i < count; i += nt) f(i);
        });
    for (auto& t : th) t.join();
}

void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w)
{
    const double pi = 3.14159265358979323846;
    x.assign((size_t)q, 0.0);
    w.assign((size_t)q, 0.0);
    for (int i = 0; i < q; ++i) {
        double z = std::cos(pi * (i + 0.75) / (q + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[(size_t)i] = z;
        w[(size_t)i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

struct mbo_surface_s {
    mbo_plan_t grid = nullptr;  // 3-D plan of the periodic grid: workspace Z, passes, tables
    int n = 3, p = 1, w = 6, Ng = 8, pk = 0;
    mbo_precision prec = MBO_F64;
    size_t esz = 8;
    hipStream_t stream = nullptr;
    double R = 1.0, dx = 0.1, tau = 0.01, eps = 1e-6, wb = 0.0, beta = 0.0, h = 0.0, y0 = 0.0;
    int64_t m = 0, cells = 0;
    std::vector<double> xq, xc, wq;  // canonical order, host
    struct Bins {
        void* pos = nullptr;
        void* wts = nullptr;
        int64_t* perm = nullptr;
        int64_t* start = nullptr;
        int* bin = nullptr;
        int nbins = 0;
    } spread, interp, cellbins;
    // cell spreading (the default): nodes dx n_a and weight factors dx w_a per
    // axis, union stencil width U, waves per workgroup (0: spread sample by
    // sample instead)
    void* nodes = nullptr;
    void* nwts = nullptr;
    int U = 0, cell_waves = 0, cell_chunk = 1;
    bool cell_lines = false;
    // spreading tiles of every (listed bin, plane) and the bin -> listed index map
    void* tiles = nullptr;
    int* binmap = nullptr;
    int tile_edge = 0;
    void* tmp = nullptr;        // [n*n][m]
    int8_t* sgn = nullptr;      // [m]
    unsigned long long* counters = nullptr;
    // volume-preserving step: integer volume weights (host and device), their
    // total, Delta E, the selection state, digit histogram and tie chunk sums
    std::vector<int64_t> Wh;
    int64_t Wtotal = 0;
    int64_t* Wd = nullptr;
    void* de = nullptr;
    WSelState* wsel = nullptr;
    unsigned long long* whist = nullptr;
    long long* wcsum = nullptr;
    std::string err;
};

namespace {

mbo_status sfail(mbo_surface_t s, mbo_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_plan_error = buf;
    return st;
}

#define SHIP(surf, expr)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return sfail(surf, e_ == hipErrorOutOfMemory ? MBO_ERR_ALLOC : MBO_ERR_HIP,       \
                         "%s failed: %s", #expr, hipGetErrorString(e_));                      \
    } while (0)

void surface_free(mbo_surface_t s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_dev(s->nodes);
    free_dev(s->nwts);
    free_dev(s->tiles);
    free_dev(s->binmap);
    free_dev(s->Wd);
    free_dev(s->de);
    free_dev(s->wsel);
    free_dev(s->whist);
    free_dev(s->wcsum);
    for (auto* b : {&s->spread, &s->interp, &s->cellbins}) {
        free_dev(b->pos);
        free_dev(b->wts);
        free_dev(b->perm);
        free_dev(b->start);
        free_dev(b->bin);
    }
    free_dev(s->tmp);
    free_dev(s->sgn);
    free_dev(s->counters);
    if (s->grid) destroy(s->grid);
    delete s;
}

// Upload T-typed copies of host doubles.
mbo_status upload_as(mbo_surface_t s, void** dst, const std::vector<double>& h)
{
    SHIP(s, hipMalloc(dst, h.size() * s->esz + 8));
    if (s->esz == 8) {
        SHIP(s, hipMemcpy(*dst, h.data(), h.size() * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(h.size());
        for (size_t i = 0; i < h.size(); ++i) f[i] = (float)h[i];
        SHIP(s, hipMemcpy(*dst, f.data(), f.size() * 4, hipMemcpyHostToDevice));
    }
    return MBO_OK;
}

// Sort the points pts ([3][m], canonical order) by their SURF_BIN^3 bin of the
// grid and upload positions, weights (nullable), permutation, bin starts and
// the coordinates of the non-empty bins.  The grid coordinate of a point is
// computed here exactly as the kernels compute it (in T from the T-rounded
// position), so that every stencil lies in its bin's tile.
// Within a bin the points are ordered by their stencil start (x, then y, then
// z): the lanes of a wave then read the same few z-lines of the tile, as LDS
// broadcasts or consecutive banks.
template <typename T>
mbo_status build_bins_t(mbo_surface_t s, const std::vector<double>& pts, const std::vector<double>* wts,
                        mbo_surface_s::Bins& B)
{
    const int64_t m = s->m;
    const int nb = (s->Ng + SURF_BIN - 1) / SURF_BIN;
    const T y0 = (T)s->y0, invh = (T)(1.0 / s->h);
    std::vector<std::pair<int64_t, int64_t>> key((size_t)m);
    std::vector<int64_t> sub((size_t)m);
    const T half = (T)s->w * (T)0.5;
    for (int64_t q = 0; q < m; ++q) {
        int64_t id = 0, st = 0;
        for (int a = 0; a < 3; ++a) {
            const T u = ((T)pts[(size_t)(a * m + q)] - y0) * invh;
            if (!(u >= (T)1 && u < (T)(s->Ng - 1)))
                return sfail(s, MBO_ERR_INVALID_ARG, "sample %lld lies outside the grid", (long long)q);
            const int bi = (int)std::floor(u / (T)SURF_BIN);
            id = id * nb + bi;
            st = st * (s->Ng + 64) + ((int64_t)std::ceil(u - half) + 32);
        }
        key[(size_t)q] = {id, q};
        sub[(size_t)q] = st;
    }
    std::sort(key.begin(), key.end(), [&](const std::pair<int64_t, int64_t>& x, const std::pair<int64_t, int64_t>& y) {
        if (x.first != y.first) return x.first < y.first;
        const int64_t sx = sub[(size_t)x.second], sy = sub[(size_t)y.second];
        return sx != sy ? sx < sy : x.second < y.second;
    });
    std::vector<int64_t> perm((size_t)m), start;
    std::vector<int> bins;
    std::vector<double> pos((size_t)(3 * m)), w;
    if (wts) w.resize((size_t)m);
    for (int64_t i = 0; i < m; ++i) {
        const int64_t q = key[(size_t)i].second;
        perm[(size_t)i] = q;
        for (int a = 0; a < 3; ++a) pos[(size_t)(a * m + i)] = pts[(size_t)(a * m + q)];
        if (wts) w[(size_t)i] = (*wts)[(size_t)q];
        if (i == 0 || key[(size_t)i].first != key[(size_t)i - 1].first) {
            start.push_back(i);
            const int64_t id = key[(size_t)i].first;
            bins.push_back((int)(id / ((int64_t)nb * nb)));
            bins.push_back((int)((id / nb) % nb));
            bins.push_back((int)(id % nb));
        }
    }
    start.push_back(m);
    B.nbins = (int)(start.size() - 1);
    mbo_status st;
    if ((st = upload_as(s, &B.pos, pos)) != MBO_OK) return st;
    if (wts && (st = upload_as(s, &B.wts, w)) != MBO_OK) return st;
    SHIP(s, hipMalloc((void**)&B.perm, (size_t)m * 8 + 8));
    SHIP(s, hipMemcpy(B.perm, perm.data(), (size_t)m * 8, hipMemcpyHostToDevice));
    SHIP(s, hipMalloc((void**)&B.start, start.size() * 8));
    SHIP(s, hipMemcpy(B.start, start.data(), start.size() * 8, hipMemcpyHostToDevice));
    SHIP(s, hipMalloc((void**)&B.bin, bins.size() * sizeof(int) + 4));
    SHIP(s, hipMemcpy(B.bin, bins.data(), bins.size() * sizeof(int), hipMemcpyHostToDevice));
    return MBO_OK;
}

mbo_status build_bins(mbo_surface_t s, const std::vector<double>& pts, const std::vector<double>* wts,
                      mbo_surface_s::Bins& B)
{
    return s->esz == 8 ? build_bins_t<double>(s, pts, wts, B) : build_bins_t<float>(s, pts, wts, B);
}

// Bin the band cells (corners [3][cells], canonical order) by the grid
// coordinate of their first node, computed as the cell kernel computes it, and
// upload corners (sorted), cell indices, bin starts and bin coordinates.
template <typename T>
mbo_status build_cell_bins_t(mbo_surface_t s, const std::vector<double>& corners, double node0)
{
    const int64_t nc = s->cells;
    const int nb = (s->Ng + SURF_BIN - 1) / SURF_BIN;
    const T y0 = (T)s->y0, invh = (T)(1.0 / s->h), n0 = (T)node0;
    std::vector<std::pair<int64_t, int64_t>> key((size_t)nc);
    for (int64_t c = 0; c < nc; ++c) {
        int64_t id = 0;
        for (int a = 0; a < 3; ++a) {
            const T u = ((T)corners[(size_t)(a * nc + c)] + n0 - y0) * invh;
            if (!(u >= (T)1 && u < (T)(s->Ng - 1)))
                return sfail(s, MBO_ERR_INVALID_ARG, "cell %lld lies outside the grid", (long long)c);
            id = id * nb + (int)std::floor(u / (T)SURF_BIN);
        }
        key[(size_t)c] = {id, c};
    }
    std::stable_sort(key.begin(), key.end());
    std::vector<int64_t> perm((size_t)nc), start;
    std::vector<int> bins;
    std::vector<double> pos((size_t)(3 * nc));
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t c = key[(size_t)i].second;
        perm[(size_t)i] = c;
        for (int a = 0; a < 3; ++a) pos[(size_t)(a * nc + i)] = corners[(size_t)(a * nc + c)];
        if (i == 0 || key[(size_t)i].first != key[(size_t)i - 1].first) {
            start.push_back(i);
            const int64_t id = key[(size_t)i].first;
            bins.push_back((int)(id / ((int64_t)nb * nb)));
            bins.push_back((int)((id / nb) % nb));
            bins.push_back((int)(id % nb));
        }
    }
    start.push_back(nc);
    mbo_surface_s::Bins& B = s->cellbins;
    B.nbins = (int)(start.size() - 1);
    mbo_status st;
    if ((st = upload_as(s, &B.pos, pos)) != MBO_OK) return st;
    SHIP(s, hipMalloc((void**)&B.perm, (size_t)nc * 8 + 8));
    SHIP(s, hipMemcpy(B.perm, perm.data(), (size_t)nc * 8, hipMemcpyHostToDevice));
    SHIP(s, hipMalloc((void**)&B.start, start.size() * 8));
    SHIP(s, hipMemcpy(B.start, start.data(), start.size() * 8, hipMemcpyHostToDevice));
    SHIP(s, hipMalloc((void**)&B.bin, bins.size() * sizeof(int) + 4));
    SHIP(s, hipMemcpy(B.bin, bins.data(), bins.size() * sizeof(int), hipMemcpyHostToDevice));
    return MBO_OK;
}

SurfArgs surf_args(mbo_surface_t s, const mbo_surface_s::Bins& B)
{
    SurfArgs a;
    std::memset(&a, 0, sizeof a);
    a.m = s->m;
    a.n = s->n;
    a.PL = s->grid->PL;
    a.Ng = s->Ng;
    a.w = s->w;
    a.beta = s->beta;
    a.y0 = s->y0;
    a.h = s->h;
    a.pos = B.pos;
    a.wts = B.wts;
    a.perm = B.perm;
    a.start = B.start;
    a.bin = B.bin;
    a.nbins = B.nbins;
    a.Z = s->grid->Z;
    return a;
}

// Device state of the volume-preserving step, allocated on first use.
mbo_status ensure_surface_volume(mbo_surface_t s)
{
    if (s->wsel) return MBO_OK;
    const int64_t nch = (s->m + WSEL_CHUNK - 1) / WSEL_CHUNK;
    SHIP(s, hipMalloc((void**)&s->Wd, (size_t)s->m * 8 + 8));
    SHIP(s, hipMemcpy(s->Wd, s->Wh.data(), (size_t)s->m * 8, hipMemcpyHostToDevice));
    SHIP(s, hipMalloc(&s->de, (size_t)s->m * s->esz + 8));
    SHIP(s, hipMalloc((void**)&s->whist, 256 * sizeof(unsigned long long)));
    SHIP(s, hipMemset(s->whist, 0, 256 * sizeof(unsigned long long)));
    SHIP(s, hipMalloc((void**)&s->wcsum, (size_t)nch * 8 + 8));
    SHIP(s, hipMalloc((void**)&s->wsel, sizeof(WSelState)));
    return MBO_OK;
}

SurfVolArgs surf_vol_args(mbo_surface_t s)
{
    SurfVolArgs a;
    std::memset(&a, 0, sizeof a);
    a.m = s->m;
    a.D = s->tmp;
    a.de = s->de;
    a.W = s->Wd;
    a.sel = s->wsel;
    a.hist = s->whist;
    a.csum = s->wcsum;
    a.nonfinite = s->counters;
    a.fallback = s->prec == MBO_F32_F64FALLBACK;
    a.sigma_fb = 1e-3;
    return a;
}

// out = S_tau in at the closest points: spread, forward FFT, symbol, inverse
// FFT, interpolate.
hipError_t enqueue_surface_diffuse(mbo_surface_t s, const void* in, void* out, hipStream_t st)
{
    mbo_plan_t g = s->grid;
    hipError_t e;
    const int PL = g->PL;
    const bool cells = s->cell_waves > 0 || s->cell_lines;
    const mbo_surface_s::Bins& sb = cells ? s->cellbins : s->spread;
    SurfArgs a = surf_args(s, sb);
    a.A = in;
    a.pl0 = 0;
    a.pl1 = PL;
    a.tiles = s->tiles;
    a.binmap = s->binmap;
    if (cells) {
        a.p = s->p;
        a.U = s->U;
        a.TE = SURF_BIN + s->U;
        a.nodes = s->nodes;
        a.nwts = s->nwts;
        a.chunk = s->cell_chunk;
        if ((e = launch_surface_spread_cells(s->pk, a, s->cell_lines ? 0 : s->cell_waves, st)) != hipSuccess)
            return e;
    } else if ((e = launch_surface_spread(s->pk, a, st)) != hipSuccess) {
        return e;
    }
    if ((e = launch_surface_gather(s->pk, a, s->tile_edge, st)) != hipSuccess) return e;
    RowArgs r = row_args(g);
    r.flags = RF_FORWARD;
    if ((e = run_row_relax(g, r, st)) != hipSuccess) return e;
    ColArgs y = col_args(g, g->ypass);
    if ((e = run_col(g, g->ypass, CM_FORWARD, y, st)) != hipSuccess) return e;
    ColArgs hh = col_args(g, g->heat);
    if ((e = run_col(g, g->heat, CM_HEAT, hh, st)) != hipSuccess) return e;
    if ((e = run_col(g, g->ypass, CM_INVERSE, y, st)) != hipSuccess) return e;
    r.flags = RF_INVERSE | RF_STORE_Z;
    if ((e = run_row_relax(g, r, st)) != hipSuccess) return e;
    SurfArgs ia = surf_args(s, s->interp);
    ia.out = out;
    ia.pl0 = 0;
    ia.pl1 = PL;
    if ((e = launch_surface_interp(s->pk, ia, st)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* mbo_status_string(mbo_status s)
{
    switch (s) {
    case MBO_OK: return "MBO_OK";
    case MBO_ERR_INVALID_ARG: return "MBO_ERR_INVALID_ARG";
    case MBO_ERR_UNSUPPORTED: return "MBO_ERR_UNSUPPORTED";
    case MBO_ERR_ALLOC: return "MBO_ERR_ALLOC";
    case MBO_ERR_HIP: return "MBO_ERR_HIP";
    case MBO_ERR_NONFINITE: return "MBO_ERR_NONFINITE";
    case MBO_ERR_SCRATCH: return "MBO_ERR_SCRATCH";
    }
    return "MBO_ERR_UNKNOWN";
}

const char* mbo_last_error(mbo_plan_t plan)
{
    if (plan) return plan->err.c_str();
    return g_static_failed ? g_static_error : g_plan_error.c_str();
}

mbo_status mbo_plan(mbo_plan_t* out, int d, const int64_t* N, int n, int64_t batch, double tau,
                    mbo_precision prec, double sigma_fallback, void* hip_stream)
{
    g_plan_error.clear();
    g_static_failed = false;
    if (!out) return fail(nullptr, MBO_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!N) return fail(nullptr, MBO_ERR_INVALID_ARG, "N is NULL");
    if (batch < 1) return fail(nullptr, MBO_ERR_INVALID_ARG, "batch must be >= 1");
    if (!valid_precision(prec))
        return fail(nullptr, MBO_ERR_INVALID_ARG, "unknown precision %d", raw_enum(prec));
    const mbo_status cs = check_shape(d, N, n, tau);
    if (cs != MBO_OK) return cs;

    mbo_plan_t p = new mbo_plan_s();
    set_shape(p, d, N, n, batch, tau, prec, sigma_fallback, hip_stream);
    const mbo_status st = plan_init(p, nullptr);
    if (st != MBO_OK) {
        g_plan_error = p->err;
        destroy(p);
        return st;
    }
    *out = p;
    return MBO_OK;
}

mbo_status mbo_plan_batched(mbo_plan_t* out, int count, const mbo_field_desc* descs, mbo_precision prec,
                            double sigma_fallback, int autotune, void* hip_stream)
{
    g_plan_error.clear();
    g_static_failed = false;
    if (!out) return fail(nullptr, MBO_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !descs) return fail(nullptr, MBO_ERR_INVALID_ARG, "count < 1 or descs is NULL");
    if (!valid_precision(prec))
        return fail(nullptr, MBO_ERR_INVALID_ARG, "unknown precision %d", raw_enum(prec));
    for (int f = 0; f < count; ++f) {
        const mbo_status cs = check_shape(descs[f].d, descs[f].N, descs[f].n, descs[f].tau);
        if (cs != MBO_OK) {
            g_plan_error = "field " + std::to_string(f) + ": " + g_plan_error;
            return cs;
        }
    }
    mbo_plan_t g = new mbo_plan_s();
    g->group = true;
    g->batch = count;
    g->prec = prec;
    g->stream = (hipStream_t)hip_stream;
    auto bail = [&](mbo_status st, const std::string& msg) {
        g_plan_error = msg;
        destroy(g);
        return st;
    };
    hipError_t he = hipGetDevice(&g->device);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (he != hipSuccess) return bail(MBO_ERR_HIP, std::string("device set-up: ") + hipGetErrorString(he));

    // classes of equal (d, N, n), in order of first appearance; the fields are
    // concatenated in the caller's order
    std::vector<int> rep_of;  // representative field of each class
    int64_t off = 0;
    for (int f = 0; f < count; ++f) {
        const mbo_field_desc& df = descs[f];
        int c = -1;
        for (size_t k = 0; k < rep_of.size() && c < 0; ++k) {
            const mbo_field_desc& dr = descs[rep_of[k]];
            bool same = dr.d == df.d && dr.n == df.n;
            for (int a = 0; a < df.d && same; ++a) same = dr.N[a] == df.N[a];
            if (same) c = (int)k;
        }
        if (c < 0) {
            c = (int)rep_of.size();
            rep_of.push_back(f);
        }
        g->f_member.push_back(c);
        g->f_off.push_back(off);
        int64_t pts = 1;
        for (int a = 0; a < df.d; ++a) pts *= df.N[a];
        off += (int64_t)df.n * df.n * pts;
    }
    g->f_index.assign((size_t)count, 0);
    for (size_t c = 0; c < rep_of.size(); ++c) {
        const mbo_field_desc& dr = descs[rep_of[c]];
        std::vector<double> taus;
        std::vector<int64_t> foff;
        for (int f = 0; f < count; ++f)
            if (g->f_member[(size_t)f] == (int)c) {
                g->f_index[(size_t)f] = (int)taus.size();
                taus.push_back(descs[f].tau);
                foff.push_back(g->f_off[(size_t)f]);
            }
        mbo_plan_t m = new mbo_plan_s();
        set_shape(m, dr.d, dr.N, dr.n, (int64_t)taus.size(), taus[0], prec, sigma_fallback, hip_stream);
        m->per_field_tau = true;
        m->taus = taus;
        g->members.push_back(m);
        mbo_status st = plan_init(m, foff.data());
        if (st == MBO_OK && autotune) st = autotune_plan(m);
        if (st != MBO_OK) return bail(st, "field class " + std::to_string(c) + ": " + m->err);
    }
    const mbo_status ss = setup_side_streams(g);
    if (ss != MBO_OK) return bail(ss, g->err);
    *out = g;
    return MBO_OK;
}

mbo_status mbo_plan_autotune(mbo_plan_t p)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    HIP_TRY(p, hipSetDevice(p->device));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (p->group) {
        for (mbo_plan_t m : p->members) {
            const mbo_status s = autotune_plan(m);
            if (s != MBO_OK) return fail(p, s, "%s", m->err.c_str());
        }
        drop_graph(p);
        return MBO_OK;
    }
    return autotune_plan(p);
}

mbo_status mbo_plan_tuning(mbo_plan_t p, int field, int* rows_per_group, int* row_threads,
                           int* heat_lines_per_group, int* xcd_order)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (field < 0 || field >= (int)p->batch) return fail(p, MBO_ERR_INVALID_ARG, "field out of range");
    mbo_plan_t m = p->group ? p->members[(size_t)p->f_member[(size_t)field]] : p;
    if (rows_per_group) *rows_per_group = m->row_rpw;
    if (row_threads) *row_threads = (int)m->row_block.x;
    if (heat_lines_per_group) *heat_lines_per_group = m->fast ? m->fast_tx : m->heat.TX;
    if (xcd_order) *xcd_order = m->xcd_remap;
    return MBO_OK;
}

mbo_status mbo_plan_destroy(mbo_plan_t plan)
{
    destroy(plan);
    return MBO_OK;
}

mbo_status mbo_plan_set_tau(mbo_plan_t p, double tau)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "the fields of a batched plan keep their own tau");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(p, MBO_ERR_INVALID_ARG, "tau must be finite and > 0");
    HIP_TRY(p, hipSetDevice(p->device));
    HIP_TRY(p, hipStreamSynchronize(p->stream));  // tables may be in use by queued work
    p->tau = tau;
    drop_graph(p);  // the energy reduction bakes tau into its arguments
    mbo_status s = build_symbol_tables(p);
    if (s != MBO_OK) return s;
    // the kept modes depend on tau (the logs' partial count may change with them)
    drop_logs(p);
    config_fast(p);
    if ((s = build_fast_tables(p)) != MBO_OK) return s;
    prepare_fast_kernels(p);
    return MBO_OK;
}

mbo_status mbo_plan_set_path(mbo_plan_t p, mbo_path path)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    const int pv = raw_enum(path);
    if (pv != MBO_PATH_GENERIC && pv != MBO_PATH_FULL && pv != MBO_PATH_BANDED)
        return fail(p, MBO_ERR_INVALID_ARG, "unknown path %d", pv);
    HIP_TRY(p, hipSetDevice(p->device));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    drop_graph(p);
    std::vector<mbo_plan_t> plans = p->group ? p->members : std::vector<mbo_plan_t>(1, p);
    for (mbo_plan_t m : plans) {
        m->path = pv;
        drop_logs(m);  // the heat pass's partial count may change
        config_fast(m);
        const mbo_status s = build_fast_tables(m);
        if (s != MBO_OK) return p == m ? s : fail(p, s, "%s", m->err.c_str());
        prepare_fast_kernels(m);
    }
    return MBO_OK;
}

mbo_status mbo_plan_path(mbo_plan_t p, int field, int* path, int* band_half_width, int* stored_modes)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (field < 0 || field >= (int)p->batch) return fail(p, MBO_ERR_INVALID_ARG, "field out of range");
    mbo_plan_t m = p->group ? p->members[(size_t)p->f_member[(size_t)field]] : p;
    if (path) *path = !m->fast ? MBO_PATH_GENERIC : (m->band_W < m->N[m->d - 1] ? MBO_PATH_BANDED : MBO_PATH_FULL);
    if (band_half_width) *band_half_width = m->band_c;
    if (stored_modes) *stored_modes = m->band_W;
    return MBO_OK;
}

mbo_status mbo_plan_set_timing(mbo_plan_t p, int enable)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group && enable) return fail(p, MBO_ERR_UNSUPPORTED, "no kernel timing for a batched plan");
    if (p->timing != (enable != 0)) drop_graph(p);
    p->timing = enable != 0;
    return MBO_OK;
}

mbo_status mbo_last_timing(mbo_plan_t p, double* row_us, double* heat_us, int* launches)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (row_us) *row_us = p->t_row_us;
    if (heat_us) *heat_us = p->t_col_us;
    if (launches) *launches = p->t_launches;
    return MBO_OK;
}

mbo_status mbo_plan_set_stream(mbo_plan_t p, void* hip_stream)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    p->stream = (hipStream_t)hip_stream;
    for (mbo_plan_t m : p->members) m->stream = (hipStream_t)hip_stream;
    return MBO_OK;
}

mbo_status mbo_diffuse(mbo_plan_t p, const void* A_in, void* A_out)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (!A_in || !A_out) return fail(p, MBO_ERR_INVALID_ARG, "A_in / A_out is NULL");
    HIP_TRY(p, hipSetDevice(p->device));
    if (p->group) {
        for (mbo_plan_t m : p->members) {
            const mbo_status s = mbo_diffuse(m, A_in, A_out);
            if (s != MBO_OK) return fail(p, s, "%s", m->err.c_str());
        }
        return MBO_OK;
    }
    HIP_TRY(p, enqueue_forward(p, A_in, 0, true, p->stream));
    ColArgs h = col_args(p, p->heat);
    HIP_TRY(p, run_col(p, p->heat, CM_HEAT, h, p->stream));
    if (p->d == 3) {
        ColArgs y = col_args(p, p->ypass);
        HIP_TRY(p, run_col(p, p->ypass, CM_INVERSE, y, p->stream));
    }
    RowArgs r = row_args(p);
    r.Aout = A_out;
    r.flags = RF_INVERSE | RF_STORE_REAL;
    HIP_TRY(p, run_row(p, r, p->stream));
    return MBO_OK;
}

mbo_status mbo_project(mbo_plan_t p, const void* A_in, void* A_out, int8_t* det_sign)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (!A_in || !A_out) return fail(p, MBO_ERR_INVALID_ARG, "A_in / A_out is NULL");
    HIP_TRY(p, hipSetDevice(p->device));
    if (p->group) {
        if (det_sign) return fail(p, MBO_ERR_UNSUPPORTED, "det_sign is not available for a batched plan");
        for (mbo_plan_t m : p->members) {
            m->last_fb = m->last_bad = 0;
        }
        for (mbo_plan_t m : p->members) {
            const mbo_status s = mbo_project(m, A_in, A_out, nullptr);
            if (s != MBO_OK) return fail(p, s, "%s", m->err.c_str());
        }
        return MBO_OK;
    }
    HIP_TRY(p, launch_fill_u64(p->counters, 4, 0ull, p->stream));
    ProjArgs a;
    a.npts = p->npts;
    a.A = A_in;
    a.Q = A_out;
    a.dsign = det_sign;
    a.nonfinite = p->counters;
    a.fallbacks = p->counters + 1;
    a.fallback = p->prec == MBO_F32_F64FALLBACK;
    a.sigma_fb = p->sigma_fb;
    a.foff = p->foff_dev;
    HIP_TRY(p, launch_project(p->pk, p->n, a, (int)p->batch, p->stream));
    unsigned long long h[4];
    HIP_TRY(p, hipMemcpyAsync(h, p->counters, sizeof h, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->last_fb = (int64_t)h[1];
    p->last_bad = (int64_t)h[0];
    if (h[0]) return fail(p, MBO_ERR_NONFINITE, "%llu points with NaN/Inf input", h[0]);
    return MBO_OK;
}

mbo_status mbo_last_project_counts(mbo_plan_t p, int64_t* fallbacks, int64_t* nonfinite)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    int64_t fb = p->last_fb, bad = p->last_bad;
    for (mbo_plan_t m : p->members) {
        fb += m->last_fb;
        bad += m->last_bad;
    }
    if (fallbacks) *fallbacks = fb;
    if (nonfinite) *nonfinite = bad;
    return MBO_OK;
}

mbo_status mbo_diffuse_dtau(mbo_plan_t p, const void* A, void* out, const void* G, double* dot)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (!A) return fail(p, MBO_ERR_INVALID_ARG, "A is NULL");
    const bool want_dot = G != nullptr && dot != nullptr;
    if (!out && !want_dot) return fail(p, MBO_ERR_INVALID_ARG, "neither out nor (G, dot) given");
    if ((G == nullptr) != (dot == nullptr)) return fail(p, MBO_ERR_INVALID_ARG, "G and dot go together");
    HIP_TRY(p, hipSetDevice(p->device));
    HIP_TRY(p, enqueue_forward(p, A, 0, true, p->stream));
    ColArgs h = col_args(p, p->heat);
    HIP_TRY(p, run_col(p, p->heat, CM_DTAU, h, p->stream));
    if (p->d == 3) {
        ColArgs y = col_args(p, p->ypass);
        HIP_TRY(p, run_col(p, p->ypass, CM_INVERSE, y, p->stream));
    }
    RowArgs r = row_args(p);
    r.Aout = out;
    r.flags = RF_INVERSE | (out ? RF_STORE_REAL : 0) | (want_dot ? RF_DOT : 0);
    r.Gdot = G;
    r.dpart = p->dpart;
    HIP_TRY(p, run_row(p, r, p->stream));
    if (want_dot) {
        HIP_TRY(p, launch_sum_rows(p->dpart, (int64_t)p->row_grid.x, (int)p->batch, p->dsum, p->stream));
        HIP_TRY(p, hipMemcpyAsync(dot, p->dsum, (size_t)p->batch * sizeof(double), hipMemcpyDeviceToHost,
                                  p->stream));
        HIP_TRY(p, hipStreamSynchronize(p->stream));
    }
    return MBO_OK;
}

mbo_status mbo_project_vjp(mbo_plan_t p, const void* A_tilde, const void* G_Q, void* G_A)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (!A_tilde || !G_Q || !G_A) return fail(p, MBO_ERR_INVALID_ARG, "A_tilde / G_Q / G_A is NULL");
    HIP_TRY(p, hipSetDevice(p->device));
    HIP_TRY(p, launch_fill_u64(p->counters, 4, 0ull, p->stream));
    VjpArgs a;
    a.npts = p->npts;
    a.A = A_tilde;
    a.G = G_Q;
    a.GA = G_A;
    a.nonfinite = p->counters;
    a.fallback = p->prec == MBO_F32_F64FALLBACK;
    a.sigma_fb = p->sigma_fb;
    HIP_TRY(p, launch_vjp(p->pk, p->n, a, (int)p->batch, p->stream));
    unsigned long long h[4];
    HIP_TRY(p, hipMemcpyAsync(h, p->counters, sizeof h, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (h[0]) return fail(p, MBO_ERR_NONFINITE, "%llu points with NaN/Inf input", h[0]);
    return MBO_OK;
}

mbo_status mbo_step(mbo_plan_t p, const void* A_prev, void* A_next)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (!A_prev || !A_next) return fail(p, MBO_ERR_INVALID_ARG, "A_prev / A_next is NULL");
    if (A_prev == A_next) return fail(p, MBO_ERR_INVALID_ARG, "A_next must not alias A_prev");
    HIP_TRY(p, hipSetDevice(p->device));
    if (p->fast) {
        // the kernels of mbo_iterate, so that a step reproduces its iterate
        FastRowArgs r0 = fast_row_args(p);
        r0.Ain = A_prev;
        r0.flags = RF_LOAD_REAL | RF_FORWARD;
        HIP_TRY(p, run_row_fast(p, r0, p->stream));
        FastColArgs hf = fast_col_args(p);
        HIP_TRY(p, run_heat_fast(p, hf, p->stream));
        FastRowArgs r1 = fast_row_args(p);
        r1.Aout = A_next;
        r1.flags = RF_INVERSE | RF_PROJECT | RF_STORE_REAL;
        if (p->prec == MBO_F32_F64FALLBACK) r1.flags |= RF_FALLBACK;
        HIP_TRY(p, run_row_fast(p, r1, p->stream));
        return MBO_OK;
    }
    HIP_TRY(p, enqueue_forward(p, A_prev, 0, true, p->stream));
    ColArgs h = col_args(p, p->heat);
    HIP_TRY(p, run_col(p, p->heat, CM_HEAT, h, p->stream));
    if (p->d == 3) {
        ColArgs y = col_args(p, p->ypass);
        HIP_TRY(p, run_col(p, p->ypass, CM_INVERSE, y, p->stream));
    }
    RowArgs r = row_args(p);
    r.Aout = A_next;
    r.flags = RF_INVERSE | RF_PROJECT | RF_STORE_REAL;
    if (p->prec == MBO_F32_F64FALLBACK) r.flags |= RF_FALLBACK;
    HIP_TRY(p, run_row(p, r, p->stream));
    return MBO_OK;
}

mbo_status mbo_step_vjp(mbo_plan_t p, const void* A_prev, void* G, double* dtau)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (!A_prev || !G) return fail(p, MBO_ERR_INVALID_ARG, "A_prev / G is NULL");
    if (A_prev == (const void*)G) return fail(p, MBO_ERR_INVALID_ARG, "G must not alias A_prev");
    HIP_TRY(p, hipSetDevice(p->device));
    const size_t fbytes = (size_t)p->batch * p->n * p->n * (size_t)p->npts * p->esz;
    if (!p->ws_a) HIP_TRY(p, hipMalloc(&p->ws_a, fbytes));
    if (!p->ws_g) HIP_TRY(p, hipMalloc(&p->ws_g, fbytes));
    hipStream_t st = p->stream;
    // A~ = e^{tau Delta} A_{s-1}
    HIP_TRY(p, enqueue_diffuse(p, A_prev, p->ws_a, st));
    // G~ = VJP of the projection at A~
    VjpArgs v;
    v.npts = p->npts;
    v.A = p->ws_a;
    v.G = G;
    v.GA = p->ws_g;
    v.nonfinite = p->counters;
    v.fallback = p->prec == MBO_F32_F64FALLBACK;
    v.sigma_fb = p->sigma_fb;
    HIP_TRY(p, launch_vjp(p->pk, p->n, v, (int)p->batch, st));
    // dL/dtau += <G~, d/dtau e^{tau Delta} A_{s-1}>
    if (dtau) HIP_TRY(p, enqueue_dtau_dot(p, A_prev, p->ws_g, dtau, st));
    // Gbar_{s-1} = e^{tau Delta} G~
    HIP_TRY(p, enqueue_diffuse(p, p->ws_g, G, st));
    return MBO_OK;
}

mbo_status mbo_energy(mbo_plan_t p, const void* A, double* E)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (!A || !E) return fail(p, MBO_ERR_INVALID_ARG, "A / E is NULL");
    HIP_TRY(p, hipSetDevice(p->device));
    if (!p->group) return energy_into(p, A, E, nullptr);
    for (size_t mi = 0; mi < p->members.size(); ++mi) {
        const std::vector<int> map = member_fields(p, (int)mi);
        const mbo_status s = energy_into(p->members[mi], A, E, &map);
        if (s != MBO_OK) return fail(p, s, "%s", p->members[mi]->err.c_str());
    }
    return MBO_OK;
}

mbo_status mbo_iterate(mbo_plan_t p, void* A, int max_iter, double tol, int* iters_done,
                       double* energy, int64_t* flips, double* delta, int64_t* fallbacks)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (!A) return fail(p, MBO_ERR_INVALID_ARG, "A is NULL");
    if (max_iter < 0) return fail(p, MBO_ERR_INVALID_ARG, "max_iter < 0");
    if (std::isnan(tol)) return fail(p, MBO_ERR_INVALID_ARG, "tol is NaN");
    HIP_TRY(p, hipSetDevice(p->device));
    const int K = max_iter;
    const bool want_energy = energy != nullptr;
    mbo_status s;
    if (p->group) {
        for (mbo_plan_t m : p->members)
            if ((s = ensure_logs(m, K)) != MBO_OK) return fail(p, s, "%s", m->err.c_str());
    } else if ((s = ensure_logs(p, K)) != MBO_OK) {
        return s;
    }
    if (p->timing && p->ev_K < K) {
        p->ev.reserve(4 * (size_t)K);
        while ((int)p->ev.size() < 4 * K) {
            hipEvent_t e;
            HIP_TRY(p, hipEventCreate(&e));
            p->ev.push_back(e);
        }
        p->ev_K = K;
        drop_graph(p);
    }
    const int key = (tol > 0.0 ? 1 : 0) | (want_energy ? 2 : 0) | (p->timing ? 4 : 0);
    // the iteration of plan q captured into its own graph (re-captured when the
    // field pointer, K, tol or the logs asked for change)
    auto ensure_graph = [&](mbo_plan_t q) -> mbo_status {
        if (q->gexec && q->g_A == A && q->g_K == K && q->g_key == key && q->g_tol == tol) return MBO_OK;
        drop_graph(q);
        hipGraph_t g = nullptr;
        HIP_TRY(q, hipStreamBeginCapture(q->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_iterate(q, A, K, tol, want_energy, q->cap);
        hipError_t e2 = hipStreamEndCapture(q->cap, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(q, MBO_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipError_t e3 = hipGraphInstantiate(&q->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) {
            q->gexec = nullptr;
            return fail(q, MBO_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
        }
        q->g_A = A;
        q->g_K = K;
        q->g_key = key;
        q->g_tol = tol;
        return MBO_OK;
    };
    if (use_graphs() && !p->timing) {
        if (!p->group) {
            if ((s = ensure_graph(p)) != MBO_OK) return s;
            HIP_TRY(p, hipGraphLaunch(p->gexec, p->stream));
        } else {
            // the field classes are independent: each runs its own graph on a
            // side stream, forked from and joined back into the plan's stream
            for (mbo_plan_t m : p->members)
                if ((s = ensure_graph(m)) != MBO_OK) return fail(p, s, "%s", m->err.c_str());
            HIP_TRY(p, hipEventRecord(p->ev_fork, p->stream));
            for (hipStream_t q : p->side) HIP_TRY(p, hipStreamWaitEvent(q, p->ev_fork, 0));
            for (size_t mi = 0; mi < p->members.size(); ++mi)
                HIP_TRY(p, hipGraphLaunch(p->members[mi]->gexec, p->side[(size_t)p->side_of[mi]]));
            for (size_t q = 0; q < p->side.size(); ++q) {
                HIP_TRY(p, hipEventRecord(p->ev_join[q], p->side[q]));
                HIP_TRY(p, hipStreamWaitEvent(p->stream, p->ev_join[q], 0));
            }
        }
    } else if (!p->group) {
        HIP_TRY(p, enqueue_iterate(p, A, K, tol, want_energy, p->stream));
    } else {
        for (mbo_plan_t m : p->members) HIP_TRY(p, enqueue_iterate(m, A, K, tol, want_energy, p->stream));
    }

    // one copy of the logs at the end
    unsigned long long bad = 0;
    if (p->group) {
        for (size_t mi = 0; mi < p->members.size(); ++mi) {
            mbo_plan_t m = p->members[mi];
            std::vector<int> map;
            for (size_t f = 0; f < p->f_member.size(); ++f)
                if (p->f_member[f] == (int)mi) map.push_back((int)f);
            if ((s = read_logs(m, K, tol, p->stream, iters_done, energy, flips, delta, fallbacks, &map,
                               &bad)) != MBO_OK)
                return fail(p, s, "%s", m->err.c_str());
        }
    } else if ((s = read_logs(p, K, tol, p->stream, iters_done, energy, flips, delta, fallbacks, nullptr,
                              &bad)) != MBO_OK) {
        return s;
    }
    if (bad) return fail(p, MBO_ERR_NONFINITE, "%llu projections met NaN/Inf input", bad);
    return MBO_OK;
}

mbo_status mbo_relaxed_flow(mbo_plan_t p, void* A, int steps, int kind, double eps, double dt)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    mbo_status s;
    if ((s = check_relax_args(p, kind, eps)) != MBO_OK) return s;
    if (!A) return fail(p, MBO_ERR_INVALID_ARG, "A is NULL");
    if (steps < 0) return fail(p, MBO_ERR_INVALID_ARG, "steps < 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, MBO_ERR_INVALID_ARG, "dt must be finite and > 0");
    HIP_TRY(p, hipSetDevice(p->device));
    if ((s = ensure_logs(p, steps)) != MBO_OK) return s;
    (void)launch_row_relax(p->pk, p->n, ilog2((int)p->N[p->d - 1]), row_args(p), p->row_grid, p->row_block,
                           p->lds_max, nullptr, true);
    (void)hipGetLastError();
    const double c = std::isinf(eps) ? 0.0 : dt / (eps * eps);
    if (use_graphs()) {
        if (!(p->rexec && p->rg_A == A && p->rg_K == steps && p->rg_kind == kind && p->rg_c == c &&
              p->rg_dt == dt)) {
            if (p->rexec) (void)hipGraphExecDestroy(p->rexec);
            p->rexec = nullptr;
            hipGraph_t g = nullptr;
            HIP_TRY(p, hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_relaxed_flow(p, A, steps, kind, c, dt, p->cap);
            hipError_t e2 = hipStreamEndCapture(p->cap, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(p, MBO_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
            }
            hipError_t e3 = hipGraphInstantiate(&p->rexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e3 != hipSuccess) {
                p->rexec = nullptr;
                return fail(p, MBO_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
            }
            p->rg_A = A;
            p->rg_K = steps;
            p->rg_kind = kind;
            p->rg_c = c;
            p->rg_dt = dt;
        }
        HIP_TRY(p, hipGraphLaunch(p->rexec, p->stream));
    } else {
        HIP_TRY(p, enqueue_relaxed_flow(p, A, steps, kind, c, dt, p->stream));
    }
    const size_t cs = (size_t)p->batch * (size_t)(steps > 0 ? steps : 1);
    std::vector<unsigned long long> h(cs);
    HIP_TRY(p, hipMemcpyAsync(h.data(), p->nonfinite, cs * 8, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    unsigned long long bad = 0;
    for (unsigned long long v : h) bad += v;
    if (bad) return fail(p, MBO_ERR_NONFINITE, "%llu points met NaN/Inf", bad);
    return MBO_OK;
}

mbo_status mbo_relaxed_energy(mbo_plan_t p, const void* A, int kind, double eps, double* E)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    mbo_status s;
    if ((s = check_relax_args(p, kind, eps)) != MBO_OK) return s;
    if (!A || !E) return fail(p, MBO_ERR_INVALID_ARG, "A / E is NULL");
    HIP_TRY(p, hipSetDevice(p->device));
    if ((s = ensure_logs(p, 0)) != MBO_OK) return s;
    const int64_t blocks = (p->npts + 255) / 256;
    if (!p->pen) HIP_TRY(p, hipMalloc((void**)&p->pen, (size_t)p->batch * (size_t)blocks * sizeof(double)));
    if (!p->pen_sum) HIP_TRY(p, hipMalloc((void**)&p->pen_sum, (size_t)p->batch * sizeof(double)));
    // (1/2) int |grad A|^2 from the spectrum (Parseval), then the mean penalty
    HIP_TRY(p, enqueue_forward(p, A, 0, true, p->stream));
    ColArgs h = col_args(p, p->heat);
    h.K = 0;
    h.slot = 0;
    h.epart = p->epart;
    HIP_TRY(p, run_col(p, p->heat, CM_DIRICHLET, h, p->stream));
    HIP_TRY(p, launch_sum_rows(p->epart, energy_partials(p), (int)p->batch, p->dsum, p->stream));
    HIP_TRY(p, launch_penalty(p->pk, p->n, A, p->npts, (int)p->batch, kind, p->pen, p->stream));
    HIP_TRY(p, launch_sum_rows(p->pen, blocks, (int)p->batch, p->pen_sum, p->stream));
    std::vector<double> dir((size_t)p->batch), pen((size_t)p->batch);
    HIP_TRY(p, hipMemcpyAsync(dir.data(), p->dsum, dir.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipMemcpyAsync(pen.data(), p->pen_sum, pen.size() * sizeof(double), hipMemcpyDeviceToHost,
                              p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    const double P = (double)p->npts;
    for (int64_t b = 0; b < p->batch; ++b)
        E[b] = 0.5 * dir[(size_t)b] / (P * P) + (std::isinf(eps) ? 0.0 : pen[(size_t)b] / (P * eps * eps));
    return MBO_OK;
}

mbo_status mbo_so2_index(mbo_plan_t p, const void* A, double* w_x, double* w_y)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (p->d != 2 || p->n != 2) return fail(p, MBO_ERR_UNSUPPORTED, "the index needs n = 2 on a 2-D grid");
    if (!A) return fail(p, MBO_ERR_INVALID_ARG, "A is NULL");
    HIP_TRY(p, hipSetDevice(p->device));
    const int64_t N0 = p->N[0], N1 = p->N[1];
    const size_t nx = (size_t)p->batch * (size_t)N1, ny = (size_t)p->batch * (size_t)N0;
    double* d = nullptr;
    HIP_TRY(p, hipMalloc((void**)&d, (nx + ny) * sizeof(double)));
    hipError_t e = launch_so2_index(p->pk, A, N0, N1, (int)p->batch, 0, d, p->stream);
    if (e == hipSuccess) e = launch_so2_index(p->pk, A, N0, N1, (int)p->batch, 1, d + nx, p->stream);
    std::vector<double> h(nx + ny);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(p, MBO_ERR_HIP, "index: %s", hipGetErrorString(e));
    if (w_x) std::memcpy(w_x, h.data(), nx * sizeof(double));
    if (w_y) std::memcpy(w_y, h.data() + nx, ny * sizeof(double));
    return MBO_OK;
}

mbo_status mbo_volume_select(mbo_plan_t p, const void* dE, const int64_t* n_plus, uint8_t* selected)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (!dE || !n_plus || !selected) return fail(p, MBO_ERR_INVALID_ARG, "dE / n_plus / selected is NULL");
    HIP_TRY(p, hipSetDevice(p->device));
    mbo_status s;
    if ((s = ensure_volume(p)) != MBO_OK) return s;
    if ((s = upload_nplus(p, n_plus)) != MBO_OK) return s;
    SelArgs a = sel_args(p, dE);
    a.mask = selected;
    HIP_TRY(p, launch_select(p->pk, a, (int)p->batch, p->stream));
    HIP_TRY(p, launch_sel_mark(p->pk, a, (int)p->batch, p->stream));
    return MBO_OK;
}

mbo_status mbo_project_volume(mbo_plan_t p, const void* A_in, void* A_out, const int64_t* n_plus, void* dE)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (!A_in || !A_out || !n_plus) return fail(p, MBO_ERR_INVALID_ARG, "A_in / A_out / n_plus is NULL");
    HIP_TRY(p, hipSetDevice(p->device));
    mbo_status s;
    if ((s = ensure_logs(p, 1)) != MBO_OK) return s;
    if ((s = ensure_volume(p)) != MBO_OK) return s;
    if ((s = upload_nplus(p, n_plus)) != MBO_OK) return s;
    HIP_TRY(p, launch_fill_u64(p->nonfinite, p->batch, 0ull, p->stream));
    HIP_TRY(p, launch_fill_u64(p->fallbacks, p->batch, 0ull, p->stream));
    RowArgs r = row_args(p);
    r.Aout = A_out;
    r.iter = 1;
    r.K = 1;
    r.nonfinite = p->nonfinite;
    r.fallbacks = p->fallbacks;
    r.flags = RF_STORE_REAL;
    HIP_TRY(p, enqueue_volume_step(p, RF_LOAD_REAL, A_in, dE ? dE : p->vde, r, p->stream));
    std::vector<unsigned long long> h((size_t)p->batch);
    HIP_TRY(p, hipMemcpyAsync(h.data(), p->nonfinite, h.size() * 8, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    unsigned long long bad = 0;
    for (unsigned long long v : h) bad += v;
    if (bad) return fail(p, MBO_ERR_NONFINITE, "%llu points with NaN/Inf input", bad);
    return MBO_OK;
}

mbo_status mbo_iterate_volume(mbo_plan_t p, void* A, int max_iter, const int64_t* n_plus, int64_t* n_plus_used,
                              double* energy, int64_t* flips, int64_t* fallbacks)
{
    if (!p) return MBO_ERR_INVALID_ARG;
    if (p->group) return fail(p, MBO_ERR_UNSUPPORTED, "not available for a batched plan");
    if (!A) return fail(p, MBO_ERR_INVALID_ARG, "A is NULL");
    if (max_iter < 0) return fail(p, MBO_ERR_INVALID_ARG, "max_iter < 0");
    HIP_TRY(p, hipSetDevice(p->device));
    const int K = max_iter;
    const bool want_energy = energy != nullptr;
    const bool from_a0 = n_plus == nullptr;
    mbo_status s;
    if ((s = ensure_logs(p, K)) != MBO_OK) return s;
    if ((s = ensure_volume(p)) != MBO_OK) return s;
    if (!from_a0 && (s = upload_nplus(p, n_plus)) != MBO_OK) return s;
    const int key = (want_energy ? 1 : 0) | (from_a0 ? 2 : 0);
    if (use_graphs()) {
        if (!(p->vexec && p->vg_A == A && p->vg_K == K && p->vg_key == key)) {
            if (p->vexec) (void)hipGraphExecDestroy(p->vexec);
            p->vexec = nullptr;
            hipGraph_t g = nullptr;
            HIP_TRY(p, hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_iterate_volume(p, A, K, from_a0, want_energy, p->cap);
            hipError_t e2 = hipStreamEndCapture(p->cap, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(p, MBO_ERR_HIP, "graph capture failed: %s",
                            hipGetErrorString(e != hipSuccess ? e : e2));
            }
            hipError_t e3 = hipGraphInstantiate(&p->vexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e3 != hipSuccess) {
                p->vexec = nullptr;
                return fail(p, MBO_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
            }
            p->vg_A = A;
            p->vg_K = K;
            p->vg_key = key;
        }
        HIP_TRY(p, hipGraphLaunch(p->vexec, p->stream));
    } else {
        HIP_TRY(p, enqueue_iterate_volume(p, A, K, from_a0, want_energy, p->stream));
    }
    std::vector<long long> used((size_t)p->batch);
    HIP_TRY(p, hipMemcpyAsync(used.data(), p->vnplus, used.size() * sizeof(long long), hipMemcpyDeviceToHost,
                              p->stream));
    unsigned long long bad = 0;
    if ((s = read_logs(p, K, 0.0, p->stream, nullptr, energy, flips, nullptr, fallbacks, nullptr, &bad)) != MBO_OK)
        return s;
    if (n_plus_used)
        for (int64_t b = 0; b < p->batch; ++b) n_plus_used[b] = (int64_t)used[(size_t)b];
    if (bad) return fail(p, MBO_ERR_NONFINITE, "%llu projections met NaN/Inf input", bad);
    return MBO_OK;
}

}  // extern "C"

namespace {

enum SurfaceKind { SURF_SPHERE = 0, SURF_PEANUT = 1 };

// The surface object of either kind: sample set on the host, then the grid
// plan, symbol tables, bins and buffers.
mbo_status surface_create(mbo_surface_t* out, int kind, double radius, double dx, int p, double tau, double eps,
                          int n, mbo_precision prec, void* hip_stream)
{
    g_plan_error.clear();
    g_static_failed = false;
    if (!out) return sfail(nullptr, MBO_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!(radius > 0.0) || !(dx > 0.0) || !(tau > 0.0) || !(eps > 0.0 && eps < 0.5) || !std::isfinite(radius) ||
        !std::isfinite(dx) || !std::isfinite(tau))
        return sfail(nullptr, MBO_ERR_INVALID_ARG, "radius, dx, tau must be finite and > 0, eps in (0, 0.5)");
    if (p < 1 || p > 8) return sfail(nullptr, MBO_ERR_INVALID_ARG, "p must be in [1, 8]");
    if (n < 1 || n > 4) return sfail(nullptr, MBO_ERR_INVALID_ARG, "n must be in [1, 4]");
    if (!valid_precision(prec))
        return sfail(nullptr, MBO_ERR_INVALID_ARG, "unknown precision %d", raw_enum(prec));
    mbo_surface_t s = new mbo_surface_s();
    auto bail = [&](mbo_status st) {
        g_plan_error = s->err;
        surface_free(s);
        return st;
    };
    s->R = radius;
    s->dx = dx;
    s->p = p;
    s->tau = tau;
    s->eps = eps;
    s->n = n;
    s->prec = prec;
    s->pk = prec == MBO_F64 ? 0 : 1;
    s->esz = prec == MBO_F64 ? 8 : 4;
    s->stream = (hipStream_t)hip_stream;
    // Algorithm 2, step 1: band width, band cells, quadrature points, closest points
    s->wb = band_width_of(tau, eps);
    double nx[8], nw[8];
    chebyshev_rule(p, nx, nw);
    // half extents of the surface per axis (the sphere: R; the peanut: tips at
    // x = +-2, largest radius 1.25)
    const double ext[3] = {kind == SURF_SPHERE ? radius : 2.0, kind == SURF_SPHERE ? radius : 1.25,
                           kind == SURF_SPHERE ? radius : 1.25};
    const double lim_x = std::ceil((ext[0] + s->wb) / dx) + 1.0, lim_r = std::ceil((ext[1] + s->wb) / dx) + 1.0;
    if (lim_x > 1500.0 || lim_r > 1500.0)  // about 2.7e10 lattice points to test
        return bail(sfail(s, MBO_ERR_UNSUPPORTED, "dx = %g is too small for a band of outer extent %g", dx,
                          ext[0] + s->wb));
    const int64_t lx = (int64_t)lim_x, lr = (int64_t)lim_r;
    std::vector<std::array<double, 3>> corners;
    if (kind == SURF_SPHERE) {
        for (int64_t i = -lx; i <= lx; ++i)
            for (int64_t j = -lr; j <= lr; ++j)
                for (int64_t k = -lr; k <= lr; ++k) {
                    const double gx = dx * (double)i, gy = dx * (double)j, gz = dx * (double)k;
                    if (std::fabs(std::sqrt(gx * gx + gy * gy + gz * gz) - radius) < s->wb)
                        corners.push_back({gx, gy, gz});
                }
    } else {
        // one slab of constant i per task, lexicographic order kept by slab
        const int64_t ni = 2 * lx + 1;
        std::vector<std::vector<std::array<double, 3>>> slab_c((size_t)ni);
        const double wb = s->wb;
        parallel_for(ni, [&](int64_t ii) {
            const int64_t i = ii - lx;
            for (int64_t j = -lr; j <= lr; ++j)
                for (int64_t k = -lr; k <= lr; ++k) {
                    const double gx = dx * (double)i, gy = dx * (double)j, gz = dx * (double)k;
                    double c[3];
                    if (peanut_cp(gx, gy, gz, c) < wb) slab_c[(size_t)ii].push_back({gx, gy, gz});
                }
        });
        for (int64_t ii = 0; ii < ni; ++ii)
            corners.insert(corners.end(), slab_c[(size_t)ii].begin(), slab_c[(size_t)ii].end());
    }
    s->cells = (int64_t)corners.size();
    const int64_t m = s->cells * p * p * p;
    s->m = m;
    if (m == 0) return bail(sfail(s, MBO_ERR_INVALID_ARG, "the band holds no grid point"));
    if (m > ((int64_t)1 << 31) - 1)
        return bail(sfail(s, MBO_ERR_UNSUPPORTED, "%lld samples: at most 2^31 - 1", (long long)m));
    s->xq.assign((size_t)(3 * m), 0.0);
    s->xc.assign((size_t)(3 * m), 0.0);
    s->wq.assign((size_t)m, 0.0);
    const int p3 = p * p * p;
    parallel_for(s->cells, [&](int64_t ci) {
        const auto& c = corners[(size_t)ci];
        int64_t q = ci * p3;
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b)
                for (int e = 0; e < p; ++e, ++q) {
                    const double x = c[0] + dx * nx[a], y = c[1] + dx * nx[b], z = c[2] + dx * nx[e];
                    double cp[3];
                    if (kind == SURF_SPHERE) {
                        const double r = std::sqrt(x * x + y * y + z * z);
                        cp[0] = r > 0.0 ? radius * x / r : radius;
                        cp[1] = r > 0.0 ? radius * y / r : 0.0;
                        cp[2] = r > 0.0 ? radius * z / r : 0.0;
                    } else {
                        peanut_cp(x, y, z, cp);
                    }
                    s->xq[(size_t)q] = x;
                    s->xq[(size_t)(m + q)] = y;
                    s->xq[(size_t)(2 * m + q)] = z;
                    s->xc[(size_t)q] = cp[0];
                    s->xc[(size_t)(m + q)] = cp[1];
                    s->xc[(size_t)(2 * m + q)] = cp[2];
                    s->wq[(size_t)q] = dx * dx * dx * nw[a] * nw[b] * nw[e];
                }
    });
    // integer volume weights (Algorithm 3): the quadrature weight in units of
    // 2^-30 dx^3, so that sums of them are exact
    s->Wh.resize((size_t)m);
    s->Wtotal = 0;
    for (int64_t q = 0; q < m; ++q) {
        s->Wh[(size_t)q] = (int64_t)std::llround(s->wq[(size_t)q] / (dx * dx * dx) * 1073741824.0);
        s->Wtotal += s->Wh[(size_t)q];
    }
    // the periodic grid.  Gridding tolerance eg = eps / 10 (the gridding error
    // at a target grows with the strength of the sources within reach, about
    // (4 pi tau)^{-3/2} times the band volume, so it gets a tenth of the band's
    // tolerance), kernel width w for eg, spacing at most that of a 2x
    // oversampled band limit of the heat kernel (exp(-tau k^2) = eg at half
    // the Nyquist wavenumber), box wide enough that (a) no periodic image of
    // G_tau reaches a target (its tail mass beyond band_width_of(tau, eg) is eg)
    // and (b) every sample lies inside the box with a grid point to spare
    const double pi = 3.14159265358979323846;
    const double eg = std::max(0.1 * eps, prec == MBO_F64 ? 1e-11 : 1e-7);
    s->w = std::max(3, std::min(12, (int)std::ceil(std::log10(1.0 / eg)) + 1));
    s->beta = 2.30 * s->w;
    const double L = std::log(1.0 / eg);
    const double hmax = pi / (2.0 * std::sqrt(L / tau));
    // per axis: sources reach ext + w_b + sqrt(3) dx, targets ext
    double span = 0.0, reach = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double ra = ext[a] + s->wb + dx * std::sqrt(3.0);
        span = std::max(span, ext[a] + ra);
        reach = std::max(reach, ra);
    }
    const double need = std::max(span + band_width_of(tau, eg), 2.0 * reach + 4.0 * hmax);
    int Ng = 64;  // at least the spreading tiles plus a bin
    while (Ng * hmax < need) Ng *= 2;
    if (Ng > 512)
        return bail(sfail(s, MBO_ERR_UNSUPPORTED, "the grid would need %d > 512 points per axis", Ng));
    s->Ng = Ng;
    s->h = need / Ng;  // the whole power-of-two grid oversamples further
    s->y0 = -0.5 * need;
    const int64_t N3[3] = {Ng, Ng, Ng};
    mbo_status st = mbo_plan(&s->grid, 3, N3, n, 1, tau, prec, 0.0, hip_stream);
    if (st != MBO_OK) {
        s->err = g_plan_error;
        return bail(st);
    }
    mbo_plan_t g = s->grid;
    // symbol per axis: exp(-tau k^2) / (Ng h psihat(k h)^2), k = 2 pi m' / (Ng h);
    // psihat(xi) = int_{-W}^{W} psi(z) cos(xi z) dz by Gauss-Legendre
    std::vector<double> gx, gw;
    gauss_legendre(200, gx, gw);
    const double W = 0.5 * s->w;
    std::vector<double> f((size_t)Ng);
    for (int mm = 0; mm < Ng; ++mm) {
        const int mw = 2 * mm < Ng ? mm : mm - Ng;
        const double k = 2.0 * pi * mw / (Ng * s->h);
        double ph = 0.0;
        for (size_t i = 0; i < gx.size(); ++i) {
            const double z = W * gx[i];
            const double r = gx[i];
            ph += W * gw[i] * std::exp(s->beta * (std::sqrt(std::max(0.0, 1.0 - r * r)) - 1.0)) * std::cos(k * s->h * z);
        }
        f[(size_t)mm] = tau * k * k > 3.0 * L ? 0.0 : std::exp(-tau * k * k) / (Ng * s->h * ph * ph);
    }
    std::vector<double> inner((size_t)Ng * Ng);
    for (int a = 0; a < Ng; ++a)
        for (int b = 0; b < Ng; ++b) inner[(size_t)a * Ng + b] = f[(size_t)a] * f[(size_t)b];
    if ((st = upload(g, g->lam_row, f)) != MBO_OK || (st = upload(g, g->lam_inner, inner)) != MBO_OK) {
        s->err = g->err;
        return bail(st);
    }
    (void)launch_row_relax(g->pk, n, ilog2(Ng), row_args(g), g->row_grid, g->row_block, g->lds_max, nullptr, true);
    (void)hipGetLastError();
    // spreading: whole cells when the cell kernel's LDS (tile plus per-wave
    // scratch) fits with at least one wave, else sample by sample
    s->U = s->w + (int)std::ceil(dx * (nx[p - 1] - nx[0]) / s->h * (1.0 + 1e-4) + 1e-4);
    // the line-owner variant (no LDS atomics) when its tile fits in the
    // registers of a 512-thread workgroup, else one wave per cell
    s->cell_waves = 0;
    s->cell_lines = p <= 4 && SURF_BIN + s->U <= 22 &&
                    surface_lines_lds(p, s->U, 64, s->esz) <= g->lds_max;
    if (s->cell_lines) s->cell_chunk = 64;
    for (int wv = 4; wv >= 1 && !s->cell_waves && !s->cell_lines && SURF_BIN + s->U <= 4 * SURF_BIN; wv /= 2) {
        const size_t fixed = surface_cell_lds(p, s->U, wv, 0, s->esz);
        const size_t per_cell = (size_t)(3 + 2 * p * p * p) * s->esz + 8;
        const size_t ch = fixed < g->lds_max ? (g->lds_max - fixed) / per_cell : 0;
        if (ch >= (size_t)wv) {
            s->cell_waves = wv;
            s->cell_chunk = (int)std::min<size_t>(ch, 64);
        }
    }
    if (s->cell_waves || s->cell_lines) {
        std::vector<double> cflat((size_t)(3 * s->cells)), nd((size_t)p), nwv((size_t)p);
        for (int64_t c = 0; c < s->cells; ++c)
            for (int a = 0; a < 3; ++a) cflat[(size_t)(a * s->cells + c)] = corners[(size_t)c][(size_t)a];
        for (int a = 0; a < p; ++a) {
            nd[(size_t)a] = dx * nx[a];
            nwv[(size_t)a] = dx * nw[a];
        }
        st = s->esz == 8 ? build_cell_bins_t<double>(s, cflat, nd[0]) : build_cell_bins_t<float>(s, cflat, nd[0]);
        if (st != MBO_OK) return bail(st);
        if ((st = upload_as(s, &s->nodes, nd)) != MBO_OK || (st = upload_as(s, &s->nwts, nwv)) != MBO_OK)
            return bail(st);
    } else if ((st = build_bins(s, s->xq, &s->wq, s->spread)) != MBO_OK) {
        return bail(st);
    }
    if ((st = build_bins(s, s->xc, nullptr, s->interp)) != MBO_OK) return bail(st);
    {
        // spreading tiles and the map from bin to listed index (the gather's lookup)
        const bool cells = s->cell_waves || s->cell_lines;
        const mbo_surface_s::Bins& sb = cells ? s->cellbins : s->spread;
        s->tile_edge = SURF_BIN + (cells ? s->U : s->w);
        const int nbx = Ng / SURF_BIN;
        std::vector<int> coords((size_t)(3 * sb.nbins)), map((size_t)nbx * nbx * nbx, -1);
        if (sb.nbins > 0)
            SHIP(s, hipMemcpy(coords.data(), sb.bin, coords.size() * sizeof(int), hipMemcpyDeviceToHost));
        for (int b = 0; b < sb.nbins; ++b)
            map[((size_t)coords[(size_t)(3 * b)] * nbx + coords[(size_t)(3 * b + 1)]) * nbx +
                coords[(size_t)(3 * b + 2)]] = b;
        const size_t te3 = (size_t)s->tile_edge * s->tile_edge * s->tile_edge;
        SHIP(s, hipMalloc(&s->tiles, (size_t)sb.nbins * g->PL * te3 * 2 * s->esz + 16));
        SHIP(s, hipMalloc((void**)&s->binmap, map.size() * sizeof(int)));
        SHIP(s, hipMemcpy(s->binmap, map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    const size_t te = (size_t)(SURF_BIN + s->w);
    if (2 * te * te * (te | 1) * s->esz > g->lds_max)
        return bail(sfail(s, MBO_ERR_UNSUPPORTED, "kernel width %d needs more LDS than the device has", s->w));
    if (hipMalloc(&s->tmp, (size_t)(n * n) * (size_t)m * s->esz) != hipSuccess ||
        hipMalloc((void**)&s->sgn, (size_t)m) != hipSuccess ||
        hipMalloc((void**)&s->counters, 4 * sizeof(unsigned long long)) != hipSuccess)
        return bail(sfail(s, MBO_ERR_ALLOC, "device allocation failed"));
    *out = s;
    return MBO_OK;
}

}  // namespace

extern "C" {

mbo_status mbo_surface_sphere(mbo_surface_t* out, double radius, double dx, int p, double tau, double eps, int n,
                              mbo_precision prec, void* hip_stream)
{
    return surface_create(out, SURF_SPHERE, radius, dx, p, tau, eps, n, prec, hip_stream);
}

mbo_status mbo_surface_peanut(mbo_surface_t* out, double dx, int p, double tau, double eps, int n,
                              mbo_precision prec, void* hip_stream)
{
    return surface_create(out, SURF_PEANUT, 1.0, dx, p, tau, eps, n, prec, hip_stream);
}

mbo_status mbo_surface_destroy(mbo_surface_t s)
{
    surface_free(s);
    return MBO_OK;
}

const char* mbo_surface_last_error(mbo_surface_t s) { return s ? s->err.c_str() : g_plan_error.c_str(); }

mbo_status mbo_surface_info(mbo_surface_t s, int64_t* samples, int64_t* cells, int* grid, double* band_width)
{
    if (!s) return MBO_ERR_INVALID_ARG;
    if (samples) *samples = s->m;
    if (cells) *cells = s->cells;
    if (grid) *grid = s->Ng;
    if (band_width) *band_width = s->wb;
    return MBO_OK;
}

mbo_status mbo_surface_points(mbo_surface_t s, double* xq, double* xc, double* w)
{
    if (!s) return MBO_ERR_INVALID_ARG;
    if (xq) std::memcpy(xq, s->xq.data(), s->xq.size() * sizeof(double));
    if (xc) std::memcpy(xc, s->xc.data(), s->xc.size() * sizeof(double));
    if (w) std::memcpy(w, s->wq.data(), s->wq.size() * sizeof(double));
    return MBO_OK;
}

mbo_status mbo_surface_diffuse(mbo_surface_t s, const void* A_in, void* A_out)
{
    if (!s) return MBO_ERR_INVALID_ARG;
    if (!A_in || !A_out) return sfail(s, MBO_ERR_INVALID_ARG, "A_in / A_out is NULL");
    if (A_in == A_out) return sfail(s, MBO_ERR_INVALID_ARG, "A_out must not alias A_in");
    SHIP(s, hipSetDevice(s->grid->device));
    SHIP(s, enqueue_surface_diffuse(s, A_in, A_out, s->stream));
    return MBO_OK;
}

mbo_status mbo_surface_volume_weights(mbo_surface_t s, int64_t* W)
{
    if (!s || !W) return MBO_ERR_INVALID_ARG;
    std::memcpy(W, s->Wh.data(), s->Wh.size() * sizeof(int64_t));
    return MBO_OK;
}

mbo_status mbo_surface_volume_select(mbo_surface_t s, const void* dE, int64_t V, uint8_t* selected)
{
    if (!s) return MBO_ERR_INVALID_ARG;
    if (!dE || !selected) return sfail(s, MBO_ERR_INVALID_ARG, "dE / selected is NULL");
    SHIP(s, hipSetDevice(s->grid->device));
    mbo_status st = ensure_surface_volume(s);
    if (st != MBO_OK) return st;
    SurfVolArgs a = surf_vol_args(s);
    a.de = const_cast<void*>(dE);
    a.selected = selected;
    SHIP(s, launch_wsel(s->pk, a, (long long)V, (long long)s->Wtotal, s->stream));
    SHIP(s, launch_wsel_mark(s->pk, a, s->stream));
    SHIP(s, hipStreamSynchronize(s->stream));
    return MBO_OK;
}

mbo_status mbo_surface_iterate_volume(mbo_surface_t s, void* A, int K, const int64_t* V, int64_t* V_used,
                                      int64_t* flips)
{
    if (!s) return MBO_ERR_INVALID_ARG;
    if (!A) return sfail(s, MBO_ERR_INVALID_ARG, "A is NULL");
    if (K < 0) return sfail(s, MBO_ERR_INVALID_ARG, "K < 0");
    SHIP(s, hipSetDevice(s->grid->device));
    mbo_status st = ensure_surface_volume(s);
    if (st != MBO_OK) return st;
    SHIP(s, launch_fill_u64(s->counters, 4, 0ull, s->stream));
    std::vector<int8_t> prev, cur;
    int64_t vol = V ? *V : 0;
    if (!V || flips) {
        // det signs of A_0 (its projection into tmp is discarded)
        ProjArgs a0;
        std::memset(&a0, 0, sizeof a0);
        a0.npts = s->m;
        a0.A = A;
        a0.Q = s->tmp;
        a0.dsign = s->sgn;
        a0.nonfinite = s->counters + 2;
        a0.fallbacks = s->counters + 3;
        SHIP(s, launch_project(s->pk, s->n, a0, 1, s->stream));
        prev.resize((size_t)s->m);
        SHIP(s, hipMemcpyAsync(prev.data(), s->sgn, (size_t)s->m, hipMemcpyDeviceToHost, s->stream));
        SHIP(s, hipStreamSynchronize(s->stream));
        if (!V) {
            vol = 0;
            for (int64_t q = 0; q < s->m; ++q) vol += prev[(size_t)q] > 0 ? s->Wh[(size_t)q] : 0;
        }
    }
    if (V_used) *V_used = vol;
    for (int it = 0; it < K; ++it) {
        SHIP(s, enqueue_surface_diffuse(s, A, s->tmp, s->stream));
        SurfVolArgs a = surf_vol_args(s);
        a.A = A;
        a.sgn = s->sgn;
        SHIP(s, launch_surf_vp_key(s->pk, s->n, a, s->stream));
        SHIP(s, launch_wsel(s->pk, a, (long long)vol, (long long)s->Wtotal, s->stream));
        SHIP(s, launch_surf_vp_apply(s->pk, s->n, a, s->stream));
        if (flips) {
            cur.resize((size_t)s->m);
            SHIP(s, hipMemcpyAsync(cur.data(), s->sgn, (size_t)s->m, hipMemcpyDeviceToHost, s->stream));
            SHIP(s, hipStreamSynchronize(s->stream));
            int64_t f = 0;
            for (int64_t i = 0; i < s->m; ++i) f += cur[(size_t)i] != prev[(size_t)i];
            flips[it] = f;
            prev.swap(cur);
        }
    }
    unsigned long long h[4];
    SHIP(s, hipMemcpyAsync(h, s->counters, sizeof h, hipMemcpyDeviceToHost, s->stream));
    SHIP(s, hipStreamSynchronize(s->stream));
    if (h[0]) return sfail(s, MBO_ERR_NONFINITE, "%llu samples with NaN/Inf values", h[0]);
    return MBO_OK;
}

mbo_status mbo_surface_iterate(mbo_surface_t s, void* A, int K, int64_t* flips)
{
    if (!s) return MBO_ERR_INVALID_ARG;
    if (!A) return sfail(s, MBO_ERR_INVALID_ARG, "A is NULL");
    if (K < 0) return sfail(s, MBO_ERR_INVALID_ARG, "K < 0");
    SHIP(s, hipSetDevice(s->grid->device));
    std::vector<int8_t> prev, cur;
    if (flips && K > 0) {
        ProjArgs a0;
        std::memset(&a0, 0, sizeof a0);
        a0.npts = s->m;
        a0.A = A;
        a0.Q = s->tmp;
        a0.dsign = s->sgn;
        a0.nonfinite = s->counters;
        a0.fallbacks = s->counters + 1;
        SHIP(s, launch_project(s->pk, s->n, a0, 1, s->stream));  // det signs of A_0 (projection discarded)
        prev.resize((size_t)s->m);
        SHIP(s, hipMemcpyAsync(prev.data(), s->sgn, (size_t)s->m, hipMemcpyDeviceToHost, s->stream));
        SHIP(s, hipStreamSynchronize(s->stream));
    }
    SHIP(s, launch_fill_u64(s->counters, 4, 0ull, s->stream));
    for (int it = 0; it < K; ++it) {
        SHIP(s, enqueue_surface_diffuse(s, A, s->tmp, s->stream));
        ProjArgs a;
        std::memset(&a, 0, sizeof a);
        a.npts = s->m;
        a.A = s->tmp;
        a.Q = A;
        a.dsign = flips ? s->sgn : nullptr;
        a.nonfinite = s->counters;
        a.fallbacks = s->counters + 1;
        a.fallback = s->prec == MBO_F32_F64FALLBACK;
        a.sigma_fb = 1e-3;
        SHIP(s, launch_project(s->pk, s->n, a, 1, s->stream));
        if (flips) {
            cur.resize((size_t)s->m);
            SHIP(s, hipMemcpyAsync(cur.data(), s->sgn, (size_t)s->m, hipMemcpyDeviceToHost, s->stream));
            SHIP(s, hipStreamSynchronize(s->stream));
            int64_t f = 0;
            for (int64_t i = 0; i < s->m; ++i) f += cur[(size_t)i] != prev[(size_t)i];
            flips[it] = f;
            prev.swap(cur);
        }
    }
    unsigned long long h[4];
    SHIP(s, hipMemcpyAsync(h, s->counters, sizeof h, hipMemcpyDeviceToHost, s->stream));
    SHIP(s, hipStreamSynchronize(s->stream));
    if (h[0]) return sfail(s, MBO_ERR_NONFINITE, "%llu points with NaN/Inf input", h[0]);
    return MBO_OK;
}

}  // extern "C"
