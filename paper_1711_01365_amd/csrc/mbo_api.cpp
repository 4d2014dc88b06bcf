// Host runtime and C ABI of libmbo (declared in include/mbo.h).
//
// The plan owns: the packed spectra workspace Z (ceil(n^2/2) complex planes per
// field), per-point det signs, twiddle tables per axis length, the heat-symbol
// tables, the device logs of mbo_iterate, and one cached HIP graph of the whole
// iteration.  All device work goes to the plan's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mbo.h"
#include "mbo_internal.hpp"

using namespace mbo;

namespace {

thread_local std::string g_plan_error;  // failures of mbo_plan (no plan to hold them)

int ilog2(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }

int lds_len(int L) { return (L - 1) + ((L - 1) >> 3) + 1; }  // lds_pad(L-1) + 1

struct ColCfg {
    int L = 0, TX = 1, pitch = 0;
    int64_t S = 0, outer = 0;
    dim3 grid, block;
    size_t lds = 0;
    int axis = 0;
};

}  // namespace

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

// Energy partials per field and iterate: one per wave of the heat pass.
int energy_partials(mbo_plan_t p)
{
    const unsigned bx = p->heat.block.x;
    return (int)(p->heat.grid.x * ((bx % 64) ? 1 : bx / 64));  // = col_args(p, p->heat).nwg
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
    p->log_K = -1;
}

mbo_status ensure_logs(mbo_plan_t p, int K)
{
    if (K <= p->log_K) return MBO_OK;
    drop_logs(p);
    const size_t slots = (size_t)p->batch * (size_t)(K + 1);
    const int nwg = energy_partials(p);
    HIP_TRY(p, hipMalloc((void**)&p->epart, slots * (size_t)nwg * sizeof(double)));
    HIP_TRY(p, hipMalloc((void**)&p->energy, slots * sizeof(double)));
    const size_t cslots = (size_t)p->batch * (size_t)(K > 0 ? K : 1);
    HIP_TRY(p, hipMalloc((void**)&p->flips, cslots * sizeof(unsigned long long)));
    HIP_TRY(p, hipMalloc((void**)&p->fallbacks, cslots * sizeof(unsigned long long)));
    HIP_TRY(p, hipMalloc((void**)&p->nonfinite, cslots * sizeof(unsigned long long)));
    HIP_TRY(p, hipMalloc((void**)&p->delta_bits, cslots * sizeof(unsigned long long)));
    HIP_TRY(p, hipMalloc((void**)&p->stop_iter, (size_t)p->batch * sizeof(int)));
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

// Enqueue the whole of mbo_iterate on stream st (captured into a graph by the caller).
hipError_t enqueue_iterate(mbo_plan_t p, void* A, int K, double tol, bool want_energy, hipStream_t st)
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
mbo_status time_iterations(mbo_plan_t p, void* A, int reps, hipEvent_t e0, hipEvent_t e1, double* us)
{
    const int64_t count = p->batch * (int64_t)p->n * p->n * p->npts;
    HIP_TRY(p, launch_fill_uniform(p->pk, A, count, 0x5eedull, p->stream));
    HIP_TRY(p, enqueue_iterate(p, A, 1, 0.0, false, p->stream));  // warm-up
    HIP_TRY(p, launch_fill_uniform(p->pk, A, count, 0x5eedull, p->stream));
    HIP_TRY(p, hipEventRecord(e0, p->stream));
    HIP_TRY(p, enqueue_iterate(p, A, reps, 0.0, false, p->stream));
    HIP_TRY(p, hipEventRecord(e1, p->stream));
    HIP_TRY(p, hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(p, hipEventElapsedTime(&ms, e0, e1));
    *us = 1000.0 * ms / reps;
    return MBO_OK;
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
    // strided passes: tile width, from one line up to what the rule allows
    for (int axis = 0; axis < (p->d == 3 ? 2 : 1); ++axis) {
        ColCfg& c = axis == 0 ? p->heat : p->ypass;
        int& cap = axis == 0 ? p->tune_tx_heat : p->tune_tx_y;
        const int tx_rule = c.TX;
        cap = 1 << 20;  // widest tile the LDS and 512 threads allow
        if ((s = config_col(p, c, axis)) != MBO_OK) return done(s);
        const int tx_max = c.TX;
        int best_tx = tx_rule;
        for (int tx = 1; tx <= tx_max; tx *= 2) {
            if (tx == tx_rule) continue;  // timed above
            cap = tx;
            if ((s = config_col(p, c, axis)) != MBO_OK) return done(s);
            if ((s = time_iterations(p, A, reps, e0, e1, &t)) != MBO_OK) return done(s);
            if (t < best) {
                best = t;
                best_tx = tx;
            }
        }
        cap = best_tx;
        if ((s = config_col(p, c, axis)) != MBO_OK) return done(s);
        if (axis == 0) {
            p->xcd_remap = 0;
            if ((s = time_iterations(p, A, reps, e0, e1, &t)) != MBO_OK) return done(s);
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
            if ((s = time_iterations(p, A, reps, e0, e1, &t)) != MBO_OK) return done(s);
            if (t < best) {
                best = t;
                best_rpw = rpw;
                best_groups = groups;
            }
        }
    p->tune_rpw = best_rpw;
    p->tune_row_groups = best_groups;
    p->err.clear();
    if ((s = config_row(p)) != MBO_OK) return done(s);
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
    }
    return "MBO_ERR_UNKNOWN";
}

const char* mbo_last_error(mbo_plan_t plan)
{
    return plan ? plan->err.c_str() : g_plan_error.c_str();
}

mbo_status mbo_plan(mbo_plan_t* out, int d, const int64_t* N, int n, int64_t batch, double tau,
                    mbo_precision prec, double sigma_fallback, void* hip_stream)
{
    g_plan_error.clear();
    if (!out) return fail(nullptr, MBO_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!N) return fail(nullptr, MBO_ERR_INVALID_ARG, "N is NULL");
    if (batch < 1) return fail(nullptr, MBO_ERR_INVALID_ARG, "batch must be >= 1");
    if (prec != MBO_F64 && prec != MBO_F32 && prec != MBO_F32_F64FALLBACK)
        return fail(nullptr, MBO_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
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
    if (!out) return fail(nullptr, MBO_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !descs) return fail(nullptr, MBO_ERR_INVALID_ARG, "count < 1 or descs is NULL");
    if (prec != MBO_F64 && prec != MBO_F32 && prec != MBO_F32_F64FALLBACK)
        return fail(nullptr, MBO_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
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
    if (heat_lines_per_group) *heat_lines_per_group = m->heat.TX;
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
    return build_symbol_tables(p);
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
    if (h[0]) return fail(p, MBO_ERR_NONFINITE, "%llu points with NaN/Inf input", h[0]);
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
    auto enqueue_all = [&](hipStream_t st) -> hipError_t {
        if (!p->group) return enqueue_iterate(p, A, K, tol, want_energy, st);
        for (mbo_plan_t m : p->members) {
            hipError_t e = enqueue_iterate(m, A, K, tol, want_energy, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const int key = (tol > 0.0 ? 1 : 0) | (want_energy ? 2 : 0) | (p->timing ? 4 : 0);
    if (use_graphs() && !p->timing) {
        if (!(p->gexec && p->g_A == A && p->g_K == K && p->g_key == key && p->g_tol == tol)) {
            drop_graph(p);
            hipGraph_t g = nullptr;
            HIP_TRY(p, hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_all(p->cap);
            hipError_t e2 = hipStreamEndCapture(p->cap, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(p, MBO_ERR_HIP, "graph capture failed: %s",
                            hipGetErrorString(e != hipSuccess ? e : e2));
            }
            hipError_t e3 = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e3 != hipSuccess) {
                p->gexec = nullptr;
                return fail(p, MBO_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
            }
            p->g_A = A;
            p->g_K = K;
            p->g_key = key;
            p->g_tol = tol;
        }
        HIP_TRY(p, hipGraphLaunch(p->gexec, p->stream));
    } else {
        HIP_TRY(p, enqueue_all(p->stream));
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
