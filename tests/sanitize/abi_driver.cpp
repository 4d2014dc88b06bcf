// Drives the C ABI's argument checks (the paths that run before any device work)
// and its status strings; built with AddressSanitizer and UndefinedBehaviorSanitizer
// on the host side by tests/test_sanitizers.py and run without a GPU.
#include <cstdio>
#include <cstring>

#include "mbo.h"

static int expect(mbo_status got, mbo_status want, const char* what)
{
    if (got != want) {
        std::printf("FAIL %s: got %d want %d (%s)\n", what, (int)got, (int)want, mbo_last_error(nullptr));
        return 1;
    }
    return 0;
}

int main()
{
    int bad = 0;
    mbo_plan_t p = nullptr;
    const int64_t N[3] = {64, 64, 64}, Nodd[2] = {64, 48}, Nbig[2] = {4096, 64};
    bad |= expect(mbo_plan(nullptr, 2, N, 3, 1, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "out NULL");
    bad |= expect(mbo_plan(&p, 2, nullptr, 3, 1, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "N NULL");
    bad |= expect(mbo_plan(&p, 1, N, 3, 1, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "d = 1");
    bad |= expect(mbo_plan(&p, 4, N, 3, 1, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "d = 4");
    bad |= expect(mbo_plan(&p, 2, N, 0, 1, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "n = 0");
    bad |= expect(mbo_plan(&p, 2, N, 5, 1, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "n = 5");
    bad |= expect(mbo_plan(&p, 2, N, 3, 0, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "batch = 0");
    bad |= expect(mbo_plan(&p, 2, N, 3, 1, -1.0, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "tau < 0");
    bad |= expect(mbo_plan(&p, 2, N, 3, 1, 1.0 / 0.0, MBO_F64, 0.0, nullptr), MBO_ERR_INVALID_ARG, "tau inf");
    bad |= expect(mbo_plan(&p, 2, N, 3, 1, 1e-3, (mbo_precision)7, 0.0, nullptr), MBO_ERR_INVALID_ARG, "prec");
    bad |= expect(mbo_plan(&p, 2, Nodd, 3, 1, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_UNSUPPORTED, "N = 48");
    bad |= expect(mbo_plan(&p, 2, Nbig, 3, 1, 1e-3, MBO_F64, 0.0, nullptr), MBO_ERR_UNSUPPORTED, "N = 4096");
    if (p) bad |= 1;
    mbo_field_desc descs[2];
    std::memset(descs, 0, sizeof descs);
    descs[0].d = 2; descs[0].N[0] = 32; descs[0].N[1] = 32; descs[0].n = 3; descs[0].tau = 1e-3;
    descs[1] = descs[0];
    descs[1].n = 9;
    bad |= expect(mbo_plan_batched(&p, 2, descs, MBO_F32, 0.0, 0, nullptr), MBO_ERR_INVALID_ARG, "batched n = 9");
    bad |= expect(mbo_plan_batched(&p, 0, descs, MBO_F32, 0.0, 0, nullptr), MBO_ERR_INVALID_ARG, "batched count");
    bad |= expect(mbo_plan_batched(nullptr, 1, descs, MBO_F32, 0.0, 0, nullptr), MBO_ERR_INVALID_ARG, "batched out");
    // every call on a NULL plan is refused without touching the device
    double e = 0.0, r = 0.0, h = 0.0;
    int it = 0, l = 0, a = 0, b = 0, c = 0;
    int64_t fb = 0, nf = 0;
    bad |= expect(mbo_plan_destroy(nullptr), MBO_OK, "destroy NULL");
    bad |= expect(mbo_plan_set_tau(nullptr, 1e-3), MBO_ERR_INVALID_ARG, "set_tau");
    bad |= expect(mbo_plan_set_stream(nullptr, nullptr), MBO_ERR_INVALID_ARG, "set_stream");
    bad |= expect(mbo_plan_set_timing(nullptr, 1), MBO_ERR_INVALID_ARG, "set_timing");
    bad |= expect(mbo_plan_set_path(nullptr, MBO_PATH_FULL), MBO_ERR_INVALID_ARG, "set_path");
    bad |= expect(mbo_plan_path(nullptr, 0, &a, &b, &c), MBO_ERR_INVALID_ARG, "path");
    bad |= expect(mbo_last_timing(nullptr, &r, &h, &l), MBO_ERR_INVALID_ARG, "last_timing");
    bad |= expect(mbo_last_project_counts(nullptr, &fb, &nf), MBO_ERR_INVALID_ARG, "project counts");
    bad |= expect(mbo_diffuse(nullptr, &e, &e), MBO_ERR_INVALID_ARG, "diffuse");
    bad |= expect(mbo_project(nullptr, &e, &e, nullptr), MBO_ERR_INVALID_ARG, "project");
    bad |= expect(mbo_iterate(nullptr, &e, 3, 0.0, &it, nullptr, nullptr, nullptr, nullptr), MBO_ERR_INVALID_ARG,
                  "iterate");
    bad |= expect(mbo_energy(nullptr, &e, &e), MBO_ERR_INVALID_ARG, "energy");
    bad |= expect(mbo_plan_autotune(nullptr), MBO_ERR_INVALID_ARG, "autotune");
    bad |= expect(mbo_plan_tuning(nullptr, 0, &a, &b, &c, &l), MBO_ERR_INVALID_ARG, "tuning");
    for (int s = 0; s <= 6; ++s)
        if (!mbo_status_string((mbo_status)s) || !*mbo_status_string((mbo_status)s)) bad |= 1;
    if (!mbo_last_error(nullptr)) bad |= 1;
    std::printf("abi driver done bad=%d\n", bad);
    return bad;
}
