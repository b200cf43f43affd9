// Workgroup shapes of the ADMM transpose and projector, chosen per plan by timing
// every candidate on the device, with a text cache keyed by device, precision and
// problem shape.
//
// Both kernels read every value they need whatever the shape; the shape changes
// only how a workgroup's waves share the views (transpose) or the lines
// (projector), i.e. the order in which partial sums are added.  Slices share
// batched launches only when their plans' shapes agree.
#include <cstdio>
#include <cstring>
#include <string>

#include "common.h"
#include "kernels.h"

namespace dect {
namespace {

constexpr int kCandidates[] = {2, 4, 8};

bool valid_waves(int w) { return w == 2 || w == 4 || w == 8; }

dect_status cache_key(const dect_plan* p, std::string& key) {
    hipDeviceProp_t prop;
    DECT_HIP(hipGetDeviceProperties(&prop, p->device));
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s:%s:%s:%dx%d:%dx%d:sym%d", prop.gcnArchName,
                  p->dtype == DECT_F32 ? "f32" : "f64",
                  p->geom.kind == DECT_FAN ? "fan" : "parallel", p->nx, p->ny, p->V, p->D, p->sym);
    for (char* c = buf; *c; ++c)
        if (*c == ' ') *c = '_';
    key = buf;
    return DECT_OK;
}

// The last entry of the cache for `key`, if any.
bool cache_lookup(const char* path, const std::string& key, dect_launch& out) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512], k[300];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        dect_launch e{};
        if (line[0] == '#') continue;
        if (std::sscanf(line, "%299s %d %d %lf %lf", k, &e.bp_waves, &e.proj_waves, &e.bp_us,
                        &e.proj_us) == 5 &&
            key == k && valid_waves(e.bp_waves) && valid_waves(e.proj_waves)) {
            out = e;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

template <typename T>
dect_status time_candidates(dect_plan* p, hipStream_t s, dect_launch& out) {
    void* st = nullptr;
    DECT_HIP(hipMalloc(&st, p->layout.bytes));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    dect_status rc = DECT_OK;
    auto done = [&](dect_status r) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(st);
        return r;
    };
    if (hipMemsetAsync(st, 0, p->layout.bytes, s) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return done(fail(DECT_E_DEVICE, "tuning setup failed"));
    dect_params prm{};
    prm.cg_iters = 1;
    prm.lm_iters = 1;
    prm.rho_mode = DECT_RHO_ADAPTIVE;
    // The measurement pointers only fill the decomposition's arguments, which
    // the timed kernels do not read.
    const SliceJob<T> J = make_job<T>(p, st, st, st, st, st, &prm);
    constexpr int reps = 5;
    auto timed = [&](auto&& launch, double& us) -> dect_status {
        if (launch() != hipSuccess) return fail(DECT_E_DEVICE, "tuning launch failed");
        DECT_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r)
            if (launch() != hipSuccess) return fail(DECT_E_DEVICE, "tuning launch failed");
        DECT_HIP(hipEventRecord(e1, s));
        DECT_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        DECT_HIP(hipEventElapsedTime(&ms, e0, e1));
        us = 1e3 * ms / reps;
        return DECT_OK;
    };
    out.bp_us = out.proj_us = 1e300;
    for (int w : kCandidates) {
        double us = 0.0;
        rc = timed([&] { return launch_backproject_admm<T>(J.sym, w, EPI_Q, nullptr, J.q, 1,
                                                           J.bp_gx, J.bp_gy, s); }, us);
        if (rc) return done(rc);
        if (us < out.bp_us) {
            out.bp_us = us;
            out.bp_waves = w;
        }
        rc = timed([&] { return launch_project_pair<T>(J.sym, w, nullptr, J.orb, nullptr, J.prj, 1,
                                                       J.N, J.pj_gx, J.pj_gy, s); }, us);
        if (rc) return done(rc);
        if (us < out.proj_us) {
            out.proj_us = us;
            out.proj_waves = w;
        }
    }
    return done(DECT_OK);
}

}  // namespace
}  // namespace dect

using namespace dect;

extern "C" {

dect_status dect_plan_set_launch(dect_plan* p, int bp_waves, int proj_waves) {
    if (!p) return fail(DECT_E_ARG, "null plan");
    if (!valid_waves(bp_waves) || !valid_waves(proj_waves))
        return fail(DECT_E_ARG, "waves per workgroup must be 2, 4 or 8 (got %d, %d)", bp_waves,
                    proj_waves);
    p->bp_waves = bp_waves;
    p->pj_waves = proj_waves;
    return DECT_OK;
}

dect_status dect_plan_get_launch(const dect_plan* p, dect_launch* out) {
    if (!p || !out) return fail(DECT_E_ARG, "null argument");
    std::memset(out, 0, sizeof *out);
    out->bp_waves = p->bp_waves;
    out->proj_waves = p->pj_waves;
    return DECT_OK;
}

dect_status dect_plan_tune(dect_plan* p, const char* cache_path, int flags, dect_launch* out,
                           void* stream) {
    if (!p) return fail(DECT_E_ARG, "null plan");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::string key;
    dect_status rc = cache_key(p, key);
    if (rc) return rc;
    dect_launch best{};
    if (cache_path && !(flags & DECT_TUNE_FORCE) && cache_lookup(cache_path, key, best)) {
        best.from_cache = 1;
    } else {
        rc = p->dtype == DECT_F32 ? time_candidates<float>(p, s, best)
                                  : time_candidates<double>(p, s, best);
        if (rc) return rc;
        if (cache_path) {
            FILE* f = std::fopen(cache_path, "a");
            if (!f) return fail(DECT_E_ARG, "cannot append to tuning cache %s", cache_path);
            std::fprintf(f, "%s %d %d %.3f %.3f\n", key.c_str(), best.bp_waves, best.proj_waves,
                         best.bp_us, best.proj_us);
            std::fclose(f);
        }
    }
    p->bp_waves = best.bp_waves;
    p->pj_waves = best.proj_waves;
    if (out) *out = best;
    return DECT_OK;
}

}  // extern "C"
