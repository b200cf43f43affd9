// Workgroup shapes of the ADMM transpose and projector, chosen per plan by timing
// every candidate on the device, with a text cache keyed by device, precision and
// problem shape.
//
// Both kernels read every value they need whatever the shape; the shape changes
// only how a workgroup's waves share the views (transpose) or the lines
// (projector), i.e. the order in which partial sums are added.  Slices share
// batched launches only when their plans' shapes agree.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

#include "common.h"
#include "kernels.h"

namespace dect {
namespace {

constexpr int kWaves[] = {2, 4, 8};
constexpr int kViews[] = {1, 2, 4};
constexpr int kChunks[] = {1, 2, 4};
// The shapes used when nothing has been tuned (measured best at 512^2 / 720 x 1024).
constexpr int kBpDefault = 4, kPjDefault = 8;
// Timed repetitions: kBatches batches of kReps launches; a candidate's time is its
// median batch average, its spread (max - min) / min over the batches.
constexpr int kBatches = 3, kReps = 8;

bool valid_waves(int w) { return w == 2 || w == 4 || w == 8; }
bool valid_views(int v) { return v == 1 || v == 2 || v == 4 || v == 8; }
bool valid_chunk(int c) { return c >= 1 && c <= 16; }

dect_status cache_key(const dect_plan* p, std::string& key) {
    hipDeviceProp_t prop;
    DECT_HIP(hipGetDeviceProperties(&prop, p->device));
    char buf[256];
    std::snprintf(buf, sizeof buf, "v2:%s:%s:%s:%dx%d:%dx%d:sym%d", prop.gcnArchName,
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
        if (std::sscanf(line, "%299s %d %d %d %d %lf %lf", k, &e.bp_waves, &e.proj_waves,
                        &e.proj_views, &e.proj_chunk, &e.bp_us, &e.proj_us) == 7 &&
            key == k && valid_waves(e.bp_waves) && valid_waves(e.proj_waves) &&
            valid_views(e.proj_views) && valid_chunk(e.proj_chunk)) {
            out = e;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

struct Timing {
    double us = 1e300, spread = 0.0;
};

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
    auto timed = [&](auto&& launch, Timing& t) -> dect_status {
        for (int w = 0; w < 2; ++w)
            if (launch() != hipSuccess) return fail(DECT_E_DEVICE, "tuning launch failed");
        double avg[kBatches];
        for (int b = 0; b < kBatches; ++b) {
            DECT_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < kReps; ++r)
                if (launch() != hipSuccess) return fail(DECT_E_DEVICE, "tuning launch failed");
            DECT_HIP(hipEventRecord(e1, s));
            DECT_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            DECT_HIP(hipEventElapsedTime(&ms, e0, e1));
            avg[b] = 1e3 * ms / kReps;
        }
        std::sort(avg, avg + kBatches);
        t.us = avg[kBatches / 2];
        t.spread = (avg[kBatches - 1] - avg[0]) / avg[0];
        return DECT_OK;
    };
    // A candidate replaces the default only if it is faster by more than the larger of
    // 1 % and the two measurements' spreads.
    auto better = [](const Timing& c, const Timing& d) {
        const double margin = std::max(0.01, std::max(c.spread, d.spread));
        return c.us < d.us * (1.0 - margin);
    };
    Timing bp_def, bp_best;
    int bp_w = kBpDefault;
    for (int w : kWaves) {
        Timing t;
        rc = timed([&] { return launch_backproject_admm<T>(J.sym, w, EPI_Q, nullptr, J.q, 1,
                                                           J.bp_gx, J.bp_gy, s); }, t);
        if (rc) return done(rc);
        if (w == kBpDefault) bp_def = t;
        if (t.us < bp_best.us) {
            bp_best = t;
            bp_w = w;
        }
    }
    if (bp_w != kBpDefault && !better(bp_best, bp_def)) {
        bp_w = kBpDefault;
        bp_best = bp_def;
    }
    Timing pj_def, pj_best;
    int pj_w = kPjDefault, pj_v = kProjViewsDefault, pj_c = kProjChunkDefault;
    for (int w : kWaves)
        for (int v : kViews)
            for (int c : kChunks) {
                ProjArgs<T> a = J.prj;
                a.views = v;
                a.chunk = c;
                const int gx = proj_grid_x(p->D, v), gy = proj_grid_y(p->Vb, v);
                Timing t;
                rc = timed([&] { return launch_project_pair<T>(J.sym, w, nullptr, J.orb, nullptr, a,
                                                               1, J.N, gx, gy, s); }, t);
                if (rc) return done(rc);
                if (w == kPjDefault && v == kProjViewsDefault && c == kProjChunkDefault) pj_def = t;
                if (t.us < pj_best.us) {
                    pj_best = t;
                    pj_w = w;
                    pj_v = v;
                    pj_c = c;
                }
            }
    if ((pj_w != kPjDefault || pj_v != kProjViewsDefault || pj_c != kProjChunkDefault) &&
        !better(pj_best, pj_def)) {
        pj_w = kPjDefault;
        pj_v = kProjViewsDefault;
        pj_c = kProjChunkDefault;
        pj_best = pj_def;
    }
    out.bp_waves = bp_w;
    out.bp_us = bp_best.us;
    out.bp_us_default = bp_def.us;
    out.proj_waves = pj_w;
    out.proj_views = pj_v;
    out.proj_chunk = pj_c;
    out.proj_us = pj_best.us;
    out.proj_us_default = pj_def.us;
    return done(DECT_OK);
}

}  // namespace
}  // namespace dect

using namespace dect;

extern "C" {

dect_status dect_plan_set_launch(dect_plan* p, int bp_waves, int proj_waves, int proj_views,
                                 int proj_chunk) {
    if (!p) return fail(DECT_E_ARG, "null plan");
    if (!valid_waves(bp_waves) || !valid_waves(proj_waves))
        return fail(DECT_E_ARG, "waves per workgroup must be 2, 4 or 8 (got %d, %d)", bp_waves,
                    proj_waves);
    if (!valid_views(proj_views) || !valid_chunk(proj_chunk))
        return fail(DECT_E_ARG, "projector views per wave must be 1, 2, 4 or 8 and the chunk "
                                "1 to 16 (got %d, %d)", proj_views, proj_chunk);
    p->bp_waves = bp_waves;
    p->pj_waves = proj_waves;
    p->pj_views = proj_views;
    p->pj_chunk = proj_chunk;
    return DECT_OK;
}

dect_status dect_plan_get_launch(const dect_plan* p, dect_launch* out) {
    if (!p || !out) return fail(DECT_E_ARG, "null argument");
    std::memset(out, 0, sizeof *out);
    out->bp_waves = p->bp_waves;
    out->proj_waves = p->pj_waves;
    out->proj_views = p->pj_views;
    out->proj_chunk = p->pj_chunk;
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
            std::fprintf(f, "%s %d %d %d %d %.3f %.3f\n", key.c_str(), best.bp_waves,
                         best.proj_waves, best.proj_views, best.proj_chunk, best.bp_us,
                         best.proj_us);
            std::fclose(f);
        }
    }
    p->bp_waves = best.bp_waves;
    p->pj_waves = best.proj_waves;
    p->pj_views = best.proj_views;
    p->pj_chunk = best.proj_chunk;
    if (out) *out = best;
    return DECT_OK;
}

}  // extern "C"
