// Several slices advanced together: one launch per kernel per shape group, each
// launch covering every slice of the group through blockIdx.z, and optionally
// one outer iteration of all groups replayed from a HIP graph.
//
// Slices are independent problems (one per detector row or table position); a
// slice's kernels read only its own argument block, so its result does not
// depend on which other slices share the launches.
#include <cstring>
#include <memory>

#include "common.h"
#include "kernels.h"
#include "profile.h"
#include "runner.h"

namespace dect {

namespace {

template <typename T>
bool same_shape(const SliceJob<T>& a, const SliceJob<T>& b) {
    return a.N == b.N && a.M == b.M && a.sym == b.sym && a.bp_gx == b.bp_gx &&
           a.bp_gy == b.bp_gy && a.pj_gx == b.pj_gx && a.pj_gy == b.pj_gy &&
           a.prj.nx == b.prj.nx && a.prj.ny == b.prj.ny && a.cg_iters == b.cg_iters &&
           a.rho_mode == b.rho_mode && a.bp_waves == b.bp_waves && a.pj_waves == b.pj_waves &&
           a.pj_views == b.pj_views && a.pj_chunk == b.pj_chunk &&
           a.precond == b.precond && a.rt_sums64 == b.rt_sums64 &&
           (a.udm.joint_lim > 0.0f) == (b.udm.joint_lim > 0.0f);
}

// Byte offsets of the ten argument arrays of a group of n slices.
template <typename T>
struct ArrayOffsets {
    size_t orb, prj, rhs, q, dual, udm, vec, resc, red, pre0, pre1, end;
    ArrayOffsets(size_t base, size_t n) {
        size_t off = base;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off = (off + bytes + 255) & ~size_t(255);
            return o;
        };
        orb = take(n * sizeof(OrbitArgs<T>));
        prj = take(n * sizeof(ProjArgs<T>));
        rhs = take(n * sizeof(BpArgs<T>));
        q = take(n * sizeof(BpArgs<T>));
        dual = take(n * sizeof(BpArgs<T>));
        udm = take(n * sizeof(UdmArgs<T>));
        vec = take(n * sizeof(VecArgs<T>));
        resc = take(n * sizeof(RescaleArgs<T>));
        red = take(n * sizeof(RedArgs));
        pre0 = take(n * sizeof(PrecArgs<T>));
        pre1 = take(n * sizeof(PrecArgs<T>));
        end = off;
    }
};

template <typename F>
void put(std::vector<char>& h, size_t at, size_t k, const F& v) {
    std::memcpy(&h[at + k * sizeof(F)], &v, sizeof(F));
}

}  // namespace

template <typename T>
Runner<T>::~Runner() {
    if (mem_) (void)hipFree(mem_);
}

template <typename T>
hipError_t Runner<T>::set(const std::vector<SliceJob<T>>& jobs) {
    groups_.clear();
    n_ = (int)jobs.size();
    for (const SliceJob<T>& J : jobs) {
        Group* into = nullptr;
        for (auto& g : groups_)
            if (same_shape(g.jobs[0], J)) into = &g;
        if (!into) {
            groups_.emplace_back();
            into = &groups_.back();
        }
        into->jobs.push_back(J);
    }
    size_t total = 0;
    std::vector<ArrayOffsets<T>> offs;
    for (const Group& g : groups_) {
        offs.emplace_back(total, g.jobs.size());
        total = offs.back().end;
    }
    if (total == 0) return hipSuccess;
    if (total > cap_) {
        if (mem_) {
            hipError_t e = hipFree(mem_);
            mem_ = nullptr;
            cap_ = 0;
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipMalloc(&mem_, total);
        if (e != hipSuccess) return e;
        cap_ = total;
    }
    std::vector<char> h(total, 0);
    char* b = static_cast<char*>(mem_);
    for (size_t gi = 0; gi < groups_.size(); ++gi) {
        Group& g = groups_[gi];
        const ArrayOffsets<T>& o = offs[gi];
        for (size_t k = 0; k < g.jobs.size(); ++k) {
            const SliceJob<T>& J = g.jobs[k];
            put(h, o.orb, k, J.orb);
            put(h, o.prj, k, J.prj);
            put(h, o.rhs, k, J.rhs);
            put(h, o.q, k, J.q);
            put(h, o.dual, k, J.dual);
            put(h, o.udm, k, J.udm);
            put(h, o.vec, k, J.vec);
            put(h, o.resc, k, J.resc);
            put(h, o.red, k, J.red);
            put(h, o.pre0, k, J.pre0);
            put(h, o.pre1, k, J.pre1);
        }
        g.dev.orb = reinterpret_cast<OrbitArgs<T>*>(b + o.orb);
        g.dev.prj = reinterpret_cast<ProjArgs<T>*>(b + o.prj);
        g.dev.rhs = reinterpret_cast<BpArgs<T>*>(b + o.rhs);
        g.dev.q = reinterpret_cast<BpArgs<T>*>(b + o.q);
        g.dev.dual = reinterpret_cast<BpArgs<T>*>(b + o.dual);
        g.dev.udm = reinterpret_cast<UdmArgs<T>*>(b + o.udm);
        g.dev.vec = reinterpret_cast<VecArgs<T>*>(b + o.vec);
        g.dev.resc = reinterpret_cast<RescaleArgs<T>*>(b + o.resc);
        g.dev.red = reinterpret_cast<RedArgs*>(b + o.red);
        g.dev.pre0 = reinterpret_cast<PrecArgs<T>*>(b + o.pre0);
        g.dev.pre1 = reinterpret_cast<PrecArgs<T>*>(b + o.pre1);
    }
    return hipMemcpy(mem_, h.data(), total, hipMemcpyHostToDevice);
}

template <typename T>
hipError_t Runner<T>::enqueue(hipStream_t s) const {
    for (const Group& g : groups_) {
        // The launch structure comes from the group; every other parameter is in the
        // slices' own argument blocks and device scalars.
        dect_params prm{};
        prm.cg_iters = g.jobs[0].cg_iters;
        prm.rho_mode = g.jobs[0].rho_mode;
        prm.precond = g.jobs[0].precond;
        prm.rt_sums = g.jobs[0].rt_sums64 ? DECT_RT_SUMS_F64 : DECT_RT_SUMS_PLAN;
        hipError_t e = launch_iteration<T>(g.jobs[0], &g.dev, (int)g.jobs.size(), &prm, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t Runner<T>::settle(hipStream_t s) const {
    for (const Group& g : groups_) {
        hipError_t e = launch_settle<T>(g.jobs[0], &g.dev, (int)g.jobs.size(), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template class Runner<float>;
template class Runner<double>;

}  // namespace dect

using namespace dect;

struct dect_batch {
    dect_dtype dtype;
    int device = 0;
    dect_params prm{};
    bool use_graph = false;
    Runner<float> rf;
    Runner<double> rd;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~dect_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
    hipError_t settle(hipStream_t s) {
        return dtype == DECT_F32 ? rf.settle(s) : rd.settle(s);
    }
    hipError_t enqueue(hipStream_t s) {
        return dtype == DECT_F32 ? rf.enqueue(s) : rd.enqueue(s);
    }
};

namespace {

template <typename T>
dect_status build_groups(Runner<T>& r, int n, const dect_params* prm,
                         const dect_plan* const* plans, const void* const* mh,
                         const void* const* ml, const void* const* wh, const void* const* wl,
                         void* const* states) {
    std::vector<SliceJob<T>> jobs;
    for (int k = 0; k < n; ++k)
        jobs.push_back(make_job<T>(plans[k], mh[k], ml[k], wh[k], wl[k], states[k], prm));
    hipError_t e = r.set(jobs);
    if (e != hipSuccess)
        return fail(DECT_E_DEVICE, "batch argument upload failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

}  // namespace

namespace dect {

dect_status check_batch_params(const dect_params* prm) {
    if (!prm) return fail(DECT_E_ARG, "null params");
    if (prm->lm_iters < 1 || prm->cg_iters < 1)
        return fail(DECT_E_ARG, "lm_iters and cg_iters must be >= 1");
    if (prm->rho_mode != DECT_RHO_FIXED && prm->rho_mode != DECT_RHO_ADAPTIVE)
        return fail(DECT_E_ARG, "a batch runs fixed or adaptive rho (got mode %d)", prm->rho_mode);
    if (prm->rho_mode == DECT_RHO_ADAPTIVE && (!(prm->bal_mu > 1) || !(prm->bal_tau > 1)))
        return fail(DECT_E_ARG, "residual balancing needs mu > 1 and tau > 1");
    if (!(prm->lm_mu0 > 0)) return fail(DECT_E_ARG, "lm_mu0 must be > 0");
    if (!(prm->rho_c > 0) || !(prm->rho_p > 0) || !(prm->lambda_c >= 0) || !(prm->lambda_p >= 0))
        return fail(DECT_E_ARG, "rho must be > 0 and lambda >= 0");
    if (prm->precond != DECT_PRECOND_NONE && prm->precond != DECT_PRECOND_RAMP)
        return fail(DECT_E_ARG, "bad precond %d", prm->precond);
    if (prm->rt_sums != DECT_RT_SUMS_PLAN && prm->rt_sums != DECT_RT_SUMS_F64)
        return fail(DECT_E_ARG, "bad rt_sums %d", prm->rt_sums);
    return DECT_OK;
}

}  // namespace dect

extern "C" {

dect_status dect_batch_create(int n, const dect_plan* const* plans, const void* const* m_h,
                              const void* const* m_l, const void* const* w_h,
                              const void* const* w_l, void* const* states,
                              const dect_params* params, int use_graph, dect_batch** out) {
    if (!out) return fail(DECT_E_ARG, "null output pointer");
    *out = nullptr;
    if (n < 1) return fail(DECT_E_ARG, "a batch needs at least one slice (got %d)", n);
    if (!plans || !m_h || !m_l || !w_h || !w_l || !states) return fail(DECT_E_ARG, "null argument");
    dect_status st = check_batch_params(params);
    if (st) return st;
    for (int k = 0; k < n; ++k) {
        if (!plans[k] || !m_h[k] || !m_l[k] || !w_h[k] || !w_l[k] || !states[k])
            return fail(DECT_E_ARG, "null entry for slice %d", k);
        if (plans[k]->dtype != plans[0]->dtype)
            return fail(DECT_E_ARG, "slice %d has another precision than slice 0", k);
        if (params->precond && !plans[k]->has_precond)
            return fail(DECT_E_SHAPE, "slice %d: no preconditioner for its image size", k);
        if (reinterpret_cast<uintptr_t>(states[k]) % 256)
            return fail(DECT_E_ARG, "state of slice %d is not 256-byte aligned", k);
        for (int j = 0; j < k; ++j)
            if (states[j] == states[k]) return fail(DECT_E_ARG, "slices %d and %d share a state", j, k);
    }
    std::unique_ptr<dect_batch> b(new (std::nothrow) dect_batch());
    if (!b) return fail(DECT_E_NOMEM, "out of host memory");
    b->dtype = plans[0]->dtype;
    b->prm = *params;
    b->prm.rho_schedule = nullptr;
    b->prm.rho_schedule_len = 0;
    b->use_graph = use_graph != 0;
    DECT_HIP(hipGetDevice(&b->device));
    st = b->dtype == DECT_F32
             ? build_groups<float>(b->rf, n, &b->prm, plans, m_h, m_l, w_h, w_l, states)
             : build_groups<double>(b->rd, n, &b->prm, plans, m_h, m_l, w_h, w_l, states);
    if (st) return st;
    *out = b.release();
    return DECT_OK;
}

dect_status dect_batch_iterate(dect_batch* b, int n_iters, void* stream) {
    if (!b) return fail(DECT_E_ARG, "null batch");
    if (n_iters < 0) return fail(DECT_E_ARG, "n_iters must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Direct launches when timing per kernel (the events bracket each launch).
    // The states' duals hold their scaled values between calls.
    auto settle = [&]() -> dect_status {
        if (n_iters == 0) return DECT_OK;
        const hipError_t e = b->settle(s);
        return e == hipSuccess ? DECT_OK
                               : fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    };
    if (!b->use_graph || prof_enabled()) {
        for (int k = 0; k < n_iters; ++k) {
            hipError_t e = b->enqueue(s);
            if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
        }
        return settle();
    }
    if (!b->exec) {
        // Capture one outer iteration of every group on a private stream (a capture
        // needs a stream other than the null stream), then replay it on s.
        if (!b->cap) DECT_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        DECT_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = b->enqueue(b->cap);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(DECT_E_DEVICE, "graph capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        b->graph = g;
        DECT_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    for (int k = 0; k < n_iters; ++k) DECT_HIP(hipGraphLaunch(b->exec, s));
    return settle();
}

int dect_batch_groups(const dect_batch* b) {
    if (!b) return 0;
    return b->dtype == DECT_F32 ? b->rf.groups() : b->rd.groups();
}

void dect_batch_destroy(dect_batch* b) { delete b; }

}  // extern "C"
