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

namespace dect {
namespace {

template <typename T>
struct Group {
    std::vector<int> slices;       // indices into the batch, in launch order
    std::vector<SliceJob<T>> jobs;
    JobArrays<T> dev{};
    void* mem = nullptr;           // device storage of dev
};

template <typename T>
bool same_shape(const SliceJob<T>& a, const SliceJob<T>& b) {
    return a.N == b.N && a.M == b.M && a.sym == b.sym && a.bp_gx == b.bp_gx &&
           a.bp_gy == b.bp_gy && a.pj_gx == b.pj_gx && a.pj_gy == b.pj_gy &&
           a.prj.nx == b.prj.nx && a.prj.ny == b.prj.ny;
}

// Copy the argument blocks of a group to one device allocation.
template <typename T>
hipError_t upload(Group<T>& g) {
    const size_t n = g.jobs.size();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_orb = take(n * sizeof(OrbitArgs<T>)), o_prj = take(n * sizeof(ProjArgs<T>)),
                 o_rhs = take(n * sizeof(BpArgs<T>)), o_q = take(n * sizeof(BpArgs<T>)),
                 o_dual = take(n * sizeof(BpArgs<T>)), o_udm = take(n * sizeof(UdmArgs<T>)),
                 o_vec = take(n * sizeof(VecArgs<T>)), o_tv = take(n * sizeof(TvArgs<T>)),
                 o_resc = take(n * sizeof(RescaleArgs<T>)), o_red = take(n * sizeof(RedArgs));
    std::vector<char> h(off, 0);
    for (size_t k = 0; k < n; ++k) {
        const SliceJob<T>& J = g.jobs[k];
        std::memcpy(&h[o_orb + k * sizeof(J.orb)], &J.orb, sizeof(J.orb));
        std::memcpy(&h[o_prj + k * sizeof(J.prj)], &J.prj, sizeof(J.prj));
        std::memcpy(&h[o_rhs + k * sizeof(J.rhs)], &J.rhs, sizeof(J.rhs));
        std::memcpy(&h[o_q + k * sizeof(J.q)], &J.q, sizeof(J.q));
        std::memcpy(&h[o_dual + k * sizeof(J.dual)], &J.dual, sizeof(J.dual));
        std::memcpy(&h[o_udm + k * sizeof(J.udm)], &J.udm, sizeof(J.udm));
        std::memcpy(&h[o_vec + k * sizeof(J.vec)], &J.vec, sizeof(J.vec));
        std::memcpy(&h[o_tv + k * sizeof(J.tv)], &J.tv, sizeof(J.tv));
        std::memcpy(&h[o_resc + k * sizeof(J.resc)], &J.resc, sizeof(J.resc));
        std::memcpy(&h[o_red + k * sizeof(J.red)], &J.red, sizeof(J.red));
    }
    hipError_t e = hipMalloc(&g.mem, off);
    if (e != hipSuccess) return e;
    e = hipMemcpy(g.mem, h.data(), off, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    char* b = static_cast<char*>(g.mem);
    g.dev.orb = reinterpret_cast<OrbitArgs<T>*>(b + o_orb);
    g.dev.prj = reinterpret_cast<ProjArgs<T>*>(b + o_prj);
    g.dev.rhs = reinterpret_cast<BpArgs<T>*>(b + o_rhs);
    g.dev.q = reinterpret_cast<BpArgs<T>*>(b + o_q);
    g.dev.dual = reinterpret_cast<BpArgs<T>*>(b + o_dual);
    g.dev.udm = reinterpret_cast<UdmArgs<T>*>(b + o_udm);
    g.dev.vec = reinterpret_cast<VecArgs<T>*>(b + o_vec);
    g.dev.tv = reinterpret_cast<TvArgs<T>*>(b + o_tv);
    g.dev.resc = reinterpret_cast<RescaleArgs<T>*>(b + o_resc);
    g.dev.red = reinterpret_cast<RedArgs*>(b + o_red);
    return hipSuccess;
}

}  // namespace
}  // namespace dect

using namespace dect;

struct dect_batch {
    dect_dtype dtype;
    int n = 0;
    int device = 0;
    dect_params prm{};
    bool use_graph = false;
    std::vector<Group<float>> gf;
    std::vector<Group<double>> gd;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~dect_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        for (auto& g : gf)
            if (g.mem) (void)hipFree(g.mem);
        for (auto& g : gd)
            if (g.mem) (void)hipFree(g.mem);
    }

    template <typename T>
    std::vector<Group<T>>& groups();

    // One outer iteration of every group, enqueued on s.
    template <typename T>
    hipError_t enqueue(hipStream_t s) {
        for (const Group<T>& g : groups<T>()) {
            hipError_t e = launch_iteration<T>(g.jobs[0], &g.dev, (int)g.jobs.size(), &prm, 0, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t enqueue(hipStream_t s) {
        return dtype == DECT_F32 ? enqueue<float>(s) : enqueue<double>(s);
    }
};

template <>
std::vector<Group<float>>& dect_batch::groups<float>() { return gf; }
template <>
std::vector<Group<double>>& dect_batch::groups<double>() { return gd; }

namespace {

template <typename T>
dect_status build_groups(dect_batch* b, const dect_plan* const* plans, const void* const* mh,
                         const void* const* ml, const void* const* wh, const void* const* wl,
                         void* const* states) {
    std::vector<Group<T>>& G = b->groups<T>();
    for (int k = 0; k < b->n; ++k) {
        const SliceJob<T> J = make_job<T>(plans[k], mh[k], ml[k], wh[k], wl[k], states[k], &b->prm);
        Group<T>* into = nullptr;
        for (auto& g : G)
            if (same_shape(g.jobs[0], J)) into = &g;
        if (!into) {
            G.emplace_back();
            into = &G.back();
        }
        into->slices.push_back(k);
        into->jobs.push_back(J);
    }
    for (auto& g : G) {
        hipError_t e = upload<T>(g);
        if (e != hipSuccess)
            return fail(DECT_E_DEVICE, "batch argument upload failed: %s", hipGetErrorString(e));
    }
    return DECT_OK;
}

dect_status check_batch_params(const dect_params* prm) {
    if (!prm) return fail(DECT_E_ARG, "null params");
    if (prm->lm_iters < 1 || prm->cg_iters < 1)
        return fail(DECT_E_ARG, "lm_iters and cg_iters must be >= 1");
    if (prm->rho_mode != DECT_RHO_FIXED && prm->rho_mode != DECT_RHO_ADAPTIVE)
        return fail(DECT_E_ARG, "a batch runs fixed or adaptive rho (got mode %d)", prm->rho_mode);
    if (prm->rho_mode == DECT_RHO_ADAPTIVE && (!(prm->bal_mu > 1) || !(prm->bal_tau > 1)))
        return fail(DECT_E_ARG, "residual balancing needs mu > 1 and tau > 1");
    if (!(prm->lm_mu0 > 0)) return fail(DECT_E_ARG, "lm_mu0 must be > 0");
    return DECT_OK;
}

}  // namespace

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
        if (reinterpret_cast<uintptr_t>(states[k]) % 256)
            return fail(DECT_E_ARG, "state of slice %d is not 256-byte aligned", k);
        for (int j = 0; j < k; ++j)
            if (states[j] == states[k]) return fail(DECT_E_ARG, "slices %d and %d share a state", j, k);
    }
    std::unique_ptr<dect_batch> b(new (std::nothrow) dect_batch());
    if (!b) return fail(DECT_E_NOMEM, "out of host memory");
    b->dtype = plans[0]->dtype;
    b->n = n;
    b->prm = *params;
    b->prm.rho_schedule = nullptr;
    b->prm.rho_schedule_len = 0;
    b->use_graph = use_graph != 0;
    DECT_HIP(hipGetDevice(&b->device));
    st = b->dtype == DECT_F32 ? build_groups<float>(b.get(), plans, m_h, m_l, w_h, w_l, states)
                              : build_groups<double>(b.get(), plans, m_h, m_l, w_h, w_l, states);
    if (st) return st;
    *out = b.release();
    return DECT_OK;
}

dect_status dect_batch_iterate(dect_batch* b, int n_iters, void* stream) {
    if (!b) return fail(DECT_E_ARG, "null batch");
    if (n_iters < 0) return fail(DECT_E_ARG, "n_iters must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Direct launches when timing per kernel (the events bracket each launch).
    if (!b->use_graph || prof_enabled()) {
        for (int k = 0; k < n_iters; ++k) {
            hipError_t e = b->enqueue(s);
            if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
        }
        return DECT_OK;
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
    return DECT_OK;
}

int dect_batch_groups(const dect_batch* b) {
    if (!b) return 0;
    return b->dtype == DECT_F32 ? (int)b->gf.size() : (int)b->gd.size();
}

void dect_batch_destroy(dect_batch* b) { delete b; }

}  // extern "C"
