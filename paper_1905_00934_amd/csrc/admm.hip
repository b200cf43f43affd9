// One ADMM outer iteration of the splitting scheme (Sec. 3.3) on one slice:
// image-side kernels, deterministic reductions, the host driver, and the C ABI.
//
// Per outer iteration (n CG steps, m LM steps), all on the caller's stream and
// with every scalar (CG step sizes, rho, dual rescale) kept in device memory:
//   R^T t + image terms -> r0 = p0, |r0|^2          (Eq. (12) right-hand side; R^T t is
//                                                    tracked as h + u, no transpose)
//   n x { R p ; R^T R p + D^T D p + p ; alpha ;
//         except after the last: x += alpha p, h -= alpha R^T R p ; beta }
//   per-ray LM on Eq. (13) with R x += alpha R p and u^a (one lane per ray), and in
//   the same launch y, z, u^y, u^z (Eq. (9)-(11)) with their partials (one lane per
//   pixel), reading x through the pending last CG step
//   R^T da + D^T dy + dz                             (dual residual; R^T da also goes to h;
//                                                    per pixel also the last CG step
//                                                    x += alpha p, h -= alpha R^T R p,
//                                                    and u += h)
//   residuals, rho and the log                        (one workgroup)
// The dual rescale after a change of rho, kappa = rho_old / rho_new, is left pending:
// the next iteration's readers of u, u^a, u^y, u^z scale them as they read them, and
// the end of a call applies what is still pending (k_settle).
#include <cmath>
#include <cstring>

#include "common.h"
#include "epilogue.h"
#include "kernels.h"
#include "profile.h"
#include "reduce.h"

namespace dect {

namespace {

__global__ __launch_bounds__(256) void k_zero(uint32_t* p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_set_scalars(double* s, double rc, double rp, double lc, double lp) {
    if (threadIdx.x != 0) return;
    for (int k = 0; k < S_COUNT; ++k) s[k] = 0.0;
    s[S_RHO] = rc;
    s[S_RHO + 1] = rp;
    s[S_KAPPA] = 1.0;
    s[S_KAPPA + 1] = 1.0;
    s[S_LAM] = lc;
    s[S_LAM + 1] = lp;
}

// x += alpha p; with FULL also r -= alpha q and block partials of r.r.
template <typename T, bool FULL, bool BATCH>
__global__ __launch_bounds__(256) void k_cg_step(const VecArgs<T>* __restrict__ dev, VecArgs<T> one) {
    using V2 = vec<T, 2>;
    const VecArgs<T> A = pick_args<BATCH>(dev, one);
    if ((long)blockIdx.x * blockDim.x >= A.N) return;  // beyond this slice (whole block)
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const T al[2] = {(T)A.scal[S_ALPHA], (T)A.scal[S_ALPHA + 1]};
    double part[2] = {0.0, 0.0};
    if (i < A.N) {
        V2 xv = reinterpret_cast<V2*>(A.x)[i];
        const V2 pv = reinterpret_cast<const V2*>(A.p)[i];
#pragma unroll
        for (int c = 0; c < 2; ++c) xv.v[c] = fma(al[c], pv.v[c], xv.v[c]);
        reinterpret_cast<V2*>(A.x)[i] = xv;
        // R x moves by alpha R p, so the tracked R^T (a - R x) by -alpha R^T R p.
        const V2 rr = reinterpret_cast<const V2*>(A.rtrp)[i];
#pragma unroll
        for (int c = 0; c < 2; ++c)
            A.h[2 * i + c] = fma(-A.scal[S_ALPHA + c], (double)rr.v[c], A.h[2 * i + c]);
        if constexpr (FULL) {
            V2 rv = reinterpret_cast<V2*>(A.r)[i];
            const V2 qv = reinterpret_cast<const V2*>(A.q)[i];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                rv.v[c] -= al[c] * qv.v[c];
                part[c] = (double)rv.v[c] * (double)rv.v[c];
            }
            reinterpret_cast<V2*>(A.r)[i] = rv;
        }
    }
    if constexpr (FULL) block_sum_store<2>(part, A.partials + (size_t)blockIdx.x * kPartialSlots);
}

// R x += alpha R p (tracking, so no extra projection of x is needed).
template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_rx_step(const VecArgs<T>* __restrict__ dev, VecArgs<T> one) {
    using V2 = vec<T, 2>;
    const VecArgs<T> A = pick_args<BATCH>(dev, one);
    const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= A.M) return;
    const long i = std_ray(l, A.sym, A.Vb, A.D);
    V2 a = reinterpret_cast<V2*>(A.Rx)[i];
    const V2 b = reinterpret_cast<const V2*>(A.Rp)[l];
    a.v[0] += (T)A.scal[S_ALPHA] * b.v[0];
    a.v[1] += (T)A.scal[S_ALPHA + 1] * b.v[1];
    reinterpret_cast<V2*>(A.Rx)[i] = a;
}

// p = z + beta p (z = r for plain CG, M r for PCG).
template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_p_step(const VecArgs<T>* __restrict__ dev, VecArgs<T> one) {
    using V2 = vec<T, 2>;
    const VecArgs<T> A = pick_args<BATCH>(dev, one);
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.N) return;
    V2 a = reinterpret_cast<V2*>(A.p)[i];
    const V2 b = reinterpret_cast<const V2*>(A.zp)[i];
    a.v[0] = b.v[0] + (T)A.scal[S_BETA] * a.v[0];
    a.v[1] = b.v[1] + (T)A.scal[S_BETA + 1] * a.v[1];
    reinterpret_cast<V2*>(A.p)[i] = a;
}

// The pending dual rescale kappa = rho_old / rho_new applied to the stored duals:
// u (R^T u^a), u^a, u^y, u^z.  Every element is scaled as its reader in the next
// iteration would scale it, so the iterations continue bitwise as without it.
template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_settle(const RescaleArgs<T>* __restrict__ dev,
                                                RescaleArgs<T> one) {
    using V2 = vec<T, 2>;
    using V4 = vec<T, 4>;
    const RescaleArgs<T> A = pick_args<BATCH>(dev, one);
    const long M = A.M, N = A.N;
    if ((long)blockIdx.x * blockDim.x >= (M > N ? M : N)) return;
    const double k0 = A.scal[S_KAPPA], k1 = A.scal[S_KAPPA + 1];
    if (k0 == 1.0 && k1 == 1.0) return;
    const T kc[2] = {(T)k0, (T)k1};
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) {
        V2 u = reinterpret_cast<V2*>(A.ua)[i];
#pragma unroll
        for (int c = 0; c < 2; ++c) u.v[c] = mul_rn(kc[c], u.v[c]);
        reinterpret_cast<V2*>(A.ua)[i] = u;
    }
    if (i < N) {
        A.u[2 * i] = mul_rn(k0, A.u[2 * i]);
        A.u[2 * i + 1] = mul_rn(k1, A.u[2 * i + 1]);
        V4 u4 = reinterpret_cast<V4*>(A.uy)[i];
#pragma unroll
        for (int k = 0; k < 4; ++k) u4.v[k] = mul_rn(kc[k & 1], u4.v[k]);
        reinterpret_cast<V4*>(A.uy)[i] = u4;
        V2 u2 = reinterpret_cast<V2*>(A.uz)[i];
        u2.v[0] = mul_rn(kc[0], u2.v[0]);
        u2.v[1] = mul_rn(kc[1], u2.v[1]);
        reinterpret_cast<V2*>(A.uz)[i] = u2;
    }
}

// kappa = 1 once k_settle has applied it (a launch of its own: every thread of
// k_settle reads kappa).
template <typename T, bool BATCH>
__global__ void k_settle_done(const RescaleArgs<T>* __restrict__ dev, RescaleArgs<T> one) {
    const RescaleArgs<T> A = pick_args<BATCH>(dev, one);
    if (threadIdx.x == 0) {
        A.scal[S_KAPPA] = 1.0;
        A.scal[S_KAPPA + 1] = 1.0;
    }
}


template <bool BATCH>
__global__ __launch_bounds__(256) void k_reduce(const RedArgs* __restrict__ dev, RedArgs one,
                                                int mode) {
    const RedArgs A = pick_args<BATCH>(dev, one);
    if (mode == RED_ALPHA)
        reduce_alpha(A);
    else if (mode == RED_BETA)
        reduce_beta(A);
    else
        reduce_final(A);
}

// Initial CG residual of Eq. (12): r0 = R^T t + D^T (y + u^y - D x) + (z + u^z - x)
// with R^T t = h + u (the tracked R^T (a - R x) and R^T u^a), per pixel; block
// partials of |r0|^2 per 256 pixels.
template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_rhs(const BpArgs<T>* __restrict__ dev, BpArgs<T> one) {
    const BpArgs<T> a = pick_args<BATCH>(dev, one);
    const long N = (long)a.nx * a.ny;
    if ((long)blockIdx.x * blockDim.x >= N) return;  // beyond this slice (whole block)
    const long pix = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double part[2] = {0.0, 0.0};
    if (pix < N) {
        T res[2];
        rhs_tracked(a, (size_t)pix, res);
        int pi, pj;
        pixel_ij(pix, a.nx, pi, pj);
        epilogue<T, EPI_RHS>(a, pi, pj, res, part);
    }
    block_sum_store<2>(part, a.part_img + (size_t)blockIdx.x * kPartialSlots);
}

// The tracked right-hand side at the start: h = R^T t with t = a + u^a - R x (u^a = 0
// then, so h = R^T (a - R x)), u = 0.
__global__ __launch_bounds__(256) void k_zero_f64(double* __restrict__ p, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename T>
SliceJob<T> make_job(const dect_plan* p, const void* mh, const void* ml, const void* wh,
                     const void* wl, void* st, const dect_params* prm) {
    const dect_layout& L = p->layout;
    T* x = at<T>(st, L.x);
    T* y = at<T>(st, L.y);
    T* uy = at<T>(st, L.uy);
    T* z = at<T>(st, L.z);
    T* uz = at<T>(st, L.uz);
    T* a = at<T>(st, L.a);
    T* ua = at<T>(st, L.ua);
    T* Rx = at<T>(st, L.Rx);
    double* scal = at<double>(st, L.scalars);
    T* pp = at<T>(st, p->off_p);
    T* pO = at<T>(st, p->off_pO);
    T* pOT = at<T>(st, p->off_pOT);
    T* r = at<T>(st, p->off_r);
    T* q = at<T>(st, p->off_q);
    T* dy = at<T>(st, p->off_dy);
    T* dz = at<T>(st, p->off_dz);
    T* Rp = at<T>(st, p->off_Rp);
    T* t = at<T>(st, p->off_t);
    T* da = at<T>(st, p->off_da);
    T* zb = at<T>(st, p->off_z);
    double* hh = at<double>(st, p->off_h);
    double* uu = at<double>(st, p->off_u);
    T* rtrp = at<T>(st, p->off_rtrp);
    double* part = at<double>(st, p->off_partials);
    const Partials P{part, part + (size_t)p->nb_sino * kPartialSlots,
                     part + (size_t)(p->nb_sino + p->nb_img) * kPartialSlots,
                     part + (size_t)(p->nb_sino + p->nb_img + p->nb_tiles) * kPartialSlots};
    const int n = prm->cg_iters;
    const bool pre = prm->precond == DECT_PRECOND_RAMP;

    SliceJob<T> J{};
    J.cg_iters = prm->cg_iters;
    J.rho_mode = prm->rho_mode;
    J.precond = pre ? 1 : 0;
    J.rt_sums64 = prm->rt_sums == DECT_RT_SUMS_F64 ? 1 : 0;
    J.N = p->N;
    J.M = p->M;
    J.sym = p->sym;
    J.bp_waves = p->bp_waves;
    J.pj_waves = p->pj_waves;
    J.pj_views = p->pj_views;
    J.pj_chunk = p->pj_chunk;
    J.pj_gx = proj_grid_x(p->D, p->pj_views);
    J.pj_gy = proj_grid_y(p->Vb, p->pj_views);
    J.orb = OrbitArgs<T>{pp, pO, pOT, p->nx, p->ny};
    J.prj = ProjArgs<T>{static_cast<const RayParam<T>*>(p->rays), pO, pOT, Rp, p->nx, p->ny,
                        p->Vb, p->D, p->pj_views, p->pj_chunk};
    // Right-hand side of Eq. (12) and the initial CG residual.
    BpArgs<T> b{};
    fill_bp_plan<T>(p, b);
    J.bp_gx = b.gx;
    J.bp_gy = b.gy;
    b.partials = P.tiles;
    J.rhs = b;
    J.rhs.sino = t;
    // CG: p0 = r0 (and r = r0 when more steps follow); PCG: r = r0, p0 = M r0 next.
    J.rhs.out = pre ? r : pp;
    J.rhs.out2 = (!pre && n > 1) ? r : nullptr;
    J.rhs.x = x;
    J.rhs.y = y;
    J.rhs.uy = uy;
    J.rhs.z = z;
    J.rhs.uz = uz;
    // (R^T R + D^T D + I) p and p . q
    J.q = b;
    J.q.sino = Rp;
    J.q.out = n > 1 ? q : nullptr;
    J.q.x = pp;
    // Dual residual R^T da + D^T dy + dz
    J.dual = b;
    J.dual.sino = da;
    J.dual.y = dy;
    J.dual.z = dz;
    // The tracked right-hand side: the RHS kernel reads h + u, the q transpose stores
    // R^T R p, the dual transpose adds R^T da to h.
    J.rhs.h = hh;
    J.rhs.u = uu;
    J.rhs.part_img = P.img;
    J.q.raw = rtrp;
    J.dual.h = hh;
    J.rhs.scal = scal;
    // The last CG step of the iteration (x += alpha p, h -= alpha R^T R p) is applied
    // by the dual transpose's epilogue, and read through by the TV update before it;
    // the same epilogue adds the new h to u.
    J.dual.u = uu;
    J.dual.scal = scal;
    J.dual.step_x = x;
    J.dual.step_p = pp;
    J.dual.step_rtrp = rtrp;
    // The scalar steps (CG step sizes; residuals, rho and the log) run as one
    // workgroup per slice.
    J.red = RedArgs{P.tiles, p->nb_tiles, P.img, p->nb_img, P.sino, p->nb_sino, P.pre, p->nb_pre,
                    pre ? 1 : 0, scal,
                    at<double>(st, p->off_log), prm->rho_mode,
                    prm->rho_mode == DECT_RHO_ADAPTIVE ? 1 : 0, prm->bal_mu, prm->bal_tau,
                    0.0, 0.0};
    // a-update (Eq. (13)) fused with R x += alpha R p, u^a and the next t.
    UdmArgs<T>& u = J.udm;
    fill_udm_tables<T>(p, u);
    u.M = p->M;
    u.sym = p->sym;
    u.Vb = p->Vb;
    u.D = p->D;
    u.mh = static_cast<const T*>(mh);
    u.ml = static_cast<const T*>(ml);
    u.wh = static_cast<const T*>(wh);
    u.wl = static_cast<const T*>(wl);
    u.a = a;
    u.ua = ua;
    u.Rx = Rx;
    u.Rp = Rp;
    u.t = nullptr;  // R^T t is tracked in h + u
    u.da = da;
    u.fg = at<T>(st, p->off_fg);
    u.lmbits = at<uint8_t>(st, L.lm_accept);
    u.scal = scal;
    u.partials = P.sino;
    u.iters = prm->lm_iters;
    u.mu0 = prm->lm_mu0;
    J.vec = VecArgs<T>{p->N, p->M, p->sym, p->Vb, p->D, x, pp, r, pre ? zb : r, q, Rx, Rp, scal,
                       P.img, hh, rtrp, pre ? P.pre : P.img, pre ? p->nb_pre : p->nb_img,
                       P.tiles, p->nb_tiles};
    if (pre) {
        fill_precond_plan<T>(p, J.pre0);
        J.pre0.W = at<T>(st, p->off_fftw);
        J.pre0.r = r;
        J.pre0.partials = P.pre;
        J.pre1 = J.pre0;
        J.pre0.z = pp;
        J.pre1.z = zb;
    }
    J.tv = TvArgs<T>{p->nx, p->ny, x, y, uy, dy, z, uz, dz, scal, P.img, pp};
    // The TV/z/dual update runs in the a-update's launch, after its blocks.
    u.udm_blocks = (int)nblk(p->M);
    u.tv = J.tv;
    // The iterations keep R^T t tracked in h + u, not t itself (t is set at the start).
    J.resc = RescaleArgs<T>{p->M, p->N, ua, uy, uz, uu, scal};
    return J;
}

namespace {

template <typename T, bool BATCH>
hipError_t iteration_t(const SliceJob<T>& J, const JobArrays<T>* dev, int nsl,
                       const dect_params* prm, long it, hipStream_t s) {
    const int n = prm->cg_iters;
    const unsigned z = (unsigned)nsl;
    auto reduce = [&](int mode) -> hipError_t {
        RedArgs A = J.red;
        if (mode == RED_FINAL && prm->rho_mode == DECT_RHO_SCHEDULE) {
            A.next_rho_c = prm->rho_schedule[2 * (it + 1)];
            A.next_rho_p = prm->rho_schedule[2 * (it + 1) + 1];
        }
        ProfScope ps("reduce", s);
        hipLaunchKernelGGL(k_reduce<BATCH>, dim3(1, 1, z), dim3(256), 0, s,
                           dev ? dev->red : nullptr, A, mode);
        return hipGetLastError();
    };
#define DECT_TRY(e)                          \
    do {                                     \
        hipError_t e_ = (e);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)
    const dim3 gN(nblk(J.N), 1, z), gM(nblk(J.M), 1, z);
    const VecArgs<T>* dvec = dev ? dev->vec : nullptr;
    // CG (not PCG) starts from p0 = r0: on a quarter-turn symmetric slice the
    // right-hand-side kernel also writes the orbit images of r0 the projector reads.
    const bool fused = !J.precond && rhs_orbit_fits(J.sym, J.rhs.nx, J.rhs.ny);
    if (fused) {
        ProfScope ps("rhs_orbit", s);
        DECT_TRY(launch_rhs_orbit<T>(dev ? dev->rhs : nullptr, J.rhs, dev ? dev->orb : nullptr,
                                     J.orb, nsl, s));
    } else {
        // R^T t of the right-hand side is tracked (h + u), so no transpose is needed.
        ProfScope ps("rhs", s);
        hipLaunchKernelGGL((k_rhs<T, BATCH>), gN, dim3(256), 0, s, dev ? dev->rhs : nullptr,
                           J.rhs);
        DECT_TRY(hipGetLastError());
    }
    if (J.precond) DECT_TRY(launch_precond<T>(dev ? dev->pre0 : nullptr, J.pre0, nsl, s));
    for (int c = 0; c < n; ++c) {
        DECT_TRY(launch_project_pair<T>(J.sym, J.pj_waves, dev ? dev->orb : nullptr, J.orb,
                                        dev ? dev->prj : nullptr, J.prj, nsl, J.N, J.pj_gx,
                                        J.pj_gy, s, !(fused && c == 0)));
        DECT_TRY(launch_backproject_admm<T>(J.sym, J.bp_waves, EPI_Q, dev ? dev->q : nullptr, J.q,
                                            nsl, J.bp_gx, J.bp_gy, s, J.rt_sums64 != 0));
        DECT_TRY(reduce(RED_ALPHA));
        if (c < n - 1) {
            ProfScope ps("cg_vector", s);
            hipLaunchKernelGGL((k_rx_step<T, BATCH>), gM, dim3(256), 0, s, dvec, J.vec);
            hipLaunchKernelGGL((k_cg_step<T, true, BATCH>), gN, dim3(256), 0, s, dvec, J.vec);
            if (J.precond) DECT_TRY(launch_precond<T>(dev ? dev->pre1 : nullptr, J.pre1, nsl, s));
            DECT_TRY(reduce(RED_BETA));
            hipLaunchKernelGGL((k_p_step<T, BATCH>), gN, dim3(256), 0, s, dvec, J.vec);
        }
        // The last step's x and h updates are applied by the dual transpose.
        DECT_TRY(hipGetLastError());
    }
    // The a-update (Eq. (13)) and, in the same launch, the TV/z/dual update.
    if (dev)
        DECT_TRY(launch_udm_batch<T>(dev->udm, nsl, (int)(nblk(J.M) + nblk(J.N)),
                                      J.udm.joint_lim > 0.0f, s));
    else
        DECT_TRY(launch_udm<T>(nullptr, 2, J.udm, s));
    // R^T da: the dual residual (adaptive rho) and the tracked h in every mode.
    DECT_TRY(launch_backproject_admm<T>(J.sym, J.bp_waves, EPI_DUAL, dev ? dev->dual : nullptr,
                                        J.dual, nsl, J.bp_gx, J.bp_gy, s, J.rt_sums64 != 0));
    DECT_TRY(reduce(RED_FINAL));
#undef DECT_TRY
    return hipSuccess;
}

template <typename T, bool BATCH>
hipError_t settle_t(const SliceJob<T>& J, const JobArrays<T>* dev, int nsl, hipStream_t s) {
    ProfScope ps("settle", s);
    const unsigned z = (unsigned)nsl;
    hipLaunchKernelGGL((k_settle<T, BATCH>), dim3(nblk(J.M > J.N ? J.M : J.N), 1, z), dim3(256), 0,
                       s, dev ? dev->resc : nullptr, J.resc);
    hipLaunchKernelGGL((k_settle_done<T, BATCH>), dim3(1, 1, z), dim3(64), 0, s,
                       dev ? dev->resc : nullptr, J.resc);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_settle(const SliceJob<T>& J, const JobArrays<T>* dev, int nsl, hipStream_t s) {
    return dev ? settle_t<T, true>(J, dev, nsl, s) : settle_t<T, false>(J, nullptr, 1, s);
}

template <typename T>
hipError_t launch_iteration(const SliceJob<T>& J, const JobArrays<T>* dev, int nsl,
                            const dect_params* prm, long it, hipStream_t s) {
    return dev ? iteration_t<T, true>(J, dev, nsl, prm, it, s)
               : iteration_t<T, false>(J, dev, nsl, prm, it, s);
}

template <typename T>
hipError_t launch_track_init(const dect_plan* p, void* st, hipStream_t s, bool sums64) {
    double* hh = at<double>(st, p->off_h);
    hipLaunchKernelGGL(k_zero_f64, dim3(nblk(2 * p->N)), dim3(256), 0, s, hh, 2 * p->N);
    BpArgs<T> b{};
    fill_bp_plan<T>(p, b);
    b.sino = at<T>(st, p->off_t);
    b.y = at<T>(st, p->off_dy);  // zero at the start
    b.z = at<T>(st, p->off_dz);  // zero at the start
    b.h = hh;
    b.partials = at<double>(st, p->off_partials) + (size_t)(p->nb_sino + p->nb_img) * kPartialSlots;
    return launch_backproject_admm<T>(p->sym, p->bp_waves, EPI_DUAL, nullptr, b, 1, b.gx, b.gy, s,
                                      sums64);
}

#define DECT_INST(T)                                                                            \
    template SliceJob<T> make_job<T>(const dect_plan*, const void*, const void*, const void*,    \
                                     const void*, void*, const dect_params*);                    \
    template hipError_t launch_iteration<T>(const SliceJob<T>&, const JobArrays<T>*, int,        \
                                            const dect_params*, long, hipStream_t);              \
    template hipError_t launch_settle<T>(const SliceJob<T>&, const JobArrays<T>*, int,           \
                                         hipStream_t);                                           \
    template hipError_t launch_track_init<T>(const dect_plan*, void*, hipStream_t, bool);
DECT_INST(float)
DECT_INST(double)
#undef DECT_INST

namespace {

template <typename T>
dect_status iterate_T(const dect_plan* p, const void* mh, const void* ml, const void* wh,
                      const void* wl, void* st, const dect_params* prm, int n_iters,
                      dect_iter_log* log, hipStream_t s) {
    double* scal = at<double>(st, p->layout.scalars);
    double* dlog = at<double>(st, p->off_log);
    long it0 = 0;
    if (prm->rho_mode == DECT_RHO_SCHEDULE || log) {
        DECT_HIP(hipStreamSynchronize(s));
        double v = 0.0;
        DECT_HIP(hipMemcpy(&v, scal + S_ITER, sizeof v, hipMemcpyDeviceToHost));
        it0 = (long)v;
    }
    if (prm->rho_mode == DECT_RHO_SCHEDULE &&
        (!prm->rho_schedule || it0 + n_iters >= (long)prm->rho_schedule_len))
        return fail(DECT_E_ARG, "rho schedule of length %d does not reach iteration %ld",
                    prm->rho_schedule_len, it0 + n_iters);
    const SliceJob<T> J = make_job<T>(p, mh, ml, wh, wl, st, prm);
    for (int k = 0; k < n_iters; ++k) {
        const hipError_t e = launch_iteration<T>(J, nullptr, 1, prm, it0 + k, s);
        if (e != hipSuccess)
            return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    }
    // The state's duals hold their scaled values between calls.
    if (n_iters > 0) {
        const hipError_t e = launch_settle<T>(J, nullptr, 1, s);
        if (e != hipSuccess)
            return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    }
    if (log) {
        DECT_HIP(hipStreamSynchronize(s));
        std::vector<double> h((size_t)kLogCap * kLogStride);
        DECT_HIP(hipMemcpy(h.data(), dlog, h.size() * sizeof(double), hipMemcpyDeviceToHost));
        bool bad = false;
        for (int k = 0; k < n_iters; ++k) {
            const long it = it0 + k;
            const double* e = &h[(size_t)(it % kLogCap) * kLogStride];
            dect_iter_log& o = log[k];
            o.iter = (int32_t)e[0];
            o.flags = (int32_t)e[1];
            o.rho[0] = e[2];
            o.rho[1] = e[3];
            o.r_primal[0] = e[4];
            o.r_primal[1] = e[5];
            o.s_dual[0] = e[6];
            o.s_dual[1] = e[7];
            o.data_cost = e[8];
            o.tv_cost = e[9];
            bad = bad || (o.flags & 1);
        }
        if (bad) return fail(DECT_E_NONFINITE, "a non-finite residual or objective was produced");
    }
    return DECT_OK;
}

template <typename T>
dect_status init_T(const dect_plan* p, const void* mh, const void* ml, const void* wh,
                   const void* wl, void* st, const dect_params* prm, hipStream_t s) {
    const size_t words = p->layout.bytes / 4;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                       static_cast<uint32_t*>(st), words);
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, at<double>(st, p->layout.scalars),
                       prm->rho_c, prm->rho_p, prm->lambda_c, prm->lambda_p);
    UdmArgs<T> u{};
    u.M = p->M;
    u.sym = p->sym;
    u.Vb = p->Vb;
    u.D = p->D;
    u.mh = static_cast<const T*>(mh);
    u.ml = static_cast<const T*>(ml);
    u.wh = static_cast<const T*>(wh);
    u.wl = static_cast<const T*>(wl);
    u.a = at<T>(st, p->layout.a);
    u.t = at<T>(st, p->off_t);
    u.fg = at<T>(st, p->off_fg);
    u.iters = 10;
    u.mu0 = prm->lm_mu0;
    // Inverse of the linearisation at a = 0: rows (mean f_KN, mean f_p) per spectrum.
    const double hc = p->mean_f[0][0], hp = p->mean_f[0][1];
    const double lc = p->mean_f[1][0], lp = p->mean_f[1][1];
    const double det = hc * lp - hp * lc;
    u.lin[0] = lp / det;
    u.lin[1] = -hp / det;
    u.lin[2] = -lc / det;
    u.lin[3] = hc / det;
    hipError_t e = launch_udm<T>(p, 1, u, s);
    if (e == hipSuccess) e = launch_track_init<T>(p, st, s, prm->rt_sums == DECT_RT_SUMS_F64);
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status check_params(const dect_params* prm) {
    if (!prm) return fail(DECT_E_ARG, "null params");
    if (prm->lm_iters < 1 || prm->cg_iters < 1)
        return fail(DECT_E_ARG, "lm_iters and cg_iters must be >= 1");
    if (prm->rho_mode < DECT_RHO_FIXED || prm->rho_mode > DECT_RHO_SCHEDULE)
        return fail(DECT_E_ARG, "bad rho_mode %d", prm->rho_mode);
    if (!(prm->rho_c > 0) || !(prm->rho_p > 0) || !(prm->lambda_c >= 0) || !(prm->lambda_p >= 0))
        return fail(DECT_E_ARG, "rho must be > 0 and lambda >= 0");
    if (prm->rho_mode == DECT_RHO_ADAPTIVE && (!(prm->bal_mu > 1) || !(prm->bal_tau > 1)))
        return fail(DECT_E_ARG, "residual balancing needs mu > 1 and tau > 1");
    if (!(prm->lm_mu0 > 0)) return fail(DECT_E_ARG, "lm_mu0 must be > 0");
    if (prm->precond != DECT_PRECOND_NONE && prm->precond != DECT_PRECOND_RAMP)
        return fail(DECT_E_ARG, "bad precond %d", prm->precond);
    if (prm->rt_sums != DECT_RT_SUMS_PLAN && prm->rt_sums != DECT_RT_SUMS_F64)
        return fail(DECT_E_ARG, "bad rt_sums %d", prm->rt_sums);
    return DECT_OK;
}

bool bad_ch(int ch) { return ch != 1 && ch != 2 && ch != 4; }

}  // namespace
}  // namespace dect

using namespace dect;

extern "C" {

dect_status dect_project(const dect_plan* p, const void* img, void* sino, int ch, void* stream) {
    if (!p || !img || !sino) return fail(DECT_E_ARG, "null argument");
    if (bad_ch(ch)) return fail(DECT_E_ARG, "ch must be 1, 2 or 4 (got %d)", ch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = p->dtype == DECT_F32 ? launch_project<float>(p, img, sino, ch, s)
                                        : launch_project<double>(p, img, sino, ch, s);
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status dect_backproject(const dect_plan* p, const void* sino, void* img, int ch,
                             void* stream) {
    if (!p || !img || !sino) return fail(DECT_E_ARG, "null argument");
    if (bad_ch(ch)) return fail(DECT_E_ARG, "ch must be 1, 2 or 4 (got %d)", ch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (p->dtype == DECT_F32) {
        BpArgs<float> a{};
        a.sino = static_cast<const float*>(sino);
        a.out = static_cast<float*>(img);
        e = launch_backproject<float>(p, ch, a, s);
    } else {
        BpArgs<double> a{};
        a.sino = static_cast<const double*>(sino);
        a.out = static_cast<double*>(img);
        e = launch_backproject<double>(p, ch, a, s);
    }
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status dect_decompose_rays(const dect_plan* p, const void* m_h, const void* m_l,
                                const void* w_h, const void* w_l, const void* v, double rho_c,
                                double rho_p, int lm_iters, void* a, void* cost, void* stream) {
    if (!p || !m_h || !m_l || !w_h || !w_l || !a) return fail(DECT_E_ARG, "null argument");
    if (lm_iters < 0) return fail(DECT_E_ARG, "lm_iters must be >= 0");
    if (v && (!(rho_c >= 0) || !(rho_p >= 0))) return fail(DECT_E_ARG, "rho must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (p->dtype == DECT_F32) {
        UdmArgs<float> u{};
        u.M = p->M;
        u.sym = 1;
        u.Vb = p->V;
        u.D = p->D;
        u.mh = static_cast<const float*>(m_h);
        u.ml = static_cast<const float*>(m_l);
        u.wh = static_cast<const float*>(w_h);
        u.wl = static_cast<const float*>(w_l);
        u.a = static_cast<float*>(a);
        u.v = static_cast<const float*>(v);
        u.cost = static_cast<float*>(cost);
        u.rho_c = rho_c;
        u.rho_p = rho_p;
        u.iters = lm_iters;
        u.mu0 = 1e-3;
        e = launch_udm<float>(p, 0, u, s);
    } else {
        UdmArgs<double> u{};
        u.M = p->M;
        u.sym = 1;
        u.Vb = p->V;
        u.D = p->D;
        u.mh = static_cast<const double*>(m_h);
        u.ml = static_cast<const double*>(m_l);
        u.wh = static_cast<const double*>(w_h);
        u.wl = static_cast<const double*>(w_l);
        u.a = static_cast<double*>(a);
        u.v = static_cast<const double*>(v);
        u.cost = static_cast<double*>(cost);
        u.rho_c = rho_c;
        u.rho_p = rho_p;
        u.iters = lm_iters;
        u.mu0 = 1e-3;
        e = launch_udm<double>(p, 0, u, s);
    }
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status dect_ingest_counts(const dect_plan* p, const void* counts_h, const void* counts_l,
                               double i0_h, double i0_l, void* m_h, void* m_l, void* w_h,
                               void* w_l, void* stream) {
    if (!p || !counts_h || !counts_l || !m_h || !m_l || !w_h || !w_l)
        return fail(DECT_E_ARG, "null argument");
    if (!(i0_h > 0) || !(i0_l > 0)) return fail(DECT_E_ARG, "I0 must be positive");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = p->dtype == DECT_F32
                       ? launch_ingest<float>(p, counts_h, counts_l, i0_h, i0_l, m_h, m_l, w_h, w_l, s)
                       : launch_ingest<double>(p, counts_h, counts_l, i0_h, i0_l, m_h, m_l, w_h, w_l, s);
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status dect_admm_init(const dect_plan* p, const void* m_h, const void* m_l,
                           const void* w_h, const void* w_l, void* state,
                           const dect_params* prm, void* stream) {
    if (!p || !m_h || !m_l || !w_h || !w_l || !state) return fail(DECT_E_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(state) % 256)
        return fail(DECT_E_ARG, "state buffer must be 256-byte aligned");
    dect_status st = check_params(prm);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return p->dtype == DECT_F32 ? init_T<float>(p, m_h, m_l, w_h, w_l, state, prm, s)
                                : init_T<double>(p, m_h, m_l, w_h, w_l, state, prm, s);
}

dect_status dect_admm_init_image(const dect_plan* p, const void* m_h, const void* m_l,
                                 const void* w_h, const void* w_l, const void* x0, void* state,
                                 const dect_params* prm, void* stream) {
    if (!x0) return fail(DECT_E_ARG, "null argument");
    dect_status st = dect_admm_init(p, m_h, m_l, w_h, w_l, state, prm, stream);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool sums64 = prm->rt_sums == DECT_RT_SUMS_F64;
    const hipError_t e = p->dtype == DECT_F32 ? launch_init_image<float>(p, x0, state, s, sums64)
                                              : launch_init_image<double>(p, x0, state, s, sums64);
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status dect_admm_iterate(const dect_plan* p, const void* m_h, const void* m_l,
                              const void* w_h, const void* w_l, void* state,
                              const dect_params* prm, int n_iters, dect_iter_log* log,
                              void* stream) {
    if (!p || !m_h || !m_l || !w_h || !w_l || !state) return fail(DECT_E_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(state) % 256)
        return fail(DECT_E_ARG, "state buffer must be 256-byte aligned");
    dect_status st = check_params(prm);
    if (st) return st;
    if (prm->precond && !p->has_precond)
        return fail(DECT_E_SHAPE, "no preconditioner for a %dx%d image", p->nx, p->ny);
    if (n_iters < 0) return fail(DECT_E_ARG, "n_iters must be >= 0");
    if (log && n_iters > kLogCap)
        return fail(DECT_E_ARG, "a log holds at most %d iterations per call", kLogCap);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return p->dtype == DECT_F32
               ? iterate_T<float>(p, m_h, m_l, w_h, w_l, state, prm, n_iters, log, s)
               : iterate_T<double>(p, m_h, m_l, w_h, w_l, state, prm, n_iters, log, s);
}

dect_status dect_state_log(const dect_plan* p, const void* state, int64_t first, int n,
                           dect_iter_log* log, void* stream) {
    if (!p || !state || (!log && n > 0)) return fail(DECT_E_ARG, "null argument");
    if (n < 0 || first < 0) return fail(DECT_E_ARG, "first and n must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DECT_HIP(hipStreamSynchronize(s));
    const char* base = static_cast<const char*>(state);
    double done = 0.0;
    DECT_HIP(hipMemcpy(&done, base + p->layout.scalars + S_ITER * sizeof(double), sizeof done,
                       hipMemcpyDeviceToHost));
    const int64_t it_done = (int64_t)done;
    if (first + n > it_done || first < it_done - kLogCap)
        return fail(DECT_E_ARG, "iterations [%lld, %lld) are not in the log (%lld done, last %d kept)",
                    (long long)first, (long long)(first + n), (long long)it_done, kLogCap);
    std::vector<double> h((size_t)kLogCap * kLogStride);
    DECT_HIP(hipMemcpy(h.data(), base + p->off_log, h.size() * sizeof(double),
                       hipMemcpyDeviceToHost));
    for (int k = 0; k < n; ++k) {
        const double* e = &h[(size_t)((first + k) % kLogCap) * kLogStride];
        dect_iter_log& o = log[k];
        o.iter = (int32_t)e[0];
        o.flags = (int32_t)e[1];
        o.rho[0] = e[2];
        o.rho[1] = e[3];
        o.r_primal[0] = e[4];
        o.r_primal[1] = e[5];
        o.s_dual[0] = e[6];
        o.s_dual[1] = e[7];
        o.data_cost = e[8];
        o.tv_cost = e[9];
    }
    return DECT_OK;
}

}  // extern "C"
