// Per-ray unconstrained decomposition (Eq. (13)) by Levenberg-Marquardt, and the
// count-to-measurement ingest, for gfx950.
//
// One ray per lane.  The energy-bin tables are read with wave-uniform indices,
// so they come from scalar loads and every lane runs the same bin loop; the
// only divergence is the per-ray accept/reject of the LM step.  The polychromatic
// transform f_s(a) = -ln sum_k omega_k exp(-f_KN[k] a_c - f_p[k] a_p) (Eq. (3))
// is a log-sum-exp evaluated in base 2 with a shift factored out, which keeps metal
// rays (exponents below -700) finite in single precision.  Where the plan has a
// joint table both spectra come from one exponential per bin; a ray whose shift
// left the range is evaluated again exactly by its whole wave.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "profile.h"
#include "tv.h"

// No contraction into fused multiply-adds beyond the fma() calls written out: the
// compiler could fuse a sum of products differently in different instantiations of a
// kernel, and the batched and single-slice a-updates must agree bit for bit.
#pragma clang fp contract(off)

namespace dect {

namespace {

template <typename T> struct Cst;
template <> struct Cst<float> {
    // Raw hardware exp2/log2: arguments stay in the normal range by construction
    // (the largest exponent is shifted to <= 0 and the sum of terms is >= 2^-110),
    // and a result below 2^-126 only drops a term smaller than 2^-126 of the sum.
    __device__ static float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
    __device__ static float log2(float x) { return __builtin_amdgcn_logf(x); }
};
template <> struct Cst<double> {
    __device__ static double exp2(double x) { return ::exp2(x); }
    __device__ static double log2(double x) { return ::log2(x); }
};

// f and gradient of one spectrum at (ac, ap), tables in base-2 units:
//   f = -ln2 (M + log2 sum_k 2^(e_k - M)),  e_k = lw_k - kc_k ac - kp_k ap,
//   grad f = ln2 sum_k 2^(e_k - M) (kc_k, kp_k) / sum_k 2^(e_k - M).
// Any shift M gives the same value; M must keep every e_k - M below the
// overflow threshold and the largest above underflow.  With exact = true M is
// the largest exponent (one extra pass); otherwise the caller's M is used.
template <typename T>
__device__ inline void spectrum_eval(const T* __restrict__ lw_, const T* __restrict__ kc_,
                                     const T* __restrict__ kp_, int n, T ac, T ap, T shift,
                                     bool exact, T& f, T& gc, T& gp) {
    // The tables are read-only for the whole launch: read them through the constant
    // address space, so they stay on scalar loads whatever else the kernel stores.
    using CT = const __attribute__((address_space(4))) T;
    CT* lw = (CT*)lw_;
    CT* kc = (CT*)kc_;
    CT* kp = (CT*)kp_;
    constexpr T ln2 = T(0.6931471805599453);
    T m = shift;
    if (exact) {
        m = -INFINITY;
#pragma unroll 8
        for (int k = 0; k < n; ++k) m = fmax(m, fma(-kp[k], ap, fma(-kc[k], ac, lw[k])));
    }
    T z = T(0), sc = T(0), sp = T(0);
#pragma unroll 8
    for (int k = 0; k < n; ++k) {
        const T q = Cst<T>::exp2(fma(-kp[k], ap, fma(-kc[k], ac, lw[k] - m)));
        z += q;
        sc = fma(q, kc[k], sc);
        sp = fma(q, kp[k], sp);
    }
    f = -(m + Cst<T>::log2(z)) * ln2;
    // sum_k q_k f_KN[k] / z = ln2 * sum_k q_k kc[k] / z, since kc = f_KN / ln2.
    const T iz = ln2 / z;
    gc = sc * iz;
    gp = sp * iz;
}

template <typename T>
struct Point {
    T ac, ap, fh, fl, ghc, ghp, glc, glp, phi;
};

// Both spectra on one energy grid (the plan's joint table, [jb + jh + jl][8]).
template <typename T>
struct JointTab {
    const T* tab;
    int jb, jh, jl;
    float lim;       // largest log2 distance from the shift to a log-sum-exp (0: never)
    float kc0, kc1;  // smallest and largest kc of the table
    float kp0, kp1;  // smallest and largest kp
};

// f and gradient of both spectra at (ac, ap) with one exponential per energy bin:
// A_k = 2^(-kc_k ac - kp_k ap - s) is shared by the spectra, which differ only in their
// weights, so f_s = -ln2 (s + log2 sum_k w_sk A_k) and grad f_s = ln2 sum_k w_sk A_k
// (kc_k, kp_k) / sum_k w_sk A_k, with the products w_sk kc_k, w_sk kp_k from the table
// (one record of 8 values per bin, read with one scalar load).  Returns whether the shift
// s kept the evaluation in range: every sum finite (no A_k overflowed) and both
// normalising sums at least 2^-90, so that terms lost below 2^-126 are below 2^-36 of
// their sum.
template <typename T, int U = 4>
__device__ inline bool spectra_eval_joint(const JointTab<T>& J, T ac, T ap, T s, T& fh, T& ghc,
                                          T& ghp, T& fl, T& glc, T& glp) {
    using CT = const __attribute__((address_space(4))) T;
    CT* rec = (CT*)J.tab;
    const int nj = J.jb + J.jh + J.jl;
    constexpr T ln2 = T(0.6931471805599453);
    const T ns = -s;
    T zh = T(0), ah = T(0), bh = T(0), zl = T(0), al = T(0), bl = T(0);
    int k = 0;
#pragma unroll U
    for (; k < J.jb; ++k) {
        CT* r = rec + 8 * k;
        const T A = Cst<T>::exp2(fma(-r[1], ap, fma(-r[0], ac, ns)));
        zh = fma(r[2], A, zh);
        ah = fma(r[3], A, ah);
        bh = fma(r[4], A, bh);
        zl = fma(r[5], A, zl);
        al = fma(r[6], A, al);
        bl = fma(r[7], A, bl);
    }
#pragma unroll 2
    for (; k < J.jb + J.jh; ++k) {
        CT* r = rec + 8 * k;
        const T A = Cst<T>::exp2(fma(-r[1], ap, fma(-r[0], ac, ns)));
        zh = fma(r[2], A, zh);
        ah = fma(r[3], A, ah);
        bh = fma(r[4], A, bh);
    }
#pragma unroll 2
    for (; k < nj; ++k) {
        CT* r = rec + 8 * k;
        const T A = Cst<T>::exp2(fma(-r[1], ap, fma(-r[0], ac, ns)));
        zl = fma(r[5], A, zl);
        al = fma(r[6], A, al);
        bl = fma(r[7], A, bl);
    }
    fh = -(s + Cst<T>::log2(zh)) * ln2;
    fl = -(s + Cst<T>::log2(zl)) * ln2;
    const T ih = ln2 / zh, il = ln2 / zl;
    ghc = ah * ih;
    ghp = bh * ih;
    glc = al * il;
    glp = bl * il;
    constexpr T tiny = T(8.077935669463161e-28);  // 2^-90
    return zh >= tiny && zl >= tiny && isfinite(((zh + zl) + (ah + bh)) + (al + bl));
}

// Sum and maximum over the 64 lanes of a wave, in a fixed butterfly order that gives every
// lane the same bits; every lane of the wave must be active.
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// f and gradient of one spectrum at the wave-uniform point (ac, ap), its bins spread over
// the lanes of the wave (lane t takes bins t, t + 64, ...), with the largest exponent as
// the shift: the exact form of spectrum_eval for one ray, at a wave's cost of a few bins.
// Every lane of the wave must be active; every lane returns the same values.
template <typename T>
__device__ inline void wave_spectrum_eval(const T* __restrict__ lw, const T* __restrict__ kc,
                                          const T* __restrict__ kp, int n, T ac, T ap, T& f,
                                          T& gc, T& gp) {
    constexpr T ln2 = T(0.6931471805599453);
    const int t = (int)(threadIdx.x & 63u);
    __builtin_amdgcn_sched_barrier(0);
    T m = -INFINITY;
#pragma unroll 1
    for (int k = t; k < n; k += 64) m = fmax(m, fma(-kp[k], ap, fma(-kc[k], ac, lw[k])));
    m = wave_max<T>(m);
    T z = T(0), sc = T(0), sp = T(0);
#pragma unroll 1
    for (int k = t; k < n; k += 64) {
        const T q = Cst<T>::exp2(fma(-kp[k], ap, fma(-kc[k], ac, lw[k] - m)));
        z += q;
        sc = fma(q, kc[k], sc);
        sp = fma(q, kp[k], sp);
    }
    z = wave_sum<T>(z);
    sc = wave_sum<T>(sc);
    sp = wave_sum<T>(sp);
    f = -(m + Cst<T>::log2(z)) * ln2;
    const T iz = ln2 / z;
    gc = sc * iz;
    gp = sp * iz;
    __builtin_amdgcn_sched_barrier(0);
}

// Largest |kc| and |kp| over both spectra (bounds the exponent change of a step).
struct StepBound {
    float kcmax, kpmax;
};

template <typename T>
__device__ inline void evaluate(const T* __restrict__ spec, int kmax, int kh, int kl, T mh, T ml,
                                T wh, T wl, T vc, T vp, T rc, T rp, T shift_h, T shift_l,
                                bool exact, Point<T>& P) {
    spectrum_eval<T>(spec, spec + kmax, spec + 2 * kmax, kh, P.ac, P.ap, shift_h, exact, P.fh,
                     P.ghc, P.ghp);
    spectrum_eval<T>(spec + 3 * kmax, spec + 4 * kmax, spec + 5 * kmax, kl, P.ac, P.ap, shift_l,
                     exact, P.fl, P.glc, P.glp);
    const T rh = P.fh - mh, rl = P.fl - ml, dc = P.ac - vc, dp = P.ap - vp;
    P.phi = T(0.5) * (wh * rh * rh + wl * rl * rl) + T(0.5) * (rc * dc * dc + rp * dp * dp);
}

// a*d - b*c with the rounding error of b*c compensated (Kahan).
template <typename T>
__device__ inline T det2(T a, T d, T b, T c) {
    const T w = b * c;
    const T e = fma(-b, c, w);
    const T f = fma(a, d, -w);
    return f + e;
}

// m Levenberg-Marquardt iterations from P (evaluated); P ends at the last accepted
// point.  A trial point is evaluated in one pass, shifted by the log-sum-exp of
// the current point: the exponents then change by at most
// B = kcmax |d_c| + kpmax |d_p|, so for B <= 96 nothing overflows and the largest
// term stays above 2^-(96 + log2 K).  Larger steps take the two-pass form.
//
// JT (the plan has a joint table): every trial point is evaluated with the joint table
// (spectra_eval_joint) for both spectra with one shift placed between bounds of their
// log-sum-exps at the trial point.  A ray for which that shift left the range (a step
// across which the bounds are too far apart, a non-finite current point) is evaluated
// again exactly, by the whole wave (wave_spectrum_eval); every lane of the wave must call
// lm_solve together.  Without a joint table (a weight below 2^-24 of its spectrum) the
// spectra are evaluated apart.
//
// CONSTR (the constrained decomposition, a >= 0): a coordinate at zero whose
// gradient is positive is held at zero and the damped step is taken in the other
// coordinate alone; trial points are projected onto a >= 0.
//
// accepted: bit k set when LM iteration k (k < 32) accepted its trial point.
template <typename T, bool CONSTR, bool JT>
__device__ inline void lm_solve(const T* __restrict__ spec, int kmax, int kh, int kl,
                                const JointTab<T>& jt, T mh, T ml, T wh, T wl, T vc, T vp,
                                T rc, T rp, int iters, T mu, StepBound sb, Point<T>& P,
                                unsigned& accepted) {
    constexpr T log2e = T(1.4426950408889634);
    accepted = 0u;
    // The iterations are predicated rather than left early, so that all lanes of a wave
    // reach the spectra evaluation together (the joint path's fallback is wave-wide).
    bool stop = false;  // CONSTR: stationary at the corner
    for (int it = 0; it < iters; ++it) {
        const T rh = P.fh - mh, rl = P.fl - ml;
        const T Gc = wh * rh * P.ghc + wl * rl * P.glc + rc * (P.ac - vc);
        const T Gp = wh * rh * P.ghp + wl * rl * P.glp + rp * (P.ap - vp);
        const T Acc = wh * P.ghc * P.ghc + wl * P.glc * P.glc;
        const T App = wh * P.ghp * P.ghp + wl * P.glp * P.glp;
        const T Hcc = Acc + rc, Hpp = App + rp;
        const T Hcp = wh * P.ghc * P.ghp + wl * P.glc * P.glp;
        const T Dcc = (T(1) + mu) * Hcc, Dpp = (T(1) + mu) * Hpp;
        bool fix_c = false, fix_p = false;
        if constexpr (CONSTR) {
            fix_c = P.ac == T(0) && Gc > T(0);
            fix_p = P.ap == T(0) && Gp > T(0);
            stop = stop || (fix_c && fix_p);
        }
        T dc = T(0), dp = T(0);
        bool bad;  // singular or non-finite damped system: no step, mu grows
        if (fix_c || fix_p) {
            const T d1 = fix_c ? Dpp : Dcc;
            bad = !(d1 > T(0)) || !(d1 < INFINITY);
            if (!bad) {
                dc = fix_c ? T(0) : -Gc / d1;
                dp = fix_p ? T(0) : -Gp / d1;
            }
        } else {
            // det(H + mu diag H) as a sum of nonnegative terms (no cancellation):
            // w_h w_l (g_h x g_l)^2 + rc App + rp Acc + rc rp + mu (2 + mu) Hcc Hpp.
            const T cr = det2<T>(P.ghc, P.glp, P.ghp, P.glc);
            const T det = wh * wl * cr * cr + rc * App + rp * Acc + rc * rp +
                          mu * (T(2) + mu) * Hcc * Hpp;
            bad = !(det > T(0)) || !(det < INFINITY);
            if (!bad) {
                const T id = T(1) / det;
                dc = -(Dpp * Gc - Hcp * Gp) * id;
                dp = -(Dcc * Gp - Hcp * Gc) * id;
            }
        }
        const bool skip = stop || bad;  // no trial point in this iteration
        if (!stop && bad) mu *= T(10);
        Point<T> Q;
        Q.ac = P.ac + dc;
        Q.ap = P.ap + dp;
        if constexpr (CONSTR) {
            Q.ac = fmax(Q.ac, T(0));
            Q.ap = fmax(Q.ap, T(0));
            dc = Q.ac - P.ac;
            dp = Q.ap - P.ap;
        }
        const T sh = -P.fh * log2e, sl = -P.fl * log2e;
        if constexpr (JT) {
            // Each spectrum's log-sum-exp at Q lies between its first-order prediction
            // from P (the log-sum-exp is convex in a) and its value at P plus the largest
            // change of any exponent.  The shift, halfway between the predictions, is
            // moved so that the highest bound is at most lim above it and the lowest at
            // most 90 below it; both hold when the bounds are within lim + 90.
            const T up = (dc >= T(0) ? -(T)jt.kc0 * dc : -(T)jt.kc1 * dc) +
                         (dp >= T(0) ? -(T)jt.kp0 * dp : -(T)jt.kp1 * dp);
            const T lh = -(P.fh + P.ghc * dc + P.ghp * dp) * log2e;
            const T ll = -(P.fl + P.glc * dc + P.glp * dp) * log2e;
            const T s = fmin(fmax(T(0.5) * (lh + ll), fmax(sh, sl) + up - (T)jt.lim),
                             fmin(lh, ll) + T(90));
            const bool ok =
                spectra_eval_joint<T>(jt, Q.ac, Q.ap, s, Q.fh, Q.ghc, Q.ghp, Q.fl, Q.glc, Q.glp);
            // A ray whose sums left the range is evaluated again by the whole wave, its
            // bins spread over the lanes, so that a few such rays do not hold up the wave.
            unsigned long long need = __ballot(!ok && !skip);
            const int t = (int)(threadIdx.x & 63u);
            while (need) {
                const int j = __ffsll((long long)need) - 1;
                need &= need - 1;
                const T ac = __shfl(Q.ac, j, 64), ap = __shfl(Q.ap, j, 64);
                T f0, g0, g1;
                wave_spectrum_eval<T>(spec, spec + kmax, spec + 2 * kmax, kh, ac, ap, f0, g0,
                                      g1);
                if (t == j) {
                    Q.fh = f0;
                    Q.ghc = g0;
                    Q.ghp = g1;
                }
                wave_spectrum_eval<T>(spec + 3 * kmax, spec + 4 * kmax, spec + 5 * kmax, kl, ac,
                                      ap, f0, g0, g1);
                if (t == j) {
                    Q.fl = f0;
                    Q.glc = g0;
                    Q.glp = g1;
                }
            }
            const T rh = Q.fh - mh, rl = Q.fl - ml, ec = Q.ac - vc, ep = Q.ap - vp;
            Q.phi = T(0.5) * (wh * rh * rh + wl * rl * rl) + T(0.5) * (rc * ec * ec + rp * ep * ep);
        } else if (!skip) {
            const T bound = (T)sb.kcmax * fabs(dc) + (T)sb.kpmax * fabs(dp);
            // A non-finite current value gives no usable shift either.
            const bool exact = !(bound <= T(96)) || !(isfinite(P.fh) && isfinite(P.fl));
            evaluate<T>(spec, kmax, kh, kl, mh, ml, wh, wl, vc, vp, rc, rp, sh, sl, exact, Q);
        }
        if (!skip) {
            if (Q.phi < P.phi) {
                P = Q;
                mu *= T(0.1);
                if (it < 32) accepted |= 1u << it;
            } else {
                mu *= T(10);
            }
        }
    }
}

// JT: the plan has a joint table (joint_lim > 0); see lm_solve.
template <typename T, int MODE, bool BATCH, bool JT>
__global__ __launch_bounds__(256) void k_udm(const UdmArgs<T>* __restrict__ dev, UdmArgs<T> one) {
    using V2 = vec<T, 2>;
    using V4 = vec<T, 4>;
    const UdmArgs<T> A = pick_args<BATCH>(dev, one);
    if constexpr (MODE == 2) {
        // Blocks past the a-update's run the image's TV/z/dual update.
        if ((int)blockIdx.x >= A.udm_blocks) {
            if (A.tv.x) tv_dual_block<T>(A.tv, (long)blockIdx.x - A.udm_blocks);
            return;
        }
    }
    const T* __restrict__ spec = A.spec;
    const int kmax = A.kmax, kh = A.kh, kl = A.kl;
    const StepBound sb{A.kc_max, A.kp_max};
    if ((long)blockIdx.x * blockDim.x >= A.M) return;  // beyond this slice (whole block)
    // l: internal ray index (t, da, R p, f cache); i: standard [V][D] index (m, w, a,
    // u^a, R x).
    // With JT every lane of a wave takes part in the LM iterations (their fallback is
    // wave-wide): lanes past the last ray repeat it and store nothing.
    const long l0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = l0 < A.M;
    const long l = live ? l0 : A.M - 1;
    const long i = live || JT ? std_ray(l, A.sym, A.Vb, A.D) : 0;
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (live || JT) {
        const T mh = A.mh[i], ml = A.ml[i], wh = A.wh[i], wl = A.wl[i];
        V2* a2 = reinterpret_cast<V2*>(A.a);
        Point<T> P;
        T vc = T(0), vp = T(0), rc = T(0), rp = T(0);
        V2 rx;
        V2 ua;
        const V2 a_prev = a2[i];
        if constexpr (MODE == 1 || MODE == 3) {
            // Start at the solution of the linearisation at a = 0 (CDM: projected).
            P.ac = (T)(A.lin[0] * (double)mh + A.lin[1] * (double)ml);
            P.ap = (T)(A.lin[2] * (double)mh + A.lin[3] * (double)ml);
            if constexpr (MODE == 3) {
                P.ac = fmax(P.ac, T(0));
                P.ap = fmax(P.ap, T(0));
            }
        } else {
            P.ac = a_prev.v[0];
            P.ap = a_prev.v[1];
        }
        if constexpr (MODE == 0) {
            if (A.v) {
                const V2 v2 = reinterpret_cast<const V2*>(A.v)[i];
                vc = v2.v[0];
                vp = v2.v[1];
                rc = (T)A.rho_c;
                rp = (T)A.rho_p;
            }
        } else if constexpr (MODE == 2) {
            // R x after the last CG step (tracked: R x += alpha R p), v = R x - u^a.
            const V2 rx0 = reinterpret_cast<const V2*>(A.Rx)[i];
            const V2 rp2 = reinterpret_cast<const V2*>(A.Rp)[l];
            // u^a as rescaled by the pending kappa (stored below with its update).
            ua = reinterpret_cast<const V2*>(A.ua)[i];
            ua.v[0] = mul_rn((T)A.scal[S_KAPPA], ua.v[0]);
            ua.v[1] = mul_rn((T)A.scal[S_KAPPA + 1], ua.v[1]);
            rx.v[0] = rx0.v[0] + (T)A.scal[S_ALPHA] * rp2.v[0];
            rx.v[1] = rx0.v[1] + (T)A.scal[S_ALPHA + 1] * rp2.v[1];
            vc = rx.v[0] - ua.v[0];
            vp = rx.v[1] - ua.v[1];
            rc = (T)A.scal[S_RHO];
            rp = (T)A.scal[S_RHO + 1];
        }
        if constexpr (MODE == 2) {
            // f and its gradient at the current a were computed by the previous
            // a-update (a has not changed since) and are kept per ray.
            const V4 c0 = reinterpret_cast<const V4*>(A.fg)[2 * l];
            const V2 c1 = reinterpret_cast<const V2*>(A.fg)[4 * l + 2];
            P.fh = c0.v[0];
            P.fl = c0.v[1];
            P.ghc = c0.v[2];
            P.ghp = c0.v[3];
            P.glc = c1.v[0];
            P.glp = c1.v[1];
            const T rh = P.fh - mh, rl = P.fl - ml, dc = P.ac - vc, dp = P.ap - vp;
            P.phi = T(0.5) * (wh * rh * rh + wl * rl * rl) + T(0.5) * (rc * dc * dc + rp * dp * dp);
        } else {
            evaluate<T>(spec, kmax, kh, kl, mh, ml, wh, wl, vc, vp, rc, rp, T(0), T(0), true, P);
        }
        unsigned accepted;
        const JointTab<T> jt{A.joint,  A.jb,      A.jh,      A.jl,     A.joint_lim,
                             A.jkc[0], A.jkc[1], A.jkp[0], A.jkp[1]};
        lm_solve<T, MODE == 3, JT>(spec, kmax, kh, kl, jt, mh, ml, wh, wl, vc, vp, rc, rp, A.iters,
                               (T)A.mu0, sb, P, accepted);
        if (live) {
            if constexpr (MODE == 2) {
                if (A.lmbits) A.lmbits[i] = (uint8_t)(accepted & 0xffu);
            }
            V2 an;
            an.v[0] = P.ac;
            an.v[1] = P.ap;
            a2[i] = an;
            if constexpr (MODE == 1 || MODE == 2) {
                V4 c0;
                V2 c1;
                c0.v[0] = P.fh;
                c0.v[1] = P.fl;
                c0.v[2] = P.ghc;
                c0.v[3] = P.ghp;
                c1.v[0] = P.glc;
                c1.v[1] = P.glp;
                reinterpret_cast<V4*>(A.fg)[2 * l] = c0;
                reinterpret_cast<V2*>(A.fg)[4 * l + 2] = c1;
            }
            if constexpr (MODE == 0 || MODE == 3) {
                if (A.cost) A.cost[i] = P.phi;
            } else if constexpr (MODE == 1) {
                reinterpret_cast<V2*>(A.t)[l] = an;  // u^a = R x = 0
            } else {
                V2 un, tn, dn;
    #pragma unroll
                for (int c = 0; c < 2; ++c) {
                    un.v[c] = ua.v[c] + an.v[c] - rx.v[c];        // Eq. (11), a-block
                    tn.v[c] = an.v[c] + un.v[c] - rx.v[c];        // next R^T right-hand side
                    dn.v[c] = an.v[c] - a_prev.v[c];
                    part[c] = (double)(an.v[c] - rx.v[c]) * (double)(an.v[c] - rx.v[c]);
                }
                reinterpret_cast<V2*>(A.ua)[i] = un;
                reinterpret_cast<V2*>(A.Rx)[i] = rx;
                if (A.t) reinterpret_cast<V2*>(A.t)[l] = tn;
                reinterpret_cast<V2*>(A.da)[l] = dn;
                const T rh = P.fh - mh, rl = P.fl - ml;
                part[2] = 0.5 * ((double)wh * (double)rh * (double)rh + (double)wl * (double)rl * (double)rl);
                const bool finite = isfinite(P.ac) && isfinite(P.ap) && isfinite(part[2]);
                part[3] = finite ? 0.0 : 1.0;
            }
        }
    }
    if constexpr (MODE == 2) block_sum_store<4>(part, A.partials + (size_t)blockIdx.x * kPartialSlots);
}

// f and its gradient of both spectra at (a_c, a_p) = (at, ao) (basis 0) or (ao, at)
// (basis 1), for the LM x CG scheme: cache[k][M], k = (f_h, f_l, df_h/da_c,
// df_h/da_p, df_l/da_c, df_l/da_p); block partials of 1/2 sum_s w_s (f_s - m_s)^2.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_eval(const T* __restrict__ spec, int kmax, int kh,
                                                 int kl, long M, int basis,
                                                 const T* __restrict__ at,
                                                 const T* __restrict__ ao, const T* __restrict__ mh,
                                                 const T* __restrict__ ml, const T* __restrict__ wh,
                                                 const T* __restrict__ wl, T* __restrict__ cache,
                                                 double* __restrict__ partials) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < M) {
        Point<T> P;
        P.ac = basis == 0 ? at[i] : ao[i];
        P.ap = basis == 0 ? ao[i] : at[i];
        evaluate<T>(spec, kmax, kh, kl, mh[i], ml[i], wh[i], wl[i], T(0), T(0), T(0), T(0), T(0),
                    T(0), true, P);
        cache[i] = P.fh;
        cache[M + i] = P.fl;
        cache[2 * M + i] = P.ghc;
        cache[3 * M + i] = P.ghp;
        cache[4 * M + i] = P.glc;
        cache[5 * M + i] = P.glp;
        const double eh = (double)P.fh - (double)mh[i], el = (double)P.fl - (double)ml[i];
        v[0] = 0.5 * ((double)wh[i] * eh * eh + (double)wl[i] * el * el);
        v[1] = (isfinite(P.fh) && isfinite(P.fl)) ? 0.0 : 1.0;
    }
    block_sum_store<4>(v, partials + (size_t)blockIdx.x * kPartialSlots);
}

template <typename T>
__global__ __launch_bounds__(256) void k_ingest(long M, const T* __restrict__ ch,
                                                const T* __restrict__ cl, T i0h, T i0l, T* mh,
                                                T* ml, T* wh, T* wl) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const T h = ch[i], l = cl[i];
    mh[i] = log(i0h / fmax(h, T(1)));
    ml[i] = log(i0l / fmax(l, T(1)));
    wh[i] = h / i0h;
    wl[i] = l / i0l;
}

}  // namespace

template <typename T>
void fill_udm_tables(const dect_plan* p, UdmArgs<T>& a) {
    a.spec = static_cast<const T*>(p->spec);
    a.kmax = p->kmax;
    a.kh = p->kh;
    a.kl = p->kl;
    a.kc_max = (float)p->kc_max;
    a.kp_max = (float)p->kp_max;
    a.joint = static_cast<const T*>(p->joint);
    a.jb = p->jb;
    a.jh = p->jh;
    a.jl = p->jl;
    a.joint_lim = (float)p->joint_lim;
    for (int e = 0; e < 2; ++e) {
        a.jkc[e] = (float)p->joint_kc[e];
        a.jkp[e] = (float)p->joint_kp[e];
    }
}

template <typename T>
hipError_t launch_udm(const dect_plan* p, int mode, const UdmArgs<T>& a0, hipStream_t s) {
    UdmArgs<T> a = a0;
    if (p) fill_udm_tables<T>(p, a);  // else the tables are already in a
    a.udm_blocks = (int)((a.M + 255) / 256);
    const long tvb = mode == 2 && a.tv.x ? ((long)a.tv.nx * a.tv.ny + 255) / 256 : 0;
    dim3 g((unsigned)(a.udm_blocks + tvb));
    ProfScope ps(mode == 1 ? "udm_init" : (mode == 3 ? "cdm" : "udm"), s);
    const bool jt = a.joint_lim > 0.0f;
    if (mode == 0 && jt)
        hipLaunchKernelGGL((k_udm<T, 0, false, true>), g, dim3(256), 0, s, nullptr, a);
    else if (mode == 0)
        hipLaunchKernelGGL((k_udm<T, 0, false, false>), g, dim3(256), 0, s, nullptr, a);
    else if (mode == 3 && jt)
        hipLaunchKernelGGL((k_udm<T, 3, false, true>), g, dim3(256), 0, s, nullptr, a);
    else if (mode == 3)
        hipLaunchKernelGGL((k_udm<T, 3, false, false>), g, dim3(256), 0, s, nullptr, a);
    else if (mode == 1 && jt)
        hipLaunchKernelGGL((k_udm<T, 1, false, true>), g, dim3(256), 0, s, nullptr, a);
    else if (mode == 1)
        hipLaunchKernelGGL((k_udm<T, 1, false, false>), g, dim3(256), 0, s, nullptr, a);
    else if (jt)
        hipLaunchKernelGGL((k_udm<T, 2, false, true>), g, dim3(256), 0, s, nullptr, a);
    else
        hipLaunchKernelGGL((k_udm<T, 2, false, false>), g, dim3(256), 0, s, nullptr, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_udm_batch(const UdmArgs<T>* args, int n, int blocks, bool joint,
                            hipStream_t s) {
    ProfScope ps("udm", s);
    if (joint)
        hipLaunchKernelGGL((k_udm<T, 2, true, true>), dim3(blocks, 1, n), dim3(256), 0, s, args,
                           UdmArgs<T>{});
    else
        hipLaunchKernelGGL((k_udm<T, 2, true, false>), dim3(blocks, 1, n), dim3(256), 0, s, args,
                           UdmArgs<T>{});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lm_eval(const dect_plan* p, int basis, const T* at, const T* ao, const T* mh,
                          const T* ml, const T* wh, const T* wl, T* cache, double* partials,
                          hipStream_t s) {
    ProfScope ps("lm_eval", s);
    hipLaunchKernelGGL((k_lm_eval<T>), dim3((unsigned)((p->M + 255) / 256)), dim3(256), 0, s,
                       static_cast<const T*>(p->spec), p->kmax, p->kh, p->kl, p->M, basis, at, ao,
                       mh, ml, wh, wl, cache, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ingest(const dect_plan* p, const void* ch, const void* cl, double i0h,
                         double i0l, void* mh, void* ml, void* wh, void* wl, hipStream_t s) {
    dim3 g((unsigned)((p->M + 255) / 256));
    hipLaunchKernelGGL((k_ingest<T>), g, dim3(256), 0, s, p->M, static_cast<const T*>(ch),
                       static_cast<const T*>(cl), (T)i0h, (T)i0l, static_cast<T*>(mh),
                       static_cast<T*>(ml), static_cast<T*>(wh), static_cast<T*>(wl));
    return hipGetLastError();
}

template void fill_udm_tables<float>(const dect_plan*, UdmArgs<float>&);
template void fill_udm_tables<double>(const dect_plan*, UdmArgs<double>&);
template hipError_t launch_udm<float>(const dect_plan*, int, const UdmArgs<float>&, hipStream_t);
template hipError_t launch_udm<double>(const dect_plan*, int, const UdmArgs<double>&, hipStream_t);
template hipError_t launch_lm_eval<float>(const dect_plan*, int, const float*, const float*,
                                          const float*, const float*, const float*,
                                          const float*, float*, double*, hipStream_t);
template hipError_t launch_lm_eval<double>(const dect_plan*, int, const double*, const double*,
                                           const double*, const double*, const double*,
                                           const double*, double*, double*, hipStream_t);
template hipError_t launch_udm_batch<float>(const UdmArgs<float>*, int, int, bool, hipStream_t);
template hipError_t launch_udm_batch<double>(const UdmArgs<double>*, int, int, bool, hipStream_t);
template hipError_t launch_ingest<float>(const dect_plan*, const void*, const void*, double, double,
                                         void*, void*, void*, void*, hipStream_t);
template hipError_t launch_ingest<double>(const dect_plan*, const void*, const void*, double,
                                          double, void*, void*, void*, void*, hipStream_t);

}  // namespace dect
