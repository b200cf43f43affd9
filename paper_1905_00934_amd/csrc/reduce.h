// The scalar steps of an ADMM iteration: fixed-order sums of block partials and the
// updates they feed (CG step sizes; residuals, rho and the log).  Run by one
// workgroup per slice (k_reduce); every thread of the workgroup must call them,
// thread 0 stores the results.
#pragma once

#include <cmath>

#include "kernels.h"

namespace dect {

// alpha = gamma / (p . q) of a CG step: gamma = r . z (r . r without the
// preconditioner) from the image or preconditioner partials, p . q from the q
// transpose's tile partials.
__device__ inline void reduce_alpha(const RedArgs& A) {
    double* s = A.scal;
    if (!s) return;  // empty slot
    double g[2], pq[2], none[1];
    partial_sums<2, 2, 1>(A.precond ? A.pre : A.img, A.precond ? A.nb_pre : A.nb_img, g,
                          A.tiles, A.nb_tiles, pq, nullptr, 0, none);
    if (threadIdx.x == 0)
        for (int c = 0; c < 2; ++c) {
            s[S_GAMMA + c] = g[c];
            s[S_PQ + c] = pq[c];
            s[S_ALPHA + c] = (pq[c] > 0.0 && g[c] > 0.0) ? g[c] / pq[c] : 0.0;
        }
}

// beta = gamma' / gamma of a CG step, gamma <- gamma'.
__device__ inline void reduce_beta(const RedArgs& A) {
    double* s = A.scal;
    if (!s) return;
    double g[2];
    if (A.precond)
        partial_sum<2>(A.pre, A.nb_pre, g);
    else
        partial_sum<2>(A.img, A.nb_img, g);
    if (threadIdx.x == 0)
        for (int c = 0; c < 2; ++c) {
            s[S_BETA + c] = s[S_GAMMA + c] > 0.0 ? g[c] / s[S_GAMMA + c] : 0.0;
            s[S_GAMMA + c] = g[c];
        }
}

// End of an outer iteration: the primal residual r = |(a - R x, y - D x, z - x)|, the
// dual residual s = rho |R^T da + D^T dy + dz| (adaptive rho; its partials are the
// dual transpose's tiles), the data and TV costs, the non-finite flag and the log
// entry; the residual-balancing rho update (or the scheduled rho) and the pending
// dual rescale kappa = rho_old / rho_new.
__device__ inline void reduce_final(const RedArgs& A) {
    double* s = A.scal;
    if (!s) return;
    double sn[4], im[4], du[2];
    partial_sums<4, 4, 2>(A.sino, A.nb_sino, sn, A.img, A.nb_img, im, A.tiles,
                          A.dual ? A.nb_tiles : 0, du);
    if (threadIdx.x != 0) return;
    const double rho[2] = {s[S_RHO], s[S_RHO + 1]};
    double r[2], sd[2], nr[2];
    for (int c = 0; c < 2; ++c) {
        r[c] = sqrt(sn[c] + im[c]);
        sd[c] = rho[c] * sqrt(du[c]);
        nr[c] = rho[c];
        if (A.rho_mode == DECT_RHO_ADAPTIVE) {
            if (r[c] > A.bal_mu * sd[c]) nr[c] = rho[c] * A.bal_tau;
            else if (sd[c] > A.bal_mu * r[c]) nr[c] = rho[c] / A.bal_tau;
        }
    }
    if (A.rho_mode == DECT_RHO_SCHEDULE) {
        nr[0] = A.next_rho_c;
        nr[1] = A.next_rho_p;
    }
    const double data = sn[2];
    const double tv = s[S_LAM] * im[2] + s[S_LAM + 1] * im[3];
    bool bad = sn[3] > 0.0;
    for (int c = 0; c < 2; ++c) bad = bad || !isfinite(r[c]) || !isfinite(sd[c]);
    bad = bad || !isfinite(data) || !isfinite(tv);
    const long it = (long)s[S_ITER];
    double* L = A.log + (size_t)(it % kLogCap) * kLogStride;
    L[0] = (double)it;
    L[1] = bad ? 1.0 : 0.0;
    L[2] = rho[0];
    L[3] = rho[1];
    L[4] = r[0];
    L[5] = r[1];
    L[6] = sd[0];
    L[7] = sd[1];
    L[8] = data;
    L[9] = tv;
    for (int c = 0; c < 2; ++c) {
        s[S_KAPPA + c] = rho[c] / nr[c];
        s[S_RHO + c] = nr[c];
    }
    if (bad) s[S_FLAGS] = (double)((long)s[S_FLAGS] | 1L);
    s[S_ITER] = (double)(it + 1);
}

}  // namespace dect
