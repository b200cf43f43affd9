// Image-side epilogues of the ADMM transposes (CH = 2), shared by the transposed
// projector and the right-hand-side kernel.
#pragma once

#include "common.h"
#include "kernels.h"

namespace dect {

// The tracked R^T t = h + u of the right-hand side at pixel pix: u is read scaled by
// the pending kappa (scal == nullptr: 1) and stored back scaled.
template <typename T>
__device__ inline void rhs_tracked(const BpArgs<T>& a, size_t pix, T (&res)[2]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double u = a.u[2 * pix + c];
        if (a.scal) {
            u = mul_rn(a.scal[S_KAPPA + c], u);
            a.u[2 * pix + c] = u;
        }
        res[c] = (T)(a.h[2 * pix + c] + u);
    }
}

// Image-side terms added to R^T at pixel (i, j) for the ADMM epilogues (CH = 2).
// Adds the per-channel partial sums of the finished values to part.
template <typename T, int EPI>
__device__ inline void epilogue(const BpArgs<T>& a, int i, int j, T (&res)[2], double (&part)[2]) {
    using V2 = vec<T, 2>;
    using V4 = vec<T, 4>;
    const int nx = a.nx, ny = a.ny;
    const size_t pix = (size_t)j * nx + i;
    const V2* x2 = reinterpret_cast<const V2*>(a.x);
    if constexpr (EPI == EPI_RHS) {
        // r0 = R^T t + D^T (y + u^y - D x) + (z + u^z - x), Eq. (12), with u^y and u^z
        // scaled by the pending kappa as they are read (their stored values are
        // scaled by the TV update that follows).
        const T k0 = a.scal ? (T)a.scal[S_KAPPA] : T(1), k1 = a.scal ? (T)a.scal[S_KAPPA + 1] : T(1);
        const V4* y4 = reinterpret_cast<const V4*>(a.y);
        const V4* uy4 = reinterpret_cast<const V4*>(a.uy);
        auto u4 = [&](size_t q) {
            V4 v = uy4[q];
            v.v[0] = mul_rn(k0, v.v[0]);
            v.v[1] = mul_rn(k1, v.v[1]);
            v.v[2] = mul_rn(k0, v.v[2]);
            v.v[3] = mul_rn(k1, v.v[3]);
            return v;
        };
        const V2 xc = x2[pix];
        const V2 z = reinterpret_cast<const V2*>(a.z)[pix];
        V2 uz = reinterpret_cast<const V2*>(a.uz)[pix];
        uz.v[0] = mul_rn(k0, uz.v[0]);
        uz.v[1] = mul_rn(k1, uz.v[1]);
        const V4 yc = y4[pix], uc = u4(pix);
#pragma unroll
        for (int c = 0; c < 2; ++c) res[c] += z.v[c] + uz.v[c] - xc.v[c];
        if (i < nx - 1) {
            const V2 xr = x2[pix + 1];
#pragma unroll
            for (int c = 0; c < 2; ++c) res[c] -= yc.v[c] + uc.v[c] - (xr.v[c] - xc.v[c]);
        }
        if (i > 0) {
            const V2 xl = x2[pix - 1];
            const V4 yl = y4[pix - 1], ul = u4(pix - 1);
#pragma unroll
            for (int c = 0; c < 2; ++c) res[c] += yl.v[c] + ul.v[c] - (xc.v[c] - xl.v[c]);
        }
        if (j < ny - 1) {
            const V2 xd = x2[pix + nx];
#pragma unroll
            for (int c = 0; c < 2; ++c) res[c] -= yc.v[2 + c] + uc.v[2 + c] - (xd.v[c] - xc.v[c]);
        }
        if (j > 0) {
            const V2 xu = x2[pix - nx];
            const V4 yu = y4[pix - nx], uu = u4(pix - nx);
#pragma unroll
            for (int c = 0; c < 2; ++c) res[c] += yu.v[2 + c] + uu.v[2 + c] - (xc.v[c] - xu.v[c]);
        }
        V2 o;
        o.v[0] = res[0];
        o.v[1] = res[1];
        reinterpret_cast<V2*>(a.out)[pix] = o;
        if (a.out2) reinterpret_cast<V2*>(a.out2)[pix] = o;
        part[0] += (double)res[0] * (double)res[0];
        part[1] += (double)res[1] * (double)res[1];
    } else if constexpr (EPI == EPI_Q) {
        // q = R^T R p + D^T D p + p; a.x holds p.  raw: R^T R p itself.
        if (a.raw) {
            V2 o;
            o.v[0] = res[0];
            o.v[1] = res[1];
            reinterpret_cast<V2*>(a.raw)[pix] = o;
        }
        const V2 pc = x2[pix];
#pragma unroll
        for (int c = 0; c < 2; ++c) res[c] += pc.v[c];
        if (i < nx - 1) { const V2 q = x2[pix + 1]; for (int c = 0; c < 2; ++c) res[c] += pc.v[c] - q.v[c]; }
        if (i > 0) { const V2 q = x2[pix - 1]; for (int c = 0; c < 2; ++c) res[c] += pc.v[c] - q.v[c]; }
        if (j < ny - 1) { const V2 q = x2[pix + nx]; for (int c = 0; c < 2; ++c) res[c] += pc.v[c] - q.v[c]; }
        if (j > 0) { const V2 q = x2[pix - nx]; for (int c = 0; c < 2; ++c) res[c] += pc.v[c] - q.v[c]; }
        if (a.out) {
            V2 o;
            o.v[0] = res[0];
            o.v[1] = res[1];
            reinterpret_cast<V2*>(a.out)[pix] = o;
        }
        part[0] += (double)pc.v[0] * (double)res[0];
        part[1] += (double)pc.v[1] * (double)res[1];
    } else {  // EPI_DUAL: s = R^T da + D^T dy + dz; h += R^T da
        if (a.h) {
            double hv[2] = {a.h[2 * pix] + (double)res[0], a.h[2 * pix + 1] + (double)res[1]};
            if (a.step_x) {
                // The iteration's last CG step: x += alpha p, and R x having moved by
                // alpha R p, the tracked R^T (a - R x) by -alpha R^T R p.  Then the
                // a-block dual update u^a += a - R x in R^T form, u += h; its rescale by
                // kappa (not known before this launch's partials are summed) is left to
                // the readers of u.
                const double al[2] = {a.scal[S_ALPHA], a.scal[S_ALPHA + 1]};
                V2 xv = reinterpret_cast<V2*>(a.step_x)[pix];
                const V2 pv = reinterpret_cast<const V2*>(a.step_p)[pix];
                const V2 rr = reinterpret_cast<const V2*>(a.step_rtrp)[pix];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    xv.v[c] = fma((T)al[c], pv.v[c], xv.v[c]);
                    hv[c] = fma(-al[c], (double)rr.v[c], hv[c]);
                    a.u[2 * pix + c] = a.u[2 * pix + c] + hv[c];
                }
                reinterpret_cast<V2*>(a.step_x)[pix] = xv;
            }
            a.h[2 * pix] = hv[0];
            a.h[2 * pix + 1] = hv[1];
        }
        const V4* d4 = reinterpret_cast<const V4*>(a.y);
        const V4 dc = d4[pix];
        const V2 dz = reinterpret_cast<const V2*>(a.z)[pix];
#pragma unroll
        for (int c = 0; c < 2; ++c) res[c] += dz.v[c];
        if (i < nx - 1) for (int c = 0; c < 2; ++c) res[c] -= dc.v[c];
        if (i > 0) { const V4 dl = d4[pix - 1]; for (int c = 0; c < 2; ++c) res[c] += dl.v[c]; }
        if (j < ny - 1) for (int c = 0; c < 2; ++c) res[c] -= dc.v[2 + c];
        if (j > 0) { const V4 du = d4[pix - nx]; for (int c = 0; c < 2; ++c) res[c] += du.v[2 + c]; }
        part[0] += (double)res[0] * (double)res[0];
        part[1] += (double)res[1] * (double)res[1];
    }
}

}  // namespace dect
