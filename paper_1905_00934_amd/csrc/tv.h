// TV/z/dual update of the ADMM image (Eqs. (9)-(11)), run by extra blocks of the
// a-update's launch (the two are independent).
#pragma once
#include "kernels.h"

namespace dect {

template <typename T>
__device__ inline T soft(T v, T t) {
    const T m = fabs(v) - t;
    return m > T(0) ? copysign(m, v) : T(0);
}

// y = shrink(D x - u^y, lambda/rho) (Eq. (9)), z = max(0, x - u^z) (Eq. (10)),
// u^y += y - D x, u^z += z - x (Eq. (11)); dy, dz = changes of y, z, for the pixels of
// image block blk.  Partials: |y - Dx|^2 + |z - x|^2 per basis, |y_c|_1, |y_p|_1.
// Every thread of the block must call it.
template <typename T>
__device__ inline void tv_dual_block(const TvArgs<T>& A, long blk) {
    using V2 = vec<T, 2>;
    using V4 = vec<T, 4>;
    const int nx = A.nx, ny = A.ny;
    const long N = (long)nx * ny;
    if (blk * (long)blockDim.x >= N) return;  // beyond this slice (whole block)
    const T* __restrict__ x = A.x;
    T* __restrict__ y = A.y;
    T* __restrict__ uy = A.uy;
    T* __restrict__ dy = A.dy;
    T* __restrict__ z = A.z;
    T* __restrict__ uz = A.uz;
    T* __restrict__ dz = A.dz;
    const double* __restrict__ scal = A.scal;
    const long pix = blk * (long)blockDim.x + threadIdx.x;
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (pix < N) {
        int i, j;
        pixel_ij(pix, nx, i, j);
        const V2* x2 = reinterpret_cast<const V2*>(x);
        const V2* p2 = reinterpret_cast<const V2*>(A.step_p);
        // x after the iteration's last CG step, x + alpha p, when that step is still
        // pending (the dual transpose's epilogue stores it with the same fma).
        const T al[2] = {(T)scal[S_ALPHA], (T)scal[S_ALPHA + 1]};
        auto xat = [&](long q) {
            V2 v = x2[q];
            if (p2) {
                const V2 pv = p2[q];
#pragma unroll
                for (int c = 0; c < 2; ++c) v.v[c] = fma(al[c], pv.v[c], v.v[c]);
            }
            return v;
        };
        const V2 xc = xat(pix);
        V4 Dx;
        if (i < nx - 1) {
            const V2 xr = xat(pix + 1);
            Dx.v[0] = xr.v[0] - xc.v[0];
            Dx.v[1] = xr.v[1] - xc.v[1];
        } else {
            Dx.v[0] = Dx.v[1] = T(0);
        }
        if (j < ny - 1) {
            const V2 xd = xat(pix + nx);
            Dx.v[2] = xd.v[0] - xc.v[0];
            Dx.v[3] = xd.v[1] - xc.v[1];
        } else {
            Dx.v[2] = Dx.v[3] = T(0);
        }
        const T th[2] = {(T)(scal[S_LAM] / scal[S_RHO]), (T)(scal[S_LAM + 1] / scal[S_RHO + 1])};
        // u^y and u^z as rescaled by the pending kappa (stored below with their update).
        const T kc[2] = {(T)scal[S_KAPPA], (T)scal[S_KAPPA + 1]};
        V4 u = reinterpret_cast<V4*>(uy)[pix];
#pragma unroll
        for (int k = 0; k < 4; ++k) u.v[k] = mul_rn(kc[k & 1], u.v[k]);
        const V4 yo = reinterpret_cast<V4*>(y)[pix];
        V4 yn, d;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            yn.v[k] = soft<T>(Dx.v[k] - u.v[k], th[k & 1]);
            u.v[k] += yn.v[k] - Dx.v[k];
            d.v[k] = yn.v[k] - yo.v[k];
            const double e = (double)(yn.v[k] - Dx.v[k]);
            part[k & 1] += e * e;
            part[2 + (k & 1)] += fabs((double)yn.v[k]);
        }
        reinterpret_cast<V4*>(y)[pix] = yn;
        reinterpret_cast<V4*>(uy)[pix] = u;
        reinterpret_cast<V4*>(dy)[pix] = d;
        V2 w = reinterpret_cast<V2*>(uz)[pix];
        w.v[0] = mul_rn(kc[0], w.v[0]);
        w.v[1] = mul_rn(kc[1], w.v[1]);
        const V2 zo = reinterpret_cast<V2*>(z)[pix];
        V2 zn, dzv;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            zn.v[c] = fmax(T(0), xc.v[c] - w.v[c]);
            w.v[c] += zn.v[c] - xc.v[c];
            dzv.v[c] = zn.v[c] - zo.v[c];
            const double e = (double)(zn.v[c] - xc.v[c]);
            part[c] += e * e;
        }
        reinterpret_cast<V2*>(z)[pix] = zn;
        reinterpret_cast<V2*>(uz)[pix] = w;
        reinterpret_cast<V2*>(dz)[pix] = dzv;
    }
    block_sum_store<4>(part, A.partials + (size_t)blk * kPartialSlots);
}

}  // namespace dect
