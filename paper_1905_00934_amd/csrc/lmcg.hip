// The baseline LM(m) x CG(n) splitting (Eqs. (7)-(8), Table 1) on the device.
//
// One outer iteration: x_c by Eq. (7) with x_p fixed, then x_p by Eq. (8) with the
// new x_c; each is m Levenberg-Marquardt iterations on
//   Phi(x_b) = 1/2 ||f(R x_c, R x_p) - m||^2_Sigma + rho_b/2 ||[y_b; z_b] - [D; I] x_b + u_b||^2,
// whose Gauss-Newton system (R^T W R + rho_b (D^T D + I) + mu kappa I) d = -grad Phi
// (W = sum_s w_s (df_s/da_b)^2 per ray, kappa = g'Hg / g'g the curvature along the
// gradient, taken in the first CG step) is solved by n CG steps from d = 0 with the
// single-channel R and R^T; the trial x + d is projected, f is evaluated there, and
// the step is kept if Phi decreases (mu / 10) or dropped (mu * 10).  f and its
// gradient at R x are cached per ray, so an LM iteration evaluates f once.  Then
// y, z and the scaled duals (Eqs. (9)-(11) with C = [D; I]) and rho from the
// residuals, as in the proposed scheme but with no a-block.
//
// Every scalar (CG alpha, beta, kappa, mu, the accept decision, rho) stays on the
// device; the launch sequence is fixed, so an iteration is one host call.  Images
// are planar per basis ([2][ny][nx]; y and u^y [2][2][ny][nx] with the horizontal
// then the vertical difference), sinograms [2][V][D] in standard order.
#include <cstring>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "profile.h"

namespace dect {
namespace {

enum LmScalar : int {
    L_RHO = 0,     // [2] rho in force
    L_LAM = 2,     // [2] lambda
    L_SCALE = 4,   // [2] pending dual rescale rho_old / rho_new
    L_MU = 6,      // LM damping of the basis being updated
    L_KAPPA = 7,   // curvature along the gradient
    L_FIRST = 8,   // 1 until the first CG step of an LM iteration has set kappa
    L_RR = 9,      // r . r
    L_ALPHA = 10,
    L_BETA = 11,
    L_PHI = 12,    // Phi at the current x
    L_DATA = 13,   // data term at the current R x
    L_ACC = 14,    // 1 if the last trial was accepted
    L_ITER = 15,
    L_FLAGS = 16,  // bit 0: non-finite value met
    L_MU0 = 17,
    L_COUNT = 24
};

enum LmReduce : int { LR_GRAD = 0, LR_Q = 1, LR_UPD = 2, LR_TRIAL = 3, LR_FINAL = 4 };

struct LmLayout {
    size_t bytes;
    size_t x, y, uy, z, uz, Rx, scalars;  // public
    size_t r, pv, q, d, xt, tmp, dy, dz;  // images
    size_t t, W, Rp, at;                  // sinograms
    size_t fc, ft;                        // f caches [6][M]
    size_t part, log;
    int nb_s, nb_i;
};

LmLayout lm_layout(const dect_plan* p) {
    const size_t e = p->elem, N = (size_t)p->N, M = (size_t)p->M;
    LmLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    L.x = take(2 * N * e);
    L.y = take(4 * N * e);
    L.uy = take(4 * N * e);
    L.z = take(2 * N * e);
    L.uz = take(2 * N * e);
    L.Rx = take(2 * M * e);
    L.scalars = take(L_COUNT * sizeof(double));
    L.r = take(N * e);
    L.pv = take(N * e);
    L.q = take(N * e);
    L.d = take(N * e);
    L.xt = take(N * e);
    L.tmp = take(N * e);
    L.dy = take(4 * N * e);
    L.dz = take(2 * N * e);
    L.t = take(M * e);
    L.W = take(M * e);
    L.Rp = take(M * e);
    L.at = take(M * e);
    L.fc = take(6 * M * e);
    L.ft = take(6 * M * e);
    L.nb_s = (int)((M + 255) / 256);
    L.nb_i = (int)((N + 255) / 256);
    L.part = take((size_t)(L.nb_s + 2 * L.nb_i) * kPartialSlots * sizeof(double));
    L.log = take((size_t)kLogCap * kLogStride * sizeof(double));
    L.bytes = off;
    return L;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

// (D^T D v) at pixel k = (j, i): D^T of the forward differences (zero at the last
// column and row).
template <typename T>
__device__ inline T dtd(const T* __restrict__ v, int i, int j, int nx, int ny, long k) {
    const T c = v[k];
    T s = T(0);
    if (i < nx - 1) s -= v[k + 1] - c;
    if (i > 0) s += c - v[k - 1];
    if (j < ny - 1) s -= v[k + nx] - c;
    if (j > 0) s += c - v[k - nx];
    return s;
}

// D^T (h, v) at pixel k, with h's last column and v's last row ignored.
template <typename T>
__device__ inline T dt(const T* __restrict__ h, const T* __restrict__ v, int i, int j, int nx,
                       int ny, long k) {
    T s = T(0);
    if (i < nx - 1) s -= h[k];
    if (i > 0) s += h[k - 1];
    if (j < ny - 1) s -= v[k];
    if (j > 0) s += v[k - nx];
    return s;
}

template <typename T>
__device__ inline T soft(T v, T t) {
    const T m = fabs(v) - t;
    return m > T(0) ? copysign(m, v) : T(0);
}

// Penalty terms of Phi at image v: 1/2 rho (|y - D v + u^y|^2 + |z - v + u^z|^2) at k.
template <typename T>
__device__ inline double pen_at(const T* __restrict__ v, const T* __restrict__ yh,
                                const T* __restrict__ yv, const T* __restrict__ uyh,
                                const T* __restrict__ uyv, const T* __restrict__ z,
                                const T* __restrict__ uz, int i, int j, int nx, int ny, long k,
                                double rho) {
    const T c = v[k];
    const T dxh = i < nx - 1 ? v[k + 1] - c : T(0);
    const T dxv = j < ny - 1 ? v[k + nx] - c : T(0);
    const double eh = (double)(yh[k] - dxh + uyh[k]);
    const double ev = (double)(yv[k] - dxv + uyv[k]);
    const double ez = (double)(z[k] - c + uz[k]);
    return 0.5 * rho * (eh * eh + ev * ev + ez * ez);
}

struct ImgArgs {
    int nx, ny;
    long N;
};

// Per ray, from the f cache at the current R x: the gradient sinogram
// t = sum_s w_s (f_s - m_s) df_s/da_b, W = sum_s w_s (df_s/da_b)^2, and the data term.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_setup(long M, int b, const T* __restrict__ mh,
                                                  const T* __restrict__ ml,
                                                  const T* __restrict__ wh,
                                                  const T* __restrict__ wl,
                                                  const T* __restrict__ fc, T* __restrict__ t,
                                                  T* __restrict__ W, double* __restrict__ part) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < M) {
        const T eh = fc[i] - mh[i], el = fc[M + i] - ml[i];
        const T jh = fc[(2 + b) * M + i], jl = fc[(4 + b) * M + i];
        t[i] = wh[i] * eh * jh + wl[i] * el * jl;
        W[i] = wh[i] * jh * jh + wl[i] * jl * jl;
        const double deh = (double)fc[i] - (double)mh[i], del = (double)fc[M + i] - (double)ml[i];
        v[0] = 0.5 * ((double)wh[i] * deh * deh + (double)wl[i] * del * del);
    }
    block_sum_store<4>(v, part + (size_t)blockIdx.x * kPartialSlots);
}

// g = R^T t + rho (D^T D x + x - D^T (y + u^y) - z - u^z); r = p = -g; d = 0.
// Partials: g . g, the penalty at x.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_grad(ImgArgs I, int b, const T* __restrict__ bp,
                                                 const T* __restrict__ x,
                                                 const T* __restrict__ yh,
                                                 const T* __restrict__ yv,
                                                 const T* __restrict__ uyh,
                                                 const T* __restrict__ uyv,
                                                 const T* __restrict__ z,
                                                 const T* __restrict__ uz,
                                                 const double* __restrict__ sc, T* __restrict__ r,
                                                 T* __restrict__ p, T* __restrict__ d,
                                                 double* __restrict__ part) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (k < I.N) {
        int i, j;
        pixel_ij(k, I.nx, i, j);
        const int nx = I.nx, ny = I.ny;
        const double rho_d = sc[L_RHO + b];
        const T rho = (T)rho_d;
        T s = T(0);
        if (i < nx - 1) s -= yh[k] + uyh[k];
        if (i > 0) s += yh[k - 1] + uyh[k - 1];
        if (j < ny - 1) s -= yv[k] + uyv[k];
        if (j > 0) s += yv[k - nx] + uyv[k - nx];
        const T g = bp[k] + rho * (dtd(x, i, j, nx, ny, k) + x[k] - s - z[k] - uz[k]);
        r[k] = -g;
        p[k] = -g;
        d[k] = T(0);
        v[0] = (double)g * (double)g;
        v[1] = pen_at(x, yh, yv, uyh, uyv, z, uz, i, j, nx, ny, k, rho_d);
    }
    block_sum_store<4>(v, part + (size_t)blockIdx.x * kPartialSlots);
}

template <typename T>
__global__ __launch_bounds__(256) void k_lm_wmul(long M, const T* __restrict__ W,
                                                 T* __restrict__ Rp) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) Rp[i] *= W[i];
}

// H p = R^T W R p + rho (D^T D p + p) (undamped) into q; partials p . Hp, p . p.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_hp(ImgArgs I, int b, const T* __restrict__ bp,
                                               const T* __restrict__ p,
                                               const double* __restrict__ sc, T* __restrict__ q,
                                               double* __restrict__ part) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (k < I.N) {
        int i, j;
        pixel_ij(k, I.nx, i, j);
        const T rho = (T)sc[L_RHO + b];
        const T hp = bp[k] + rho * (dtd(p, i, j, I.nx, I.ny, k) + p[k]);
        q[k] = hp;
        v[0] = (double)p[k] * (double)hp;
        v[1] = (double)p[k] * (double)p[k];
    }
    block_sum_store<4>(v, part + (size_t)blockIdx.x * kPartialSlots);
}

// q = H p + mu kappa p; d += alpha p; r -= alpha q; partial r . r.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_step(long N, const double* __restrict__ sc,
                                                 const T* __restrict__ p, const T* __restrict__ q,
                                                 T* __restrict__ d, T* __restrict__ r,
                                                 double* __restrict__ part) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (k < N) {
        const T damp = (T)(sc[L_MU] * sc[L_KAPPA]), alpha = (T)sc[L_ALPHA];
        const T pk = p[k];
        const T qk = q[k] + damp * pk;
        d[k] += alpha * pk;
        const T rk = r[k] - alpha * qk;
        r[k] = rk;
        v[0] = (double)rk * (double)rk;
    }
    block_sum_store<4>(v, part + (size_t)blockIdx.x * kPartialSlots);
}

template <typename T>
__global__ __launch_bounds__(256) void k_lm_dir(long N, const double* __restrict__ sc,
                                                const T* __restrict__ r, T* __restrict__ p) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N) p[k] = r[k] + (T)sc[L_BETA] * p[k];
}

// Trial image xt = x + d; partial: the penalty at xt.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_trial_x(ImgArgs I, int b, const T* __restrict__ x,
                                                    const T* __restrict__ d,
                                                    const T* __restrict__ yh,
                                                    const T* __restrict__ yv,
                                                    const T* __restrict__ uyh,
                                                    const T* __restrict__ uyv,
                                                    const T* __restrict__ z,
                                                    const T* __restrict__ uz,
                                                    const double* __restrict__ sc,
                                                    T* __restrict__ xt, double* __restrict__ part) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (k < I.N) {
        int i, j;
        pixel_ij(k, I.nx, i, j);
        const int nx = I.nx, ny = I.ny;
        const T c = x[k] + d[k];
        xt[k] = c;
        // The penalty at x + d, from x and d (xt is being written by other threads).
        const T dxh = i < nx - 1 ? (x[k + 1] + d[k + 1]) - c : T(0);
        const T dxv = j < ny - 1 ? (x[k + nx] + d[k + nx]) - c : T(0);
        const double eh = (double)(yh[k] - dxh + uyh[k]);
        const double ev = (double)(yv[k] - dxv + uyv[k]);
        const double ez = (double)(z[k] - c + uz[k]);
        v[0] = 0.5 * sc[L_RHO + b] * (eh * eh + ev * ev + ez * ez);
    }
    block_sum_store<4>(v, part + (size_t)blockIdx.x * kPartialSlots);
}

template <typename T>
__global__ __launch_bounds__(256) void k_lm_accept_img(long N, const double* __restrict__ sc,
                                                       const T* __restrict__ xt,
                                                       T* __restrict__ x) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N && sc[L_ACC] != 0.0) x[k] = xt[k];
}

template <typename T>
__global__ __launch_bounds__(256) void k_lm_accept_sino(long M, const double* __restrict__ sc,
                                                        const T* __restrict__ at,
                                                        const T* __restrict__ ft,
                                                        T* __restrict__ Rx, T* __restrict__ fc) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M || sc[L_ACC] == 0.0) return;
    Rx[i] = at[i];
#pragma unroll
    for (int c = 0; c < 6; ++c) fc[c * M + i] = ft[c * M + i];
}

// y = shrink(D x - u^y, lambda / rho), z = max(0, x - u^z), u^y += y - D x, u^z += z - x
// for both bases (Eqs. (9)-(11)); dy, dz keep the changes of y and z.  Partials:
// |y - D x|^2 + |z - x|^2 per basis, |y|_1 per basis.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_tv(ImgArgs I, const T* __restrict__ x,
                                               T* __restrict__ y, T* __restrict__ uy,
                                               T* __restrict__ z, T* __restrict__ uz,
                                               T* __restrict__ dy, T* __restrict__ dz,
                                               const double* __restrict__ sc,
                                               double* __restrict__ part) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (k < I.N) {
        const long N = I.N;
        int i, j;
        pixel_ij(k, I.nx, i, j);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const T* xb = x + b * N;
            const T th = (T)(sc[L_LAM + b] / sc[L_RHO + b]);
            const T c = xb[k];
            const T dx[2] = {i < I.nx - 1 ? xb[k + 1] - c : T(0),
                             j < I.ny - 1 ? xb[k + I.nx] - c : T(0)};
            double res = 0.0, l1 = 0.0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const long o = (2 * b + a) * N + k;
                const T yn = soft<T>(dx[a] - uy[o], th);
                dy[o] = yn - y[o];
                y[o] = yn;
                uy[o] += yn - dx[a];
                res += (double)(yn - dx[a]) * (double)(yn - dx[a]);
                l1 += fabs((double)yn);
            }
            const long o = b * N + k;
            const T zn = fmax(c - uz[o], T(0));
            dz[o] = zn - z[o];
            z[o] = zn;
            uz[o] += zn - c;
            res += (double)(zn - c) * (double)(zn - c);
            v[b] = res;
            v[2 + b] = l1;
        }
    }
    block_sum_store<4>(v, part + (size_t)blockIdx.x * kPartialSlots);
}

// |D^T dy + dz|^2 per basis (the dual residual without an R^T term).
template <typename T>
__global__ __launch_bounds__(256) void k_lm_dual(ImgArgs I, const T* __restrict__ dy,
                                                 const T* __restrict__ dz,
                                                 double* __restrict__ part) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (k < I.N) {
        const long N = I.N;
        int i, j;
        pixel_ij(k, I.nx, i, j);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const T s = dt(dy + 2 * b * N, dy + (2 * b + 1) * N, i, j, I.nx, I.ny, k) + dz[b * N + k];
            v[b] = (double)s * (double)s;
        }
    }
    block_sum_store<4>(v, part + (size_t)blockIdx.x * kPartialSlots);
}

template <typename T>
__global__ __launch_bounds__(256) void k_lm_rescale(long N, const double* __restrict__ sc,
                                                    T* __restrict__ uy, T* __restrict__ uz) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const T f = (T)sc[L_SCALE + b];
        uy[2 * b * N + k] *= f;
        uy[(2 * b + 1) * N + k] *= f;
        uz[b * N + k] *= f;
    }
}


struct RedLm {
    double* sc;
    const double* sino;  // per-ray partials (nb_s blocks)
    const double* img;   // per-pixel partials (nb_i blocks)
    const double* dual;  // dual-residual partials (nb_i blocks)
    int nb_s, nb_i;
    int rho_mode;
    double bal_mu, bal_tau;
    double* log;
};

__global__ __launch_bounds__(256) void k_lm_reduce(RedLm A, int mode, int reset_mu) {
    double* s = A.sc;
    if (mode == LR_GRAD) {
        double dn[4], im[4];
        partial_sum<4>(A.sino, A.nb_s, dn);
        partial_sum<4>(A.img, A.nb_i, im);
        if (threadIdx.x == 0) {
            s[L_DATA] = dn[0];
            s[L_PHI] = dn[0] + im[1];
            s[L_RR] = im[0];
            s[L_FIRST] = 1.0;
            if (reset_mu) s[L_MU] = s[L_MU0];
        }
    } else if (mode == LR_Q) {
        double im[4];
        partial_sum<4>(A.img, A.nb_i, im);
        if (threadIdx.x == 0) {
            const double php = im[0], pp = im[1];
            if (s[L_FIRST] != 0.0) {
                s[L_KAPPA] = pp > 0.0 ? php / pp : 0.0;
                s[L_FIRST] = 0.0;
            }
            const double pq = php + s[L_MU] * s[L_KAPPA] * pp;
            s[L_ALPHA] = pq > 0.0 ? s[L_RR] / pq : 0.0;
        }
    } else if (mode == LR_UPD) {
        double im[4];
        partial_sum<4>(A.img, A.nb_i, im);
        if (threadIdx.x == 0) {
            s[L_BETA] = s[L_RR] > 0.0 ? im[0] / s[L_RR] : 0.0;
            s[L_RR] = im[0];
        }
    } else if (mode == LR_TRIAL) {
        double dn[4], im[4];
        partial_sum<4>(A.sino, A.nb_s, dn);
        partial_sum<4>(A.img, A.nb_i, im);
        if (threadIdx.x == 0) {
            const double phit = dn[0] + im[0];
            const bool acc = phit < s[L_PHI];
            s[L_ACC] = acc ? 1.0 : 0.0;
            if (acc) {
                s[L_DATA] = dn[0];
                s[L_MU] /= 10.0;
            } else {
                s[L_MU] *= 10.0;
            }
            if (dn[1] > 0.0 || !isfinite(phit)) s[L_FLAGS] = (double)((long)s[L_FLAGS] | 1L);
        }
    } else {
        double im[4], du[4];
        partial_sum<4>(A.img, A.nb_i, im);
        partial_sum<4>(A.dual, A.nb_i, du);
        if (threadIdx.x == 0) {
            const double rho[2] = {s[L_RHO], s[L_RHO + 1]};
            double r[2], sd[2], nr[2];
            for (int c = 0; c < 2; ++c) {
                r[c] = sqrt(im[c]);
                sd[c] = A.rho_mode == DECT_RHO_ADAPTIVE ? rho[c] * sqrt(du[c]) : 0.0;
                nr[c] = rho[c];
                if (A.rho_mode == DECT_RHO_ADAPTIVE) {
                    if (r[c] > A.bal_mu * sd[c]) nr[c] = rho[c] * A.bal_tau;
                    else if (sd[c] > A.bal_mu * r[c]) nr[c] = rho[c] / A.bal_tau;
                }
            }
            const double data = s[L_DATA];
            const double tv = s[L_LAM] * im[2] + s[L_LAM + 1] * im[3];
            bool bad = ((long)s[L_FLAGS] & 1L) != 0;
            for (int c = 0; c < 2; ++c) bad = bad || !isfinite(r[c]) || !isfinite(sd[c]);
            bad = bad || !isfinite(data) || !isfinite(tv);
            const long it = (long)s[L_ITER];
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
                s[L_SCALE + c] = rho[c] / nr[c];
                s[L_RHO + c] = nr[c];
            }
            if (bad) s[L_FLAGS] = (double)((long)s[L_FLAGS] | 1L);
            s[L_ITER] = (double)(it + 1);
        }
    }
}

// x (planar) and z from the pair image x0 [N][2] (or zero), y = D x, u = 0.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_init(ImgArgs I, const T* __restrict__ x0,
                                                 T* __restrict__ x, T* __restrict__ y,
                                                 T* __restrict__ uy, T* __restrict__ z,
                                                 T* __restrict__ uz) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= I.N) return;
    const long N = I.N;
    int i, j;
    pixel_ij(k, I.nx, i, j);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const T c = x0 ? x0[2 * k + b] : T(0);
        const T r = (x0 && i < I.nx - 1) ? x0[2 * (k + 1) + b] - c : T(0);
        const T u = (x0 && j < I.ny - 1) ? x0[2 * (k + I.nx) + b] - c : T(0);
        x[b * N + k] = c;
        z[b * N + k] = c;
        uz[b * N + k] = T(0);
        y[2 * b * N + k] = r;
        y[(2 * b + 1) * N + k] = u;
        uy[2 * b * N + k] = T(0);
        uy[(2 * b + 1) * N + k] = T(0);
    }
}

__global__ void k_lm_scalars(double* s, double rc, double rp, double lc, double lp, double mu0) {
    if (threadIdx.x != 0) return;
    for (int k = 0; k < L_COUNT; ++k) s[k] = 0.0;
    s[L_RHO] = rc;
    s[L_RHO + 1] = rp;
    s[L_LAM] = lc;
    s[L_LAM + 1] = lp;
    s[L_SCALE] = s[L_SCALE + 1] = 1.0;
    s[L_MU0] = mu0;
    s[L_MU] = mu0;
}

template <typename T>
struct LmPtrs {
    T *x, *y, *uy, *z, *uz, *Rx, *r, *pv, *q, *d, *xt, *tmp, *dy, *dz, *t, *W, *Rp, *at, *fc, *ft;
    double *sc, *psino, *pimg, *pdual, *log;
};

template <typename T>
LmPtrs<T> lm_ptrs(const LmLayout& L, void* st) {
    LmPtrs<T> P;
    P.x = at<T>(st, L.x);
    P.y = at<T>(st, L.y);
    P.uy = at<T>(st, L.uy);
    P.z = at<T>(st, L.z);
    P.uz = at<T>(st, L.uz);
    P.Rx = at<T>(st, L.Rx);
    P.r = at<T>(st, L.r);
    P.pv = at<T>(st, L.pv);
    P.q = at<T>(st, L.q);
    P.d = at<T>(st, L.d);
    P.xt = at<T>(st, L.xt);
    P.tmp = at<T>(st, L.tmp);
    P.dy = at<T>(st, L.dy);
    P.dz = at<T>(st, L.dz);
    P.t = at<T>(st, L.t);
    P.W = at<T>(st, L.W);
    P.Rp = at<T>(st, L.Rp);
    P.at = at<T>(st, L.at);
    P.fc = at<T>(st, L.fc);
    P.ft = at<T>(st, L.ft);
    P.sc = at<double>(st, L.scalars);
    P.psino = at<double>(st, L.part);
    P.pimg = P.psino + (size_t)L.nb_s * kPartialSlots;
    P.pdual = P.pimg + (size_t)L.nb_i * kPartialSlots;
    P.log = at<double>(st, L.log);
    return P;
}

template <typename T>
hipError_t bp1(const dect_plan* p, const T* sino, T* img, hipStream_t s) {
    BpArgs<T> a{};
    a.sino = sino;
    a.out = img;
    return launch_backproject<T>(p, 1, a, s);
}

#define LM_TRY(expr)                          \
    do {                                      \
        const hipError_t e_ = (expr);         \
        if (e_ != hipSuccess) return e_;      \
    } while (0)

template <typename T>
hipError_t lm_iteration(const dect_plan* p, const LmLayout& L, const LmPtrs<T>& P,
                        const T* mh, const T* ml, const T* wh, const T* wl,
                        const dect_params* prm, hipStream_t s) {
    const long N = p->N, M = p->M;
    const ImgArgs I{p->nx, p->ny, N};
    const dim3 gi(nblk(N)), gs(nblk(M)), b256(256);
    RedLm R{P.sc, P.psino, P.pimg, P.pdual, L.nb_s, L.nb_i, prm->rho_mode, prm->bal_mu,
            prm->bal_tau, P.log};
    for (int b = 0; b < 2; ++b) {
        T* xb = P.x + b * N;
        const T* yh = P.y + 2 * b * N;
        const T* yv = P.y + (2 * b + 1) * N;
        const T* uyh = P.uy + 2 * b * N;
        const T* uyv = P.uy + (2 * b + 1) * N;
        const T* zb = P.z + b * N;
        const T* uzb = P.uz + b * N;
        T* Rxb = P.Rx + b * M;
        const T* Rxo = P.Rx + (1 - b) * M;
        for (int l = 0; l < prm->lm_iters; ++l) {
            {
                ProfScope ps("lm_vec", s);
                hipLaunchKernelGGL((k_lm_setup<T>), gs, b256, 0, s, M, b, mh, ml, wh, wl, P.fc,
                                   P.t, P.W, P.psino);
            }
            LM_TRY(bp1<T>(p, P.t, P.tmp, s));
            {
                ProfScope ps("lm_vec", s);
                hipLaunchKernelGGL((k_lm_grad<T>), gi, b256, 0, s, I, b, P.tmp, xb, yh, yv, uyh,
                                   uyv, zb, uzb, P.sc, P.r, P.pv, P.d, P.pimg);
            }
            {
                ProfScope ps("lm_reduce", s);
                hipLaunchKernelGGL(k_lm_reduce, dim3(1), b256, 0, s, R, (int)LR_GRAD,
                                   l == 0 ? 1 : 0);
            }
            for (int c = 0; c < prm->cg_iters; ++c) {
                LM_TRY(launch_project<T>(p, P.pv, P.Rp, 1, s));
                {
                    ProfScope ps("lm_vec", s);
                    hipLaunchKernelGGL((k_lm_wmul<T>), gs, b256, 0, s, M, P.W, P.Rp);
                }
                LM_TRY(bp1<T>(p, P.Rp, P.tmp, s));
                ProfScope ps("lm_vec", s);
                hipLaunchKernelGGL((k_lm_hp<T>), gi, b256, 0, s, I, b, P.tmp, P.pv, P.sc, P.q,
                                   P.pimg);
                hipLaunchKernelGGL(k_lm_reduce, dim3(1), b256, 0, s, R, (int)LR_Q, 0);
                hipLaunchKernelGGL((k_lm_step<T>), gi, b256, 0, s, N, P.sc, P.pv, P.q, P.d, P.r,
                                   P.pimg);
                hipLaunchKernelGGL(k_lm_reduce, dim3(1), b256, 0, s, R, (int)LR_UPD, 0);
                hipLaunchKernelGGL((k_lm_dir<T>), gi, b256, 0, s, N, P.sc, P.r, P.pv);
            }
            {
                ProfScope ps("lm_vec", s);
                hipLaunchKernelGGL((k_lm_trial_x<T>), gi, b256, 0, s, I, b, xb, P.d, yh, yv, uyh,
                                   uyv, zb, uzb, P.sc, P.xt, P.pimg);
            }
            LM_TRY(launch_project<T>(p, P.xt, P.at, 1, s));
            LM_TRY(launch_lm_eval<T>(p, b, P.at, Rxo, mh, ml, wh, wl, P.ft, P.psino, s));
            ProfScope ps("lm_vec", s);
            hipLaunchKernelGGL(k_lm_reduce, dim3(1), b256, 0, s, R, (int)LR_TRIAL, 0);
            hipLaunchKernelGGL((k_lm_accept_img<T>), gi, b256, 0, s, N, P.sc, P.xt, xb);
            hipLaunchKernelGGL((k_lm_accept_sino<T>), gs, b256, 0, s, M, P.sc, P.at, P.ft, Rxb,
                               P.fc);
        }
    }
    ProfScope ps("lm_tv", s);
    hipLaunchKernelGGL((k_lm_tv<T>), gi, b256, 0, s, I, P.x, P.y, P.uy, P.z, P.uz, P.dy, P.dz,
                       P.sc, P.pimg);
    hipLaunchKernelGGL((k_lm_dual<T>), gi, b256, 0, s, I, P.dy, P.dz, P.pdual);
    hipLaunchKernelGGL(k_lm_reduce, dim3(1), b256, 0, s, R, (int)LR_FINAL, 0);
    hipLaunchKernelGGL((k_lm_rescale<T>), gi, b256, 0, s, N, P.sc, P.uy, P.uz);
    return hipGetLastError();
}

template <typename T>
hipError_t lm_init(const dect_plan* p, const LmLayout& L, const LmPtrs<T>& P, const T* mh,
                   const T* ml, const T* wh, const T* wl, const T* x0, const dect_params* prm,
                   hipStream_t s) {
    const long N = p->N, M = p->M;
    const ImgArgs I{p->nx, p->ny, N};
    hipLaunchKernelGGL(k_lm_scalars, dim3(1), dim3(64), 0, s, P.sc, prm->rho_c, prm->rho_p,
                       prm->lambda_c, prm->lambda_p, prm->lm_mu0);
    hipLaunchKernelGGL((k_lm_init<T>), dim3(nblk(N)), dim3(256), 0, s, I, x0, P.x, P.y, P.uy,
                       P.z, P.uz);
    LM_TRY(hipGetLastError());
    LM_TRY(launch_project<T>(p, P.x, P.Rx, 1, s));
    LM_TRY(launch_project<T>(p, P.x + N, P.Rx + M, 1, s));
    return launch_lm_eval<T>(p, 0, P.Rx, P.Rx + M, mh, ml, wh, wl, P.fc, P.psino, s);
}

dect_status check_lm_params(const dect_params* prm) {
    if (!prm) return fail(DECT_E_ARG, "null params");
    if (prm->lm_iters < 1 || prm->cg_iters < 1)
        return fail(DECT_E_ARG, "lm_iters and cg_iters must be >= 1");
    if (prm->rho_mode != DECT_RHO_FIXED && prm->rho_mode != DECT_RHO_ADAPTIVE)
        return fail(DECT_E_ARG, "the LM x CG scheme takes rho_mode FIXED or ADAPTIVE (got %d)",
                    prm->rho_mode);
    if (!(prm->rho_c > 0) || !(prm->rho_p > 0) || !(prm->lambda_c >= 0) || !(prm->lambda_p >= 0))
        return fail(DECT_E_ARG, "rho must be > 0 and lambda >= 0");
    if (prm->rho_mode == DECT_RHO_ADAPTIVE && (!(prm->bal_mu > 1) || !(prm->bal_tau > 1)))
        return fail(DECT_E_ARG, "residual balancing needs mu > 1 and tau > 1");
    if (!(prm->lm_mu0 >= 0)) return fail(DECT_E_ARG, "lm_mu0 must be >= 0");
    if (prm->precond != DECT_PRECOND_NONE)
        return fail(DECT_E_ARG, "the LM x CG scheme has no preconditioner");
    return DECT_OK;
}

}  // namespace
}  // namespace dect

using namespace dect;

extern "C" {

size_t dect_lmcg_state_bytes(const dect_plan* p) { return p ? lm_layout(p).bytes : 0; }

dect_status dect_lmcg_state_layout(const dect_plan* p, dect_lmcg_layout* out) {
    if (!p || !out) return fail(DECT_E_ARG, "null argument");
    const LmLayout L = lm_layout(p);
    std::memset(out, 0, sizeof *out);
    out->bytes = L.bytes;
    out->x = L.x;
    out->y = L.y;
    out->uy = L.uy;
    out->z = L.z;
    out->uz = L.uz;
    out->Rx = L.Rx;
    out->scalars = L.scalars;
    return DECT_OK;
}

dect_status dect_lmcg_init(const dect_plan* p, const void* m_h, const void* m_l, const void* w_h,
                           const void* w_l, const void* x0, void* state, const dect_params* prm,
                           void* stream) {
    if (!p || !m_h || !m_l || !w_h || !w_l || !state) return fail(DECT_E_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(state) % 256)
        return fail(DECT_E_ARG, "state buffer must be 256-byte aligned");
    dect_status st = check_lm_params(prm);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const LmLayout L = lm_layout(p);
    hipError_t e;
    if (p->dtype == DECT_F32)
        e = lm_init<float>(p, L, lm_ptrs<float>(L, state), static_cast<const float*>(m_h),
                           static_cast<const float*>(m_l), static_cast<const float*>(w_h),
                           static_cast<const float*>(w_l), static_cast<const float*>(x0), prm, s);
    else
        e = lm_init<double>(p, L, lm_ptrs<double>(L, state), static_cast<const double*>(m_h),
                            static_cast<const double*>(m_l), static_cast<const double*>(w_h),
                            static_cast<const double*>(w_l), static_cast<const double*>(x0), prm,
                            s);
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status dect_lmcg_iterate(const dect_plan* p, const void* m_h, const void* m_l,
                              const void* w_h, const void* w_l, void* state,
                              const dect_params* prm, int n_iters, dect_iter_log* log,
                              void* stream) {
    if (!p || !m_h || !m_l || !w_h || !w_l || !state) return fail(DECT_E_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(state) % 256)
        return fail(DECT_E_ARG, "state buffer must be 256-byte aligned");
    dect_status st = check_lm_params(prm);
    if (st) return st;
    if (n_iters < 0) return fail(DECT_E_ARG, "n_iters must be >= 0");
    if (log && n_iters > kLogCap)
        return fail(DECT_E_ARG, "a log holds at most %d iterations per call", kLogCap);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const LmLayout L = lm_layout(p);
    long it0 = 0;
    double* scal = at<double>(state, L.scalars);
    if (log) {
        DECT_HIP(hipStreamSynchronize(s));
        double v = 0.0;
        DECT_HIP(hipMemcpy(&v, scal + L_ITER, sizeof v, hipMemcpyDeviceToHost));
        it0 = (long)v;
    }
    for (int k = 0; k < n_iters; ++k) {
        hipError_t e;
        if (p->dtype == DECT_F32)
            e = lm_iteration<float>(p, L, lm_ptrs<float>(L, state), static_cast<const float*>(m_h),
                                    static_cast<const float*>(m_l), static_cast<const float*>(w_h),
                                    static_cast<const float*>(w_l), prm, s);
        else
            e = lm_iteration<double>(p, L, lm_ptrs<double>(L, state),
                                     static_cast<const double*>(m_h),
                                     static_cast<const double*>(m_l),
                                     static_cast<const double*>(w_h),
                                     static_cast<const double*>(w_l), prm, s);
        if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    }
    if (log) {
        DECT_HIP(hipStreamSynchronize(s));
        std::vector<double> h((size_t)kLogCap * kLogStride);
        DECT_HIP(hipMemcpy(h.data(), at<double>(state, L.log), h.size() * sizeof(double),
                           hipMemcpyDeviceToHost));
        bool bad = false;
        for (int k = 0; k < n_iters; ++k) {
            const double* e = &h[(size_t)((it0 + k) % kLogCap) * kLogStride];
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

}  // extern "C"
