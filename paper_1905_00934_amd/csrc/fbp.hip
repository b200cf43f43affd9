// The projection-wise baseline and initial image (Sec. 2, CDM; Sec. 4, set-up):
// constrained per-ray decomposition, filtered backprojection of the line integrals,
// and the ADMM start from an image.
//
// FBP (textbook parallel and equispaced-fan formulas): each view's row, weighted by
// D / sqrt(D^2 + u^2) for a fan (u on the detector scaled to the isocentre), is
// convolved with the discrete Ram-Lak kernel by an FFT of the zero-padded row (two
// channels as one complex row; the kernel is real and even); then every pixel
// gathers, over the views, the filtered row linearly interpolated at its detector
// coordinate, weighted by U^-2 = (D / L)^2 for a fan (L the distance from the
// source to the pixel along the central ray), and the sum is scaled by span / V.
#include "common.h"
#include "fftcore.h"
#include "kernels.h"
#include "profile.h"

namespace dect {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_fbp_filter(const T* __restrict__ sino, int ch, int D,
                                                    int lg, const T* __restrict__ H,
                                                    const T* __restrict__ tw,
                                                    const T* __restrict__ wpre, T* __restrict__ Q) {
    extern __shared__ char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const int v = blockIdx.x, P = 1 << lg;
    const T* row = sino + (size_t)v * D * ch;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        cx<T> x{T(0), T(0)};
        if (i < D) {
            x.re = row[(size_t)i * ch] * wpre[i];
            if (ch == 2) x.im = row[(size_t)i * ch + 1] * wpre[i];
        }
        buf[bitrev(i, lg)] = x;
    }
    fft_lds<T>(buf, 1, lg, tw, false);
    for (int k = threadIdx.x; k < P; k += blockDim.x) {
        buf[k].re *= H[k];
        buf[k].im *= H[k];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < P; k += blockDim.x) {
        const int kr = bitrev(k, lg);
        if (k < kr) {
            const cx<T> a = buf[k];
            buf[k] = buf[kr];
            buf[kr] = a;
        }
    }
    fft_lds<T>(buf, 1, lg, tw, true);
    cx<T>* q = reinterpret_cast<cx<T>*>(Q) + (size_t)v * D;
    for (int b = threadIdx.x; b < D; b += blockDim.x) q[b] = buf[b];
}

template <typename T>
__device__ inline T recip(T d) {
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_rcpf(d);  // 1 ulp; the bin position is good to ~1e-4 bins
    else
        return T(1) / d;
}

// One thread per pixel of a 16 x 16 tile (the tile's pixels read a narrow band of
// bins per view, which stays in L1); the views are walked in order.
template <typename T, bool FAN>
__global__ __launch_bounds__(256) void k_fbp_back(const T* __restrict__ Q, int nx, int ny, int V,
                                                  int D, T b0, const T* __restrict__ view,
                                                  T dtheta, int ch, T* __restrict__ img) {
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= nx || j >= ny) return;
    const T ic = (T)i - T(0.5) * (T)(nx - 1), jc = (T)j - T(0.5) * (T)(ny - 1);
    const cx<T>* q = reinterpret_cast<const cx<T>*>(Q);
    T ac = T(0), ap = T(0);
#pragma unroll 4
    for (int v = 0; v < V; ++v) {
        const T* e = view + 4 * v;
        T r = T(1), w = T(1);
        if constexpr (FAN) {
            r = recip<T>(fma(e[1], jc, fma(e[0], ic, T(1))));
            w = r * r;
        }
        const T b = fma(fma(e[3], jc, e[2] * ic), r, b0);
        const T fb = floor(b);
        const T al = b - fb;
        const int k = (int)fb;
        cx<T> q0{T(0), T(0)}, q1{T(0), T(0)};
        const cx<T>* row = q + (size_t)v * D;
        if (k >= 0 && k < D) q0 = row[k];
        if (k + 1 >= 0 && k + 1 < D) q1 = row[k + 1];
        ac = fma(w, fma(al, q1.re - q0.re, q0.re), ac);
        ap = fma(w, fma(al, q1.im - q0.im, q0.im), ap);
    }
    const long pix = (long)j * nx + i;
    if (ch == 2) {
        img[2 * pix] = ac * dtheta;
        img[2 * pix + 1] = ap * dtheta;
    } else {
        img[pix] = ac * dtheta;
    }
}

// Sums of a_c and a_p over all rays in a fixed order: kRaySumBlocks block partials
// (grid-strided), then one block adds them into the slot after the partials.
template <typename T>
__global__ __launch_bounds__(256) void k_ray_sums(const T* __restrict__ a, long M,
                                                  double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (long)gridDim.x * blockDim.x) {
        v[0] += (double)a[2 * i];
        v[1] += (double)a[2 * i + 1];
    }
    block_sum_store<2>(v, part + (size_t)blockIdx.x * kPartialSlots);
}

__global__ __launch_bounds__(256) void k_ray_sums_total(double* __restrict__ part, int nb) {
    double v[2] = {0.0, 0.0};
    if ((int)threadIdx.x < nb) {
        v[0] = part[(size_t)threadIdx.x * kPartialSlots];
        v[1] = part[(size_t)threadIdx.x * kPartialSlots + 1];
    }
    block_sum_store<2>(v, part + (size_t)nb * kPartialSlots);
}

// x0 = (x_c, s x_c) with s = sum a_p / sum a_c.
template <typename T>
__global__ __launch_bounds__(256) void k_start_image(const T* __restrict__ fbp, long N,
                                                     const double* __restrict__ sums,
                                                     T* __restrict__ x0) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T sc = (T)(sums[0] != 0.0 ? sums[1] / sums[0] : 0.0);
    const T xc = fbp[2 * i];
    x0[2 * i] = xc;
    x0[2 * i + 1] = sc * xc;
}

// x = z = x0 and y = D x0 (forward differences, zero at the last column and row).
template <typename T>
__global__ __launch_bounds__(256) void k_init_image(const T* __restrict__ x0, int nx, int ny,
                                                    T* __restrict__ x, T* __restrict__ z,
                                                    T* __restrict__ y) {
    const long pix = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= (long)nx * ny) return;
    int i, j;
    pixel_ij(pix, nx, i, j);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T v = x0[2 * pix + c];
        x[2 * pix + c] = v;
        z[2 * pix + c] = v;
        y[4 * pix + c] = i < nx - 1 ? x0[2 * (pix + 1) + c] - v : T(0);
        y[4 * pix + 2 + c] = j < ny - 1 ? x0[2 * (pix + nx) + c] - v : T(0);
    }
}

// The next right-hand side t = a + u^a - R x with u^a = 0 (internal ray order l).
template <typename T>
__global__ __launch_bounds__(256) void k_init_t(const T* __restrict__ a, const T* __restrict__ Rx,
                                                long M, int sym, int Vb, int D, T* __restrict__ t) {
    const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= M) return;
    const long i = std_ray(l, sym, Vb, D);
    t[2 * l] = a[2 * i] - Rx[2 * i];
    t[2 * l + 1] = a[2 * i + 1] - Rx[2 * i + 1];
}

template <typename T>
hipError_t fbp_t(const dect_plan* p, const void* sino, void* img, int ch, hipStream_t s) {
    ProfScope ps("fbp", s);
    const size_t lds = (size_t)p->fbp_P * sizeof(cx<T>);
    hipLaunchKernelGGL((k_fbp_filter<T>), dim3(p->V), dim3(256), lds, s,
                       static_cast<const T*>(sino), ch, p->D, p->fbp_lg,
                       static_cast<const T*>(p->fbp_H), static_cast<const T*>(p->fbp_tw),
                       static_cast<const T*>(p->fbp_wpre), static_cast<T*>(p->scratch_Q));
    const dim3 g((unsigned)((p->nx + 15) / 16), (unsigned)((p->ny + 15) / 16));
    const dect_geometry& G = p->geom;
    const T dtheta = (T)(G.span / p->V);
    if (G.kind == DECT_FAN)
        hipLaunchKernelGGL((k_fbp_back<T, true>), g, dim3(256), 0, s,
                           static_cast<const T*>(p->scratch_Q), p->nx, p->ny, p->V, p->D,
                           (T)p->fbp_b0, static_cast<const T*>(p->fbp_view), dtheta, ch,
                           static_cast<T*>(img));
    else
        hipLaunchKernelGGL((k_fbp_back<T, false>), g, dim3(256), 0, s,
                           static_cast<const T*>(p->scratch_Q), p->nx, p->ny, p->V, p->D,
                           (T)p->fbp_b0, static_cast<const T*>(p->fbp_view), dtheta, ch,
                           static_cast<T*>(img));
    return hipGetLastError();
}

template <typename T>
hipError_t cdm_t(const dect_plan* p, const void* mh, const void* ml, const void* wh,
                 const void* wl, int iters, void* a, void* cost, hipStream_t s) {
    UdmArgs<T> u{};
    u.M = p->M;
    u.sym = 1;
    u.Vb = p->V;
    u.D = p->D;
    u.mh = static_cast<const T*>(mh);
    u.ml = static_cast<const T*>(ml);
    u.wh = static_cast<const T*>(wh);
    u.wl = static_cast<const T*>(wl);
    u.a = static_cast<T*>(a);
    u.cost = static_cast<T*>(cost);
    u.iters = iters;
    u.mu0 = 1e-3;
    // Inverse of the linearisation at a = 0: rows (mean f_KN, mean f_p) per spectrum.
    const double hc = p->mean_f[0][0], hp = p->mean_f[0][1];
    const double lc = p->mean_f[1][0], lp = p->mean_f[1][1];
    const double det = hc * lp - hp * lc;
    u.lin[0] = lp / det;
    u.lin[1] = -hp / det;
    u.lin[2] = -lc / det;
    u.lin[3] = hc / det;
    return launch_udm<T>(p, 3, u, s);
}

template <typename T>
hipError_t start_t(const dect_plan* p, const void* a, void* fbp, void* x0, hipStream_t s) {
    static_assert(kRaySumBlocks <= 256, "one block adds the partials");
    hipLaunchKernelGGL((k_ray_sums<T>), dim3(kRaySumBlocks), dim3(256), 0, s,
                       static_cast<const T*>(a), p->M, p->scratch_part);
    hipLaunchKernelGGL(k_ray_sums_total, dim3(1), dim3(256), 0, s, p->scratch_part,
                       kRaySumBlocks);
    hipLaunchKernelGGL((k_start_image<T>), dim3((unsigned)((p->N + 255) / 256)), dim3(256), 0, s,
                       static_cast<const T*>(fbp), p->N,
                       p->scratch_part + (size_t)kRaySumBlocks * kPartialSlots,
                       static_cast<T*>(x0));
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_init_image(const dect_plan* p, const void* x0, void* state, hipStream_t s,
                             bool sums64) {
    const dect_layout& L = p->layout;
    char* st = static_cast<char*>(state);
    T* Rx = reinterpret_cast<T*>(st + L.Rx);
    hipLaunchKernelGGL((k_init_image<T>), dim3((unsigned)((p->N + 255) / 256)), dim3(256), 0, s,
                       static_cast<const T*>(x0), p->nx, p->ny, reinterpret_cast<T*>(st + L.x),
                       reinterpret_cast<T*>(st + L.z), reinterpret_cast<T*>(st + L.y));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // R x0 into the state's R x (standard [V][D][2] order), then t = a - R x0.
    e = launch_project<T>(p, x0, Rx, 2, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_init_t<T>), dim3((unsigned)((p->M + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const T*>(st + L.a), Rx, p->M, p->sym, p->Vb, p->D,
                       reinterpret_cast<T*>(st + p->off_t));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_track_init<T>(p, state, s, sums64);
}

template hipError_t launch_init_image<float>(const dect_plan*, const void*, void*, hipStream_t,
                                             bool);
template hipError_t launch_init_image<double>(const dect_plan*, const void*, void*, hipStream_t,
                                              bool);

}  // namespace dect

using namespace dect;

extern "C" {

dect_status dect_cdm(const dect_plan* p, const void* m_h, const void* m_l, const void* w_h,
                     const void* w_l, int lm_iters, void* a, void* cost, void* stream) {
    if (!p || !m_h || !m_l || !w_h || !w_l || !a) return fail(DECT_E_ARG, "null argument");
    if (lm_iters < 0) return fail(DECT_E_ARG, "lm_iters must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = p->dtype == DECT_F32
                             ? cdm_t<float>(p, m_h, m_l, w_h, w_l, lm_iters, a, cost, s)
                             : cdm_t<double>(p, m_h, m_l, w_h, w_l, lm_iters, a, cost, s);
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status dect_fbp(const dect_plan* p, const void* sino, void* img, int ch, void* stream) {
    if (!p || !sino || !img) return fail(DECT_E_ARG, "null argument");
    if (ch != 1 && ch != 2) return fail(DECT_E_ARG, "ch must be 1 or 2 (got %d)", ch);
    if (!p->has_fbp)
        return fail(DECT_E_SHAPE, "no FBP filter for %d bins (padded row > %d)", p->D, kMaxFbp);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = p->dtype == DECT_F32 ? fbp_t<float>(p, sino, img, ch, s)
                                              : fbp_t<double>(p, sino, img, ch, s);
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

dect_status dect_cdm_fbp_start(const dect_plan* p, const void* m_h, const void* m_l,
                               const void* w_h, const void* w_l, int cdm_iters, void* a,
                               void* x0, void* fbp_out, void* stream) {
    if (!p || !m_h || !m_l || !w_h || !w_l || !a || !x0) return fail(DECT_E_ARG, "null argument");
    if (cdm_iters < 0) return fail(DECT_E_ARG, "cdm_iters must be >= 0");
    if (!p->has_fbp)
        return fail(DECT_E_SHAPE, "no FBP filter for %d bins (padded row > %d)", p->D, kMaxFbp);
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* f = fbp_out ? fbp_out : x0;
    hipError_t e;
    if (p->dtype == DECT_F32) {
        e = cdm_t<float>(p, m_h, m_l, w_h, w_l, cdm_iters, a, nullptr, s);
        if (e == hipSuccess) e = fbp_t<float>(p, a, f, 2, s);
        if (e == hipSuccess) e = start_t<float>(p, a, f, x0, s);
    } else {
        e = cdm_t<double>(p, m_h, m_l, w_h, w_l, cdm_iters, a, nullptr, s);
        if (e == hipSuccess) e = fbp_t<double>(p, a, f, 2, s);
        if (e == hipSuccess) e = start_t<double>(p, a, f, x0, s);
    }
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

}  // extern "C"
