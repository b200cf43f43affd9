// Joseph projector R (ray-driven) and its exact transpose R^T (pixel-driven
// gather, no atomics), for gfx950.
//
// Projector: one lane per ray, a workgroup covers 256 consecutive bins of one
// view, so sinogram writes are coalesced along the detector.  A ray that steps
// along columns reads the transposed image [nx][ny] so that neighbouring lanes
// (neighbouring bins) read neighbouring addresses of one image line.
//
// Transpose: one lane per pixel of a 16x16 tile; for every view the lane finds
// the bins whose Joseph samples can touch its pixel from the central projection
// of the two-pixel segment around it, then re-evaluates each candidate's
// interpolation weight with the projector's own fma on the same table values.
// The weights are therefore bit-identical to the projector's, and R^T is the
// transpose of R up to summation order.
#include "common.h"
#include "kernels.h"
#include "profile.h"

namespace dect {

namespace {

// Extra bins scanned on each side of a pixel's analytic footprint.  Rounding of
// the table values and of the footprint moves bin coordinates by < 1e-3 bins.
constexpr float kFootprintMargin = 0.05f;

template <typename T, int CH>
__device__ inline void zero(vec<T, CH>& a) {
#pragma unroll
    for (int c = 0; c < CH; ++c) a.v[c] = T(0);
}

template <typename T, int CH>
__global__ __launch_bounds__(256) void k_project(const RayParam<T>* __restrict__ rays,
                                                 const vec<T, CH>* __restrict__ img,
                                                 const vec<T, CH>* __restrict__ imgT,
                                                 vec<T, CH>* __restrict__ sino, int nx, int ny,
                                                 int D) {
    const int v = blockIdx.y;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= D) return;
    const RayParam<T> r = rays[(size_t)v * D + b];
    const bool xs = r.pad == T(0);
    const int n_steps = xs ? nx : ny;   // samples along the ray
    const int n_lines = xs ? ny : nx;   // interpolation axis
    const vec<T, CH>* src = xs ? imgT : img;  // [n_steps][n_lines]
    // Samples can touch the image only where phi lies in [-1, n_lines).
    // Outside [k0, k1] both taps of every sample are outside the image, so the
    // restriction changes no term; the one-step margin absorbs rounding.
    int k0 = 0, k1 = n_steps - 1;
    if (r.slope != T(0)) {
        const T t1 = (T(-1) - r.phi0) / r.slope;
        const T t2 = (T(n_lines) - r.phi0) / r.slope;
        const T lo = fmax(t1 < t2 ? t1 : t2, T(-2));
        const T hi = fmin(t1 < t2 ? t2 : t1, T(n_steps + 1));
        const int kl = (int)floor(lo) - 1, kh = (int)ceil(hi) + 1;
        k0 = kl > 0 ? kl : 0;
        k1 = kh < n_steps - 1 ? kh : n_steps - 1;
    } else if (!(r.phi0 >= T(-1) && r.phi0 < T(n_lines))) {
        k1 = -1;
    }
    T acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = T(0);
    for (int k = k0; k <= k1; ++k) {
        const T phi = fma(r.slope, (T)k, r.phi0);
        T fl = floor(phi);
        const T al = phi - fl;
        fl = fmin(fmax(fl, T(-2)), T(n_lines + 1));
        const int j0 = (int)fl;
        const vec<T, CH>* line = src + (size_t)k * n_lines;
        vec<T, CH> a0, a1;
        zero(a0);
        zero(a1);
        if ((unsigned)j0 < (unsigned)n_lines) a0 = line[j0];
        if ((unsigned)(j0 + 1) < (unsigned)n_lines) a1 = line[j0 + 1];
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] += a0.v[c] + al * (a1.v[c] - a0.v[c]);
    }
    vec<T, CH> out;
#pragma unroll
    for (int c = 0; c < CH; ++c) out.v[c] = acc[c] * r.step;
    sino[(size_t)v * D + b] = out;
}

// Image transpose [ny][nx] -> [nx][ny] through LDS, 32x32 tiles.
template <typename T, int CH>
__global__ __launch_bounds__(256) void k_transpose(const vec<T, CH>* __restrict__ in,
                                                   vec<T, CH>* __restrict__ out, int nx, int ny) {
    __shared__ vec<T, CH> tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int r = ty; r < 32; r += 8) {
        const int j = by + r, i = bx + tx;
        if (j < ny && i < nx) tile[r][tx] = in[(size_t)j * nx + i];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bx + r, j = by + tx;
        if (i < nx && j < ny) out[(size_t)i * ny + j] = tile[tx][r];
    }
}

// Gather of all Joseph weights of pixel (i, j) times the sinogram.
template <typename T, int CH>
__device__ inline void gather_pixel(const RayParam<T>* __restrict__ rays,
                                    const ViewParam<T>* __restrict__ views,
                                    const vec<T, CH>* __restrict__ sino, int V, int D, int i,
                                    int j, T ip, T jp, T (&acc)[CH]) {
    const T fi = (T)i, fj = (T)j;
    for (int v = 0; v < V; ++v) {
        const ViewParam<T> w = views[v];
        const T num = w.ni * ip + w.nj * jp;
        const T den = w.d0 + w.di * ip + w.dj * jp;
        const RayParam<T>* rv = rays + (size_t)v * D;
        const vec<T, CH>* sv = sino + (size_t)v * D;
        if (w.xb1 > w.xb0) {
            // Column i: bins whose row coordinate lies in [j-1, j+1).
            const T b1 = (num - w.nj) / (den - w.dj) + w.boff;
            const T b2 = (num + w.nj) / (den + w.dj) + w.boff;
            const T bl = (b1 < b2 ? b1 : b2) - T(kFootprintMargin);
            const T bh = (b1 < b2 ? b2 : b1) + T(kFootprintMargin);
            int lo = (int)ceil(fmax(bl, T(-1)));
            int hi = (int)floor(fmin(bh, T(D)));
            lo = lo > w.xb0 ? lo : w.xb0;
            hi = hi < w.xb1 - 1 ? hi : w.xb1 - 1;
            for (int b = lo; b <= hi; ++b) {
                const RayParam<T> r = rv[b];
                const T phi = fma(r.slope, fi, r.phi0);
                const T fl = floor(phi);
                const T al = phi - fl;
                T wt = fl == fj ? T(1) - al : (fl == fj - T(1) ? al : T(0));
                wt *= r.step;
                const vec<T, CH> s = sv[b];
#pragma unroll
                for (int c = 0; c < CH; ++c) acc[c] += wt * s.v[c];
            }
        }
        if (w.yb1 > w.yb0) {
            // Row j: bins whose column coordinate lies in [i-1, i+1).
            const T b1 = (num - w.ni) / (den - w.di) + w.boff;
            const T b2 = (num + w.ni) / (den + w.di) + w.boff;
            const T bl = (b1 < b2 ? b1 : b2) - T(kFootprintMargin);
            const T bh = (b1 < b2 ? b2 : b1) + T(kFootprintMargin);
            int lo = (int)ceil(fmax(bl, T(-1)));
            int hi = (int)floor(fmin(bh, T(D)));
            lo = lo > w.yb0 ? lo : w.yb0;
            hi = hi < w.yb1 - 1 ? hi : w.yb1 - 1;
            for (int b = lo; b <= hi; ++b) {
                const RayParam<T> r = rv[b];
                const T phi = fma(r.slope, fj, r.phi0);
                const T fl = floor(phi);
                const T al = phi - fl;
                T wt = fl == fi ? T(1) - al : (fl == fi - T(1) ? al : T(0));
                wt *= r.step;
                const vec<T, CH> s = sv[b];
#pragma unroll
                for (int c = 0; c < CH; ++c) acc[c] += wt * s.v[c];
            }
        }
    }
}

}  // namespace

namespace {

// R^T followed by an optional image-side epilogue (basis pairs, CH = 2 except EPI_NONE).
template <typename T, int CH, int EPI>
__global__ __launch_bounds__(256) void k_backproject(BpArgs<T> a) {
    using V2 = vec<T, 2>;
    using V4 = vec<T, 4>;
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    const int nx = a.nx, ny = a.ny;
    const bool inside = i < nx && j < ny;
    T acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = T(0);
    if (inside)
        gather_pixel<T, CH>(a.rays, a.views, reinterpret_cast<const vec<T, CH>*>(a.sino), a.V,
                            a.D, i, j, (T)i - T(0.5) * (T)(nx - 1), (T)j - T(0.5) * (T)(ny - 1),
                            acc);
    const size_t pix = (size_t)j * nx + i;
    if constexpr (EPI == EPI_NONE) {
        if (inside) {
            vec<T, CH> o;
#pragma unroll
            for (int c = 0; c < CH; ++c) o.v[c] = acc[c];
            reinterpret_cast<vec<T, CH>*>(a.out)[pix] = o;
        }
    } else {
        double part[2] = {0.0, 0.0};
        if (inside) {
            T res[2] = {acc[0], acc[1]};
            const V2* x2 = reinterpret_cast<const V2*>(a.x);
            auto X = [&](int jj, int ii) { return x2[(size_t)jj * nx + ii]; };
            if constexpr (EPI == EPI_RHS) {
                // r0 = R^T t + D^T (y + u^y - D x) + (z + u^z - x), Eq. (12).
                const V4* y4 = reinterpret_cast<const V4*>(a.y);
                const V4* u4 = reinterpret_cast<const V4*>(a.uy);
                const V2 xc = X(j, i);
                const V2 z = reinterpret_cast<const V2*>(a.z)[pix];
                const V2 uz = reinterpret_cast<const V2*>(a.uz)[pix];
                const V4 yc = y4[pix], uc = u4[pix];
#pragma unroll
                for (int c = 0; c < 2; ++c) res[c] += z.v[c] + uz.v[c] - xc.v[c];
                if (i < nx - 1) {  // -W_h(j, i)
                    const V2 xr = X(j, i + 1);
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        res[c] -= yc.v[c] + uc.v[c] - (xr.v[c] - xc.v[c]);
                }
                if (i > 0) {  // +W_h(j, i-1)
                    const V2 xl = X(j, i - 1);
                    const V4 yl = y4[pix - 1], ul = u4[pix - 1];
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        res[c] += yl.v[c] + ul.v[c] - (xc.v[c] - xl.v[c]);
                }
                if (j < ny - 1) {  // -W_v(j, i)
                    const V2 xd = X(j + 1, i);
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        res[c] -= yc.v[2 + c] + uc.v[2 + c] - (xd.v[c] - xc.v[c]);
                }
                if (j > 0) {  // +W_v(j-1, i)
                    const V2 xu = X(j - 1, i);
                    const V4 yu = y4[pix - nx], uu = u4[pix - nx];
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        res[c] += yu.v[2 + c] + uu.v[2 + c] - (xc.v[c] - xu.v[c]);
                }
                V2 o;
                o.v[0] = res[0];
                o.v[1] = res[1];
                reinterpret_cast<V2*>(a.out)[pix] = o;
                if (a.out2) reinterpret_cast<V2*>(a.out2)[pix] = o;
                part[0] = (double)res[0] * (double)res[0];
                part[1] = (double)res[1] * (double)res[1];
            } else if constexpr (EPI == EPI_Q) {
                // q = R^T R p + D^T D p + p; a.x holds p.
                const V2 pc = X(j, i);
#pragma unroll
                for (int c = 0; c < 2; ++c) res[c] += pc.v[c];
                if (i < nx - 1) { const V2 q = X(j, i + 1); for (int c = 0; c < 2; ++c) res[c] += pc.v[c] - q.v[c]; }
                if (i > 0) { const V2 q = X(j, i - 1); for (int c = 0; c < 2; ++c) res[c] += pc.v[c] - q.v[c]; }
                if (j < ny - 1) { const V2 q = X(j + 1, i); for (int c = 0; c < 2; ++c) res[c] += pc.v[c] - q.v[c]; }
                if (j > 0) { const V2 q = X(j - 1, i); for (int c = 0; c < 2; ++c) res[c] += pc.v[c] - q.v[c]; }
                if (a.out) {
                    V2 o;
                    o.v[0] = res[0];
                    o.v[1] = res[1];
                    reinterpret_cast<V2*>(a.out)[pix] = o;
                }
                part[0] = (double)pc.v[0] * (double)res[0];
                part[1] = (double)pc.v[1] * (double)res[1];
            } else {  // EPI_DUAL: s = R^T da + D^T dy + dz
                const V4* d4 = reinterpret_cast<const V4*>(a.y);
                const V4 dc = d4[pix];
                const V2 dz = reinterpret_cast<const V2*>(a.z)[pix];
#pragma unroll
                for (int c = 0; c < 2; ++c) res[c] += dz.v[c];
                if (i < nx - 1) for (int c = 0; c < 2; ++c) res[c] -= dc.v[c];
                if (i > 0) { const V4 dl = d4[pix - 1]; for (int c = 0; c < 2; ++c) res[c] += dl.v[c]; }
                if (j < ny - 1) for (int c = 0; c < 2; ++c) res[c] -= dc.v[2 + c];
                if (j > 0) { const V4 du = d4[pix - nx]; for (int c = 0; c < 2; ++c) res[c] += du.v[2 + c]; }
                part[0] = (double)res[0] * (double)res[0];
                part[1] = (double)res[1] * (double)res[1];
            }
        }
        double p4[2] = {part[0], part[1]};
        block_sum_store<2>(p4, a.partials + (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * kPartialSlots);
    }
}

}  // namespace

template <typename T, int CH>
hipError_t project_ch(const dect_plan* p, const void* img, void* imgT, void* sino, hipStream_t s) {
    using VV = vec<T, CH>;
    const int nx = p->nx, ny = p->ny;
    {
        ProfScope pt("transpose", s);
        hipLaunchKernelGGL((k_transpose<T, CH>), dim3((nx + 31) / 32, (ny + 31) / 32), dim3(256),
                           0, s, static_cast<const VV*>(img), static_cast<VV*>(imgT), nx, ny);
    }
    ProfScope pp("project", s);
    hipLaunchKernelGGL((k_project<T, CH>), dim3((p->D + 255) / 256, p->V), dim3(256), 0, s,
                       static_cast<const RayParam<T>*>(p->rays), static_cast<const VV*>(img),
                       static_cast<const VV*>(imgT), static_cast<VV*>(sino), nx, ny, p->D);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_project(const dect_plan* p, const void* img, void* sino, int ch, hipStream_t s) {
    switch (ch) {
        case 1: return project_ch<T, 1>(p, img, p->scratch_imgT, sino, s);
        case 2: return project_ch<T, 2>(p, img, p->scratch_imgT, sino, s);
        case 4: return project_ch<T, 4>(p, img, p->scratch_imgT, sino, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_project_pair(const dect_plan* p, const void* img, void* imgT, void* sino,
                               hipStream_t s) {
    return project_ch<T, 2>(p, img, imgT, sino, s);
}

template <typename T>
hipError_t launch_backproject(const dect_plan* p, int ch, int epi, const BpArgs<T>& a0,
                              hipStream_t s) {
    BpArgs<T> a = a0;
    a.rays = static_cast<const RayParam<T>*>(p->rays);
    a.views = static_cast<const ViewParam<T>*>(p->views);
    a.nx = p->nx;
    a.ny = p->ny;
    a.V = p->V;
    a.D = p->D;
    dim3 g((p->nx + 15) / 16, (p->ny + 15) / 16);
    static const char* names[4] = {"backproject", "backproject_rhs", "backproject_q",
                                   "backproject_dual"};
    ProfScope ps(names[epi & 3], s);
    if (epi == EPI_NONE) {
        switch (ch) {
            case 1: hipLaunchKernelGGL((k_backproject<T, 1, EPI_NONE>), g, dim3(256), 0, s, a); break;
            case 2: hipLaunchKernelGGL((k_backproject<T, 2, EPI_NONE>), g, dim3(256), 0, s, a); break;
            case 4: hipLaunchKernelGGL((k_backproject<T, 4, EPI_NONE>), g, dim3(256), 0, s, a); break;
            default: return hipErrorInvalidValue;
        }
    } else if (epi == EPI_RHS) {
        hipLaunchKernelGGL((k_backproject<T, 2, EPI_RHS>), g, dim3(256), 0, s, a);
    } else if (epi == EPI_Q) {
        hipLaunchKernelGGL((k_backproject<T, 2, EPI_Q>), g, dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_backproject<T, 2, EPI_DUAL>), g, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template hipError_t launch_project<float>(const dect_plan*, const void*, void*, int, hipStream_t);
template hipError_t launch_project<double>(const dect_plan*, const void*, void*, int, hipStream_t);
template hipError_t launch_project_pair<float>(const dect_plan*, const void*, void*, void*, hipStream_t);
template hipError_t launch_project_pair<double>(const dect_plan*, const void*, void*, void*, hipStream_t);
template hipError_t launch_backproject<float>(const dect_plan*, int, int, const BpArgs<float>&, hipStream_t);
template hipError_t launch_backproject<double>(const dect_plan*, int, int, const BpArgs<double>&, hipStream_t);

}  // namespace dect
