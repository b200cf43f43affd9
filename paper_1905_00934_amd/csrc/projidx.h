// Index arithmetic of the ray-driven projector, shared by the kernel and by the
// host-side check of its bounds: the Joseph parameters of a ray, the workgroup order,
// a ray's sample range inside the image, a wave's share of its workgroup's lines and
// the taps of one sample.  Plain C++ (no runtime calls), so it also compiles for the
// host alone.
#pragma once

#include <cmath>

#include "dect.h"

#if defined(__HIPCC__)
#define DECT_HD __host__ __device__
#else
#define DECT_HD
#endif

namespace dect {

// Joseph parameters of a ray in double precision.  An x-stepped ray (|d_x| >= |d_y|)
// is sampled at every pixel column i at the fractional row phi0 + slope * i; a
// y-stepped ray at every row j at the fractional column phi0 + slope * j; each sample
// is weighted by step, the ray length between two samples.
struct HostRay {
    double phi0, slope, step;
    bool xstep;
};

// Ray (v, b) of the geometry: its line in scanner coordinates (view angle angle0 + v
// span / n_views; bin centre u_b = (b - (n_det - 1)/2 + det_offset) det_cm; parallel
// rays p.(cos t, sin t) = u_b, fan rays from the source at src_iso_cm (cos t, sin t) to
// the bin on the flat detector), in pixel units of the image grid.
inline HostRay host_ray(const dect_geometry& g, int v, int b) {
    const double t = g.angle0 + (double)v * g.span / (double)g.n_views;
    const double c = std::cos(t), s = std::sin(t);
    const double u = ((double)b - 0.5 * (double)(g.n_det - 1) + g.det_offset) * g.det_cm;
    double ox, oy, dx, dy;
    if (g.kind == DECT_PARALLEL) {
        ox = u * c;
        oy = u * s;
        dx = -s;
        dy = c;
    } else {
        ox = g.src_iso_cm * c;
        oy = g.src_iso_cm * s;
        const double qx = -(g.src_det_cm - g.src_iso_cm) * c - u * s;
        const double qy = -(g.src_det_cm - g.src_iso_cm) * s + u * c;
        dx = qx - ox;
        dy = qy - oy;
    }
    const double d = g.pixel_cm, cx = 0.5 * (g.nx - 1), cy = 0.5 * (g.ny - 1);
    HostRay r;
    if (std::fabs(dx) >= std::fabs(dy)) {
        // Row coordinate where the ray crosses column i: linear in i.
        r.xstep = true;
        r.slope = dy / dx;
        r.phi0 = (oy - ox * r.slope) / d - cx * r.slope + cy;
    } else {
        r.xstep = false;
        r.slope = dx / dy;
        r.phi0 = (ox - oy * r.slope) / d - cy * r.slope + cx;
    }
    r.step = d * std::sqrt(1.0 + r.slope * r.slope);
    return r;
}

// Projector workgroups: 64 / views consecutive bins of `views` consecutive base views
// (lane = bin * views + view; views = 1, 2, 4, 8, ..., 64), so the lanes of a wave read
// nearby image rows at every step.  Measured at 512^2 / 720 x 1024 with 8 waves, each
// taking its share of the lines the workgroup's rays cross: 1 view (64 bins) 147 us,
// 2 views (32 bins) 120 us, 4 views 141 us, 8 views 145 us; the tuner chooses per plan.
constexpr int kProjViewsDefault = 2;
DECT_HD inline bool proj_views_ok(int views) {
    return views >= 1 && views <= 64 && (views & (views - 1)) == 0;
}
DECT_HD inline int proj_grid_x(int D, int views) { return (D + 64 / views - 1) / (64 / views); }
DECT_HD inline int proj_grid_y(int Vb, int views) { return (Vb + views - 1) / views; }

// Projector workgroup order.  The dispatcher hands consecutive workgroup ids to the
// kXcds XCDs in turn, each with its own L2.  The gx bin groups form chunks of `chunk`;
// XCD x takes chunks x, x + kXcds, ... and runs every view group of a chunk before the
// next one.  The rays in flight on one XCD then pass through a few narrow annuli of the
// image, whose part of the orbit images its L2 can hold, and each XCD still gets bins
// from across the whole detector, so the XCDs' shares of ray length balance.
// Measured at 512^2 / 720 x 1024: chunks of 1, 2, 4, 8 and 16 bin groups (of 8 bins,
// 8 views per wave) took 146, 149, 153, 160 and 244 us against 163 us in the plain
// bins-then-views order; 16 leaves one chunk per XCD and unequal ray lengths.
constexpr int kXcds = 8;
constexpr int kProjChunkDefault = 1;
// Workgroups of one slice's projector launch (a multiple of kXcds; ids whose chunk
// lies past the last bin group exit at once).
DECT_HD inline unsigned proj_blocks(int gx, int gy, int chunk) {
    const int chunks = (gx + chunk - 1) / chunk;
    return (unsigned)(kXcds * ((chunks + kXcds - 1) / kXcds) * chunk * gy);
}

// Bin group bg and view group vg of workgroup `id` (bg >= gx: none).
DECT_HD inline void proj_tile(unsigned id, int gy, int chunk, int& bg, int& vg) {
    const int xcd = (int)(id % kXcds), nth = (int)(id / kXcds);
    const int c = xcd + kXcds * (nth / (chunk * gy)), within = nth % (chunk * gy);
    bg = c * chunk + within / gy;
    vg = within % gy;
}

// Sample k of a ray (phi0, slope) on a line of n_lines >= 2 pixels: Joseph's linear
// interpolation at phi = phi0 + slope k between taps floor(phi) and floor(phi) + 1,
// with the line extended by zeros.  Returned as two taps j0, j0 + 1 that always lie
// inside the line (0 <= j0 <= n_lines - 2) and their weights w0, w1, each the tent
// max(0, 1 - |phi - j|): 1 - alpha and alpha for an interior sample (alpha = phi -
// floor(phi)), alpha on tap 0 when only floor(phi) + 1 = 0 is inside, 1 - alpha on tap
// n_lines - 1 when only floor(phi) = n_lines - 1 is, and zero for a sample with no tap
// inside.  So the loads need no bounds test.
// The median of three values (no NaN): the hardware's three-operand median on the
// device in single precision, the same selection elsewhere.
template <typename T>
DECT_HD inline T med3(T a, T b, T c) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_fmed3f(a, b, c);
#endif
    return fmax(fmin(a, b), fmin(fmax(a, b), c));
}
template <typename T>
DECT_HD inline int proj_taps(T phi0, T slope, T k, int n_lines, T& w0, T& w1) {
    const T ph = fma(slope, k, phi0);
    const T j0 = med3<T>(floor(ph), T(0), T(n_lines - 2));
    const T t = ph - j0;
    w0 = fmax(T(0), T(1) - fabs(t));  // the tent at j0
    w1 = med3<T>(t, T(2) - t, T(0));  // the tent at j0 + 1: max(0, min(t, 2 - t))
    return (int)j0;
}

// Staged image lines of the projector.  A wave whose rays all step along the same
// axis reads, at sample k, line k of one orbit image; its 64 lanes stage the
// kProjWin taps s(k) .. s(k) + kProjWin - 1 of that line into LDS (one each) and
// read their two taps from there.  s(k) centres the window on the mean trajectory
// of lanes 0 and 63 (the first bin of the first view and the last bin of the last:
// the extreme rays of the wave), so that a wave's rays fall inside as long as they
// spread over fewer than about kProjWin - 2 pixels of the line; a lane whose taps
// are outside loads them directly.  The trajectory is held in fixed point with
// kProjWinFrac fraction bits, so that the window start of each line is integer
// arithmetic on the wave's scalar unit (any start is correct: it only decides which
// taps come from LDS).
constexpr int kProjWin = 64;
constexpr int kProjWinFrac = 8;
DECT_HD inline int proj_window(int A, int B, int k) {
    return ((A + B * k) >> kProjWinFrac) - (kProjWin / 2 - 1);
}
// The centre trajectory (A + B k) / 2^kProjWinFrac from the (phi0, slope) of lanes 0
// and 63, clamped so that A + B k cannot overflow for k < 2^15.
template <typename T>
DECT_HD inline void proj_window_line(T phi0_first, T slope_first, T phi0_last, T slope_last,
                                     int& A, int& B) {
    const T scale = T(1 << kProjWinFrac);
    const T ac = fmin(fmax(T(0.5) * (phi0_first + phi0_last), T(-(1 << 20))), T(1 << 20));
    const T bc = fmin(fmax(T(0.5) * (slope_first + slope_last), T(-2)), T(2));
    A = (int)floor(ac * scale);
    B = (int)floor(bc * scale);
}

// The samples k0..k1 of a ray (phi0, slope) with n_steps samples over n_lines image
// lines that have a tap inside the image: outside [k0, k1] both taps of every sample
// are outside (the range is first taken with a one-step margin, which absorbs
// rounding, then trimmed at both ends to samples with a nonzero weight as proj_taps
// evaluates them); k1 < k0 if none.
template <typename T>
DECT_HD inline void proj_ray_range(T phi0, T slope, int n_steps, int n_lines, int& k0, int& k1) {
    k0 = 0;
    k1 = n_steps - 1;
    if (slope != T(0)) {
        const T t1 = (T(-1) - phi0) / slope;
        const T t2 = (T(n_lines) - phi0) / slope;
        const T lo = fmax(t1 < t2 ? t1 : t2, T(-2));
        const T hi = fmin(t1 < t2 ? t2 : t1, T(n_steps + 1));
        const int kl = (int)floor(lo) - 1, kh = (int)ceil(hi) + 1;
        k0 = kl > 0 ? kl : 0;
        k1 = kh < n_steps - 1 ? kh : n_steps - 1;
    } else if (!(phi0 >= T(-1) && phi0 < T(n_lines))) {
        k1 = -1;
    }
    auto inside = [&](int k) {
        T w0, w1;
        proj_taps<T>(phi0, slope, (T)k, n_lines, w0, w1);
        return w0 > T(0) || w1 > T(0);
    };
    while (k0 <= k1 && !inside(k0)) ++k0;
    while (k1 >= k0 && !inside(k1)) --k1;
}

// Wave `wave` of KS takes lines c0..c1 of the union s0..s1 of its workgroup's ray
// ranges (s1 < s0: none; every wave then gets an empty share).
DECT_HD inline void proj_wave_share(int s0, int s1, int wave, int KS, int& c0, int& c1) {
    if (s1 < s0) s0 = 0, s1 = -1;
    const int len = s1 - s0 + 1;
    c0 = s0 + wave * len / KS;
    c1 = s0 + (wave + 1) * len / KS - 1;
}

}  // namespace dect
