// Internal declarations of the dual-energy CT ADMM library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "dect.h"

namespace dect {

// ---------------------------------------------------------------- errors ---
void set_error(const char* fmt, ...);
dect_status fail(dect_status st, const char* fmt, ...);

#define DECT_HIP(expr)                                                               \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::dect::fail(DECT_E_DEVICE, "%s failed: %s (%s:%d)", #expr,       \
                                hipGetErrorString(e_), __FILE__, __LINE__);          \
    } while (0)

#define DECT_LAUNCH_CHECK()                                                          \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess)                                                        \
            return ::dect::fail(DECT_E_DEVICE, "kernel launch failed: %s (%s:%d)",   \
                                hipGetErrorString(e_), __FILE__, __LINE__);          \
    } while (0)

// ------------------------------------------------------------ vector types ---
// N values of T stored together, aligned so that one load moves all of them.
template <typename T, int N>
struct alignas(sizeof(T) * N) vec {
    T v[N];
};

// -------------------------------------------------------------- plan tables ---
// Joseph parameters of one ray.  An x-stepped ray (|d_x| >= |d_y|) is sampled at
// every pixel column i at the fractional row phi(i) = phi0 + slope * i; a
// y-stepped ray at every row j at the fractional column phi0 + slope * j.  Each
// sample is weighted by `step`, the ray length between two samples.  The forward
// projector and the plain transposed gather both evaluate phi with one fma on these
// values; the weights they then form differ only by rounding (the projector
// interpolates a0 + alpha (a1 - a0) and scales by step at the end).
template <typename T>
struct alignas(sizeof(T) * 4) RayParam {
    T phi0, slope, step, pad;
};

// A ray as the transpose weighs it: the signed minor-axis distance from the sample
// to the pixel (i, j) is d = phi0 + ci i + cj j (x-stepped: ci = slope, cj = -1;
// y-stepped: ci = -1, cj = slope), and the weight is step max(0, 1 - |d|).
template <typename T>
struct alignas(sizeof(T) * 4) BpRay {
    T phi0, ci, cj, step;
};

// Per-view data for the pixel-driven transpose.  The detector coordinate (in
// bins) of the ray through the point with centred pixel coordinates (i', j') is
//   beta = (ni i' + nj j') / (d0 + di i' + dj j') + boff
// (fan beam: central projection from the source; parallel: d0 = 1, di = dj = 0).
// Bins [xb0, xb1) of the view are x-stepped, [yb0, yb1) y-stepped.
template <typename T>
struct ViewParam {
    T ni, nj, d0, di, dj, boff;
    int xb0, xb1, yb0, yb1;
};

// Energy-bin tables of one spectrum in base-2 units: the normalised weight as
// lw = log2(omega), and kc = f_KN log2(e), kp = f_p log2(e), nonzero bins only.
template <typename T>
struct SpecTables {
    const T* lw;
    const T* kc;
    const T* kp;
    int n;
};

}  // namespace dect

// The plan: everything that depends on geometry, spectra and precision only.
struct dect_plan {
    dect_geometry geom;
    dect_dtype dtype;
    int device;
    size_t elem;            // bytes per scalar
    int nx, ny, V, D;
    long N, M;              // pixels, rays
    // Rotational symmetry order (4: views v + k V/4 are quarter turns of base
    // view v; 1: none) and the number of base views Vb = V / sym.
    int sym = 1, Vb = 0;
    double margin = 0.05;   // footprint margin of the transpose, in bins
    // Workgroup shapes of the ADMM transpose (waves splitting the views) and
    // projector (waves splitting the lines): 2, 4 or 8, set by dect_plan_tune.
    int bp_waves = 4, pj_waves = 8;
    // Projector lane layout (base views per wave) and XCD chunk (bin groups per XCD
    // turn), also set by dect_plan_tune.
    int pj_views = 2, pj_chunk = 1;
    // device tables
    void* rays = nullptr;   // RayParam<T>[Vb * D]
    void* views = nullptr;  // ViewParam<T>[Vb]
    void* bp_rays = nullptr;  // BpRay<T>[Vb * D]: the transpose's form of the rays
    void* spec = nullptr;   // T[6 * Kmax]: lw_h, kc_h, kp_h, lw_l, kc_l, kp_l
    int kh = 0, kl = 0, kmax = 0;
    // Both spectra on one energy grid, for evaluating them with one exponential per
    // energy: T[nj][8] = kc, kp, w_h, w_h kc, w_h kp, w_l, w_l kc, w_l kp (w: normalised
    // weight, linear; kc, kp: f_KN, f_p times log2(e)) over the bins where both spectra
    // are nonzero (jb of them), then where only the high one is (jh), then only the low
    // one (jl).  joint_lim: the largest log2 distance from the shift to a spectrum's
    // log-sum-exp for which no A_k overflows, 124 + log2 of the smallest weight (0: the
    // joint evaluation is not used).  joint_kc, joint_kp: smallest and largest f_KN, f_p
    // times log2(e) over the bins (they bound how far a step moves any exponent).
    void* joint = nullptr;
    int jb = 0, jh = 0, jl = 0;
    double joint_lim = 0.0;
    double joint_kc[2] = {0.0, 0.0}, joint_kp[2] = {0.0, 0.0};
    double kc_max = 0.0, kp_max = 0.0;  // largest f_KN, f_p times log2(e) over used bins
    double mean_f[2][2];    // spectrum-mean (f_KN, f_p) per spectrum (h, l)
    // plan-owned scratch: orbit images of the image being projected (up to 4 channels)
    void* scratch_O = nullptr;   // T[N * 4 * sym]
    void* scratch_OT = nullptr;  // T[N * 4 * sym]
    void* scratch_sq = nullptr;  // sym == 4: T[Vb][D][4][2], a sinogram as quad records
    // preconditioner of the x-update (ramp filter on a zero-padded FFT grid of
    // px x py = 2^lpx x 2^lpy; absent when a padded side exceeds kMaxFft)
    bool has_precond = false;
    int px = 0, py = 0, lpx = 0, lpy = 0;
    void* pre_filter = nullptr;  // T[py][px]
    void* pre_twx = nullptr;     // T[px/2][2] twiddles exp(-2 pi i k / px)
    void* pre_twy = nullptr;     // T[py/2][2]
    void* scratch_W = nullptr;   // T[ny][px][2] work grid of dect_precondition
    double* scratch_part = nullptr;  // block partials of the standalone calls (>= ny, >= 4)
    // filtered backprojection (FBP rows padded to fbp_P = 2^fbp_lg; absent when
    // fbp_P exceeds kMaxFbp)
    bool has_fbp = false;
    int fbp_P = 0, fbp_lg = 0;
    double fbp_delta = 0.0;      // detector spacing at the isocentre, cm
    double fbp_b0 = 0.0;         // bin index of detector coordinate 0
    void* fbp_H = nullptr;       // T[P] filter spectrum (scaled)
    void* fbp_tw = nullptr;      // T[P/2][2] twiddles
    void* fbp_view = nullptr;    // T[V][4] (di, dj, ni, nj): bin and weight of a pixel
    void* fbp_wpre = nullptr;    // T[D] fan pre-weights (1 for parallel beams)
    void* scratch_Q = nullptr;   // T[V][D][2] filtered rows
    // state layout (bytes)
    dect_layout layout;
    size_t off_p, off_pO, off_pOT, off_r, off_q, off_dy, off_dz, off_Rp, off_t, off_da, off_fg,
        off_z, off_fftw, off_partials, off_log;
    // Tracked right-hand-side images (double [N][2]): H = R^T (a - R x), U = R^T u^a,
    // and the last CG step's R^T R p ([N][2] of the plan's type).
    size_t off_h, off_u, off_rtrp;
    int nb_sino, nb_img, nb_tiles, nb_pre;  // block counts of the reducing kernels
};

namespace dect {

// Workgroups of the transposed projector (8x8 pixel orbits each).
int bp_blocks(const dect_plan* p);

// Column i and row j of pixel pix of an image nx wide; images hold fewer than 2^30
// pixels, so the division is unsigned 32-bit.
__host__ __device__ inline void pixel_ij(long pix, int nx, int& i, int& j) {
    const unsigned u = (unsigned)pix, r = u / (unsigned)nx;
    j = (int)r;
    i = (int)(u - r * (unsigned)nx);
}

// Standard sinogram index of internal (quad-interleaved when sym = 4) index l:
// internal order is [Vb][D][sym], standard order [V][D] with view vb + k Vb.
//
// sym is 1 or 4 and a plan keeps a sinogram below 2^30 rays, so the index arithmetic
// is unsigned 32-bit (a 64-bit division costs several times as many instructions).
__host__ __device__ inline long std_ray(long l, int sym, int Vb, int D) {
    if (sym == 1) return l;
    const unsigned u = (unsigned)l, base = u >> 2, k = u & 3u;
    const unsigned vb = base / (unsigned)D, b = base - vb * (unsigned)D;
    return ((long)vb + (long)k * Vb) * D + b;
}

constexpr int kMaxFft = 2048;     // longest padded side of the preconditioner's FFT
constexpr int kMaxFbp = 4096;     // longest padded detector row of the FBP filter
constexpr int kLogCap = 256;      // iterations kept in the device log ring
constexpr int kLogStride = 12;    // doubles per log entry
constexpr int kPartialSlots = 4;  // doubles per block partial
constexpr int kRaySumBlocks = 240;  // block partials of the ray sums of the start image

// Device scalar block (doubles), at layout.scalars.
enum Scalar : int {
    S_RHO = 0,      // [2] rho in force
    S_KAPPA = 2,    // [2] pending dual rescale rho_old / rho_new
    S_GAMMA = 4,    // [2] r.r
    S_ALPHA = 6,    // [2] CG step
    S_BETA = 8,     // [2] CG direction update
    S_PQ = 10,      // [2] p.q
    S_ITER = 12,    // outer iteration counter
    S_FLAGS = 13,   // bit 0: non-finite value met
    S_LAM = 14,     // [2] lambda
    S_NEXT_RHO = 16,// [2] scheduled rho of the next iteration
    S_COUNT = 24
};

// Partial-sum sections (block partials of kPartialSlots doubles each).
struct Partials {
    double* sino;   // UDM: |a-Rx|^2 c, p; data cost; non-finite count
    double* img;    // TV: |y-Dx|^2+|z-x|^2 c, p; |y_c|_1, |y_p|_1
    double* tiles;  // backprojection epilogues: two sums per tile
    double* pre;    // preconditioner: r . z per image row
};

}  // namespace dect
