// Joseph projector R (ray-driven) and its exact transpose R^T (pixel-driven
// gather, no atomics), for gfx950.
//
// Rotational symmetry.  For a fan beam over a full turn with n_views divisible
// by 4 and a square image, view v + k V/4 is view v turned by k quarter turns,
// and the pixel grid maps onto itself.  The plan then defines the rays of those
// views as exact rotations of the V/4 base views (SYM = 4): one Joseph weight
// computation serves four views.  Otherwise SYM = 1 and every view is a base view.
//
// Projector: one lane per base ray; a wave holds consecutive bins of one to four
// neighbouring base views, so output writes are coalesced along the detector.  It
// reads an "orbit" image O[j][i] = (X[rot^k (i, j)], k < SYM) -- the SYM rotated
// copies interleaved per pixel -- or its transpose for x-stepped rays, so that one
// record per tap serves all SYM views; a wave stages the part of each image line its
// rays cross in LDS and its lanes read their taps from there.
//
// Transpose: one lane owns the rotation orbit of a pixel.  For every base view
// and every orbit member it locates, from the central projection of the
// two-pixel segment around the pixel, the bins whose samples can touch it, and
// re-evaluates each candidate's interpolation weight from the same ray geometry;
// each weight serves SYM (pixel, view) pairs.  The projector forms the two tap
// weights of a sample as tents max(0, 1 - |phi - j|) and scales by the step length at
// the end, while the transpose forms each weight step max(0, 1 - |d|) from the
// signed distance d of its own ray records, so the pair is a transpose up to rounding
// (FP64 adjointness to 1e-12), not bit for bit.  The views are split over the waves
// of a workgroup and the wave sums are added in a fixed order through LDS.
#include <mutex>

#include "common.h"
#include "epilogue.h"
#include "kernels.h"
#include "profile.h"

namespace dect {

namespace {

// Pixel (i, j) turned by k quarter turns about the image centre (n x n image).
__device__ inline void rot(int k, int n, int i, int j, int& io, int& jo) {
    switch (k & 3) {
        case 0: io = i; jo = j; break;
        case 1: io = n - 1 - j; jo = i; break;
        case 2: io = n - 1 - i; jo = n - 1 - j; break;
        default: io = j; jo = n - 1 - i; break;
    }
}

// Orbit record of pixel (i, j): component k*CH + c = channel c of X at rot^k(i, j).
template <typename T, int CH, int SYM>
__device__ inline vec<T, CH * SYM> orbit_record(const vec<T, CH>* __restrict__ X, int nx, int i,
                                                int j) {
    vec<T, CH * SYM> o;
#pragma unroll
    for (int k = 0; k < SYM; ++k) {
        int io, jo;
        rot(k, nx, i, j, io, jo);
        const vec<T, CH> x = X[(size_t)jo * nx + io];
#pragma unroll
        for (int c = 0; c < CH; ++c) o.v[k * CH + c] = x.v[c];
    }
    return o;
}

// Orbit image O[j][i] and its transpose OT[i][j] in one pass: thread idx writes
// record idx of both.  SYM = 1 gives X and X^T.
template <typename T, int CH, int SYM, bool BATCH>
__global__ __launch_bounds__(256) void k_orbit(const OrbitArgs<T>* __restrict__ dev,
                                               OrbitArgs<T> one) {
    const OrbitArgs<T> A = pick_args<BATCH>(dev, one);
    const int nx = A.nx, ny = A.ny;
    const vec<T, CH>* __restrict__ X = reinterpret_cast<const vec<T, CH>*>(A.X);
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nx * ny) return;
    reinterpret_cast<vec<T, CH * SYM>*>(A.O)[idx] =
        orbit_record<T, CH, SYM>(X, nx, (int)(idx % nx), (int)(idx / nx));
    reinterpret_cast<vec<T, CH * SYM>*>(A.OT)[idx] =
        orbit_record<T, CH, SYM>(X, nx, (int)(idx / ny), (int)(idx % ny));
}

// The same two orbit images for the quarter-turn symmetric square image, by tiles of
// TS x TS pixels: the four rotated TS x TS regions of X that a tile's records draw on
// are loaded into LDS with coalesced reads (each along its own contiguous axis), then
// the tile's records are written to O along i and to OT along j, both coalesced.
template <typename T, int CH, bool BATCH>
__global__ __launch_bounds__(256) void k_orbit_tiled(const OrbitArgs<T>* __restrict__ dev,
                                                     OrbitArgs<T> one) {
    using X1 = vec<T, CH>;
    using R = vec<T, CH * 4>;
    constexpr int TS = 16;
    __shared__ X1 xs[4][TS][TS + 1];  // xs[k][a][b] = X at rot^k(i0 + b, j0 + a)
    const OrbitArgs<T> A = pick_args<BATCH>(dev, one);
    const int n = A.nx;
    const int tiles = (n + TS - 1) / TS;
    if ((int)blockIdx.x >= tiles * tiles) return;  // beyond this slice (whole block)
    const int i0 = (int)(blockIdx.x % tiles) * TS, j0 = (int)(blockIdx.x / tiles) * TS;
    const X1* __restrict__ X = reinterpret_cast<const X1*>(A.X);
    for (int t = threadIdx.x; t < TS * TS; t += blockDim.x) {
        const int u = t / TS, w = t % TS;  // w is the fast index of this pass
        // rot^0 (i, j) and rot^2 (n-1-i, n-1-j): X rows follow a, columns follow b.
        // rot^1 (n-1-j, i) and rot^3 (j, n-1-i): X rows follow b, columns follow a.
        {
            const int a = u, b = w, i = i0 + b, j = j0 + a;
            if (i < n && j < n) {
                xs[0][a][b] = X[(size_t)j * n + i];
                xs[2][a][b] = X[(size_t)(n - 1 - j) * n + (n - 1 - i)];
            }
        }
        {
            const int b = u, a = w, i = i0 + b, j = j0 + a;
            if (i < n && j < n) {
                xs[1][a][b] = X[(size_t)i * n + (n - 1 - j)];
                xs[3][a][b] = X[(size_t)(n - 1 - i) * n + j];
            }
        }
    }
    __syncthreads();
    auto rec = [&](int a, int b) {
        R o;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < CH; ++c) o.v[k * CH + c] = xs[k][a][b].v[c];
        return o;
    };
    for (int t = threadIdx.x; t < TS * TS; t += blockDim.x) {
        {
            const int a = t / TS, b = t % TS, i = i0 + b, j = j0 + a;  // along i
            if (i < n && j < n) reinterpret_cast<R*>(A.O)[(size_t)j * n + i] = rec(a, b);
        }
        {
            const int b = t / TS, a = t % TS, i = i0 + b, j = j0 + a;  // along j
            if (i < n && j < n) reinterpret_cast<R*>(A.OT)[(size_t)i * n + j] = rec(a, b);
        }
    }
}

// The CG right-hand side of Eq. (12) (what k_rhs computes) and the orbit images of
// it (what k_orbit_tiled writes) in one launch, for a quarter-turn symmetric square
// image with n % 16 == 0.  A workgroup owns an 8x8 tile of the first quadrant and its
// three rotations: wave k computes r0 on rotation k of the tile in memory order, the
// four tiles' values meet in LDS, and every record of the four tiles is written to O
// along i and to OT along j.  Each partial of |r0|^2 covers the workgroup's 256
// pixels.  The quadrant's tiles are dealt to the XCDs in bands of consecutive tiles,
// so that most stencil neighbours of a tile are read through the same L2.
template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_rhs_orbit(const BpArgs<T>* __restrict__ dev,
                                                   BpArgs<T> one,
                                                   const OrbitArgs<T>* __restrict__ odev,
                                                   OrbitArgs<T> oone) {
    using V2 = vec<T, 2>;
    using R = vec<T, 8>;
    constexpr int TS = 8;
    __shared__ V2 xs[4][TS][TS + 1];  // xs[k][a][b] = r0 at rot^k(i0 + b, j0 + a)
    const BpArgs<T> A = pick_args<BATCH>(dev, one);
    const OrbitArgs<T> Ob = pick_args<BATCH>(odev, oone);
    const int n = A.nx;
    const unsigned h = (unsigned)n / (2 * TS), tiles = h * h, id = blockIdx.x;
    if (id >= tiles) return;  // beyond this slice (whole block)
    const unsigned tile =
        tiles % kXcds == 0 ? (id % kXcds) * (tiles / kXcds) + id / kXcds : id;
    const int i0 = (int)(tile % h) * TS, j0 = (int)(tile / h) * TS;
    const int k = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    // Lower corner (ci, cj) of rotation k of the tile [i0, i0 + TS) x [j0, j0 + TS).
    int ci, cj;
    switch (k) {
        case 0: ci = i0; cj = j0; break;
        case 1: ci = n - TS - j0; cj = i0; break;
        case 2: ci = n - TS - i0; cj = n - TS - j0; break;
        default: ci = j0; cj = n - TS - i0; break;
    }
    const int back = (4 - k) & 3;  // rot^back undoes rot^k
    {
        const int pi = ci + (l & (TS - 1)), pj = cj + (l >> 3);
        const size_t pix = (size_t)pj * n + pi;
        T res[2];
        rhs_tracked(A, pix, res);
        double part[2] = {0.0, 0.0};
        epilogue<T, EPI_RHS>(A, pi, pj, res, part);
        int ib, jb;
        rot(back, n, pi, pj, ib, jb);
        V2& d = xs[k][jb - j0][ib - i0];
        d.v[0] = res[0];
        d.v[1] = res[1];
        block_sum_store<2>(part, A.part_img + (size_t)tile * kPartialSlots);
    }
    __syncthreads();
    // The record of pixel P = rot^k(B), B = (i0 + b, j0 + a): component kk of it is r0
    // at rot^kk(P) = rot^(kk + k)(B).
    auto rec = [&](int pi, int pj) {
        int ib, jb;
        rot(back, n, pi, pj, ib, jb);
        const int a = jb - j0, b = ib - i0;
        R o;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int c = 0; c < 2; ++c) o.v[kk * 2 + c] = xs[(kk + k) & 3][a][b].v[c];
        return o;
    };
    {
        const int pi = ci + (l & (TS - 1)), pj = cj + (l >> 3);  // along i
        reinterpret_cast<R*>(Ob.O)[(size_t)pj * n + pi] = rec(pi, pj);
    }
    {
        const int pi = ci + (l >> 3), pj = cj + (l & (TS - 1));  // along j
        reinterpret_cast<R*>(Ob.OT)[(size_t)pi * n + pj] = rec(pi, pj);
    }
}

// The value of x in lane l (uniform).
__device__ inline float lane_value(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ inline double lane_value(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// R for base rays: QUAD = true writes [Vb][D][SYM][CH] records, false writes the
// standard [V][D][CH] layout (view v + k*Vb for rotation k).  A workgroup owns
// 64 / views consecutive bins of `views` consecutive base views (one ray per lane),
// in the XCD-aware order of proj_blocks; its KS waves step through KS
// disjoint ranges of the image lines its rays cross (so the lanes of a wave read
// one image line together) and wave 0 adds the KS partial sums in order.
template <typename T, int CH, int SYM, bool QUAD, int KS, bool BATCH>
__global__ __launch_bounds__(64 * KS) void k_project(const ProjArgs<T>* __restrict__ dev,
                                                     ProjArgs<T> one) {
    constexpr int W = CH * SYM;
    using V = vec<T, W>;
    // Each wave's staged line window, a tap record split into NCH chunks of up to 16
    // bytes held in separate arrays: the lanes of a wave read nearby records, and
    // 16-byte records put records r and r + 8 (not r + 4) on the same LDS banks.
    // After the sample loops wave w > 0 leaves its partial sums in its own window for
    // wave 0.
    constexpr int CE = W * (int)sizeof(T) > 16 ? 16 / (int)sizeof(T) : W;  // values per chunk
    constexpr int NCH = W / CE;
    using VC = vec<T, CE>;
    __shared__ VC s_win[KS][NCH][kProjWin];
    const ProjArgs<T> A = pick_args<BATCH>(dev, one);
    const int nx = A.nx, ny = A.ny, Vb = A.Vb, D = A.D;
    const int BV = A.views, lbv = __builtin_ctz((unsigned)A.views);
    const int BB = 64 >> lbv;
    int bg, vg;
    proj_tile(blockIdx.x, proj_grid_y(Vb, BV), A.chunk, bg, vg);
    if (bg >= proj_grid_x(D, BV)) return;  // past the last bin group of this slice
    const RayParam<T>* __restrict__ rays = A.rays;
    const vec<T, W>* __restrict__ O = reinterpret_cast<const vec<T, W>*>(A.O);
    const vec<T, W>* __restrict__ OT = reinterpret_cast<const vec<T, W>*>(A.OT);
    T* __restrict__ sino = A.sino;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int v = vg * BV + (lane & (BV - 1));
    const int b = bg * BB + (lane >> lbv);
    const bool valid = b < D && v < Vb;
    RayParam<T> r = rays[(size_t)(v < Vb ? v : Vb - 1) * D + (b < D ? b : D - 1)];
    const bool xs = r.pad == T(0);
    const int n_steps = xs ? nx : ny;   // samples along the ray
    const int n_lines = xs ? ny : nx;   // interpolation axis
    const vec<T, W>* src = xs ? OT : O;  // [n_steps][n_lines]
    // Outside [k0, k1] both taps of every sample are outside the image, so the
    // restriction changes no term.
    int k0, k1;
    proj_ray_range<T>(r.phi0, r.slope, n_steps, n_lines, k0, k1);
    // This wave's share of the lines: every wave holds the same 64 rays, so each
    // computes the same union [s0, s1] of their ranges and takes its KS-th of it
    // (an even split of all lines would leave most waves idle on short chords).
    // An empty union gives [0, -1], so no wave enters the sample loops.
    const bool any = valid && k0 <= k1;
    int s0 = any ? k0 : 1 << 30, s1 = any ? k1 : -1;
    for (int off = 32; off > 0; off >>= 1) {
        const int a = __shfl_xor(s0, off, 64), c = __shfl_xor(s1, off, 64);
        s0 = a < s0 ? a : s0;
        s1 = c > s1 ? c : s1;
    }
    int c0, c1;
    proj_wave_share(s0, s1, wave, KS, c0, c1);
    c0 = __builtin_amdgcn_readfirstlane(c0);  // the same in every lane
    c1 = __builtin_amdgcn_readfirstlane(c1);
    k0 = k0 > c0 ? k0 : c0;
    k1 = k1 < c1 ? k1 : c1;
    if (!valid) k1 = -1;
    T acc[W];
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = T(0);
    auto add = [&](T w0, const V& a0, T w1, const V& a1) {
#pragma unroll
        for (int c = 0; c < W; ++c) {
            acc[c] = fma(w0, a0.v[c], acc[c]);
            acc[c] = fma(w1, a1.v[c], acc[c]);
        }
    };
    const unsigned long long vmask = __ballot(valid);
    const unsigned long long xmask = __ballot(valid && xs);
    if (vmask != 0ull && (xmask == 0ull || xmask == vmask)) {
        // Every ray of the wave steps along the same axis: stage each line's window
        // (proj_window) in LDS, one tap per lane, the next line's loads in flight
        // while the current line is summed.
        using GV = const __attribute__((address_space(1))) V;
        GV* __restrict__ wimg = (GV*)(xmask != 0ull ? OT : O);
        const int wl = xmask != 0ull ? ny : nx;  // this wave's interpolation axis
        int wa, wb;
        proj_window_line<T>(lane_value(r.phi0, 0), lane_value(r.slope, 0),
                            lane_value(r.phi0, 63), lane_value(r.slope, 63), wa, wb);
        wa = __builtin_amdgcn_readfirstlane(wa);
        wb = __builtin_amdgcn_readfirstlane(wb);
        auto load = [&](GV* q) {
            V o;
#pragma unroll
            for (int c = 0; c < W; ++c) o.v[c] = q->v[c];
            return o;
        };
        // Tap t of line k, addressed from the line's start (uniform) by a 32-bit byte
        // offset.
        using GC = const __attribute__((address_space(1))) char;
        auto tap = [&](int k, int t) {
            GC* line = (GC*)(wimg + (size_t)k * wl);
            return load((GV*)(line + (unsigned)t * (unsigned)sizeof(V)));
        };
        V staged;
        int s_next = 0;
        if (c0 <= c1) {
            s_next = proj_window(wa, wb, c0);
            staged = tap(c0, min(max(s_next + lane, 0), wl - 1));
        }
        for (int k = c0; k <= c1; ++k) {
            const int s0w = s_next;
#pragma unroll
            for (int h = 0; h < NCH; ++h)
#pragma unroll
                for (int c = 0; c < CE; ++c) s_win[wave][h][lane].v[c] = staged.v[h * CE + c];
            // LDS operations of one wave complete in order; the barrier only keeps
            // the compiler from moving the reads above the write.
            __builtin_amdgcn_wave_barrier();
            if (k < c1) {
                s_next = proj_window(wa, wb, k + 1);
                staged = tap(k + 1, min(max(s_next + lane, 0), wl - 1));
            }
            if (k >= k0 && k <= k1) {
                T w0, w1;
                const int j = proj_taps<T>(r.phi0, r.slope, (T)k, wl, w0, w1);
                const int idx = j - s0w;
                if ((unsigned)idx <= (unsigned)(kProjWin - 2)) {
                    V a0, a1;
#pragma unroll
                    for (int h = 0; h < NCH; ++h) {
                        const VC x0 = s_win[wave][h][idx], x1 = s_win[wave][h][idx + 1];
#pragma unroll
                        for (int c = 0; c < CE; ++c) {
                            a0.v[h * CE + c] = x0.v[c];
                            a1.v[h * CE + c] = x1.v[c];
                        }
                    }
                    add(w0, a0, w1, a1);
                } else {
                    add(w0, tap(k, j), w1, tap(k, j + 1));
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    } else {
        // Rays of both orientations: each lane reads its own taps.
        const V* __restrict__ img = xs ? OT : O;
        for (int k = k0; k <= k1; ++k) {
            T w0, w1;
            const int j = proj_taps<T>(r.phi0, r.slope, (T)k, n_lines, w0, w1);
            const V* line = img + (size_t)k * n_lines;
            add(w0, line[j], w1, line[j + 1]);
        }
    }
    if constexpr (KS > 1) {
        if (wave > 0)
#pragma unroll
            for (int c = 0; c < W; ++c) s_win[wave][c / CE][lane].v[c % CE] = acc[c];
        __syncthreads();
        if (wave != 0) return;
        for (int w = 1; w < KS; ++w)
#pragma unroll
            for (int c = 0; c < W; ++c) acc[c] += s_win[w][c / CE][lane].v[c % CE];
    }
    if (!valid) return;
    if constexpr (QUAD) {
        vec<T, W> out;
#pragma unroll
        for (int c = 0; c < W; ++c) out.v[c] = acc[c] * r.step;
        reinterpret_cast<vec<T, W>*>(sino)[(size_t)v * D + b] = out;
    } else {
#pragma unroll
        for (int s = 0; s < SYM; ++s) {
            vec<T, CH> out;
#pragma unroll
            for (int c = 0; c < CH; ++c) out.v[c] = acc[s * CH + c] * r.step;
            reinterpret_cast<vec<T, CH>*>(sino)[(size_t)(v + s * Vb) * D + b] = out;
        }
    }
}

template <typename T>
__device__ inline T fast_rcp(T x) { return T(1) / x; }
template <>
__device__ inline float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// Sum over the base views of this wave (v = wave, wave + VS, ...) for the orbit
// of pixel (i, j), reading a standard [V][D][CH] sinogram.  Pixel rot^k(p) seen
// from view v + k' Vb has the weight of base view v at pixel rot^(k - k')(p), so
// for every orbit member p_m = rot^m(p) the base-view weights are evaluated once
// and routed to acc[(m + k') mod SYM] with sinogram row v + k' Vb, for all k'.
//
// Candidates are the bins within h = max|d beta / d pixel| + margin of the
// member's detector coordinate beta (a ray more than one pixel step away along
// its minor axis has no tap on the pixel); the footprint needs only ~1e-3-bin
// accuracy, which the margin covers, hence the hardware reciprocal.  The ray's
// type says which pixel coordinate it samples along, and the weight
// max(0, step (1 - |phi - p|)) is the projector's linear-interpolation weight of
// the pixel at minor coordinate p for the sample at phi, phi computed with the
// same fma on the same table entries as the projector's sample position.
template <typename T, typename A, int CH, int SYM, int VS>
__device__ inline void gather_orbit(const BpArgs<T>& a, int wave, int i, int j,
                                    A (&acc)[SYM][CH]) {
    const T m = (T)a.margin;
    const int D = a.D, Vb = a.Vb, n = a.nx;
    const T cx = T(0.5) * (T)(a.nx - 1), cy = T(0.5) * (T)(a.ny - 1);
    const vec<T, CH>* __restrict__ sv = reinterpret_cast<const vec<T, CH>*>(a.sino);
    for (int v = wave; v < Vb; v += VS) {
        const ViewParam<T> w = a.views[v];
        const RayParam<T>* __restrict__ rv = a.rays + (size_t)v * D;
#pragma unroll
        for (int mm = 0; mm < SYM; ++mm) {
            int im, jm;
            rot(mm, n, i, j, im, jm);
            const T fi = (T)im, fj = (T)jm;
            const T ip = fi - cx, jp = fj - cy;
            const T inv = fast_rcp<T>(w.d0 + w.di * ip + w.dj * jp);
            const T bq = (w.ni * ip + w.nj * jp) * inv;
            const T bc = bq + w.boff;
            // d(beta) for one pixel step along y and along x.
            const T dby = (w.nj - bq * w.dj) * inv;
            const T dbx = (w.ni - bq * w.di) * inv;
            const T h = fmax(fabs(dby), fabs(dbx)) + m;
            const int lo0 = (int)ceil(fmax(bc - h, T(-1)));
            const int hi0 = (int)floor(fmin(bc + h, T(D)));
            const int lo = lo0 > 0 ? lo0 : 0, hi = hi0 < D - 1 ? hi0 : D - 1;
            for (int b = lo; b <= hi; ++b) {
                const RayParam<T> r = rv[b];
                const bool xs = r.pad == T(0);
                const T phi = fma(r.slope, xs ? fi : fj, r.phi0);
                const T wt = fmax(T(0), fma(-r.step, fabs(phi - (xs ? fj : fi)), r.step));
#pragma unroll
                for (int kp = 0; kp < SYM; ++kp) {
                    const vec<T, CH> t = sv[(size_t)(v + kp * Vb) * D + b];
#pragma unroll
                    for (int c = 0; c < CH; ++c)
                        acc[(mm + kp) % SYM][c] = fma((A)wt, (A)t.v[c], acc[(mm + kp) % SYM][c]);
                }
            }
        }
    }
}

// Quarter turns of a real point about the image centre, as rot() for pixels.
template <typename T>
__device__ inline void rotf(int k, int n, T i, T j, T& io, T& jo) {
    const T e = (T)(n - 1);
    switch (k & 3) {
        case 0: io = i; jo = j; break;
        case 1: io = e - j; jo = i; break;
        case 2: io = e - i; jo = e - j; break;
        default: io = j; jo = e - i; break;
    }
}

// As gather_orbit for quad sinograms, with each view's candidate records staged in
// LDS.  A wave covers the 64 orbits of its block: per view and orbit member their
// candidate bins lie within a few bins of the block centre's detector coordinate,
// so WIN records around it (ray parameters and the quad of sinogram values) are
// loaded once per view by WIN lanes and read by every lane from LDS instead of
// each lane loading them again.  The loads for the wave's next view are issued
// before the current view is accumulated, so their latency is hidden.  A candidate
// outside the window (a steep footprint near the source) is loaded directly.
template <typename T, typename A, int CH, int SYM, int VS>
__device__ inline void gather_orbit_staged(const BpArgs<T>& a, int wave, int lane, int i, int j,
                                           int bx, int by, bool inside, A (&acc)[SYM][CH]) {
    constexpr int WIN = 16;
    using Q = vec<T, SYM * CH>;
    __shared__ RayParam<T> s_ray[VS][WIN * SYM];
    __shared__ Q s_sino[VS][WIN * SYM];
    const T m = (T)a.margin;
    const int D = a.D, Vb = a.Vb, n = a.nx;
    const T cx = T(0.5) * (T)(a.nx - 1), cy = T(0.5) * (T)(a.ny - 1);
    const Q* __restrict__ sino = reinterpret_cast<const Q*>(a.sino);
    // This lane stages bin sk of the window of orbit member sm, centred on the
    // detector coordinate of the block centre seen as that member.
    const int sm = lane / WIN, sk = lane % WIN;
    const bool stager = lane < WIN * SYM;
    T icm, jcm;
    rotf<T>(sm, n, (T)(bx * 8) + T(3.5), (T)(by * 8) + T(3.5), icm, jcm);
    const T ipc = icm - cx, jpc = jcm - cy;
    RayParam<T> pr{};
    Q pq;
    int pL = 0;
    auto stage = [&](int v) {
        const ViewParam<T> w = a.views[v];
        const T bq = (w.ni * ipc + w.nj * jpc) / (w.d0 + w.di * ipc + w.dj * jpc);
        pL = (int)floor(bq + w.boff) - (WIN / 2 - 1);
        const int b = pL + sk;
        if (stager && b >= 0 && b < D) {
            pr = a.rays[(size_t)v * D + b];
            pq = sino[(size_t)v * D + b];
        } else {
            pr = RayParam<T>{};
#pragma unroll
            for (int c = 0; c < SYM * CH; ++c) pq.v[c] = T(0);
        }
    };
    if (wave < Vb) stage(wave);
    for (int v = wave; v < Vb; v += VS) {
        int L[SYM];
#pragma unroll
        for (int mm = 0; mm < SYM; ++mm) L[mm] = __builtin_amdgcn_readlane(pL, mm * WIN);
        if (stager) {
            s_ray[wave][lane] = pr;
            s_sino[wave][lane] = pq;
        }
        // LDS operations of one wave complete in order; the barrier only keeps the
        // compiler from moving the reads above the writes.
        __builtin_amdgcn_wave_barrier();
        if (v + VS < Vb) stage(v + VS);
        if (inside) {
            const ViewParam<T> w = a.views[v];
            const RayParam<T>* __restrict__ rv = a.rays + (size_t)v * D;
            const Q* __restrict__ sq = sino + (size_t)v * D;
#pragma unroll
            for (int mm = 0; mm < SYM; ++mm) {
                int im, jm;
                rot(mm, n, i, j, im, jm);
                const T fi = (T)im, fj = (T)jm;
                const T ip = fi - cx, jp = fj - cy;
                const T inv = fast_rcp<T>(w.d0 + w.di * ip + w.dj * jp);
                const T bq = (w.ni * ip + w.nj * jp) * inv;
                const T bc = bq + w.boff;
                const T dby = (w.nj - bq * w.dj) * inv;
                const T dbx = (w.ni - bq * w.di) * inv;
                const T h = fmax(fabs(dby), fabs(dbx)) + m;
                const int lo0 = (int)ceil(fmax(bc - h, T(-1)));
                const int hi0 = (int)floor(fmin(bc + h, T(D)));
                const int lo = lo0 > 0 ? lo0 : 0, hi = hi0 < D - 1 ? hi0 : D - 1;
                for (int b = lo; b <= hi; ++b) {
                    const int idx = b - L[mm];
                    RayParam<T> r;
                    Q s;
                    if ((unsigned)idx < (unsigned)WIN) {
                        r = s_ray[wave][mm * WIN + idx];
                        s = s_sino[wave][mm * WIN + idx];
                    } else {
                        r = rv[b];
                        s = sq[b];
                    }
                    const bool xs = r.pad == T(0);
                    const T phi = fma(r.slope, xs ? fi : fj, r.phi0);
                    const T wt = fmax(T(0), fma(-r.step, fabs(phi - (xs ? fj : fi)), r.step));
#pragma unroll
                    for (int kp = 0; kp < SYM; ++kp)
#pragma unroll
                        for (int c = 0; c < CH; ++c)
                            acc[(mm + kp) % SYM][c] =
                                fma((A)wt, (A)s.v[kp * CH + c], acc[(mm + kp) % SYM][c]);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// gather_orbit_staged with a 32-bin window for the quarter-turn symmetric fan: a
// block's candidates span about 8 sqrt(2) pixels times the magnification
// |d beta / d pixel| plus the footprint, ~14 bins at the centre of the fan and up to
// ~35 for blocks near the source, so 16 bins left most waves loading some
// candidates directly; with 32 that is rare.

// A staged candidate of the wide window: its ray record and its quad of sinogram
// values side by side (48 bytes for two FP32 channels), so that one address steps
// through the window.
template <typename T, int CH, int SYM>
struct alignas(sizeof(T) * 4) Staged {
    BpRay<T> r;
    T s[SYM * CH];
};
constexpr int kWideWin = 32;
// Candidates every lane takes from its window before looping over the rest: most
// footprints hold two or three, and a candidate past a pixel's footprint has weight
// exactly zero (its ray passes more than a pixel step away), so the loop's control
// flow is saved where most lanes need it least.  Each orbit member's window is
// followed by kBpFixed zero records, so that those reads never leave it.
#ifndef DECT_BP_FIXED
#define DECT_BP_FIXED 0
#endif
constexpr int kBpFixed = DECT_BP_FIXED;
constexpr int kWideStride = kWideWin + kBpFixed;

// Each lane stages WIN * SYM / 64 records.  s_win: the workgroup's staging windows,
// [VS][SYM members][kWideStride]; each wave uses only its own row.
template <typename T, typename A, int CH, int SYM, int VS>
__device__ inline void gather_orbit_staged_wide(const BpArgs<T>& a, int wave, int lane, int i, int j,
                                                int bx, int by, bool inside, A (&acc)[SYM][CH],
                                                Staged<T, CH, SYM> (*s_win)[kWideStride * SYM]) {
    constexpr int WIN = kWideWin;
    constexpr int REC = WIN * SYM;
    constexpr int PER = (REC + 63) / 64;
    static_assert(WIN % 16 == 0 && (REC <= 64 || REC % 64 == 0), "window layout");
    static_assert(kBpFixed * SYM <= 64, "padding records per wave");
    if constexpr (kBpFixed > 0) {
        if (lane < kBpFixed * SYM) {  // the zero records after each window
            Staged<T, CH, SYM>& z =
                s_win[wave][(lane / kBpFixed) * kWideStride + WIN + lane % kBpFixed];
            z.r = BpRay<T>{};
#pragma unroll
            for (int c = 0; c < SYM * CH; ++c) z.s[c] = T(0);
        }
    }
    using Q = vec<T, SYM * CH>;
    const T m = (T)a.margin;
    const int D = a.D, Vb = a.Vb, n = a.nx;
    const T cx = T(0.5) * (T)(a.nx - 1), cy = T(0.5) * (T)(a.ny - 1);
    const Q* __restrict__ sino = reinterpret_cast<const Q*>(a.sino);
    // Record lane + 64 q of the window is bin (rec % WIN) of orbit member rec / WIN,
    // centred on the detector coordinate of the block centre seen as that member.
    T ipc[PER], jpc[PER];
    int sk[PER];
    bool stager[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int rec = lane + 64 * q;
        stager[q] = rec < REC;
        sk[q] = rec % WIN;
        T icm, jcm;
        rotf<T>(rec / WIN, n, (T)(bx * 8) + T(3.5), (T)(by * 8) + T(3.5), icm, jcm);
        ipc[q] = icm - cx;
        jpc[q] = jcm - cy;
    }
    BpRay<T> pr[PER];
    Q pq[PER];
    int pL[PER];
    auto stage = [&](int v) {
        const ViewParam<T> w = a.views[v];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            // Only the window's placement depends on this value (candidates outside
            // it are loaded directly), so the hardware reciprocal is accurate enough.
            const T bq = (w.ni * ipc[q] + w.nj * jpc[q]) *
                         fast_rcp<T>(w.d0 + w.di * ipc[q] + w.dj * jpc[q]);
            pL[q] = (int)floor(bq + w.boff) - (WIN / 2 - 1);
            const int b = pL[q] + sk[q];
            if (stager[q] && b >= 0 && b < D) {
                pr[q] = a.brays[(size_t)v * D + b];
                pq[q] = sino[(size_t)v * D + b];
            } else {
                pr[q] = BpRay<T>{};
#pragma unroll
                for (int c = 0; c < SYM * CH; ++c) pq[q].v[c] = T(0);
            }
        }
    };
    if (wave < Vb) stage(wave);
    for (int v = wave; v < Vb; v += VS) {
        int L[SYM];
#pragma unroll
        for (int mm = 0; mm < SYM; ++mm)
            L[mm] = __builtin_amdgcn_readlane(pL[(mm * WIN) / 64], (mm * WIN) % 64);
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (stager[q]) {
                const int rec = lane + 64 * q;
                Staged<T, CH, SYM>& d = s_win[wave][(rec / WIN) * kWideStride + rec % WIN];
                d.r = pr[q];
#pragma unroll
                for (int c = 0; c < SYM * CH; ++c) d.s[c] = pq[q].v[c];
            }
        // LDS operations of one wave complete in order; the barrier only keeps the
        // compiler from moving the reads above the writes.
        __builtin_amdgcn_wave_barrier();
        if (v + VS < Vb) stage(v + VS);
        if (inside) {
            const ViewParam<T> w = a.views[v];
            const BpRay<T>* __restrict__ rv = a.brays + (size_t)v * D;
            const Q* __restrict__ sq = sino + (size_t)v * D;
            // Orbit member mm of the centred pixel (ip, jp) is (ip, jp), (-jp, ip),
            // (-ip, -jp), (jp, -ip), so its projective denominator and numerator are
            // signed combinations of four products shared by the members.
            const T ip0 = (T)i - cx, jp0 = (T)j - cy;
            const T pa = w.di * ip0 + w.dj * jp0, pb = w.dj * ip0 - w.di * jp0;
            const T na = w.ni * ip0 + w.nj * jp0, nb = w.nj * ip0 - w.ni * jp0;
#pragma unroll
            for (int mm = 0; mm < SYM; ++mm) {
                int im, jm;
                rot(mm, n, i, j, im, jm);
                const T fi = (T)im, fj = (T)jm;
                const T dq = (mm & 1) ? pb : pa, nq = (mm & 1) ? nb : na;
                // The denominator is positive for every image pixel (the plan keeps a
                // fan's source outside the image), so |d beta / d i| and
                // |d beta / d j| share the factor inv.
                const T inv = fast_rcp<T>(mm & 2 ? w.d0 - dq : w.d0 + dq);
                const T bq = (mm & 2 ? -nq : nq) * inv;
                const T h = fma(fmax(fabs(w.nj - bq * w.dj), fabs(w.ni - bq * w.di)), inv, m);
                auto add = [&](const BpRay<T>& r, const T* s) {
                    const T d = fma(r.ci, fi, fma(r.cj, fj, r.phi0));
                    const T wt = fmax(T(0), fma(-r.step, fabs(d), r.step));
#pragma unroll
                    for (int kp = 0; kp < SYM; ++kp)
#pragma unroll
                        for (int c = 0; c < CH; ++c)
                            acc[(mm + kp) % SYM][c] =
                                fma((A)wt, (A)s[kp * CH + c], acc[(mm + kp) % SYM][c]);
                };
                // Candidates in the window come from LDS, in window coordinates (bins
                // of the window past the detector's ends hold zero records and add
                // nothing).  The rest (a steep footprint near the source, rare) are
                // loaded directly, after them, when some lane of the wave has any.
                const T x = bq + (w.boff - (T)L[mm]);
                const int ilo = min((int)ceil(fmax(x - h, T(0))), WIN);
                const int ihi = (int)floor(fmin(x + h, T(WIN - 1)));
                const Staged<T, CH, SYM>* sw = &s_win[wave][mm * kWideStride];
                const Staged<T, CH, SYM>* c = sw + ilo;
#pragma unroll
                for (int t = 0; t < kBpFixed; ++t) add(c[t].r, c[t].s);
                for (c += kBpFixed; c <= sw + ihi; ++c) add(c->r, c->s);
                if (__any(x - h < T(0) || x + h > T(WIN - 1))) {
                    const T bc = bq + w.boff;
                    const int lo = (int)ceil(fmax(bc - h, T(0)));
                    const int hi = (int)floor(fmin(bc + h, T(D - 1)));
                    const int below = min(hi, L[mm] - 1), above = max(lo, L[mm] + WIN);
                    for (int b = lo; b <= below; ++b) add(rv[b], sq[b].v);
                    for (int b = above; b <= hi; ++b) add(rv[b], sq[b].v);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}


// R^T (+ epilogue).  A workgroup owns an 8x8 block of pixel orbits (the block
// lies in the first quadrant when SYM = 4) and has VS waves, each summing a
// disjoint subset of the base views; wave 0 adds the others' sums in order.  A: the
// type the sums are kept in (T, or double for an FP32 plan's sums in double precision:
// each product of two FP32 values is exact in double, so only the sums round); the
// finished values are rounded to T once.
template <typename T, int CH, int SYM, bool QUAD, int EPI, int VS, bool BATCH, typename A = T>
__global__ __launch_bounds__(64 * VS) void k_backproject(const BpArgs<T>* __restrict__ dev,
                                                         BpArgs<T> one, unsigned nslices) {
    // The ADMM epilogues (q, dual) run one orbit member per wave; the plain transpose
    // keeps the reduction into wave 0.
    constexpr bool kFinish = EPI == EPI_Q || EPI == EPI_DUAL;
    constexpr bool kWide = QUAD && SYM == 4;
    // The wide staging windows, one row per wave.  For the ADMM epilogues each wave
    // then stores its view sums over its own (by then idle) row.
    using St = Staged<T, CH, SYM>;
    __shared__ St s_win[kWide ? VS : 1][kWide ? kWideStride * SYM : 1];
    constexpr int kRed = kFinish ? (kWide ? 1 : VS) : (VS > 1 ? VS - 1 : 1);
    __shared__ A red_own[kRed][64][SYM * CH];
    static_assert(!kWide || sizeof(A) * 64 * SYM * CH <= sizeof(St) * kWideStride * SYM,
                  "a wave's view sums fit in its staging row");
    auto red = [&](int w) -> A(*)[SYM * CH] {
        if constexpr (kFinish && kWide) return reinterpret_cast<A(*)[SYM * CH]>(&s_win[w][0]);
        else return red_own[w];
    };
    // The orbit block (bx, by) of this workgroup: its 2-D grid position for one slice;
    // in a batch, a 1-D grid that gives each XCD an equal contiguous share of the
    // slices' blocks (one.gx, one.gy: the group's block grid, the same for all its
    // slices).
    int bx, by;
    unsigned slice = 0;
    if constexpr (BATCH) {
        unsigned tile;
        if (!xcd_slice_tile(blockIdx.x, (unsigned)(one.gx * one.gy), nslices, slice, tile))
            return;
        bx = (int)(tile % (unsigned)one.gx);
        by = (int)(tile / (unsigned)one.gx);
    } else {
        bx = (int)blockIdx.x;
        by = (int)blockIdx.y;
    }
    const BpArgs<T> a = pick_args<BATCH>(dev, one, slice);
    if (bx >= a.gx || by >= a.gy) return;  // beyond this slice
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = bx * 8 + (lane & 7);
    const int j = by * 8 + (lane >> 3);
    const int dom_x = SYM == 4 ? a.nx / 2 : a.nx, dom_y = SYM == 4 ? a.ny / 2 : a.ny;
    const bool inside = i < dom_x && j < dom_y;
    A acc[SYM][CH];
#pragma unroll
    for (int k = 0; k < SYM; ++k)
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[k][c] = A(0);
    if constexpr (kWide)
        gather_orbit_staged_wide<T, A, CH, SYM, VS>(a, wave, lane, i, j, bx, by, inside, acc, s_win);
    else if constexpr (QUAD)
        gather_orbit_staged<T, A, CH, SYM, VS>(a, wave, lane, i, j, bx, by, inside, acc);
    else if (inside)
        gather_orbit<T, A, CH, SYM, VS>(a, wave, i, j, acc);
    if constexpr (kFinish) {
        // Every wave's view sums go to LDS; wave w then finishes orbit members w, w + VS,
        // ...: it adds the waves' sums in wave order, runs the epilogue of its member
        // and reduces its partials over its lanes; thread 0 adds the members' partials
        // in member order.
        __shared__ double wpart[SYM][2];
        {
            A(*mine)[SYM * CH] = red(wave);
#pragma unroll
            for (int k = 0; k < SYM; ++k)
#pragma unroll
                for (int c = 0; c < CH; ++c) mine[lane][k * CH + c] = acc[k][c];
        }
        __syncthreads();
        for (int k = wave; k < SYM; k += VS) {
            A sum[2] = {A(0), A(0)};
            for (int w = 0; w < VS; ++w)
#pragma unroll
                for (int c = 0; c < 2; ++c) sum[c] += red(w)[lane][k * CH + (CH > 1 ? c : 0)];
            T res[2] = {(T)sum[0], (T)sum[1]};
            double part[2] = {0.0, 0.0};
            if (inside) {
                int io, jo;
                rot(k, a.nx, i, j, io, jo);
                epilogue<T, EPI>(a, io, jo, res, part);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
                for (int off = 32; off > 0; off >>= 1) part[c] += __shfl_down(part[c], off, 64);
            if (lane == 0) {
                wpart[k][0] = part[0];
                wpart[k][1] = part[1];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double o0 = 0.0, o1 = 0.0;
            for (int k = 0; k < SYM; ++k) {
                o0 += wpart[k][0];
                o1 += wpart[k][1];
            }
            double* o = a.partials + (size_t)(by * a.gx + bx) * kPartialSlots;
            o[0] = o0;
            o[1] = o1;
        }
        return;
    } else {
        if constexpr (VS > 1) {
            if (wave > 0)
#pragma unroll
                for (int k = 0; k < SYM; ++k)
#pragma unroll
                    for (int c = 0; c < CH; ++c) red_own[wave - 1][lane][k * CH + c] = acc[k][c];
            __syncthreads();
            if (wave == 0)
                for (int w = 0; w < VS - 1; ++w)
#pragma unroll
                    for (int k = 0; k < SYM; ++k)
#pragma unroll
                        for (int c = 0; c < CH; ++c) acc[k][c] += red_own[w][lane][k * CH + c];
        }
        if (wave != 0) return;
        double part[2] = {0.0, 0.0};
        if (inside) {
#pragma unroll
            for (int k = 0; k < SYM; ++k) {
                int io, jo;
                rot(k, a.nx, i, j, io, jo);
                if constexpr (EPI == EPI_NONE) {
                    vec<T, CH> o;
#pragma unroll
                    for (int c = 0; c < CH; ++c) o.v[c] = (T)acc[k][c];
                    reinterpret_cast<vec<T, CH>*>(a.out)[(size_t)jo * a.nx + io] = o;
                } else {
                    T res[2] = {(T)acc[k][0], (T)acc[k][CH > 1 ? 1 : 0]};
                    epilogue<T, EPI>(a, io, jo, res, part);
                }
            }
        }
        if constexpr (EPI != EPI_NONE) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
                for (int off = 32; off > 0; off >>= 1) part[c] += __shfl_down(part[c], off, 64);
            if (lane == 0) {
                double* o = a.partials + (size_t)(by * a.gx + bx) * kPartialSlots;
                o[0] = part[0];
                o[1] = part[1];
            }
        }
    }
}

// Waves per workgroup of the plain transposed projector and projector; the ADMM
// kernels take theirs from the plan (2, 4 or 8; see dect_plan_tune).  8 projector
// waves took the LM1 x CG1 iteration at 512^2 from 1.01 to 0.96 ms against 4.
constexpr int kViewSplit = 4;
constexpr int kLineSplit = 8;

template <typename T, int CH, int SYM, bool QUAD, bool BATCH, int KS>
void project_launch(const OrbitArgs<T>* odev, const OrbitArgs<T>& oone, const ProjArgs<T>* pdev,
                    const ProjArgs<T>& pone, int n, long pixels, int gx, int gy, hipStream_t s,
                    bool orbit) {
    if (orbit) {
        ProfScope pt("orbit", s);
        if constexpr (SYM == 4) {
            constexpr int TS = 16;
            const unsigned tiles = (unsigned)((oone.nx + TS - 1) / TS);
            hipLaunchKernelGGL((k_orbit_tiled<T, CH, BATCH>), dim3(tiles * tiles, 1, n), dim3(256),
                               0, s, odev, oone);
        } else {
            hipLaunchKernelGGL((k_orbit<T, CH, SYM, BATCH>), dim3((unsigned)((pixels + 255) / 256), 1, n),
                               dim3(256), 0, s, odev, oone);
        }
    }
    ProfScope pp("project", s);
    hipLaunchKernelGGL((k_project<T, CH, SYM, QUAD, KS, BATCH>), dim3(proj_blocks(gx, gy, pone.chunk), 1, n), dim3(64 * KS),
                       0, s, pdev, pone);
}

template <typename T, int CH, int SYM, bool QUAD, int KS>
hipError_t project_t(const OrbitArgs<T>* odev, const OrbitArgs<T>& oone,
                     const ProjArgs<T>* pdev, const ProjArgs<T>& pone, int n, long pixels, int gx,
                     int gy, hipStream_t s, bool orbit = true) {
    if (odev)
        project_launch<T, CH, SYM, QUAD, true, KS>(odev, oone, pdev, pone, n, pixels, gx, gy, s,
                                                   orbit);
    else
        project_launch<T, CH, SYM, QUAD, false, KS>(odev, oone, pdev, pone, n, pixels, gx, gy, s,
                                                    orbit);
    return hipGetLastError();
}

// A standard [V][D][CH] sinogram as quad records [Vb][D][4][CH] (view v + k Vb is
// rotation k of base view v), the layout the staged transpose reads.
template <typename T, int CH>
__global__ __launch_bounds__(256) void k_quad_records(const T* __restrict__ sino, int Vb, int D,
                                                      T* __restrict__ quad) {
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;  // (vb, b, k)
    if (r >= (long)Vb * D * 4) return;
    const int k = (int)(r & 3);
    const long vb_b = r >> 2;
    const int vb = (int)(vb_b / D), b = (int)(vb_b % D);
    const T* src = sino + ((size_t)(vb + k * Vb) * D + b) * CH;
#pragma unroll
    for (int c = 0; c < CH; ++c) quad[r * CH + c] = src[c];
}

// R^T of one or two channels on a quarter-turn symmetric plan: the sinogram is
// reordered into quad records in the plan's scratch and gathered by the staged
// transpose with `waves` waves per workgroup.
template <typename T, int CH, int VS>
hipError_t bp_quad_plain(const BpArgs<T>& one, T* quad, hipStream_t s) {
    const long recs = (long)one.Vb * one.D * 4;
    hipLaunchKernelGGL((k_quad_records<T, CH>), dim3((unsigned)((recs + 255) / 256)), dim3(256),
                       0, s, one.sino, one.Vb, one.D, quad);
    BpArgs<T> a = one;
    a.sino = quad;
    hipLaunchKernelGGL((k_backproject<T, CH, 4, true, EPI_NONE, VS, false>), dim3(a.gx, a.gy),
                       dim3(64 * VS), 0, s, nullptr, a, 1u);
    return hipGetLastError();
}

template <typename T, int CH>
hipError_t bp_quad_plain_w(int waves, const BpArgs<T>& one, T* quad, hipStream_t s) {
    switch (waves) {
        case 2: return bp_quad_plain<T, CH, 2>(one, quad, s);
        case 4: return bp_quad_plain<T, CH, 4>(one, quad, s);
        case 8: return bp_quad_plain<T, CH, 8>(one, quad, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int CH, int SYM>
hipError_t bp_plain(const BpArgs<T>& one, hipStream_t s) {
    hipLaunchKernelGGL((k_backproject<T, CH, SYM, false, EPI_NONE, kViewSplit, false>),
                       dim3(one.gx, one.gy), dim3(64 * kViewSplit), 0, s, nullptr, one, 1u);
    return hipGetLastError();
}

// The ADMM's own sinograms are two-channel quad records.
template <typename T, int SYM, bool BATCH, int VS, typename A>
hipError_t bp_admm_t(int epi, const BpArgs<T>* dev, const BpArgs<T>& one, int n, int gx, int gy,
                     hipStream_t s) {
    // One slice: a (gx, gy) grid.  A batch: each XCD an equal contiguous share of the
    // slices' blocks; the kernel takes the block grid from `one`, the same for every
    // slice of the group.
    if (gx != one.gx || gy != one.gy) return hipErrorInvalidValue;
    const dim3 g = BATCH ? dim3(xcd_slice_blocks((unsigned)(gx * gy), (unsigned)n)) : dim3(gx, gy);
    const dim3 blk(64 * VS);
    const unsigned nsl = (unsigned)n;
    switch (epi) {
        case EPI_Q:
            hipLaunchKernelGGL((k_backproject<T, 2, SYM, true, EPI_Q, VS, BATCH, A>), g, blk, 0, s,
                               dev, one, nsl);
            break;
        case EPI_DUAL:
            hipLaunchKernelGGL((k_backproject<T, 2, SYM, true, EPI_DUAL, VS, BATCH, A>), g, blk, 0,
                               s, dev, one, nsl);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int SYM, bool BATCH, typename A>
hipError_t bp_admm_w(int waves, int epi, const BpArgs<T>* dev, const BpArgs<T>& one, int n, int gx,
                     int gy, hipStream_t s) {
    switch (waves) {
        case 2: return bp_admm_t<T, SYM, BATCH, 2, A>(epi, dev, one, n, gx, gy, s);
        case 4: return bp_admm_t<T, SYM, BATCH, 4, A>(epi, dev, one, n, gx, gy, s);
        case 8: return bp_admm_t<T, SYM, BATCH, 8, A>(epi, dev, one, n, gx, gy, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int SYM, typename A>
hipError_t bp_admm(int waves, int epi, const BpArgs<T>* dev, const BpArgs<T>& one, int n, int gx,
                   int gy, hipStream_t s) {
    return dev ? bp_admm_w<T, SYM, true, A>(waves, epi, dev, one, n, gx, gy, s)
               : bp_admm_w<T, SYM, false, A>(waves, epi, dev, one, n, gx, gy, s);
}

template <typename T, int SYM>
hipError_t project_pair_w(int waves, const OrbitArgs<T>* odev, const OrbitArgs<T>& oone,
                          const ProjArgs<T>* pdev, const ProjArgs<T>& pone, int n, long pixels,
                          int gx, int gy, hipStream_t s, bool orbit) {
    switch (waves) {
        case 2: return project_t<T, 2, SYM, true, 2>(odev, oone, pdev, pone, n, pixels, gx, gy, s, orbit);
        case 4: return project_t<T, 2, SYM, true, 4>(odev, oone, pdev, pone, n, pixels, gx, gy, s, orbit);
        case 8: return project_t<T, 2, SYM, true, 8>(odev, oone, pdev, pone, n, pixels, gx, gy, s, orbit);
    }
    return hipErrorInvalidValue;
}

const char* bp_name(int epi) {
    static const char* names[4] = {"backproject", "backproject_rhs", "backproject_q",
                                   "backproject_dual"};
    return names[epi & 3];
}

}  // namespace

template <typename T>
void fill_bp_plan(const dect_plan* p, BpArgs<T>& a) {
    a.rays = static_cast<const RayParam<T>*>(p->rays);
    a.brays = static_cast<const BpRay<T>*>(p->bp_rays);
    a.views = static_cast<const ViewParam<T>*>(p->views);
    a.nx = p->nx;
    a.ny = p->ny;
    a.V = p->V;
    a.Vb = p->Vb;
    a.D = p->D;
    a.margin = p->margin;
    const int dx = p->sym == 4 ? p->nx / 2 : p->nx, dy = p->sym == 4 ? p->ny / 2 : p->ny;
    a.gx = (dx + 7) / 8;
    a.gy = (dy + 7) / 8;
}

// R into the standard sinogram layout, with the two orbit images of the image in O and
// OT (each N * ch * sym values of T).
template <typename T>
hipError_t launch_project_with(const dect_plan* p, const void* img, void* sino, int ch, void* O_,
                               void* OT_, hipStream_t s) {
    T* O = static_cast<T*>(O_);
    T* OT = static_cast<T*>(OT_);
    OrbitArgs<T> o{static_cast<const T*>(img), O, OT, p->nx, p->ny};
    ProjArgs<T> q{static_cast<const RayParam<T>*>(p->rays), O, OT, static_cast<T*>(sino), p->nx,
                  p->ny, p->Vb, p->D, p->pj_views, p->pj_chunk};
    const int gx = proj_grid_x(p->D, p->pj_views), gy = proj_grid_y(p->Vb, p->pj_views);
    if (p->sym == 4) {
        switch (ch) {
            case 1: return project_t<T, 1, 4, false, kLineSplit>(nullptr, o, nullptr, q, 1, p->N, gx, gy, s);
            case 2: return project_t<T, 2, 4, false, kLineSplit>(nullptr, o, nullptr, q, 1, p->N, gx, gy, s);
            case 4: return project_t<T, 4, 4, false, kLineSplit>(nullptr, o, nullptr, q, 1, p->N, gx, gy, s);
        }
    } else {
        switch (ch) {
            case 1: return project_t<T, 1, 1, false, kLineSplit>(nullptr, o, nullptr, q, 1, p->N, gx, gy, s);
            case 2: return project_t<T, 2, 1, false, kLineSplit>(nullptr, o, nullptr, q, 1, p->N, gx, gy, s);
            case 4: return project_t<T, 4, 1, false, kLineSplit>(nullptr, o, nullptr, q, 1, p->N, gx, gy, s);
        }
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_project(const dect_plan* p, const void* img, void* sino, int ch, hipStream_t s) {
    return launch_project_with<T>(p, img, sino, ch, p->scratch_O, p->scratch_OT, s);
}

template <typename T>
hipError_t launch_project_pair(int sym, int waves, const OrbitArgs<T>* odev,
                               const OrbitArgs<T>& oone, const ProjArgs<T>* pdev,
                               const ProjArgs<T>& pone, int n, long pixels, int gx, int gy,
                               hipStream_t s, bool orbit) {
    return sym == 4
               ? project_pair_w<T, 4>(waves, odev, oone, pdev, pone, n, pixels, gx, gy, s, orbit)
               : project_pair_w<T, 1>(waves, odev, oone, pdev, pone, n, pixels, gx, gy, s, orbit);
}

template <typename T>
hipError_t launch_rhs_orbit(const BpArgs<T>* dev, const BpArgs<T>& one, const OrbitArgs<T>* odev,
                            const OrbitArgs<T>& oone, int nsl, hipStream_t s) {
    if (!rhs_orbit_fits(4, one.nx, one.ny) || oone.nx != one.nx || oone.ny != one.ny ||
        (dev == nullptr) != (odev == nullptr) || nsl < 1 || (dev == nullptr && nsl != 1))
        return hipErrorInvalidValue;
    const unsigned h = (unsigned)one.nx / 16;
    const dim3 g(h * h, 1, (unsigned)nsl);
    if (dev)
        hipLaunchKernelGGL((k_rhs_orbit<T, true>), g, dim3(256), 0, s, dev, one, odev, oone);
    else
        hipLaunchKernelGGL((k_rhs_orbit<T, false>), g, dim3(256), 0, s, nullptr, one, nullptr,
                           oone);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_backproject(const dect_plan* p, int ch, const BpArgs<T>& a0, hipStream_t s) {
    BpArgs<T> a = a0;
    fill_bp_plan<T>(p, a);
    ProfScope ps(bp_name(EPI_NONE), s);
    if (p->sym == 4) {
        T* quad = static_cast<T*>(p->scratch_sq);
        switch (ch) {
            case 1: return bp_quad_plain_w<T, 1>(p->bp_waves, a, quad, s);
            case 2: return bp_quad_plain_w<T, 2>(p->bp_waves, a, quad, s);
            case 4: return bp_plain<T, 4, 4>(a, s);
        }
    } else {
        switch (ch) {
            case 1: return bp_plain<T, 1, 1>(a, s);
            case 2: return bp_plain<T, 2, 1>(a, s);
            case 4: return bp_plain<T, 4, 1>(a, s);
        }
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_backproject_admm(int sym, int waves, int epi, const BpArgs<T>* dev,
                                   const BpArgs<T>& one, int n, int gx, int gy, hipStream_t s,
                                   bool sums64) {
    ProfScope ps(bp_name(epi), s);
    if (sums64)  // an FP64 plan sums in double anyway
        return sym == 4 ? bp_admm<T, 4, double>(waves, epi, dev, one, n, gx, gy, s)
                        : bp_admm<T, 1, double>(waves, epi, dev, one, n, gx, gy, s);
    return sym == 4 ? bp_admm<T, 4, T>(waves, epi, dev, one, n, gx, gy, s)
                    : bp_admm<T, 1, T>(waves, epi, dev, one, n, gx, gy, s);
}

#define DECT_INST(T)                                                                          \
    template void fill_bp_plan<T>(const dect_plan*, BpArgs<T>&);                              \
    template hipError_t launch_project<T>(const dect_plan*, const void*, void*, int, hipStream_t); \
    template hipError_t launch_project_pair<T>(int, int, const OrbitArgs<T>*, const OrbitArgs<T>&, \
                                               const ProjArgs<T>*, const ProjArgs<T>&, int, long, \
                                               int, int, hipStream_t, bool);                      \
    template hipError_t launch_rhs_orbit<T>(const BpArgs<T>*, const BpArgs<T>&,                  \
                                            const OrbitArgs<T>*, const OrbitArgs<T>&, int,       \
                                            hipStream_t);                                        \
    template hipError_t launch_backproject<T>(const dect_plan*, int, const BpArgs<T>&, hipStream_t); \
    template hipError_t launch_backproject_admm<T>(int, int, int, const BpArgs<T>*,              \
                                                   const BpArgs<T>&, int, int, int, hipStream_t, \
                                                   bool);
DECT_INST(float)
DECT_INST(double)
#undef DECT_INST

}  // namespace dect

// ------------------------------------------------------------------------------
// R without any allocation: the orbit images live in a static device array.
//
// `scratch` is a file-scope device array of kNoAllocScratchBytes.  Each device the
// library runs on holds its own copy until the process ends.  In host code its
// name is only a stand-in for the device symbol, so the device address of each
// device's copy is looked up once (hipGetSymbolAddress, with that device current)
// and kept; kernels receive that address, never the name.
namespace dect {
namespace {

constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `device`'s copy of scratch (looked up on first use).
dect_status scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(DECT_E_DEVICE, "device %d is beyond the %d the library tracks", device,
                    kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        DECT_HIP(hipGetDevice(&cur));
        if (cur != device) DECT_HIP(hipSetDevice(device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            return fail(DECT_E_DEVICE, "no address for the static scratch on device %d: %s",
                        device, hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return DECT_OK;
}

}  // namespace
}  // namespace dect

extern "C" dect_status dect_project_noalloc(const dect_plan* p, const void* img, void* sino,
                                            int ch, void* stream) {
    using namespace dect;
    if (!p || !img || !sino) return fail(DECT_E_ARG, "null argument");
    if (ch != 1 && ch != 2 && ch != 4) return fail(DECT_E_ARG, "ch must be 1, 2 or 4 (got %d)", ch);
    // The orbit image and its transpose, the second at the next 256-byte boundary.
    const size_t image = (size_t)p->N * (size_t)ch * (size_t)p->sym * p->elem;
    const size_t second = (image + 255) / 256 * 256;
    if (second + image > kNoAllocScratchBytes)
        return fail(DECT_E_CAPACITY,
                    "the two orbit images need %zu bytes; the static scratch holds %zu "
                    "(%dx%d, %d channels, symmetry %d, %zu-byte values)",
                    second + image, kNoAllocScratchBytes, p->nx, p->ny, ch, p->sym, p->elem);
    void* base = nullptr;
    const dect_status st = scratch_address(p->device, &base);
    if (st != DECT_OK) return st;
    // Both orbit images are written in full before the projector reads them, so the
    // previous call's contents need no clearing.
    void* O = base;
    void* OT = static_cast<char*>(base) + second;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = p->dtype == DECT_F32
                             ? launch_project_with<float>(p, img, sino, ch, O, OT, s)
                             : launch_project_with<double>(p, img, sino, ch, O, OT, s);
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}
