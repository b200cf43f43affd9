// Host check of the ray-driven projector's index arithmetic, with the kernel's own
// helpers (projidx.h): for every workgroup of a launch, every wave and lane, the ray
// a lane takes, its sample range, the wave's share of the lines, the line windows a
// wave stages and every tap a lane loads.  Checks that every load (staged or direct)
// lies inside its orbit image, that a tap read from a window is the tap staged in that
// slot, that the two tap weights are those of linear interpolation on the
// zero-extended line, that the samples next to a ray's range have no tap inside the
// image, that each valid ray's samples are split over the waves exactly once with none
// lost, and that the only exit before the workgroup barrier is taken by the whole
// workgroup.  Plain C++: built with g++ by the CPU test suite.
//
// usage: projector_bounds kind nx ny pixel V D det_cm offset src_iso src_det angle0
//        span sym precision(32|64)
#include <algorithm>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "projidx.h"

using namespace dect;

template <typename T>
static int check(const dect_geometry& g, int sym, int KS, int BV, int chunk, long& taps,
                 long& trips, long& staged_lines, long& fallbacks) {
    const bool check_weights = KS == 2 && BV == 1 && chunk == 1;
    const int Vb = g.n_views / sym, D = g.n_det, nx = g.nx, ny = g.ny;
    std::vector<T> phi0((size_t)Vb * D), slope((size_t)Vb * D);
    std::vector<char> xs((size_t)Vb * D);
    for (int v = 0; v < Vb; ++v)
        for (int b = 0; b < D; ++b) {
            const HostRay r = host_ray(g, v, b);
            phi0[(size_t)v * D + b] = (T)r.phi0;
            slope[(size_t)v * D + b] = (T)r.slope;
            xs[(size_t)v * D + b] = r.xstep;
        }
    const int gx = proj_grid_x(D, BV), gy = proj_grid_y(Vb, BV);
    const unsigned blocks = proj_blocks(gx, gy, chunk);
    std::vector<int> covered((size_t)Vb * D, 0);
    std::vector<int> expected((size_t)Vb * D, 0);
    std::vector<int> seen_tile((size_t)gx * gy, 0);
    const int BB = 64 / BV;
    int errors = 0;
    for (unsigned id = 0; id < blocks; ++id) {
        int bg, vg;
        proj_tile(id, gy, chunk, bg, vg);
        if (bg >= gx) continue;  // the whole workgroup leaves before any barrier
        if (vg < 0 || vg >= gy) {
            std::printf("workgroup %u: view group %d out of range\n", id, vg);
            return 1;
        }
        seen_tile[(size_t)vg * gx + bg]++;
        // Per lane: ray, validity and sample range; the union is wave-independent.
        int k0[64], k1[64], v_[64], b_[64], ns[64], nl[64];
        bool valid[64];
        int s0 = 1 << 30, s1 = -1;
        for (int lane = 0; lane < 64; ++lane) {
            const int v = vg * BV + lane % BV, b = bg * BB + lane / BV;
            valid[lane] = b < D && v < Vb;
            const size_t ri = (size_t)(v < Vb ? v : Vb - 1) * D + (b < D ? b : D - 1);
            v_[lane] = v;
            b_[lane] = b;
            ns[lane] = xs[ri] ? nx : ny;
            nl[lane] = xs[ri] ? ny : nx;
            proj_ray_range<T>(phi0[ri], slope[ri], ns[lane], nl[lane], k0[lane], k1[lane]);
            if (valid[lane]) {
                // The samples next to the range have no tap inside the image.
                for (int k : {k0[lane] - 2, k0[lane] - 1, k1[lane] + 1, k1[lane] + 2}) {
                    if (k < 0 || k >= ns[lane] || (k >= k0[lane] && k <= k1[lane])) continue;
                    T w0, w1;
                    proj_taps<T>(phi0[ri], slope[ri], (T)k, nl[lane], w0, w1);
                    if ((w0 != T(0) || w1 != T(0)) && errors++ < 10)
                        std::printf("ray (%d,%d): sample %d outside [%d,%d] has weights %g %g\n",
                                    v, b, k, k0[lane], k1[lane], (double)w0, (double)w1);
                }
                expected[(size_t)v * D + b] = k1[lane] >= k0[lane] ? k1[lane] - k0[lane] + 1 : 0;
                if (k0[lane] <= k1[lane]) {
                    s0 = std::min(s0, k0[lane]);
                    s1 = std::max(s1, k1[lane]);
                }
            }
        }
        if (s1 < s0) s0 = 0, s1 = -1;
        // Staged windows: a wave whose valid rays all step along the same axis.
        bool any_valid = false, all_x = true, all_y = true;
        int wl = 0, wn = 0;
        for (int lane = 0; lane < 64; ++lane)
            if (valid[lane]) {
                const size_t ri = (size_t)v_[lane] * D + b_[lane];
                any_valid = true;
                all_x = all_x && xs[ri];
                all_y = all_y && !xs[ri];
                wl = nl[lane];
                wn = ns[lane];
            }
        const bool windowed = any_valid && (all_x || all_y);
        int wa = 0, wb = 0;
        {
            // Lanes 0 and 63 hold real rays even past the last bin (their ray index
            // is clamped), as in the kernel.
            auto ray_of = [&](int lane) {
                return (size_t)(v_[lane] < Vb ? v_[lane] : Vb - 1) * D +
                       (b_[lane] < D ? b_[lane] : D - 1);
            };
            const size_t r0 = ray_of(0), r63 = ray_of(63);
            proj_window_line<T>(phi0[r0], slope[r0], phi0[r63], slope[r63], wa, wb);
        }
        for (int wave = 0; wave < KS; ++wave) {
            int c0, c1;
            proj_wave_share(s0, s1, wave, KS, c0, c1);
            std::vector<int> slot(kProjWin);
            for (int k = c0; k <= c1; ++k) {
                int s = 0;
                if (windowed) {
                    // The staging loads of line k: tap clamp(s + lane) of that line.
                    if (k < 0 || k >= wn) {
                        if (errors++ < 10) std::printf("staged line %d outside [0,%d)\n", k, wn);
                        continue;
                    }
                    s = proj_window(wa, wb, k);
                    for (int lane = 0; lane < 64; ++lane)
                        slot[lane] = std::min(std::max(s + lane, 0), wl - 1);
                    ++staged_lines;
                }
                for (int lane = 0; lane < 64; ++lane) {
                    if (!valid[lane] || k < std::max(k0[lane], c0) || k > std::min(k1[lane], c1))
                        continue;
                    const size_t ri = (size_t)v_[lane] * D + b_[lane];
                    ++trips;
                    if (k >= ns[lane]) {
                        if (errors++ < 10)
                            std::printf("ray (%d,%d) sample %d outside [0,%d)\n", v_[lane],
                                        b_[lane], k, ns[lane]);
                        continue;
                    }
                    T w0, w1;
                    const int j = proj_taps<T>(phi0[ri], slope[ri], (T)k, nl[lane], w0, w1);
                    taps += 2;
                    if (j < 0 || j + 1 >= nl[lane]) {
                        if (errors++ < 10)
                            std::printf("ray (%d,%d) sample %d: taps %d, %d outside [0,%d)\n",
                                        v_[lane], b_[lane], k, j, j + 1, nl[lane]);
                        continue;
                    }
                    if (windowed) {
                        const int idx = j - s;
                        if ((unsigned)idx <= (unsigned)(kProjWin - 2)) {
                            if (slot[idx] != j || slot[idx + 1] != j + 1) {
                                if (errors++ < 10)
                                    std::printf("ray (%d,%d) sample %d: window slots %d, %d "
                                                "hold taps %d, %d, not %d, %d\n",
                                                v_[lane], b_[lane], k, idx, idx + 1, slot[idx],
                                                slot[idx + 1], j, j + 1);
                            }
                        } else {
                            ++fallbacks;
                        }
                    }
                    // The weights are those of linear interpolation on the zero-extended
                    // line, evaluated in double from the same position: taps floor(phi)
                    // and floor(phi) + 1 with 1 - alpha and alpha, zero outside the line,
                    // and no weight on a tap other than j, j + 1.  They do not depend on
                    // the launch shape, so they are checked for one of them.
                    if (!check_weights) continue;
                    const double ph = (double)std::fma(slope[ri], (T)k, phi0[ri]);
                    const double fl = std::floor(ph), al = ph - fl;
                    auto ref = [&](long t) {
                        if (t < 0 || t >= nl[lane]) return 0.0;
                        return t == (long)fl ? 1.0 - al : t == (long)fl + 1 ? al : 0.0;
                    };
                    const double tol = 8.0 * std::numeric_limits<T>::epsilon();
                    double lost = 0.0;
                    for (long t = (long)fl; t <= (long)fl + 1; ++t)
                        if (t != j && t != j + 1) lost += ref(t);
                    if (std::fabs((double)w0 - ref(j)) > tol ||
                        std::fabs((double)w1 - ref(j + 1)) > tol || lost > tol) {
                        if (errors++ < 10)
                            std::printf("ray (%d,%d) sample %d: phi %.17g taps %d,%d weights "
                                        "%.9g %.9g, expected %.9g %.9g\n",
                                        v_[lane], b_[lane], k, ph, j, j + 1, (double)w0,
                                        (double)w1, ref(j), ref(j + 1));
                    }
                }
            }
            for (int lane = 0; lane < 64; ++lane) {
                if (!valid[lane]) continue;
                const int a = std::max(k0[lane], c0), e = std::min(k1[lane], c1);
                if (e >= a) covered[(size_t)v_[lane] * D + b_[lane]] += e - a + 1;
            }
        }
    }
    for (size_t t = 0; t < seen_tile.size(); ++t)
        if (seen_tile[t] != 1) {
            if (errors++ < 10) std::printf("tile %zu run %d times\n", t, seen_tile[t]);
        }
    for (size_t r = 0; r < covered.size(); ++r)
        if (covered[r] != expected[r]) {
            if (errors++ < 10)
                std::printf("ray %zu: %d samples taken, %d in range\n", r, covered[r],
                            expected[r]);
        }
    return errors;
}

int main(int argc, char** argv) {
    if (argc != 15) {
        std::fprintf(stderr, "usage: %s kind nx ny pixel V D det_cm offset src_iso src_det "
                             "angle0 span sym precision\n", argv[0]);
        return 2;
    }
    dect_geometry g{};
    g.kind = std::atoi(argv[1]);
    g.nx = std::atoi(argv[2]);
    g.ny = std::atoi(argv[3]);
    g.pixel_cm = std::atof(argv[4]);
    g.n_views = std::atoi(argv[5]);
    g.n_det = std::atoi(argv[6]);
    g.det_cm = std::atof(argv[7]);
    g.det_offset = std::atof(argv[8]);
    g.src_iso_cm = std::atof(argv[9]);
    g.src_det_cm = std::atof(argv[10]);
    g.angle0 = std::atof(argv[11]);
    g.span = std::atof(argv[12]);
    const int sym = std::atoi(argv[13]), prec = std::atoi(argv[14]);
    int bad = 0;
    for (int KS : {2, 4, 8})
        for (int BV : {1, 2, 4, 8})
            for (int chunk : {1, 2, 4, 16}) {
                long taps = 0, trips = 0, staged = 0, fallbacks = 0;
                const int e = prec == 64
                                  ? check<double>(g, sym, KS, BV, chunk, taps, trips, staged, fallbacks)
                                  : check<float>(g, sym, KS, BV, chunk, taps, trips, staged, fallbacks);
                if (e || (BV == 2 && chunk == 1))
                    std::printf("KS=%d views=%d chunk=%d: %ld samples, %ld taps loaded, %ld "
                                "staged lines, %ld samples read outside their window, %d "
                                "errors\n", KS, BV, chunk, trips, taps, staged, fallbacks, e);
                bad |= e != 0;
            }
    std::printf(bad ? "FAILED\n" : "OK\n");
    return bad;
}
