// Host check of the ray-driven projector's index arithmetic, with the kernel's own
// helpers (projidx.h): for every workgroup of a launch, every wave and lane, the ray
// a lane takes, its sample range, the wave's share of the lines, and every tap it
// would load.  Checks that every load lies inside its orbit image line (or is skipped
// by the kernel's bounds test), that each valid ray's samples are split over the waves
// exactly once with none lost, and that the only exit before the workgroup barrier is
// taken by the whole workgroup.  Plain C++: built with g++ by the CPU test suite.
//
// usage: projector_bounds kind nx ny pixel V D det_cm offset src_iso src_det angle0
//        span sym precision(32|64)
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "projidx.h"

using namespace dect;

template <typename T>
static int check(const dect_geometry& g, int sym, int KS, int BV, int chunk, long& taps,
                 long& trips) {
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
                expected[(size_t)v * D + b] = k1[lane] >= k0[lane] ? k1[lane] - k0[lane] + 1 : 0;
                if (k0[lane] <= k1[lane]) {
                    s0 = std::min(s0, k0[lane]);
                    s1 = std::max(s1, k1[lane]);
                }
            }
        }
        if (s1 < s0) s0 = 0, s1 = -1;
        for (int wave = 0; wave < KS; ++wave) {
            int c0, c1;
            proj_wave_share(s0, s1, wave, KS, c0, c1);
            for (int lane = 0; lane < 64; ++lane) {
                if (!valid[lane]) continue;
                const size_t ri = (size_t)v_[lane] * D + b_[lane];
                const int a = std::max(k0[lane], c0), e = std::min(k1[lane], c1);
                for (int k = a; k <= e; ++k) {
                    ++trips;
                    if (k < 0 || k >= ns[lane]) {
                        if (errors++ < 10)
                            std::printf("ray (%d,%d) sample %d outside [0,%d)\n", v_[lane],
                                        b_[lane], k, ns[lane]);
                        continue;
                    }
                    T alpha;
                    const int j = proj_tap<T>(phi0[ri], slope[ri], k, nl[lane], alpha);
                    // The kernel loads tap j only if 0 <= j < n_lines, and j + 1 likewise.
                    for (int t = j; t <= j + 1; ++t)
                        if ((unsigned)t < (unsigned)nl[lane]) ++taps;
                    if (j < -2 || j > nl[lane] + 1 || !(alpha >= T(0) && alpha <= T(1))) {
                        if (errors++ < 10)
                            std::printf("ray (%d,%d) sample %d: tap %d alpha %g\n", v_[lane],
                                        b_[lane], k, j, (double)alpha);
                    }
                }
                if (e >= a) covered[ri] += e - a + 1;
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
                long taps = 0, trips = 0;
                const int e = prec == 64 ? check<double>(g, sym, KS, BV, chunk, taps, trips)
                                         : check<float>(g, sym, KS, BV, chunk, taps, trips);
                if (e || (BV == 2 && chunk == 1))
                    std::printf("KS=%d views=%d chunk=%d: %ld samples, %ld taps inside, %d "
                                "errors\n", KS, BV, chunk, trips, taps, e);
                bad |= e != 0;
            }
    std::printf(bad ? "FAILED\n" : "OK\n");
    return bad;
}
