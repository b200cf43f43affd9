/*
 * Sanitizer driver for the oracle's C part (test infrastructure only).
 *
 * Built by the CPU test suite with AddressSanitizer and UndefinedBehaviorSanitizer
 * (gcc, host code only) together with dect_oracle.c, and run as its own process:
 * every entry point is called on small parallel-beam and fan-beam geometries,
 * including ragged and degenerate ones (2x2 image, one view, detector offsets,
 * rays that miss the image), so that any out-of-bounds access, use of freed
 * memory, leak or undefined arithmetic in the oracle stops the run.  It also
 * checks <R x, y> = <x, R^T y> on each geometry, which needs every pair of
 * weights the projector visits to be found again by the transpose.
 */
#include <stdio.h>

#include "dect_oracle.c"

static unsigned long long rng_state = 0x9e3779b97f4a7c15ULL;

/* splitmix64 (Steele, Lea and Flood), mapped to [-1, 1). */
static double urand(void) {
    unsigned long long z = (rng_state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int check_geometry(const char* name, orc_geom g) {
    const long N = (long)g.nx * g.ny, M = (long)g.n_views * g.n_det;
    double* x = malloc(sizeof(double) * N);
    double* xt = malloc(sizeof(double) * N);
    double* y = malloc(sizeof(double) * M);
    double* yt = malloc(sizeof(double) * M);
    for (long i = 0; i < N; ++i) x[i] = urand();
    for (long i = 0; i < M; ++i) y[i] = urand();
    orc_project(&g, x, yt);
    orc_backproject(&g, y, xt);
    double lhs = 0.0, rhs = 0.0, ny = 0.0, nyt = 0.0;
    for (long i = 0; i < M; ++i) {
        lhs += yt[i] * y[i];
        ny += y[i] * y[i];
        nyt += yt[i] * yt[i];
    }
    for (long i = 0; i < N; ++i) rhs += x[i] * xt[i];
    const double scale = sqrt(ny * nyt) + 1e-300;
    const double err = fabs(lhs - rhs) / scale;
    printf("%-16s %4dx%-4d %4d views x %4d bins  adjointness %.2e\n", name, g.nx, g.ny,
           g.n_views, g.n_det, err);
    free(x);
    free(xt);
    free(y);
    free(yt);
    return err <= 1e-12 ? 0 : 1;
}

static int check_decompositions(void) {
    /* Three energy bins per spectrum, ln of normalised weights. */
    const double lnw_h[3] = {log(0.2), log(0.5), log(0.3)};
    const double lnw_l[3] = {log(0.6), log(0.3), log(0.1)};
    const double fkn[3] = {1.20, 1.05, 0.95};
    const double fp[3] = {8.0, 1.0, 0.2};
    enum { n = 64 };
    double mh[n], ml[n], wh[n], wl[n], vc[n], vp[n], ac[n], ap[n], phi[n];
    double fh[n], fl[n], gh[2 * n], gl[2 * n];
    for (int i = 0; i < n; ++i) {
        ac[i] = 6.0 * (urand() + 1.0);
        ap[i] = 0.2 * (urand() + 1.0);
    }
    orc_forward(3, lnw_h, fkn, fp, 3, lnw_l, fkn, fp, n, ac, ap, fh, fl, gh, gl);
    for (int i = 0; i < n; ++i) {
        mh[i] = fh[i] + 0.01 * urand();
        ml[i] = fl[i] + 0.01 * urand();
        wh[i] = i % 7 == 0 ? 0.0 : 0.5 + 0.5 * urand();  /* starved rays: zero weight */
        wl[i] = i % 5 == 0 ? 0.0 : 0.5 + 0.5 * urand();
        vc[i] = ac[i] + 0.1 * urand();
        vp[i] = ap[i] + 0.01 * urand();
        ac[i] = 0.0;
        ap[i] = 0.0;
    }
    int bad = 0;
    orc_udm(3, lnw_h, fkn, fp, 3, lnw_l, fkn, fp, n, mh, ml, wh, wl, vc, vp, 1e-3, 1e-3, 20, 1e-3,
            ac, ap, phi, NULL, NULL);
    for (int i = 0; i < n; ++i) bad |= !isfinite(ac[i]) || !isfinite(ap[i]) || !isfinite(phi[i]);
    orc_udm(3, lnw_h, fkn, fp, 3, lnw_l, fkn, fp, n, mh, ml, wh, wl, NULL, NULL, 0.0, 0.0, 5,
            1e-3, ac, ap, NULL, NULL, NULL);
    /* Replayed decisions: every first step rejected, every second accepted. */
    unsigned char force[n];
    double tie[n];
    for (int i = 0; i < n; ++i) force[i] = 2;
    orc_udm(3, lnw_h, fkn, fp, 3, lnw_l, fkn, fp, n, mh, ml, wh, wl, vc, vp, 1e-3, 1e-3, 3, 1e-3,
            ac, ap, phi, force, tie);
    for (int i = 0; i < n; ++i) bad |= !(tie[i] >= 0.0) || !isfinite(ac[i]);
    orc_cdm(3, lnw_h, fkn, fp, 3, lnw_l, fkn, fp, n, mh, ml, wh, wl, 20, 1e-3, ac, ap, phi);
    for (int i = 0; i < n; ++i) bad |= !(ac[i] >= 0.0) || !(ap[i] >= 0.0) || !isfinite(phi[i]);
    printf("decompositions: %s\n", bad ? "non-finite or infeasible result" : "ok");
    return bad;
}

int main(void) {
    int bad = 0;
    const double pi = 3.14159265358979323846;
    /* kind, nx, ny, pixel, views, bins, det_cm, offset, src_iso, src_det, angle0, span */
    bad |= check_geometry("parallel", (orc_geom){0, 24, 24, 0.5, 30, 35, 0.5, 0.0, 0, 0, 0.0, pi});
    bad |= check_geometry("ragged_parallel",
                          (orc_geom){0, 13, 19, 0.5, 17, 90, 0.17, -0.25, 0, 0, 0.05, pi});
    bad |= check_geometry("two_by_two", (orc_geom){0, 2, 2, 1.0, 7, 5, 0.8, 0.0, 0, 0, 0.0, pi});
    bad |= check_geometry("ragged_fan",
                          (orc_geom){1, 17, 11, 0.4, 25, 41, 0.45, 0.3, 30.0, 52.0, 0.1, 2 * pi});
    bad |= check_geometry("single_view_fan",
                          (orc_geom){1, 8, 8, 1.0, 1, 97, 0.3, 0.0, 40.0, 70.0, 0.0, 2 * pi});
    /* A wide detector: the outer bins' rays miss the image entirely. */
    bad |= check_geometry("wide_fan",
                          (orc_geom){1, 16, 16, 0.5, 12, 64, 0.9, 0.0, 30.0, 50.0, 0.0, 2 * pi});
    bad |= check_decompositions();
    printf(bad ? "FAILED\n" : "OK\n");
    return bad;
}
