/*
 * Plain FP64 CPU oracle for the splitting-based dual-energy CT ADMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the reconstruction library links,
 * includes or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code with the GPU path.
 *
 * It computes, slowly and in double precision:
 *   - the Joseph (linear-interpolation, ray-driven) projection R of an image,
 *     the discretisation of the line integrals in Eq. (2)-(3);
 *   - R^T as the literal transpose: the same per-ray weights scatter-added;
 *   - the polychromatic forward transform f_s(a) of Eq. (3) and its gradient;
 *   - the per-ray unconstrained decomposition (UDM) subproblem of Eq. (13),
 *     solved by Levenberg-Marquardt iterations (Sec. 3.3).
 * The ADMM loop itself (Eq. (9)-(13)) is written in numpy on top of these.
 *
 * Geometry: pixel (j, i) centre ((i-(nx-1)/2) d, (j-(ny-1)/2) d), row-major;
 * view angle t_v = angle0 + v*span/V; detector coordinate of bin b
 * u_b = (b - (D-1)/2 + offset) * det_cm.  Parallel: the ray is the line
 * p.(cos t, sin t) = u_b with direction (-sin t, cos t).  Fan (flat
 * detector): source R_so (cos t, sin t), bin at -(R_sd-R_so)(cos t, sin t)
 * + u_b (-sin t, cos t).
 *
 * Joseph's rule: a ray whose direction satisfies |d_x| >= |d_y| is sampled on
 * every pixel column x_i; the sample is the linear interpolation between the
 * two pixel rows bracketing the crossing point (rows outside the image are
 * zero), and each sample is weighted by the step length d*sqrt(1+(d_y/d_x)^2).
 * Otherwise rows and columns swap roles.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int kind; /* 0 = parallel, 1 = fan (flat detector) */
    int nx, ny;
    double pixel;
    int n_views, n_det;
    double det_cm, det_offset, src_iso, src_det, angle0, span;
} orc_geom;

/* A point on ray (v, b) and its (unnormalised) direction. */
static void ray_line(const orc_geom* g, int v, int b, double* ox, double* oy, double* dx,
                     double* dy) {
    double t = g->angle0 + (double)v * g->span / (double)g->n_views;
    double c = cos(t), s = sin(t);
    double u = ((double)b - 0.5 * (double)(g->n_det - 1) + g->det_offset) * g->det_cm;
    if (g->kind == 0) {
        *ox = u * c;
        *oy = u * s;
        *dx = -s;
        *dy = c;
    } else {
        double sx = g->src_iso * c, sy = g->src_iso * s;
        double qx = -(g->src_det - g->src_iso) * c - u * s;
        double qy = -(g->src_det - g->src_iso) * s + u * c;
        *ox = sx;
        *oy = sy;
        *dx = qx - sx;
        *dy = qy - sy;
    }
}

/* All (pixel index, weight) pairs of ray (v, b).  Returns their number
 * (at most 2*max(nx, ny)); weights may be zero. */
static int joseph_ray(const orc_geom* g, int v, int b, long* idx, double* w) {
    double ox, oy, dx, dy;
    ray_line(g, v, b, &ox, &oy, &dx, &dy);
    const double d = g->pixel;
    int n = 0;
    if (fabs(dx) >= fabs(dy)) {
        double slope = dy / dx;
        double step = d * sqrt(1.0 + slope * slope);
        for (int i = 0; i < g->nx; ++i) {
            double x = ((double)i - 0.5 * (double)(g->nx - 1)) * d;
            double y = oy + (x - ox) * slope;
            double phi = y / d + 0.5 * (double)(g->ny - 1);
            double j0 = floor(phi);
            double a = phi - j0;
            long j = (long)j0;
            if (j >= 0 && j < g->ny) {
                idx[n] = j * g->nx + i;
                w[n++] = (1.0 - a) * step;
            }
            if (j + 1 >= 0 && j + 1 < g->ny) {
                idx[n] = (j + 1) * g->nx + i;
                w[n++] = a * step;
            }
        }
    } else {
        double slope = dx / dy;
        double step = d * sqrt(1.0 + slope * slope);
        for (int j = 0; j < g->ny; ++j) {
            double y = ((double)j - 0.5 * (double)(g->ny - 1)) * d;
            double x = ox + (y - oy) * slope;
            double psi = x / d + 0.5 * (double)(g->nx - 1);
            double i0 = floor(psi);
            double a = psi - i0;
            long i = (long)i0;
            if (i >= 0 && i < g->nx) {
                idx[n] = (long)j * g->nx + i;
                w[n++] = (1.0 - a) * step;
            }
            if (i + 1 >= 0 && i + 1 < g->nx) {
                idx[n] = (long)j * g->nx + i + 1;
                w[n++] = a * step;
            }
        }
    }
    return n;
}

static int max_pairs(const orc_geom* g) { return 2 * (g->nx > g->ny ? g->nx : g->ny) + 4; }

/* sino[v*D + b] = sum over the ray's pairs of w * img[idx]. */
void orc_project(const orc_geom* g, const double* img, double* sino) {
    const int V = g->n_views, D = g->n_det;
#pragma omp parallel
    {
        long* idx = (long*)malloc(sizeof(long) * max_pairs(g));
        double* w = (double*)malloc(sizeof(double) * max_pairs(g));
#pragma omp for schedule(static)
        for (long r = 0; r < (long)V * D; ++r) {
            int n = joseph_ray(g, (int)(r / D), (int)(r % D), idx, w);
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += w[k] * img[idx[k]];
            sino[r] = acc;
        }
        free(idx);
        free(w);
    }
}

/* img = R^T sino: every ray scatter-adds w * sino into its pixels.  Views are
 * split into a fixed number of chunks, each with its own buffer, and the
 * buffers are summed in chunk order, so the result does not depend on the
 * thread count. */
#define ORC_CHUNKS 16
void orc_backproject(const orc_geom* g, const double* sino, double* img) {
    const int V = g->n_views, D = g->n_det;
    const long N = (long)g->nx * g->ny;
    double* part = (double*)calloc((size_t)ORC_CHUNKS * N, sizeof(double));
#pragma omp parallel
    {
        long* idx = (long*)malloc(sizeof(long) * max_pairs(g));
        double* w = (double*)malloc(sizeof(double) * max_pairs(g));
#pragma omp for schedule(static)
        for (int c = 0; c < ORC_CHUNKS; ++c) {
            double* out = part + (long)c * N;
            int v0 = (int)((long)V * c / ORC_CHUNKS), v1 = (int)((long)V * (c + 1) / ORC_CHUNKS);
            for (int v = v0; v < v1; ++v)
                for (int b = 0; b < D; ++b) {
                    double y = sino[(long)v * D + b];
                    int n = joseph_ray(g, v, b, idx, w);
                    for (int k = 0; k < n; ++k) out[idx[k]] += w[k] * y;
                }
        }
        free(idx);
        free(w);
    }
    for (long p = 0; p < N; ++p) {
        double acc = 0.0;
        for (int c = 0; c < ORC_CHUNKS; ++c) acc += part[(long)c * N + p];
        img[p] = acc;
    }
    free(part);
}

/* ---------------------------------------------------------------------------
 * Forward transform of Eq. (3) for one spectrum, normalised weights om[k]:
 *   f(a) = -ln sum_k om[k] exp(-fkn[k] a_c - fp[k] a_p)
 * evaluated as a log-sum-exp with the largest exponent factored out, and its
 * gradient (sum_k q_k fkn[k], sum_k q_k fp[k]), q_k the normalised terms.
 * ------------------------------------------------------------------------- */
typedef struct {
    int n;
    const double* lnw; /* ln of the normalised spectrum, nonzero bins only */
    const double* fkn;
    const double* fp;
} orc_spec;

static double spec_f(const orc_spec* s, double ac, double ap, double* gc, double* gp) {
    double m = -INFINITY;
    for (int k = 0; k < s->n; ++k) {
        double e = s->lnw[k] - s->fkn[k] * ac - s->fp[k] * ap;
        if (e > m) m = e;
    }
    double z = 0.0, sc = 0.0, sp = 0.0;
    for (int k = 0; k < s->n; ++k) {
        double q = exp(s->lnw[k] - s->fkn[k] * ac - s->fp[k] * ap - m);
        z += q;
        sc += q * s->fkn[k];
        sp += q * s->fp[k];
    }
    if (gc) *gc = sc / z;
    if (gp) *gp = sp / z;
    return -(m + log(z));
}

/* f_h, f_l and gradients for n rays (a_c, a_p). */
void orc_forward(int nh, const double* lnw_h, const double* fkn_h, const double* fp_h, int nl,
                 const double* lnw_l, const double* fkn_l, const double* fp_l, long n,
                 const double* ac, const double* ap, double* fh, double* fl, double* gh,
                 double* gl) {
    orc_spec sh = {nh, lnw_h, fkn_h, fp_h}, sl = {nl, lnw_l, fkn_l, fp_l};
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        fh[i] = spec_f(&sh, ac[i], ap[i], &gh[2 * i], &gh[2 * i + 1]);
        fl[i] = spec_f(&sl, ac[i], ap[i], &gl[2 * i], &gl[2 * i + 1]);
    }
}

/* ---------------------------------------------------------------------------
 * UDM, Eq. (13), one ray:
 *   Phi(a) = 1/2 sum_s w_s (f_s(a) - m_s)^2 + 1/2 sum_b rho_b (a_b - v_b)^2
 * with v = R x - u^a.  Levenberg-Marquardt with Gauss-Newton curvature
 *   H = sum_s w_s g_s g_s^T + diag(rho),  step  -(H + mu diag(H))^{-1} grad,
 * accepted when it lowers Phi (then mu /= 10), else rejected (mu *= 10).
 * A step whose damped determinant is not positive and finite is skipped.
 * ------------------------------------------------------------------------- */
typedef struct {
    double fh, fl, ghc, ghp, glc, glp, phi;
} orc_eval;

static void udm_eval(const orc_spec* sh, const orc_spec* sl, double mh, double ml, double wh,
                     double wl, double vc, double vp, double rc, double rp, double ac, double ap,
                     orc_eval* e) {
    e->fh = spec_f(sh, ac, ap, &e->ghc, &e->ghp);
    e->fl = spec_f(sl, ac, ap, &e->glc, &e->glp);
    double rh = e->fh - mh, rl = e->fl - ml;
    e->phi = 0.5 * (wh * rh * rh + wl * rl * rl) +
             0.5 * (rc * (ac - vc) * (ac - vc) + rp * (ap - vp) * (ap - vp));
}

/* Largest magnitude of the exponents ln omega_k - f_KN[k] a_c - f_p[k] a_p of one
 * spectrum's log-sum-exp at (a_c, a_p), bounded term by term: the rounding error of
 * f_s is a few units of it (f_s = -(M + ln Z) can be a small difference of such terms,
 * e.g. near a = 0). */
static double lse_scale(const orc_spec* s, double ac, double ap) {
    double w = 0.0, k = 0.0, p = 0.0;
    for (int i = 0; i < s->n; ++i) {
        if (fabs(s->lnw[i]) > w) w = fabs(s->lnw[i]);
        if (s->fkn[i] > k) k = s->fkn[i];
        if (s->fp[i] > p) p = s->fp[i];
    }
    return w + k * fabs(ac) + p * fabs(ap);
}

/* First-order bound, in units of the rounding unit, of the error of Phi when f_s carries
 * an absolute error of the order of its log-sum-exp's exponents and the residuals
 * f_s - m_s and a_b - v_b are formed from values each carrying a relative rounding error:
 * sum_s w_s |r_s| (|f_s| + |m_s| + lse_s) + sum_b rho_b |d_b| (|a_b| + |v_b|). */
static double phi_scale(const orc_spec* sh, const orc_spec* sl, const orc_eval* e, double mh,
                        double ml, double wh, double wl, double vc, double vp, double rc,
                        double rp, double ac, double ap) {
    return wh * fabs(e->fh - mh) * (fabs(e->fh) + fabs(mh) + lse_scale(sh, ac, ap)) +
           wl * fabs(e->fl - ml) * (fabs(e->fl) + fabs(ml) + lse_scale(sl, ac, ap)) +
           rc * fabs(ac - vc) * (fabs(ac) + fabs(vc)) + rp * fabs(ap - vp) * (fabs(ap) + fabs(vp));
}

/* Returns the number of single-spectrum f evaluations made per ray.
 *
 * force (NULL: none) replays accept decisions taken elsewhere: bit k of force[i] is the
 * decision of LM iteration k (k < 8) on ray i, 1 = the trial point was accepted.  The
 * iteration then follows that decision instead of its own comparison; where the two
 * differ, tie_out[i] (if given) receives the largest |Phi(trial) - Phi(current)| over
 * the single-precision rounding scale of the two values (2^-23 times phi_scale at both
 * points), so a caller can check that every replayed decision was a near-tie; a
 * replayed acceptance of a step this iteration cannot form (damped determinant not
 * positive and finite) gives +inf.  Without disagreements tie_out[i] = 0.  The scale
 * is phi_scale: the first-order rounding bound of Phi at single precision, including
 * the log-sum-exp's own cancellation. */
int orc_udm(int nh, const double* lnw_h, const double* fkn_h, const double* fp_h, int nl,
            const double* lnw_l, const double* fkn_l, const double* fp_l, long n,
            const double* mh, const double* ml, const double* wh, const double* wl,
            const double* vc, const double* vp, double rho_c, double rho_p, int iters,
            double mu0, double* ac, double* ap, double* phi_out, const unsigned char* force,
            double* tie_out) {
    orc_spec sh = {nh, lnw_h, fkn_h, fp_h}, sl = {nl, lnw_l, fkn_l, fp_l};
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double a_c = ac[i], a_p = ap[i];
        double v_c = vc ? vc[i] : 0.0, v_p = vp ? vp[i] : 0.0;
        orc_eval cur, tri;
        udm_eval(&sh, &sl, mh[i], ml[i], wh[i], wl[i], v_c, v_p, rho_c, rho_p, a_c, a_p, &cur);
        double mu = mu0;
        double tie = 0.0;
        for (int it = 0; it < iters; ++it) {
            const int forced = force && it < 8;
            const int want = forced ? (force[i] >> it) & 1 : 0;
            double rh = cur.fh - mh[i], rl = cur.fl - ml[i];
            double Gc = wh[i] * rh * cur.ghc + wl[i] * rl * cur.glc + rho_c * (a_c - v_c);
            double Gp = wh[i] * rh * cur.ghp + wl[i] * rl * cur.glp + rho_p * (a_p - v_p);
            double Hcc = wh[i] * cur.ghc * cur.ghc + wl[i] * cur.glc * cur.glc + rho_c;
            double Hpp = wh[i] * cur.ghp * cur.ghp + wl[i] * cur.glp * cur.glp + rho_p;
            double Hcp = wh[i] * cur.ghc * cur.ghp + wl[i] * cur.glc * cur.glp;
            double Dcc = (1.0 + mu) * Hcc, Dpp = (1.0 + mu) * Hpp;
            double det = Dcc * Dpp - Hcp * Hcp;
            if (!(det > 0.0) || !isfinite(det)) {
                if (want) tie = INFINITY;
                mu *= 10.0;
                continue;
            }
            double dc = -(Dpp * Gc - Hcp * Gp) / det;
            double dp = -(Dcc * Gp - Hcp * Gc) / det;
            double tc = a_c + dc, tp = a_p + dp;
            udm_eval(&sh, &sl, mh[i], ml[i], wh[i], wl[i], v_c, v_p, rho_c, rho_p, tc, tp, &tri);
            int take = tri.phi < cur.phi;
            if (forced && want != take) {
                const double scale =
                    ldexp(phi_scale(&sh, &sl, &cur, mh[i], ml[i], wh[i], wl[i], v_c, v_p, rho_c,
                                    rho_p, a_c, a_p) +
                              phi_scale(&sh, &sl, &tri, mh[i], ml[i], wh[i], wl[i], v_c, v_p,
                                        rho_c, rho_p, tc, tp),
                          -23);
                const double r = fabs(tri.phi - cur.phi) / (scale > 0.0 ? scale : 1e-300);
                if (r > tie) tie = r;
                take = want;
            }
            if (take) {
                a_c = tc;
                a_p = tp;
                cur = tri;
                mu /= 10.0;
            } else {
                mu *= 10.0;
            }
        }
        ac[i] = a_c;
        ap[i] = a_p;
        if (phi_out) phi_out[i] = cur.phi;
        if (tie_out) tie_out[i] = tie;
    }
    return 2 * (iters + 1);
}

/* Constrained decomposition (CDM, the projection-wise baseline of Sec. 2): per ray,
 * minimise 1/2 sum_s w_s (f_s(a) - m_s)^2 over a >= 0 by Levenberg-Marquardt with an
 * active set: a coordinate at zero whose gradient is positive is held at zero and
 * the damped Gauss-Newton step is taken in the other coordinate alone; trial points
 * are projected onto a >= 0 and accepted on a strict decrease, as in orc_udm.
 * a: start point, projected first. */
int orc_cdm(int nh, const double* lnw_h, const double* fkn_h, const double* fp_h, int nl,
            const double* lnw_l, const double* fkn_l, const double* fp_l, long n,
            const double* mh, const double* ml, const double* wh, const double* wl, int iters,
            double mu0, double* ac, double* ap, double* phi_out) {
    orc_spec sh = {nh, lnw_h, fkn_h, fp_h}, sl = {nl, lnw_l, fkn_l, fp_l};
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double a_c = fmax(ac[i], 0.0), a_p = fmax(ap[i], 0.0);
        orc_eval cur, tri;
        udm_eval(&sh, &sl, mh[i], ml[i], wh[i], wl[i], 0.0, 0.0, 0.0, 0.0, a_c, a_p, &cur);
        double mu = mu0;
        for (int it = 0; it < iters; ++it) {
            double rh = cur.fh - mh[i], rl = cur.fl - ml[i];
            double Gc = wh[i] * rh * cur.ghc + wl[i] * rl * cur.glc;
            double Gp = wh[i] * rh * cur.ghp + wl[i] * rl * cur.glp;
            double Hcc = wh[i] * cur.ghc * cur.ghc + wl[i] * cur.glc * cur.glc;
            double Hpp = wh[i] * cur.ghp * cur.ghp + wl[i] * cur.glp * cur.glp;
            double Hcp = wh[i] * cur.ghc * cur.ghp + wl[i] * cur.glc * cur.glp;
            double Dcc = (1.0 + mu) * Hcc, Dpp = (1.0 + mu) * Hpp;
            const int fix_c = a_c == 0.0 && Gc > 0.0, fix_p = a_p == 0.0 && Gp > 0.0;
            if (fix_c && fix_p) break;  /* stationary at the corner */
            double dc, dp;
            if (fix_c || fix_p) {
                const double D1 = fix_c ? Dpp : Dcc;
                if (!(D1 > 0.0) || !isfinite(D1)) {
                    mu *= 10.0;
                    continue;
                }
                dc = fix_c ? 0.0 : -Gc / D1;
                dp = fix_p ? 0.0 : -Gp / D1;
            } else {
                double det = Dcc * Dpp - Hcp * Hcp;
                if (!(det > 0.0) || !isfinite(det)) {
                    mu *= 10.0;
                    continue;
                }
                dc = -(Dpp * Gc - Hcp * Gp) / det;
                dp = -(Dcc * Gp - Hcp * Gc) / det;
            }
            double tc = fmax(a_c + dc, 0.0);
            double tp = fmax(a_p + dp, 0.0);
            udm_eval(&sh, &sl, mh[i], ml[i], wh[i], wl[i], 0.0, 0.0, 0.0, 0.0, tc, tp, &tri);
            if (tri.phi < cur.phi) {
                a_c = tc;
                a_p = tp;
                cur = tri;
                mu /= 10.0;
            } else {
                mu *= 10.0;
            }
        }
        ac[i] = a_c;
        ap[i] = a_p;
        if (phi_out) phi_out[i] = cur.phi;
    }
    return 2 * (iters + 1);
}

/* Thread count of the parallel loops above (the CPU baseline times 1 and all). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
