// Plan creation: geometry validation, Joseph ray tables, per-view footprint
// tables, spectral tables and the per-slice state layout.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "common.h"
#include "projidx.h"

namespace dect {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

dect_status fail(dect_status st, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

namespace {

template <typename T>
dect_status upload(const void* host, size_t bytes, void** dev) {
    DECT_HIP(hipMalloc(dev, bytes));
    DECT_HIP(hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice));
    return DECT_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T>
dect_status build_tables(dect_plan* p, const dect_spectra* spec) {
    const dect_geometry& g = p->geom;
    const int V = p->Vb, D = p->D;  // base views only; the others are their rotations
    std::vector<RayParam<T>> rays((size_t)V * D);
    std::vector<ViewParam<T>> views(V);
    const double d = g.pixel_cm;
    for (int v = 0; v < V; ++v) {
        int first_kind = -1, switches = 0, split = D;
        for (int b = 0; b < D; ++b) {
            HostRay r = host_ray(g, v, b);
            RayParam<T>& q = rays[(size_t)v * D + b];
            q.phi0 = (T)r.phi0;
            q.slope = (T)r.slope;
            q.step = (T)r.step;
            q.pad = (T)(r.xstep ? 0 : 1);
            int kind = r.xstep ? 0 : 1;
            if (b == 0) {
                first_kind = kind;
            } else if (kind != (int)rays[(size_t)v * D + b - 1].pad) {
                ++switches;
                split = b;
            }
        }
        if (switches > 1)
            return fail(DECT_E_SHAPE,
                        "view %d: x- and y-stepped rays interleave (%d switches); the fan is "
                        "wider than 90 degrees",
                        v, switches);
        ViewParam<T>& w = views[v];
        const int lo0 = 0, hi0 = split, lo1 = split, hi1 = D;
        if (first_kind == 0) {
            w.xb0 = lo0; w.xb1 = hi0; w.yb0 = lo1; w.yb1 = hi1;
        } else {
            w.yb0 = lo0; w.yb1 = hi0; w.xb0 = lo1; w.xb1 = hi1;
        }
        const double t = g.angle0 + (double)v * g.span / (double)g.n_views;
        const double c = std::cos(t), s = std::sin(t);
        const double boff = 0.5 * (D - 1) - g.det_offset;
        if (g.kind == DECT_PARALLEL) {
            w.ni = (T)(d * c / g.det_cm);
            w.nj = (T)(d * s / g.det_cm);
            w.d0 = (T)1;
            w.di = (T)0;
            w.dj = (T)0;
        } else {
            const double K = g.src_det_cm / g.det_cm;
            w.ni = (T)(-K * d * s);
            w.nj = (T)(K * d * c);
            w.d0 = (T)g.src_iso_cm;
            w.di = (T)(-d * c);
            w.dj = (T)(-d * s);
        }
        w.boff = (T)boff;
    }
    dect_status st = upload<T>(rays.data(), rays.size() * sizeof(rays[0]), &p->rays);
    if (st) return st;
    std::vector<BpRay<T>> brays(rays.size());
    for (size_t k = 0; k < rays.size(); ++k) {
        const RayParam<T>& r = rays[k];
        const bool xs = r.pad == T(0);
        brays[k] = BpRay<T>{r.phi0, xs ? r.slope : T(-1), xs ? T(-1) : r.slope, r.step};
    }
    st = upload<T>(brays.data(), brays.size() * sizeof(brays[0]), &p->bp_rays);
    if (st) return st;
    st = upload<T>(views.data(), views.size() * sizeof(views[0]), &p->views);
    if (st) return st;

    // Spectral tables: normalised spectra on their nonzero bins, base-2 units.
    const double log2e = 1.4426950408889634;
    std::vector<T> tab[2][3];
    const double* S[2] = {spec->s_high, spec->s_low};
    for (int h = 0; h < 2; ++h) {
        double tot = 0.0;
        for (int k = 0; k < spec->n_bins; ++k) tot += S[h][k];
        double mkn = 0.0, mp = 0.0;
        for (int k = 0; k < spec->n_bins; ++k) {
            if (!(S[h][k] > 0.0)) continue;
            const double om = S[h][k] / tot;
            tab[h][0].push_back((T)std::log2(om));
            tab[h][1].push_back((T)(spec->f_kn[k] * log2e));
            tab[h][2].push_back((T)(spec->f_p[k] * log2e));
            p->kc_max = std::fmax(p->kc_max, std::fabs(spec->f_kn[k] * log2e));
            p->kp_max = std::fmax(p->kp_max, std::fabs(spec->f_p[k] * log2e));
            mkn += om * spec->f_kn[k];
            mp += om * spec->f_p[k];
        }
        p->mean_f[h][0] = mkn;
        p->mean_f[h][1] = mp;
    }
    p->kh = (int)tab[0][0].size();
    p->kl = (int)tab[1][0].size();
    p->kmax = p->kh > p->kl ? p->kh : p->kl;
    std::vector<T> packed((size_t)6 * p->kmax, (T)0);
    for (int h = 0; h < 2; ++h)
        for (int q = 0; q < 3; ++q)
            for (size_t k = 0; k < tab[h][q].size(); ++k)
                packed[(size_t)(3 * h + q) * p->kmax + k] = tab[h][q][k];
    st = upload<T>(packed.data(), packed.size() * sizeof(T), &p->spec);
    if (st) return st;
    {
        // The joint table: bins where both spectra are nonzero, then high only, then low
        // only, each in energy order.
        double tot[2] = {0.0, 0.0};
        for (int h = 0; h < 2; ++h)
            for (int k = 0; k < spec->n_bins; ++k) tot[h] += S[h][k];
        std::vector<int> order[3];
        for (int k = 0; k < spec->n_bins; ++k) {
            const bool on_h = S[0][k] > 0.0, on_l = S[1][k] > 0.0;
            if (on_h && on_l) order[0].push_back(k);
            else if (on_h) order[1].push_back(k);
            else if (on_l) order[2].push_back(k);
        }
        p->jb = (int)order[0].size();
        p->jh = (int)order[1].size();
        p->jl = (int)order[2].size();
        const int nj = p->jb + p->jh + p->jl;
        std::vector<T> joint((size_t)8 * (nj > 0 ? nj : 1), (T)0);
        double wmin = 1.0;
        int j = 0;
        for (int r = 0; r < 3; ++r)
            for (int k : order[r]) {
                const double kc = spec->f_kn[k] * log2e, kp = spec->f_p[k] * log2e;
                const double wh = S[0][k] / tot[0], wl = S[1][k] / tot[1];
                if (S[0][k] > 0.0) wmin = std::fmin(wmin, wh);
                if (S[1][k] > 0.0) wmin = std::fmin(wmin, wl);
                const double v[8] = {kc, kp, wh, wh * kc, wh * kp, wl, wl * kc, wl * kp};
                for (int q = 0; q < 8; ++q) joint[(size_t)j * 8 + q] = (T)v[q];
                ++j;
            }
        // Every A_k is at most 2^(L - s) / w_k, L the log-sum-exp of a spectrum the bin
        // belongs to: L - s <= 124 + log2 wmin keeps it below 2^124.  The joint evaluation
        // is used when that leaves at least 100 (every weight at least 2^-24).
        const double lim = 124.0 + std::log2(wmin);
        p->joint_lim = nj > 0 && lim >= 100.0 ? lim : 0.0;
        double kcr[2] = {INFINITY, -INFINITY}, kpr[2] = {INFINITY, -INFINITY};
        for (int q = 0; q < nj; ++q) {
            kcr[0] = std::fmin(kcr[0], (double)joint[(size_t)q * 8]);
            kcr[1] = std::fmax(kcr[1], (double)joint[(size_t)q * 8]);
            kpr[0] = std::fmin(kpr[0], (double)joint[(size_t)q * 8 + 1]);
            kpr[1] = std::fmax(kpr[1], (double)joint[(size_t)q * 8 + 1]);
        }
        if (nj > 0)
            for (int e = 0; e < 2; ++e) {
                p->joint_kc[e] = kcr[e];
                p->joint_kp[e] = kpr[e];
            }
        st = upload<T>(joint.data(), joint.size() * sizeof(T), &p->joint);
        if (st) return st;
    }
    DECT_HIP(hipMalloc(&p->scratch_O, (size_t)p->N * 4 * p->sym * sizeof(T)));
    DECT_HIP(hipMalloc(&p->scratch_OT, (size_t)p->N * 4 * p->sym * sizeof(T)));
    if (p->sym == 4) DECT_HIP(hipMalloc(&p->scratch_sq, (size_t)p->M * 2 * sizeof(T)));
    return DECT_OK;
}

// Smallest power of two at least twice n (linear convolution over the image).
int pad_pow2(int n, int& lg) {
    int P = 1;
    lg = 0;
    while (P < 2 * n) {
        P *= 2;
        ++lg;
    }
    return P;
}

// Preconditioner of the x-update: the floored ramp max(|w|, 1/max(Py, Px)) on the
// zero-padded DFT grid (|w| in cycles per pixel) and the DFT twiddle factors
// exp(-2 pi i k / P), k < P / 2, of both padded sides.
template <typename T>
dect_status build_precond(dect_plan* p) {
    p->px = pad_pow2(p->nx, p->lpx);
    p->py = pad_pow2(p->ny, p->lpy);
    if (p->px > kMaxFft || p->py > kMaxFft) return DECT_OK;  // no preconditioner for this size
    const int px = p->px, py = p->py;
    const double floor_w = 1.0 / (double)(px > py ? px : py);
    std::vector<T> filt((size_t)px * py);
    for (int ky = 0; ky < py; ++ky) {
        const double fy = (ky < py / 2 ? ky : ky - py) / (double)py;
        for (int kx = 0; kx < px; ++kx) {
            const double fx = (kx < px / 2 ? kx : kx - px) / (double)px;
            filt[(size_t)ky * px + kx] = (T)std::fmax(std::sqrt(fx * fx + fy * fy), floor_w);
        }
    }
    dect_status st = upload<T>(filt.data(), filt.size() * sizeof(T), &p->pre_filter);
    if (st) return st;
    for (int axis = 0; axis < 2; ++axis) {
        const int P = axis ? py : px;
        std::vector<T> tw((size_t)P);  // (cos, -sin) pairs
        for (int k = 0; k < P / 2; ++k) {
            const double a = 6.283185307179586 * k / P;
            tw[2 * k] = (T)std::cos(a);
            tw[2 * k + 1] = (T)(-std::sin(a));
        }
        st = upload<T>(tw.data(), tw.size() * sizeof(T), axis ? &p->pre_twy : &p->pre_twx);
        if (st) return st;
    }
    DECT_HIP(hipMalloc(&p->scratch_W, (size_t)p->ny * px * 2 * sizeof(T)));
    p->has_precond = true;
    return DECT_OK;
}

// Filtered backprojection (the CDM-FBP baseline): the discrete Ram-Lak kernel of
// the detector spacing delta at the isocentre, h[0] = 1/(4 delta^2), h[n] =
// -1/(pi^2 n^2 delta^2) for odd n, zero for even n, circular over P = a power of
// two at least twice the bins; its DFT (real and even) is stored scaled by
// delta / P (and 1/2 for a fan over a full turn), so the filtered row is the
// inverse FFT of the product with no further factor.  Per view the (cos, sin) of
// its angle; per bin the fan pre-weight D / sqrt(D^2 + u^2).
template <typename T>
dect_status build_fbp(dect_plan* p) {
    const dect_geometry& g = p->geom;
    p->fbp_P = pad_pow2(p->D, p->fbp_lg);
    if (p->fbp_P > kMaxFbp) return DECT_OK;
    const int P = p->fbp_P, D = p->D, V = p->V;
    const bool fan = g.kind == DECT_FAN;
    const double delta = g.det_cm * (fan ? g.src_iso_cm / g.src_det_cm : 1.0);
    p->fbp_delta = delta;
    p->fbp_b0 = 0.5 * (D - 1) - g.det_offset;
    const double pi = 3.141592653589793;
    std::vector<double> h(P / 2 + 1, 0.0);
    h[0] = 1.0 / (4.0 * delta * delta);
    for (int n = 1; n <= P / 2; n += 2) h[n] = -1.0 / (pi * pi * (double)n * n * delta * delta);
    std::vector<T> H(P);
    const double scale = delta / P * (fan ? 0.5 : 1.0);
    for (int k = 0; k < P; ++k) {
        // h is even: H[k] = h[0] + 2 sum_{0 < n < P/2} h[n] cos(2 pi k n / P) + h[P/2] cos(pi k).
        double acc = h[0];
        for (int n = 1; n < P / 2; n += 2) acc += 2.0 * h[n] * std::cos(2.0 * pi * (double)k * n / P);
        acc += h[P / 2] * ((k & 1) ? -1.0 : 1.0);
        H[k] = (T)(acc * scale);
    }
    dect_status st = upload<T>(H.data(), H.size() * sizeof(T), &p->fbp_H);
    if (st) return st;
    std::vector<T> tw((size_t)P);
    for (int k = 0; k < P / 2; ++k) {
        tw[2 * k] = (T)std::cos(2.0 * pi * k / P);
        tw[2 * k + 1] = (T)(-std::sin(2.0 * pi * k / P));
    }
    st = upload<T>(tw.data(), tw.size() * sizeof(T), &p->fbp_tw);
    if (st) return st;
    // Per view, the detector coordinate (in bins, before b0) of the point with
    // centred pixel indices (i', j') is (ni i' + nj j') / den with den = 1 + di i' +
    // dj j', and the fan weight (D / L)^2 is 1 / den^2 (den = L / D); parallel: den = 1.
    std::vector<T> view((size_t)4 * V);
    const double kb = g.pixel_cm / delta;
    for (int v = 0; v < V; ++v) {
        const double t = g.angle0 + (double)v * g.span / V, c = std::cos(t), sn = std::sin(t);
        T* e = &view[(size_t)4 * v];
        if (fan) {
            e[0] = (T)(-g.pixel_cm * c / g.src_iso_cm);
            e[1] = (T)(-g.pixel_cm * sn / g.src_iso_cm);
            e[2] = (T)(-kb * sn);
            e[3] = (T)(kb * c);
        } else {
            e[0] = e[1] = (T)0;
            e[2] = (T)(kb * c);
            e[3] = (T)(kb * sn);
        }
    }
    st = upload<T>(view.data(), view.size() * sizeof(T), &p->fbp_view);
    if (st) return st;
    std::vector<T> wpre((size_t)D);
    for (int b = 0; b < D; ++b) {
        const double u = ((double)b - 0.5 * (D - 1) + g.det_offset) * delta;
        wpre[b] = (T)(fan ? g.src_iso_cm / std::sqrt(g.src_iso_cm * g.src_iso_cm + u * u) : 1.0);
    }
    st = upload<T>(wpre.data(), wpre.size() * sizeof(T), &p->fbp_wpre);
    if (st) return st;
    DECT_HIP(hipMalloc(&p->scratch_Q, (size_t)V * D * 2 * sizeof(T)));
    p->has_fbp = true;
    return DECT_OK;
}

void make_layout(dect_plan* p) {
    const size_t e = p->elem;
    const size_t N = (size_t)p->N, M = (size_t)p->M;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    dect_layout& L = p->layout;
    L.x = take(N * 2 * e);
    L.y = take(N * 4 * e);
    L.uy = take(N * 4 * e);
    L.z = take(N * 2 * e);
    L.uz = take(N * 2 * e);
    L.a = take(M * 2 * e);
    L.ua = take(M * 2 * e);
    L.Rx = take(M * 2 * e);
    L.scalars = take(S_COUNT * sizeof(double));
    p->off_p = take(N * 2 * e);
    p->off_pO = take(N * 2 * p->sym * e);
    p->off_pOT = take(N * 2 * p->sym * e);
    p->off_r = take(N * 2 * e);
    p->off_q = take(N * 2 * e);
    p->off_dy = take(N * 4 * e);
    p->off_dz = take(N * 2 * e);
    p->off_Rp = take(M * 2 * e);
    p->off_t = take(M * 2 * e);
    p->off_da = take(M * 2 * e);
    p->off_fg = take(M * 8 * e);
    p->off_z = take(N * 2 * e);
    p->off_h = take(N * 2 * sizeof(double));
    p->off_u = take(N * 2 * sizeof(double));
    p->off_rtrp = take(N * 2 * e);
    p->off_fftw = p->has_precond ? take((size_t)p->ny * p->px * 2 * e) : 0;
    p->nb_sino = (int)((M + 255) / 256);
    p->nb_img = (int)((N + 255) / 256);
    p->nb_tiles = bp_blocks(p);
    p->nb_pre = p->ny;
    p->off_partials = take((size_t)(p->nb_sino + p->nb_img + p->nb_tiles + p->nb_pre) *
                           kPartialSlots * sizeof(double));
    p->off_log = take((size_t)kLogCap * kLogStride * sizeof(double));
    // Accept decisions of the last a-update's LM iterations, one byte per ray.
    L.lm_accept = take(M);
    L.bytes = off;
}

}  // namespace

int bp_blocks(const dect_plan* p) {
    const int dx = p->sym == 4 ? p->nx / 2 : p->nx, dy = p->sym == 4 ? p->ny / 2 : p->ny;
    return ((dx + 7) / 8) * ((dy + 7) / 8);
}

}  // namespace dect

using namespace dect;

extern "C" {

const char* dect_last_error(void) { return g_last_error.c_str(); }

dect_status dect_plan_create(const dect_geometry* geom, const dect_spectra* spec,
                             dect_dtype dtype, dect_plan** out) {
    if (!geom || !spec || !out) return fail(DECT_E_ARG, "null argument");
    *out = nullptr;
    const dect_geometry& g = *geom;
    if (dtype != DECT_F32 && dtype != DECT_F64) return fail(DECT_E_ARG, "bad dtype %d", dtype);
    if (g.kind != DECT_PARALLEL && g.kind != DECT_FAN)
        return fail(DECT_E_ARG, "bad geometry kind %d", g.kind);
    if (g.nx < 2 || g.ny < 2 || g.n_views < 1 || g.n_det < 1)
        return fail(DECT_E_SHAPE, "image must be at least 2x2 and have views and bins");
    if ((long)g.nx * g.ny > (1L << 30) || (long)g.n_views * g.n_det > (1L << 30))
        return fail(DECT_E_SHAPE, "image or sinogram larger than 2^30 elements");
    if (!(g.pixel_cm > 0) || !(g.det_cm > 0) || !std::isfinite(g.span) ||
        !std::isfinite(g.angle0) || !std::isfinite(g.det_offset))
        return fail(DECT_E_SHAPE, "pixel and bin sizes must be positive, angles finite");
    if (g.kind == DECT_FAN) {
        const double rc = 0.5 * g.pixel_cm * std::hypot((double)g.nx, (double)g.ny);
        if (!(g.src_det_cm > g.src_iso_cm) || !(g.src_iso_cm > rc + 2.0 * g.pixel_cm))
            return fail(DECT_E_SHAPE,
                        "fan source must lie outside the image's circumscribed circle "
                        "(radius %.4g cm) by two pixels, detector beyond the centre",
                        rc);
    }
    if (spec->n_bins < 1 || !spec->s_high || !spec->s_low || !spec->f_kn || !spec->f_p)
        return fail(DECT_E_ARG, "spectra: null table or no bins");
    for (int h = 0; h < 2; ++h) {
        const double* S = h ? spec->s_low : spec->s_high;
        double tot = 0.0;
        for (int k = 0; k < spec->n_bins; ++k) {
            if (!(S[k] >= 0.0)) return fail(DECT_E_ARG, "spectrum %d bin %d negative", h, k);
            tot += S[k];
        }
        if (!(tot > 0.0)) return fail(DECT_E_ARG, "spectrum %d has no photons", h);
    }
    for (int k = 0; k < spec->n_bins; ++k)
        if (!(spec->f_kn[k] > 0.0) || !(spec->f_p[k] >= 0.0))
            return fail(DECT_E_ARG, "f_kn must be > 0 and f_p >= 0 (bin %d)", k);

    dect_plan* p = new (std::nothrow) dect_plan();
    if (!p) return fail(DECT_E_NOMEM, "host allocation failed");
    p->geom = g;
    p->dtype = dtype;
    p->elem = dtype == DECT_F32 ? 4 : 8;
    p->nx = g.nx;
    p->ny = g.ny;
    p->V = g.n_views;
    p->D = g.n_det;
    p->N = (long)g.nx * g.ny;
    p->M = (long)g.n_views * g.n_det;
    // Quarter-turn symmetry: fan beam over a full turn, views in multiples of 4,
    // square image with an even side (so the pixel grid maps onto itself).
    const double two_pi = 6.283185307179586;
    p->sym = (g.kind == DECT_FAN && std::fabs(g.span - two_pi) < 1e-12 && g.n_views % 4 == 0 &&
              g.nx == g.ny && g.nx % 2 == 0)
                 ? 4
                 : 1;
    p->Vb = g.n_views / p->sym;
    // Footprint margin of the transpose: the detector coordinate of the two-pixel
    // segment around a pixel is linearised at its centre; for a fan the error is at
    // most |d beta| * pixel / (distance to source - pixel).  Plus 0.02 bins for
    // rounding of the tables and of the footprint itself.
    p->margin = 0.02;
    if (g.kind == DECT_FAN) {
        const double rc = 0.5 * g.pixel_cm * std::hypot((double)g.nx, (double)g.ny);
        const double dmin = g.src_iso_cm - rc - 2.0 * g.pixel_cm;
        const double K = g.src_det_cm / g.det_cm;
        const double dbeta = (K * g.pixel_cm + K * rc / dmin * g.pixel_cm) / dmin;
        p->margin += 1.5 * dbeta * g.pixel_cm / (dmin - g.pixel_cm);
    }
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(DECT_E_DEVICE, "no HIP device");
    }
    dect_status st = dtype == DECT_F32 ? build_tables<float>(p, spec) : build_tables<double>(p, spec);
    if (st == DECT_OK) st = dtype == DECT_F32 ? build_precond<float>(p) : build_precond<double>(p);
    if (st == DECT_OK) st = dtype == DECT_F32 ? build_fbp<float>(p) : build_fbp<double>(p);
    if (st == DECT_OK && hipMalloc(reinterpret_cast<void**>(&p->scratch_part),
                                   (size_t)(p->ny > kRaySumBlocks ? p->ny : kRaySumBlocks + 1) *
                                       kPartialSlots *
                                       sizeof(double)) != hipSuccess)
        st = fail(DECT_E_NOMEM, "device allocation failed");
    if (st != DECT_OK) {
        dect_plan_destroy(p);
        return st;
    }
    make_layout(p);
    *out = p;
    return DECT_OK;
}

void dect_plan_destroy(dect_plan* p) {
    if (!p) return;
    (void)hipFree(p->rays);
    (void)hipFree(p->views);
    (void)hipFree(p->bp_rays);
    (void)hipFree(p->spec);
    (void)hipFree(p->joint);
    (void)hipFree(p->scratch_O);
    (void)hipFree(p->scratch_OT);
    (void)hipFree(p->scratch_sq);
    (void)hipFree(p->pre_filter);
    (void)hipFree(p->pre_twx);
    (void)hipFree(p->pre_twy);
    (void)hipFree(p->scratch_W);
    (void)hipFree(p->scratch_part);
    (void)hipFree(p->fbp_H);
    (void)hipFree(p->fbp_tw);
    (void)hipFree(p->fbp_view);
    (void)hipFree(p->fbp_wpre);
    (void)hipFree(p->scratch_Q);
    delete p;
}

dect_status dect_plan_get_info(const dect_plan* p, dect_plan_info* out) {
    if (!p || !out) return fail(DECT_E_ARG, "null argument");
    dect_plan_info info{};
    info.n_pixels = p->N;
    info.n_rays = p->M;
    info.symmetry = p->sym;
    // Same sampling rule as the projector, in double precision.
    // Views beyond the base views are rotations of them: same counts.
    for (int v = 0; v < p->Vb; ++v)
        for (int b = 0; b < p->D; ++b) {
            HostRay r = host_ray(p->geom, v, b);
            const int n_steps = r.xstep ? p->nx : p->ny, n_lines = r.xstep ? p->ny : p->nx;
            for (int k = 0; k < n_steps; ++k) {
                const double j0 = std::floor(r.phi0 + r.slope * k);
                const int in0 = (j0 >= 0 && j0 < n_lines), in1 = (j0 + 1 >= 0 && j0 + 1 < n_lines);
                info.samples += p->sym * (in0 | in1);
                info.taps += p->sym * (in0 + in1);
            }
        }
    *out = info;
    return DECT_OK;
}

size_t dect_state_bytes(const dect_plan* plan) { return plan ? plan->layout.bytes : 0; }

dect_status dect_state_layout(const dect_plan* plan, dect_layout* out) {
    if (!plan || !out) return fail(DECT_E_ARG, "null argument");
    *out = plan->layout;
    return DECT_OK;
}

}  // extern "C"
