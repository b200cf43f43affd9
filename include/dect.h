/*
 * dect.h -- C ABI of the MI355X dual-energy CT ADMM library (gfx950, HIP).
 *
 * The library implements one outer iteration of the splitting-based ADMM for
 * statistical dual-energy CT of Li, Manerikar, Prakash and Kak (Sec. 3.3):
 * the x-update by conjugate gradients on Eq. (12) with a Joseph projector R and
 * its exact transpose R^T, the per-ray decomposition of Eq. (13) by
 * Levenberg-Marquardt, the shrinkage and nonnegativity steps of Eq. (9)-(10),
 * the scaled-dual update of Eq. (11) and residual-balancing adaptation of rho.
 *
 * Conventions
 *  - Every array argument is a plain pointer.  "device" pointers address GPU
 *    memory (hipMalloc'd or a torch CUDA tensor's data_ptr()); "host" pointers
 *    address CPU memory.  Sizes are element counts.
 *  - Floating-point arrays have the plan's dtype (float for DECT_F32, double
 *    for DECT_F64).  Counts, measurements and weights too.
 *  - Images are row-major [ny][nx]; sinograms are view-major [n_views][n_det].
 *    Multi-channel arrays keep the channels innermost: an image with ch
 *    channels is [ny][nx][ch], a sinogram [n_views][n_det][ch].  The two ADMM
 *    bases (Compton c, photoelectric p) are such channel pairs (c, p).
 *  - Pixel (j, i) has its centre at ((i-(nx-1)/2) pixel_cm, (j-(ny-1)/2) pixel_cm);
 *    view v is at angle angle0 + v*span/n_views; bin b sits at detector
 *    coordinate u_b = (b - (n_det-1)/2 + det_offset) * det_cm.  Parallel beam:
 *    the ray of (v, b) is the line p.(cos t, sin t) = u_b.  Fan beam with a flat
 *    detector: source at src_iso_cm (cos t, sin t), bin at
 *    -(src_det_cm - src_iso_cm)(cos t, sin t) + u_b (-sin t, cos t).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls marked
 *    "async" only enqueue work on it; the caller keeps every buffer alive and
 *    unmodified until that work completes.
 *  - Errors: every function returns a dect_status; on failure a message is
 *    available from dect_last_error() (thread-local).  Nothing is thrown.
 *    Argument and shape checks are done at plan creation and on every call's
 *    pointer and channel arguments; faults inside kernels are reported by the
 *    HIP runtime at the next synchronising call.
 */
#ifndef DECT_H
#define DECT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DECT_OK = 0,
    DECT_NOT_READY = 1,
    DECT_E_ARG = -1,       /* null pointer, bad enum, bad channel count, bad parameter */
    DECT_E_SHAPE = -2,     /* geometry the library cannot represent */
    DECT_E_NOMEM = -3,     /* device or host allocation failed */
    DECT_E_DEVICE = -4,    /* a HIP runtime call failed */
    DECT_E_NONFINITE = -5, /* a non-finite residual or objective was produced */
    DECT_E_CAPACITY = -6   /* a request does not fit the server's memory budget */
} dect_status;

typedef enum { DECT_F32 = 0, DECT_F64 = 1 } dect_dtype;
typedef enum { DECT_PARALLEL = 0, DECT_FAN = 1 } dect_beam;

/* Scanner geometry (the projection matrix R of Eq. (2)). */
typedef struct {
    int kind;            /* dect_beam */
    int nx, ny;          /* image columns, rows */
    double pixel_cm;     /* square pixel side */
    int n_views, n_det;  /* views, detector bins */
    double det_cm;       /* bin spacing on the (flat) detector */
    double det_offset;   /* detector shift, in bins */
    double src_iso_cm;   /* fan: source to rotation centre */
    double src_det_cm;   /* fan: source to detector */
    double angle0;       /* first view angle, radians */
    double span;         /* angular range covered by the views, radians */
} dect_geometry;

/* Spectral model of Eq. (1)-(3): photon spectra S_h, S_l on an energy grid and the
 * Compton (f_KN) and photoelectric (f_p) energy multipliers.  Host arrays of
 * n_bins doubles, copied at plan creation.  S >= 0 with a positive sum; f_kn > 0;
 * f_p >= 0.  Bins where a spectrum is zero are dropped for that spectrum. */
typedef struct {
    int n_bins;
    const double* energy_kev;
    const double* s_high;
    const double* s_low;
    const double* f_kn;
    const double* f_p;
} dect_spectra;

typedef struct dect_plan dect_plan;

/* Create a plan: validated geometry, per-ray Joseph tables and per-view
 * footprint tables (device), and the spectral tables.  The plan belongs to the
 * library; it is bound to the device current at creation.  DECT_E_SHAPE if a
 * fan source lies inside the circle circumscribing the image, or if a view's
 * rays do not split into one run of x-stepped and one run of y-stepped bins. */
dect_status dect_plan_create(const dect_geometry* geom, const dect_spectra* spec,
                             dect_dtype dtype, dect_plan** out);
void dect_plan_destroy(dect_plan* plan);
const char* dect_last_error(void);

/* R: sino[v][b][c] = sum over the Joseph samples of ray (v,b) of the linearly
 * interpolated img[.][.][c] times the step length (Eq. (2), Sec. 1).
 * img: device [ny][nx][ch]; sino: device [n_views][n_det][ch] (overwritten);
 * ch in {1, 2, 4}.  async.  Uses a plan-owned scratch image, so calls with one
 * plan must not run concurrently on different streams. */
dect_status dect_project(const dect_plan* plan, const void* img, void* sino, int ch,
                         void* stream);

/* dect_project for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results as dect_project (bit for bit), but the two orbit images the
 * projector reads live in a static device array of 32 MiB that the library holds
 * on each device it runs on until the process ends, not in the plan's scratch; the
 * call allocates nothing.  Its size limits the plan: 2 * nx * ny * ch * s * bytes
 * per value (+ up to 255 bytes of alignment), with s = 4 on a quarter-turn
 * symmetric plan and 1 otherwise, must not exceed 32 MiB (e.g. 512x512 with two
 * channels in FP64 or four in FP32 on a symmetric plan); larger calls return
 * DECT_E_CAPACITY before anything is enqueued.  Every call on one device shares
 * that device's array: calls that overlap on one GPU (on different streams, or
 * from different threads) race and must not be issued; calls in order on one
 * stream are safe (each call writes the array in full before reading it).  The
 * first call on a device looks up the array's device address, with that device
 * current.  img: device [ny][nx][ch]; sino: device [n_views][n_det][ch]. async. */
dect_status dect_project_noalloc(const dect_plan* plan, const void* img, void* sino, int ch,
                                 void* stream);

/* R^T, the transpose of dect_project up to rounding, gathered per pixel with no
 * atomics: img[j][i][c] = sum over rays of weight * sino[v][b][c], each weight the
 * projector's linear-interpolation weight of the pixel re-evaluated from the same
 * ray geometry in a different but equivalent arithmetic form (so the pair is
 * adjoint to rounding: <R x, y> = <x, R^T y> to 1e-12 relative in FP64).
 * sino: device [n_views][n_det][ch]; img: device [ny][nx][ch] (overwritten);
 * ch in {1, 2, 4}.  async.  On a quarter-turn symmetric plan one or two channels
 * are first reordered into a plan-owned scratch sinogram, so calls with one plan
 * must not run concurrently on different streams. */
dect_status dect_backproject(const dect_plan* plan, const void* sino, void* img, int ch,
                             void* stream);

/* Per-ray unconstrained decomposition, Eq. (13): for every ray i minimise
 *   1/2 sum_s w_s (f_s(a) - m_s)^2 + 1/2 sum_b rho_b (a_b - v_b)^2
 * over a = (a_c, a_p), f_s the polychromatic transform of Eq. (3), by lm_iters
 * Levenberg-Marquardt iterations started at the given a (damping 1e-3, x10 on
 * rejection, /10 on acceptance, Marquardt scaling).
 * m_h, m_l, w_h, w_l: device [n_views*n_det]; v: device [..][2] or NULL (then the
 * rho terms are dropped); a: device [..][2], in/out; cost: device [..] or NULL
 * (final value of the minimised function).  async. */
dect_status dect_decompose_rays(const dect_plan* plan, const void* m_h, const void* m_l,
                                const void* w_h, const void* w_l, const void* v,
                                double rho_c, double rho_p, int lm_iters, void* a, void* cost,
                                void* stream);

/* Ingest photon counts: m = ln(I0 / max(c, 1)) and w = c / I0 (Sigma of Eq. (4) as
 * counts normalised by the unattenuated count).  All device [n_views*n_det]. async. */
dect_status dect_ingest_counts(const dect_plan* plan, const void* counts_h,
                               const void* counts_l, double i0_h, double i0_l, void* m_h,
                               void* m_l, void* w_h, void* w_l, void* stream);

/* ---------------------------------------------------------------- ADMM --- */

typedef enum {
    DECT_RHO_FIXED = 0,    /* rho stays at rho0 */
    DECT_RHO_ADAPTIVE = 1, /* residual balancing: r > mu s -> rho*tau; s > mu r -> rho/tau */
    DECT_RHO_SCHEDULE = 2  /* rho of iteration k taken from rho_schedule[2k], [2k+1] */
} dect_rho_mode;

typedef struct {
    double lambda_c, lambda_p; /* TV weights of Eq. (9) */
    double rho_c, rho_p;       /* initial penalties (used by dect_admm_init) */
    int lm_iters;              /* m: LM iterations per outer iteration, >= 1 */
    int cg_iters;              /* n: CG iterations per outer iteration, >= 1 */
    int rho_mode;              /* dect_rho_mode */
    double bal_mu, bal_tau;    /* residual balancing constants (10, 2) */
    double lm_mu0;             /* LM initial damping (1e-3) */
    const double* rho_schedule;/* host, 2*rho_schedule_len doubles, for DECT_RHO_SCHEDULE */
    int rho_schedule_len;
    int precond;               /* dect_precond: CG (0) or CG preconditioned by the ramp filter */
    int rt_sums;               /* dect_rt_sums: precision of the ADMM transposes' sums */
} dect_params;

/* Sums of the ADMM's transposes (R^T of the CG direction's projection and of the
 * change of a) on an FP32 plan.  PLAN: single precision.  F64: the products (exact
 * in double) summed in double precision and each result rounded once, at about 40 %
 * more transpose time.  The terms of R^T over the projection of a ramp-filtered
 * direction nearly cancel: with DECT_PRECOND_RAMP on an FP32 plan, F64 sums keep the
 * iterates near those of double-precision arithmetic for longer (x_c within ~3e-4
 * after 50 iterations on a 256^2 slice, against ~1.4e-3 with PLAN).  FP64 plans sum
 * in double either way.  Slices of a batch share launches only if this agrees. */
typedef enum { DECT_RT_SUMS_PLAN = 0, DECT_RT_SUMS_F64 = 1 } dect_rt_sums;

/* Preconditioner of the x-update (Sec. 3.3: the system of Eq. (12) is shift-invariant,
 * so CG is preconditioned by a high-pass filter applied by FFT).  RAMP: the image is
 * zero-padded to px x py (the powers of two at least twice each side), its 2-D DFT
 * multiplied by max(|w|, 1/max(px, py)) with |w| in cycles per pixel, transformed
 * back and cropped.  Available when both padded sides are at most 2048. */
typedef enum { DECT_PRECOND_NONE = 0, DECT_PRECOND_RAMP = 1 } dect_precond;

/* The preconditioner applied to a two-channel image: out = M img, both device
 * [ny][nx][2].  DECT_E_SHAPE if the plan has none.  async.  Uses plan-owned scratch,
 * so calls with one plan must not run concurrently on different streams. */
dect_status dect_precondition(const dect_plan* plan, const void* img, void* out, void* stream);

/* The projection-wise baseline and the initial image (Sec. 2, the constrained
 * decomposition CDM; Sec. 4, the start of the iterations). */

/* CDM: per ray, minimise 1/2 sum_s w_s (f_s(a) - m_s)^2 over a >= 0 by lm_iters
 * projected Levenberg-Marquardt iterations started at the linearised solution
 * clipped to a >= 0.  A coordinate at its bound whose gradient points out of the
 * feasible set is held there and the other one takes a 1-D damped step; every
 * accepted point is projected onto a >= 0.  m_*, w_*: device [n_views*n_det]; a:
 * device [n_views][n_det][2], out; cost: device [n_views*n_det] or NULL (final
 * objective).  async. */
dect_status dect_cdm(const dect_plan* plan, const void* m_h, const void* m_l, const void* w_h,
                     const void* w_l, int lm_iters, void* a, void* cost, void* stream);

/* Filtered backprojection of line integrals.  Parallel beam: every view row is
 * convolved with the discrete Ram-Lak kernel of the bin spacing (times the
 * spacing), the result linearly interpolated at each pixel's detector coordinate
 * (zero off the detector) and summed over views times span/n_views.  Fan beam with
 * a flat detector: the same with the detector scaled to the isocentre, each row
 * pre-weighted by D/sqrt(D^2+u^2) and halved, and each view's contribution
 * weighted by (D/L)^2, D = src_iso_cm and L the distance from the source to the
 * pixel along the central ray.  sino: device [n_views][n_det][ch]; img: device
 * [ny][nx][ch] (overwritten); ch in {1, 2}.  DECT_E_SHAPE if the row padded to a
 * power of two at least 2 n_det exceeds 4096.  async; plan-owned scratch (calls
 * with one plan must not overlap on different streams). */
dect_status dect_fbp(const dect_plan* plan, const void* sino, void* img, int ch, void* stream);

/* CDM-FBP and the initial image: a = CDM(m, w) with cdm_iters iterations, the FBP
 * of both bases, and x0 = (x_c, s x_c) with x_c the Compton FBP image and s =
 * sum(a_p) / sum(a_c) over all rays (0 if the sum of a_c is 0).  a: device
 * [n_views][n_det][2], out; x0: device [ny][nx][2], out; fbp_out: device
 * [ny][nx][2] for the FBP image pair, or NULL.  async; plan-owned scratch. */
dect_status dect_cdm_fbp_start(const dect_plan* plan, const void* m_h, const void* m_l,
                               const void* w_h, const void* w_l, int cdm_iters, void* a,
                               void* x0, void* fbp_out, void* stream);

/* As dect_admm_init, then the iterations start from the image pair x0 (device
 * [ny][nx][2]) instead of 0: x = z = x0, R x = R x0, y = D x0 (forward
 * differences as in Eq. (9)), u = 0.  async. */
dect_status dect_admm_init_image(const dect_plan* plan, const void* m_h, const void* m_l,
                                 const void* w_h, const void* w_l, const void* x0, void* state,
                                 const dect_params* params, void* stream);

/* Per-iteration record, filled when the caller passes a log buffer. */
typedef struct {
    int32_t iter;       /* outer iteration index */
    int32_t flags;      /* bit 0: a non-finite value was met */
    double rho[2];      /* rho in force during the iteration (c, p) */
    double r_primal[2]; /* ||(a - Rx, y - Dx, z - x)|| per basis */
    double s_dual[2];   /* rho ||R^T da + D^T dy + dz|| per basis (0 in fixed mode) */
    double data_cost;   /* 1/2 sum w (f(a) - m)^2 after the a-update */
    double tv_cost;     /* lambda_c |y_c|_1 + lambda_p |y_p|_1 */
} dect_iter_log;

/* The state of one slice lives in ONE caller-owned device buffer of
 * dect_state_bytes() bytes (256-byte aligned).  Its layout is described by
 * dect_state_layout: byte offsets of the named arrays; image arrays are
 * [ny][nx][2] basis pairs, y and u^y [ny][nx][4] = (c_h, p_h, c_v, p_v),
 * sinogram arrays [n_views][n_det][2].  The buffer holds everything an iteration
 * reads or writes, so copying it checkpoints the reconstruction. */
typedef struct {
    size_t bytes;
    size_t x, y, uy, z, uz;   /* images */
    size_t a, ua, Rx;         /* sinograms */
    size_t scalars;           /* device doubles: rho_c, rho_p, iteration, ... */
    size_t lm_accept;         /* uint8 [n_views][n_det]: bit k set if LM iteration k (k < 8)
                                 of the last a-update accepted its trial point */
} dect_layout;

/* Sizes of the operator, for cost accounting: Joseph samples (steps with at least
 * one tap inside the image) and nonzero taps (nonzeros of R) over all rays, and the
 * number of views that share one weight evaluation (4 on a quarter-turn symmetric
 * plan, whose views v + k n_views/4 are exact rotations of base view v; else 1). */
typedef struct {
    int64_t n_pixels, n_rays;
    int64_t samples, taps;
    int64_t symmetry;
} dect_plan_info;

/* Counted on the host on first call (a pass over every ray's samples). */
dect_status dect_plan_get_info(const dect_plan* plan, dect_plan_info* out);

size_t dect_state_bytes(const dect_plan* plan);
dect_status dect_state_layout(const dect_plan* plan, dect_layout* out);

/* Initial state: x = 0, R x = 0, y = z = u = 0, rho = (rho_c, rho_p), and a from a
 * rho = 0 decomposition (10 LM iterations) started at the linearised solution.
 * m_*, w_*: device [n_views*n_det]; state: device buffer.  async. */
dect_status dect_admm_init(const dect_plan* plan, const void* m_h, const void* m_l,
                           const void* w_h, const void* w_l, void* state,
                           const dect_params* params, void* stream);

/* n_iters outer iterations (x by CG(n) on Eq. (12), a by LM(m) on Eq. (13), y and
 * z by Eq. (9)-(10), u by Eq. (11), then rho).  log: host array of n_iters
 * records or NULL; with a log the call synchronises the stream and returns
 * DECT_E_NONFINITE if any record has the non-finite flag.  Without a log the
 * call is async.  A DECT_RHO_SCHEDULE run must cover every iteration index it
 * reaches (DECT_E_ARG otherwise).  Within a call the rescale of the scaled duals
 * after a change of rho is applied by their next readers; the call ends by applying
 * what is still pending, so between calls the state's u^a, u^y, u^z hold the scaled
 * duals of Eq. (11). */
dect_status dect_admm_iterate(const dect_plan* plan, const void* m_h, const void* m_l,
                              const void* w_h, const void* w_l, void* state,
                              const dect_params* params, int n_iters, dect_iter_log* log,
                              void* stream);

/* Records of iterations [first, first + n) of a state, from its device log ring
 * (the last 256 iterations are kept).  Synchronises the stream; DECT_E_ARG if
 * a requested iteration has not run yet or has left the ring.  log: host array
 * of n records. */
dect_status dect_state_log(const dect_plan* plan, const void* state, int64_t first, int n,
                           dect_iter_log* log, void* stream);

/* The baseline LM(m) x CG(n) splitting (Eqs. (7)-(8); Table 1 counts R 2m(n+1),
 * R^T 2m(n+1) and f 4m per iteration).  One outer iteration: x_c by m
 * Levenberg-Marquardt iterations on
 *   Phi(x_c) = 1/2 ||f(R x_c, R x_p) - m||^2_Sigma + rho_c/2 ||[y_c; z_c] - [D; I] x_c + u_c||^2
 * with x_p fixed, then x_p likewise with the new x_c.  Each LM iteration solves
 * (R^T W R + rho (D^T D + I) + mu kappa I) d = -grad Phi by cg_iters CG steps from
 * d = 0 (W = sum_s w_s (df_s/da)^2 per ray; kappa = g'Hg/g'g, the curvature along
 * the gradient; mu starts at lm_mu0 for each basis, /10 on an accepted step, x10 on
 * a rejected one: a step is accepted when Phi decreases).  f and its gradient at
 * R x are kept per ray.  Then y, z, u as in Eqs. (9)-(11) with C = [D; I], and rho
 * (DECT_RHO_FIXED or ADAPTIVE; the dual residual is rho ||D^T dy + dz||).
 * The state is one caller-owned device buffer of dect_lmcg_state_bytes() bytes
 * (256-byte aligned); images are planar per basis: x, z, u^z [2][ny][nx]; y, u^y
 * [2][2][ny][nx] (basis, then horizontal/vertical difference); R x [2][n_views][n_det]. */
typedef struct {
    size_t bytes;
    size_t x, y, uy, z, uz, Rx;
    size_t scalars;
} dect_lmcg_layout;

size_t dect_lmcg_state_bytes(const dect_plan* plan);
dect_status dect_lmcg_state_layout(const dect_plan* plan, dect_lmcg_layout* out);

/* x = x0 (device [ny][nx][2] image pair, or NULL for 0), z = x, y = D x, u = 0,
 * rho = (rho_c, rho_p), R x and f at R x.  lm_mu0 may be 0 (undamped Gauss-Newton);
 * precond must be DECT_PRECOND_NONE.  async. */
dect_status dect_lmcg_init(const dect_plan* plan, const void* m_h, const void* m_l,
                           const void* w_h, const void* w_l, const void* x0, void* state,
                           const dect_params* params, void* stream);

/* n_iters outer iterations; log as for dect_admm_iterate (the data cost is at R x). */
dect_status dect_lmcg_iterate(const dect_plan* plan, const void* m_h, const void* m_l,
                              const void* w_h, const void* w_l, void* state,
                              const dect_params* params, int n_iters, dect_iter_log* log,
                              void* stream);


/* ----------------------------------------------------------- autotuning --- */

/* Launch shapes of the ADMM's transposed projector and projector:
 *  - bp_waves: waves of a transpose workgroup, splitting the views (2, 4 or 8);
 *  - proj_waves: waves of a projector workgroup, splitting the lines its rays cross
 *    (2, 4 or 8);
 *  - proj_views: base views whose rays share a projector wave (1, 2, 4 or 8; the wave
 *    takes 64 / proj_views consecutive bins of each);
 *  - proj_chunk: bin groups an XCD takes per turn of the workgroup order (1 to 16).
 * Defaults 4, 8, 2, 1.  Every shape computes the same sums; only the order in which a
 * workgroup's partial sums are added changes.  Batches share launches only between
 * slices whose plans have the same shapes. */
typedef struct {
    int bp_waves;      /* transposed projector */
    int proj_waves;    /* projector */
    int proj_views;
    int proj_chunk;
    double bp_us;      /* timed duration of the chosen shapes (0 when not timed) */
    double proj_us;
    double bp_us_default;    /* timed duration of the default shapes (0 when not timed) */
    double proj_us_default;
    int from_cache;    /* 1 if taken from the cache without timing */
} dect_launch;

#define DECT_TUNE_FORCE 1  /* time the candidates even if the cache has an entry */

/* Choose the plan's launch shapes: from the cache file if it has an entry for this
 * device, precision and problem shape, else by timing every candidate on a scratch
 * state on `stream` (synchronises; allocates a temporary state) and appending the
 * result to the cache (cache_path NULL: no cache).  Candidates: bp_waves 2, 4, 8 for
 * the transpose; proj_waves 2, 4, 8 x proj_views 1, 2, 4 x proj_chunk 1, 2, 4 for the
 * projector; each timed as the median of 3 batches of 8 launches after 2 warm-up
 * launches.  A candidate replaces the default only if it is faster by more than the
 * larger of 1 % and the batches' spread, so run-to-run noise does not change the
 * shapes.  The plan is updated; out (may be NULL) receives the choice. */
dect_status dect_plan_tune(dect_plan* plan, const char* cache_path, int flags, dect_launch* out,
                           void* stream);
dect_status dect_plan_set_launch(dect_plan* plan, int bp_waves, int proj_waves, int proj_views,
                                 int proj_chunk);
dect_status dect_plan_get_launch(const dect_plan* plan, dect_launch* out);

/* ---------------------------------------------------------------- batch --- */

/* Independent slices advanced together.  The paper reconstructs one 2-D slice;
 * treating each slice (detector row or table position) as its own problem with no
 * data shared between slices is this library's design choice for throughput.  A batch groups its slices by shape
 * (image, views, bins); every kernel of an outer iteration is ONE launch per
 * group, all slices of the group at once, and with use_graph one outer
 * iteration of all groups is captured once into a HIP graph and replayed.  A
 * slice's arithmetic and reduction order do not depend on the other slices:
 * its state after k batch iterations is bitwise that of k dect_admm_iterate
 * calls on it alone.
 *
 * plans[k], m_h[k] .. w_l[k], states[k]: slice k's plan, measurements and state
 * (initialised by dect_admm_init); plans may repeat, states may not; all plans
 * share one dtype.  params: fixed or adaptive rho (no schedule).  The batch
 * keeps the pointers: every buffer must outlive it.  The batch owns small
 * device argument tables and, with a graph, a private capture stream. */
typedef struct dect_batch dect_batch;

dect_status dect_batch_create(int n, const dect_plan* const* plans, const void* const* m_h,
                              const void* const* m_l, const void* const* w_h,
                              const void* const* w_l, void* const* states,
                              const dect_params* params, int use_graph, dect_batch** out);
/* n_iters outer iterations of every slice, enqueued on stream.  async.  While
 * per-kernel timing is on (dect_profile_start) the kernels are launched
 * directly instead of through the graph.  As dect_admm_iterate, the call ends with
 * every slice's duals rescaled for the last change of rho. */
dect_status dect_batch_iterate(dect_batch* batch, int n_iters, void* stream);
/* Number of shape groups (launches per kernel per iteration). */
int dect_batch_groups(const dect_batch* batch);
void dect_batch_destroy(dect_batch* batch);

/* -------------------------------------------------------------- serving --- */

/* Continuous batching of slice reconstructions (each slice its own problem, as
 * in the batch above).  A server owns one worker thread and one stream on the device
 * current at creation.  Requests wait in a FIFO queue and are admitted, in
 * order, while a slot is free and their device footprint (state, measurements
 * and counts: dect_serve_footprint) fits the memory budget.  An admitted request
 * is ingested and initialised (dect_admm_init) and then advanced together with
 * every other slot, one launch per kernel per shape group, until it stops.
 * A slot is checked after every step_iters of its own iterations and at
 * max_iters: it stops when |Phi_k - Phi_(k-1)| <= tol |Phi_k| (Phi = data cost
 * + TV cost of its last two iterations), at max_iters, or on a non-finite
 * value.  The step the server runs is the smallest distance of any slot to its
 * next check, so every slot stops at exactly the iteration it would reach alone:
 * its result does not depend on the other requests in flight. */
typedef struct {
    size_t hbm_budget_bytes; /* device memory for slots; 0: half the free memory */
    int max_slots;           /* requests in flight at once, >= 1 */
    int step_iters;          /* iterations between a slot's checks, >= 1 */
    int max_queue;           /* requests waiting for admission at most (0: no limit); a
                                submit beyond it is refused with DECT_E_CAPACITY, so an
                                overloaded server sheds load instead of queueing without
                                bound */
} dect_server_config;

typedef struct {
    const dect_plan* plan;   /* geometry, spectra, dtype; must outlive the request */
    const void* counts_h;    /* host [n_views*n_det], plan dtype; copied at submit */
    const void* counts_l;
    double i0_h, i0_l;       /* unattenuated counts */
    dect_params params;      /* fixed or adaptive rho (no schedule) */
    double tol;              /* relative objective change that stops the slot */
    int max_iters;           /* outer iterations at most, >= 1 */
    void* x_out;             /* host [ny][nx][2], plan dtype; written on completion and
                                kept alive by the caller until poll/wait returns it */
} dect_request;

typedef struct {
    int32_t status;     /* DECT_OK or the error that ended the request */
    int32_t iters;      /* outer iterations run */
    double objective;   /* Phi at the last iteration */
    double rel_change;  /* |Phi_k - Phi_(k-1)| / |Phi_k| at the last check (inf if k < 2) */
    int64_t queue_ns;   /* submit to admission */
    int64_t latency_ns; /* submit to completion (x_out written) */
} dect_result;

typedef struct {
    int64_t submitted, completed, queued, in_flight, peak_in_flight, steps;
    size_t hbm_held;    /* device bytes held for slots (in use and cached) */
    int64_t rejected;   /* submits refused because the queue was full */
} dect_server_stats;

typedef struct dect_server dect_server;

dect_status dect_server_create(const dect_server_config* cfg, dect_server** out);
/* Device bytes one request of this plan holds while in flight. */
size_t dect_serve_footprint(const dect_plan* plan);
/* Queue a request; *ticket identifies it.  DECT_E_CAPACITY if its footprint
 * exceeds the whole budget or the queue holds max_queue requests, DECT_E_ARG for bad
 * arguments. */
dect_status dect_serve_submit(dect_server* server, const dect_request* req, uint64_t* ticket);
/* DECT_NOT_READY while the request is queued or running; once it has finished,
 * DECT_OK and *out, and the ticket is released (a later poll is DECT_E_ARG). */
dect_status dect_serve_poll(dect_server* server, uint64_t ticket, dect_result* out);
/* As poll, but blocks up to timeout_ms (< 0: no limit) for completion. */
dect_status dect_serve_wait(dect_server* server, uint64_t ticket, int64_t timeout_ms,
                            dect_result* out);
dect_status dect_server_get_stats(dect_server* server, dect_server_stats* out);
/* Stops the worker after its current step; unfinished requests are dropped. */
void dect_server_destroy(dect_server* server);

/* --------------------------------------------------------------- timing --- */

/* Per-kernel timing for benchmarks: between dect_profile_start and
 * dect_profile_stop every kernel the library launches is bracketed by HIP
 * events recorded on the stream it runs on.  stop waits for those events and
 * writes one record per kernel name (at most max; *n_out = number of names). */
typedef struct {
    char name[32];
    double total_ms;
    int32_t launches;
} dect_kernel_time;

dect_status dect_profile_start(void);
dect_status dect_profile_stop(dect_kernel_time* out, int max, int* n_out);

#ifdef __cplusplus
}
#endif
#endif /* DECT_H */
