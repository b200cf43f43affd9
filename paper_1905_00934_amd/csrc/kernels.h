// Kernel launchers shared by the library's translation units.
#pragma once

#include "common.h"
#include "projidx.h"

namespace dect {

enum Epilogue : int { EPI_NONE = 0, EPI_RHS = 1, EPI_Q = 2, EPI_DUAL = 3 };

// Arguments of the transposed projector and its image-side epilogues.
//  EPI_NONE: out = R^T sino (ch channels)
//  EPI_RHS : out (and out2 if set) = R^T t + D^T (y + uy - D x) + (z + uz - x);
//            partials = per-channel |out|^2.  Only the right-hand-side kernels use it,
//            with the tracked R^T t = h + u in place of a transpose; the duals u, uy, uz
//            are read scaled by the pending kappa = scal[S_KAPPA] (scal == nullptr: 1)
//  EPI_Q   : out (if set) = R^T sino + D^T D x + x, with x = p; partials = p . out;
//            raw (if set) = R^T sino
//  EPI_DUAL: y = dy, z = dz; partials = |R^T sino + D^T dy + dz|^2; h (if set) += R^T sino;
//            with step_x set also the iteration's last CG step, x += alpha step_p and
//            h -= alpha step_rtrp (alpha = scal[S_ALPHA]), and u += h (the dual update
//            of u^a in R^T form, its rescale by kappa left to the next right-hand side)
// Every kernel takes its per-slice arguments either by value (BATCH = false: one
// slice) or as a device array indexed by blockIdx.z (BATCH = true: several
// slices of one shape in one launch).  The array is read word by word through
// the constant address space, so the block-uniform loads go through the scalar
// unit into SGPRs, as a by-value argument does.  The single-slice kernels are
// separate instantiations that never touch the array.
template <bool BATCH, typename A>
__device__ inline A pick_args(const A* __restrict__ dev, const A& one, unsigned slice) {
    static_assert(sizeof(A) % 4 == 0 && alignof(A) >= 4, "argument blocks are whole words");
    if constexpr (!BATCH) {
        return one;
    } else {
        using CW = const __attribute__((address_space(4))) uint32_t;
        CW* src = (CW*)(dev + slice);
        A out;
        uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
        for (unsigned k = 0; k < sizeof(A) / 4; ++k) dst[k] = src[k];
        return out;
    }
}

template <bool BATCH, typename A>
__device__ inline A pick_args(const A* __restrict__ dev, const A& one) {
    return pick_args<BATCH>(dev, one, blockIdx.z);
}

// Workgroups of a batched launch of n slices of T workgroups each, dealt so that every
// XCD takes an equal, contiguous share of the slice-major sequence of the n T
// workgroups: the dispatcher deals consecutive workgroup ids to the kXcds XCDs in
// turn, so id = XCD + kXcds k, and XCD x takes sequence positions x P + k, with
// P = ceil(n T / kXcds).  A slice's workgroups then run on as few XCDs as that balance
// allows (on one when n is a multiple of kXcds, on about kXcds / n when n < kXcds), so
// its data passes through few L2s and no XCD idles.  Returns false for the padding
// workgroups past the n T of the sequence.
__device__ inline bool xcd_slice_tile(unsigned id, unsigned T, unsigned n, unsigned& slice,
                                      unsigned& tile) {
    const unsigned P = (n * T + kXcds - 1) / kXcds;
    const unsigned g = (id % kXcds) * P + id / kXcds;
    slice = g / T;
    tile = g % T;
    return g < n * T;
}
__host__ __device__ inline unsigned xcd_slice_blocks(unsigned T, unsigned n) {
    return kXcds * ((n * T + kXcds - 1) / kXcds);
}

template <typename T>
struct OrbitArgs {
    const T* X;   // [ny][nx][ch]
    T* O;         // orbit image [ny][nx][ch * sym]
    T* OT;        // its transpose [nx][ny][ch * sym]
    int nx, ny;
};

template <typename T>
struct ProjArgs {
    const RayParam<T>* rays;
    const T* O;
    const T* OT;
    T* sino;
    int nx, ny, Vb, D;
    int views, chunk;  // base views per wave (a power of two) and bin groups per XCD turn
};

// Fixed-order reductions of block partials and the scalar updates (one block per
// slice, or the last workgroup of a transpose).  scal == nullptr marks an empty slot.
enum RedMode : int { RED_NONE = 0, RED_ALPHA = 1, RED_BETA = 2, RED_FINAL = 3 };

struct RedArgs {
    const double* tiles;
    int nb_tiles;
    const double* img;
    int nb_img;
    const double* sino;
    int nb_sino;
    const double* pre;   // preconditioner partials (r . z), used for gamma with PCG
    int nb_pre;
    int precond;
    double* scal;
    double* log;
    int rho_mode;
    int dual;  // dual-residual partials present
    double bal_mu, bal_tau, next_rho_c, next_rho_p;
};

template <typename T>
struct BpArgs {
    const RayParam<T>* rays;
    const BpRay<T>* brays;
    const ViewParam<T>* views;
    int nx, ny, V, Vb, D;
    int gx, gy;   // this slice's grid of 8x8 orbit blocks
    double margin;
    const T* sino;
    T* out;
    T* out2;
    const T* x;
    const T* y;
    const T* uy;
    const T* z;
    const T* uz;
    double* partials;
    // Tracked right-hand side: h = R^T (a - R x), u = R^T u^a (double [N][2]);
    // raw: the plain R^T of the gathered sinogram ([N][2]) before any image term;
    // part_img: per-256-pixel partials of the right-hand-side kernel.
    double* h;
    double* u;
    T* raw;
    double* part_img;
    // The ADMM's device scalars (kappa for EPI_RHS; alpha for EPI_DUAL's CG step) and
    // the last CG step EPI_DUAL applies: x, the direction p and R^T R p (x == nullptr:
    // no step).
    const double* scal;
    T* step_x;
    const T* step_p;
    const T* step_rtrp;
};

// a * b rounded by itself: never contracted with a neighbouring add into one fma, so
// that a value scaled on the fly rounds exactly as the same value scaled and stored.
__device__ inline float mul_rn(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ inline double mul_rn(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

// Deterministic sum of K doubles over a 256-thread block (fixed shuffle and LDS
// order); thread 0 stores the K sums at out.  Every thread of the block must call it.
template <int K>
__device__ inline void block_sum_store(double (&v)[K], double* out) {
    __shared__ double sh[4][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[wid][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
}

// Fixed-order sum of K slots over nb block partials (kPartialSlots doubles each); the
// result reaches all threads.  The order is that of 256 summing threads whatever the
// block size (any multiple of 64 of at least 128; every thread must call it):
// summing thread t adds partials t, t + 256, ... in that order, the loads of 8 of them
// issued before they are added, so it waits on memory once per 8 partials; each wave
// of summing threads then adds its 64 sums by a fixed shuffle tree and the four wave
// sums are added pairwise.  A block of 128 threads runs two summing threads per
// thread, a block of 512 leaves its upper half idle.
template <int K>
__device__ inline void partial_sum(const double* __restrict__ base, int nb, double (&out)[K]) {
    __shared__ double sh[4][K];
    __shared__ double res[K];
    constexpr int NT = 256, U = 8;
    for (int t = threadIdx.x; t < NT; t += blockDim.x) {  // uniform over each wave
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = 0.0;
        int b = t;
        for (; b + (U - 1) * NT < nb; b += U * NT) {
            double w[U][K];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < K; ++k) w[u][k] = base[(size_t)(b + u * NT) * kPartialSlots + k];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] += w[u][k];
        }
        for (; b < nb; b += NT)
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] += base[(size_t)b * kPartialSlots + k];
#pragma unroll
        for (int k = 0; k < K; ++k)
            for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
        if ((t & 63) == 0)
#pragma unroll
            for (int k = 0; k < K; ++k) sh[t >> 6][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) res[k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = res[k];
    __syncthreads();
}

// partial_sum of up to three arrays in one sweep (the loads of all of them in flight
// together), each summed in exactly the order partial_sum gives it: summing thread t
// adds the partials t, t + 256, ... of every array in increasing order (an array
// shorter than the longest adds zeros past its end, which leaves its sum unchanged).
// An unused array passes nb = 0 and reads as zeros.
template <int K0, int K1, int K2>
__device__ inline void partial_sums(const double* __restrict__ b0, int n0, double (&o0)[K0],
                                    const double* __restrict__ b1, int n1, double (&o1)[K1],
                                    const double* __restrict__ b2, int n2, double (&o2)[K2]) {
    constexpr int K = K0 + K1 + K2;
    __shared__ double sh[4][K];
    __shared__ double res[K];
    constexpr int NT = 256, U = 8;
    const int nmax = max(n0, max(n1, n2));
    for (int t = threadIdx.x; t < NT; t += blockDim.x) {  // uniform over each wave
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = 0.0;
        for (int b = t; b < nmax; b += U * NT) {
            double w[U][K];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t e = (size_t)(b + u * NT);
#pragma unroll
                for (int k = 0; k < K0; ++k)
                    w[u][k] = b + u * NT < n0 ? b0[e * kPartialSlots + k] : 0.0;
#pragma unroll
                for (int k = 0; k < K1; ++k)
                    w[u][K0 + k] = b + u * NT < n1 ? b1[e * kPartialSlots + k] : 0.0;
#pragma unroll
                for (int k = 0; k < K2; ++k)
                    w[u][K0 + K1 + k] = b + u * NT < n2 ? b2[e * kPartialSlots + k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] += w[u][k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
        if ((t & 63) == 0)
#pragma unroll
            for (int k = 0; k < K; ++k) sh[t >> 6][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) res[k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K0; ++k) o0[k] = res[k];
#pragma unroll
    for (int k = 0; k < K1; ++k) o1[k] = res[K0 + k];
#pragma unroll
    for (int k = 0; k < K2; ++k) o2[k] = res[K0 + K1 + k];
    __syncthreads();
}

template <typename T>
hipError_t launch_project(const dect_plan* p, const void* img, void* sino, int ch, hipStream_t s);
// Two-channel projection of the ADMM direction into quad-interleaved records, for
// one slice (dev == nullptr: `one`) or n slices (dev: device arrays); the grid is
// (gx, gy) projector blocks of `waves` (2, 4 or 8) waves splitting the lines, and
// `pixels` orbit-image threads per slice.  orbit = false: the orbit images are
// already in place (written by launch_rhs_orbit) and only the projector runs.
template <typename T>
hipError_t launch_project_pair(int sym, int waves, const OrbitArgs<T>* odev,
                               const OrbitArgs<T>& oone, const ProjArgs<T>* pdev,
                               const ProjArgs<T>& pone, int n, long pixels, int gx, int gy,
                               hipStream_t s, bool orbit = true);
// The CG right-hand side (as the right-hand-side kernel: r0 into rhs.out and rhs.out2,
// partials of |r0|^2 per 256 pixels into rhs.part_img) and, in the same launch, the
// orbit images of r0 into orb.O and orb.OT, for quarter-turn symmetric square slices
// of side n with n % 16 == 0 (rhs_orbit_fits); one slice or nsl slices in dev arrays.
__host__ __device__ inline bool rhs_orbit_fits(int sym, int nx, int ny) {
    return sym == 4 && nx == ny && nx >= 16 && nx % 16 == 0;
}
template <typename T>
hipError_t launch_rhs_orbit(const BpArgs<T>* dev, const BpArgs<T>& one, const OrbitArgs<T>* odev,
                            const OrbitArgs<T>& oone, int nsl, hipStream_t s);
// Plain R^T of a standard-order sinogram with ch channels (one slice).
template <typename T>
hipError_t launch_backproject(const dect_plan* p, int ch, const BpArgs<T>& a, hipStream_t s);
// ADMM epilogue variants of R^T on quad records, one or n slices; `waves` (2, 4
// or 8) split the views of a workgroup.  sums64: keep the sums in double precision
// (the products of an FP32 plan are exact in double; the result is rounded once).
template <typename T>
hipError_t launch_backproject_admm(int sym, int waves, int epi, const BpArgs<T>* dev,
                                   const BpArgs<T>& one, int n, int gx, int gy, hipStream_t s,
                                   bool sums64 = false);
// Fill the plan-dependent fields of BpArgs.
template <typename T>
void fill_bp_plan(const dect_plan* p, BpArgs<T>& a);

// Per-ray decomposition.  mode 0: standalone call; 1: ADMM initialisation; 2: ADMM a-step;
// 3: constrained decomposition (a >= 0, no rho terms) from the projected linearised start.
template <typename T>
struct TvArgs {
    int nx, ny;
    const T* x;
    T* y;
    T* uy;
    T* dy;
    T* z;
    T* uz;
    T* dz;
    const double* scal;
    double* partials;
    // The pending last CG step (x + alpha p, alpha = scal[S_ALPHA]), which the dual
    // transpose's epilogue stores after this launch: the TV update reads x through it.
    // step_p == nullptr: none (x is current).
    const T* step_p;
};

template <typename T>
struct UdmArgs {
    const T* spec;     // spectral tables (plan)
    int kmax, kh, kl;
    float kc_max, kp_max;
    const T* joint;    // both spectra on one energy grid (plan; see dect_plan::joint)
    int jb, jh, jl;
    float joint_lim;
    float jkc[2], jkp[2];  // smallest and largest kc, kp of the joint table
    long M;
    int sym, Vb, D;  // internal (quad) ray order of t, da, Rp; sym = 1: standard order
    const T* mh;
    const T* ml;
    const T* wh;
    const T* wl;
    T* a;          // [M][2] in/out
    const T* v;    // [M][2] standalone proximal centre or nullptr
    T* cost;       // standalone: final Phi per ray, or nullptr
    // ADMM a-step extras
    T* ua;         // [M][2]
    T* Rx;         // [M][2], updated with alpha * Rp
    const T* Rp;   // [M][2]
    T* t;          // [M][2] next right-hand side a + u^a - R x, or nullptr (not kept)
    T* da;         // [M][2] a - a_prev
    T* fg;         // [M][8] f_h, f_l, grad f_h, grad f_l at the current a (internal order)
    uint8_t* lmbits;  // ADMM a-step: [M] accept decisions of its LM iterations, or nullptr
    const double* scal;  // device scalars (rho, alpha)
    double* partials;
    double rho_c, rho_p;  // standalone/init penalties
    int iters;
    double mu0;
    double lin[4];       // inverse of the linearisation matrix (init)
    // ADMM a-step: blocks from udm_blocks on run the TV/z/dual update of the image
    // (independent of the a-update) in the same launch; tv.x = nullptr: none.
    int udm_blocks;
    TvArgs<T> tv;
};

template <typename T>
void fill_udm_tables(const dect_plan* p, UdmArgs<T>& a);
// p: plan whose spectral tables are filled into a (nullptr: a carries them).
template <typename T>
hipError_t launch_udm(const dect_plan* p, int mode, const UdmArgs<T>& a, hipStream_t s);
// Batched a-step over n slices (args: device array), grid of `blocks` x n; joint: every
// slice's plan has a joint spectral table (joint_lim > 0).
template <typename T>
hipError_t launch_udm_batch(const UdmArgs<T>* args, int n, int blocks, bool joint, hipStream_t s);
// Preconditioner z = M r of the x-update (ramp filter by 2-D FFT, both bases as one
// complex image); partials: r . z per basis, one block per image row.
template <typename T>
struct PrecArgs {
    int nx, ny, px, py, lpx, lpy;  // image and padded grid (px = 2^lpx, py = 2^lpy)
    const T* filter;               // [py][px]
    const T* twx;                  // [px/2][2]
    const T* twy;                  // [py/2][2]
    T* W;                          // [ny][px][2] work grid
    const T* r;                    // [ny][nx][2]
    T* z;                          // [ny][nx][2]
    double* partials;
};

template <typename T>
void fill_precond_plan(const dect_plan* p, PrecArgs<T>& a);
template <typename T>
hipError_t launch_precond(const PrecArgs<T>* dev, const PrecArgs<T>& one, int n, hipStream_t s);

// Image-vector CG steps: x += alpha p, r -= alpha q, p = zp + beta p, R x += alpha R p
// (zp = r for CG, the preconditioned residual for PCG).
template <typename T>
struct VecArgs {
    long N, M;
    int sym, Vb, D;
    T* x;
    T* p;
    T* r;
    const T* zp;
    const T* q;
    T* Rx;
    const T* Rp;
    double* scal;       // device scalars; the last CG step of an iteration stores alpha
    double* partials;   // image partials
    double* h;          // tracked R^T (a - R x): minus alpha R^T R p per CG step
    const T* rtrp;      // R^T R p of the current CG step
    // Block partials of r . z (r . r without the preconditioner) and of p . q, from
    // which the last CG step of an iteration forms alpha itself.
    const double* g_part;
    int nb_g;
    const double* pq_part;
    int nb_pq;
};

// Shrinkage, nonnegativity and the y, z duals (Eq. (9)-(11)).

// The dual rescale after a change of rho, kappa = rho_old / rho_new, which the
// iterations leave pending (every reader of u, u^a, u^y, u^z scales by it on the fly
// and the next right-hand side, a-update and TV update store the scaled values):
// applied to all four at the end of a call, then kappa = 1.
template <typename T>
struct RescaleArgs {
    long M, N;
    T* ua;
    T* uy;
    T* uz;
    double* u;  // R^T u^a
    double* scal;
};

// Every argument block of one slice's outer iteration, and its launch extents.
template <typename T>
struct SliceJob {
    OrbitArgs<T> orb;
    ProjArgs<T> prj;
    BpArgs<T> rhs, q, dual;
    UdmArgs<T> udm;
    VecArgs<T> vec;
    TvArgs<T> tv;
    RescaleArgs<T> resc;
    RedArgs red;
    PrecArgs<T> pre0, pre1;  // PCG: z0 = M r0 into p; z = M r into the z buffer
    int precond;
    long N, M;
    int sym, bp_gx, bp_gy, pj_gx, pj_gy;
    int bp_waves, pj_waves;  // workgroup shapes of the plan
    int pj_views, pj_chunk;  // projector lane layout and workgroup order of the plan
    int cg_iters, rho_mode;  // launch structure: slices share launches only if these agree
    int rt_sums64;           // the ADMM transposes sum in double (dect_rt_sums)
};

// Device copies of the argument blocks of n slices of one shape, in slice order.
template <typename T>
struct JobArrays {
    OrbitArgs<T>* orb;
    ProjArgs<T>* prj;
    BpArgs<T>* rhs;
    BpArgs<T>* q;
    BpArgs<T>* dual;
    UdmArgs<T>* udm;
    VecArgs<T>* vec;
    RescaleArgs<T>* resc;
    RedArgs* red;
    PrecArgs<T>* pre0;
    PrecArgs<T>* pre1;
};

// The argument blocks of one slice for its plan, measurements and state.
template <typename T>
SliceJob<T> make_job(const dect_plan* p, const void* mh, const void* ml, const void* wh,
                     const void* wl, void* st, const dect_params* prm);
// Enqueue one outer iteration on s: of `one` (dev == nullptr) or of n slices of the
// same shape as `one` whose argument blocks are in dev.  it: iteration index (for
// a rho schedule, single slice only).
template <typename T>
hipError_t launch_iteration(const SliceJob<T>& one, const JobArrays<T>* dev, int n,
                            const dect_params* prm, long it, hipStream_t s);
// The pending dual rescale of `one` or of n slices in dev applied to the state's
// arrays (RescaleArgs), so that they hold the scaled duals between calls.
template <typename T>
hipError_t launch_settle(const SliceJob<T>& one, const JobArrays<T>* dev, int n, hipStream_t s);

// f and its gradient of both spectra at (R x_c, R x_p) for the LM x CG scheme, with
// `at` the basis' projection and `ao` the other one's; cache [6][M]; partials: data
// cost and non-finite count per block of 256 rays.
template <typename T>
hipError_t launch_lm_eval(const dect_plan* p, int basis, const T* at, const T* ao, const T* mh,
                          const T* ml, const T* wh, const T* wl, T* cache, double* partials,
                          hipStream_t s);

// The tracked right-hand side of a state whose t (= a + u^a - R x, internal ray order)
// and zero u^a, dy, dz were just set: h = R^T t, by one transpose (sums64: summed in
// double precision, as the iterations' transposes with dect_rt_sums F64).
template <typename T>
hipError_t launch_track_init(const dect_plan* p, void* state, hipStream_t s, bool sums64);

// Start of the iterations from an image pair x0: x = z = x0, y = D x0, R x = R x0,
// t = a - R x0 and h = R^T t (the state already initialised with x = 0).
template <typename T>
hipError_t launch_init_image(const dect_plan* p, const void* x0, void* state, hipStream_t s,
                             bool sums64);

template <typename T>
hipError_t launch_ingest(const dect_plan* p, const void* ch, const void* cl, double i0h,
                         double i0l, void* mh, void* ml, void* wh, void* wl, hipStream_t s);

}  // namespace dect
