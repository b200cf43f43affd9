// Kernel launchers shared by the library's translation units.
#pragma once

#include "common.h"

namespace dect {

enum Epilogue : int { EPI_NONE = 0, EPI_RHS = 1, EPI_Q = 2, EPI_DUAL = 3 };

// Arguments of the transposed projector and its image-side epilogues.
//  EPI_NONE: out = R^T sino (ch channels)
//  EPI_RHS : out (and out2 if set) = R^T sino + D^T (y + uy - D x) + (z + uz - x);
//            partials = per-channel |out|^2
//  EPI_Q   : out (if set) = R^T sino + D^T D x + x, with x = p; partials = p . out
//  EPI_DUAL: y = dy, z = dz; partials = |R^T sino + D^T dy + dz|^2
template <typename T>
struct BpArgs {
    const RayParam<T>* rays;
    const ViewParam<T>* views;
    int nx, ny, V, Vb, D;
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
};

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

template <typename T>
hipError_t launch_project(const dect_plan* p, const void* img, void* sino, int ch, hipStream_t s);
// Two-channel projection of the ADMM direction into quad-interleaved records;
// O and OT are orbit-image scratch of N * 2 * sym elements each.
template <typename T>
hipError_t launch_project_pair(const dect_plan* p, const void* img, void* O, void* OT,
                               void* sino, hipStream_t s);
template <typename T>
hipError_t launch_backproject(const dect_plan* p, int ch, int epi, const BpArgs<T>& a,
                              hipStream_t s);

// Per-ray decomposition.  mode 0: standalone call; 1: ADMM initialisation; 2: ADMM a-step.
template <typename T>
struct UdmArgs {
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
    T* t;          // [M][2] next right-hand side a + u^a - R x
    T* da;         // [M][2] a - a_prev
    T* fg;         // [M][8] f_h, f_l, grad f_h, grad f_l at the current a (internal order)
    const double* scal;  // device scalars (rho, alpha)
    double* partials;
    double rho_c, rho_p;  // standalone/init penalties
    int iters;
    double mu0;
    double lin[4];       // inverse of the linearisation matrix (init)
};

template <typename T>
hipError_t launch_udm(const dect_plan* p, int mode, const UdmArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_ingest(const dect_plan* p, const void* ch, const void* cl, double i0h,
                         double i0l, void* mh, void* ml, void* wh, void* wl, hipStream_t s);

}  // namespace dect
