// The preconditioner of the x-update (Sec. 3.3): z = M r with M the ramp filter
// applied by a 2-D FFT on the zero-padded image.
//
// The two bases of an image pair are the real and imaginary parts of one complex
// image (the [ny][nx][2] layout is already complex), and the filter is real and
// even in frequency, so one complex transform filters both: its real part stays
// the filtered c image and its imaginary part the filtered p image.
//
// Three passes over a [ny][px] complex work grid (rows beyond ny of the padded
// grid are zero and never stored):
//   rows:    forward DFT of every image row, zero-padded to px;
//   columns: forward DFT of every column (zero-padded to py), multiply by the
//            filter, inverse DFT, keep the first ny entries;
//   rows:    inverse DFT, keep the first nx entries, scale by 1/(px py); the
//            block partial sums of r . z per basis go to `partials`.
// Each transform is a radix-2 decimation-in-time FFT in LDS on bit-reversed input,
// with the twiddles exp(-2 pi i k / P) from the plan's table.
#include "common.h"
#include "fftcore.h"
#include "kernels.h"
#include "profile.h"

namespace dect {
namespace {

template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_pre_rows_fwd(const PrecArgs<T>* __restrict__ dev,
                                                      PrecArgs<T> one) {
    extern __shared__ char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const PrecArgs<T> A = pick_args<BATCH>(dev, one);
    const int j = blockIdx.x;
    if (j >= A.ny) return;  // beyond this slice (whole block)
    const cx<T>* row = reinterpret_cast<const cx<T>*>(A.r) + (size_t)j * A.nx;
    for (int i = threadIdx.x; i < A.px; i += blockDim.x)
        buf[bitrev(i, A.lpx)] = i < A.nx ? row[i] : cx<T>{T(0), T(0)};
    fft_lds<T>(buf, 1, A.lpx, A.twx, false);
    cx<T>* w = reinterpret_cast<cx<T>*>(A.W) + (size_t)j * A.px;
    for (int i = threadIdx.x; i < A.px; i += blockDim.x) w[i] = buf[i];
}

// Column groups per XCD: workgroups reach the kXcds XCDs in turn, and XCD x takes
// the x-th contiguous range of column groups, so the columns that share a cache
// line of the work grid are read through the same L2.
inline unsigned pre_col_blocks(int groups) {
    return (unsigned)(kXcds * ((groups + kXcds - 1) / kXcds));
}

// C columns per block (C consecutive columns of the work grid).
template <typename T, bool BATCH, int C>
__global__ __launch_bounds__(256) void k_pre_cols(const PrecArgs<T>* __restrict__ dev,
                                                  PrecArgs<T> one) {
    extern __shared__ char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const PrecArgs<T> A = pick_args<BATCH>(dev, one);
    const int groups = (A.px + C - 1) / C, per = (groups + kXcds - 1) / kXcds;
    const int g = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    const int c0 = g * C;
    if (g >= groups) return;  // beyond this slice (whole block)
    const int py = A.py, lg = A.lpy;
    cx<T>* W = reinterpret_cast<cx<T>*>(A.W);
    for (int t = threadIdx.x; t < C * py; t += blockDim.x) {
        const int cc = t % C, j = t / C, c = c0 + cc;
        buf[cc * py + bitrev(j, lg)] =
            (j < A.ny && c < A.px) ? W[(size_t)j * A.px + c] : cx<T>{T(0), T(0)};
    }
    fft_lds<T>(buf, C, lg, A.twy, false);
    // Filter, then back to bit-reversed order for the inverse transform.
    for (int t = threadIdx.x; t < C * py; t += blockDim.x) {
        const int cc = t / py, k = t % py, c = c0 + cc;
        const T f = c < A.px ? A.filter[(size_t)k * A.px + c] : T(0);
        buf[t].re *= f;
        buf[t].im *= f;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < C * py; t += blockDim.x) {
        const int cc = t / py, k = t % py, kr = bitrev(k, lg);
        if (k < kr) {
            const cx<T> a = buf[cc * py + k];
            buf[cc * py + k] = buf[cc * py + kr];
            buf[cc * py + kr] = a;
        }
    }
    fft_lds<T>(buf, C, lg, A.twy, true);
    for (int t = threadIdx.x; t < C * A.ny; t += blockDim.x) {
        const int cc = t % C, j = t / C, c = c0 + cc;
        if (c < A.px) W[(size_t)j * A.px + c] = buf[cc * py + j];
    }
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_pre_rows_inv(const PrecArgs<T>* __restrict__ dev,
                                                      PrecArgs<T> one) {
    extern __shared__ char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const PrecArgs<T> A = pick_args<BATCH>(dev, one);
    const int j = blockIdx.x;
    if (j >= A.ny) return;  // beyond this slice (whole block)
    const cx<T>* w = reinterpret_cast<const cx<T>*>(A.W) + (size_t)j * A.px;
    for (int i = threadIdx.x; i < A.px; i += blockDim.x) buf[bitrev(i, A.lpx)] = w[i];
    fft_lds<T>(buf, 1, A.lpx, A.twx, true);
    const T scale = T(1) / ((T)A.px * (T)A.py);
    const cx<T>* r = reinterpret_cast<const cx<T>*>(A.r) + (size_t)j * A.nx;
    cx<T>* z = reinterpret_cast<cx<T>*>(A.z) + (size_t)j * A.nx;
    double part[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < A.nx; i += blockDim.x) {
        const cx<T> v{buf[i].re * scale, buf[i].im * scale};
        const cx<T> rv = r[i];
        z[i] = v;
        part[0] += (double)rv.re * (double)v.re;
        part[1] += (double)rv.im * (double)v.im;
    }
    block_sum_store<2>(part, A.partials + (size_t)j * kPartialSlots);
}

template <typename T, bool BATCH>
void precond_launch(const PrecArgs<T>* dev, const PrecArgs<T>& one, int n, hipStream_t s) {
    // One column per block: more blocks and smaller LDS measured faster than
    // batching adjacent columns for longer row segments (C = 2, 4, 8).
    constexpr int C = 1;
    const size_t row_lds = (size_t)one.px * sizeof(cx<T>);
    const size_t col_lds = (size_t)C * one.py * sizeof(cx<T>);
    const dim3 rows((unsigned)one.ny, 1, n), cols(pre_col_blocks((one.px + C - 1) / C), 1, n);
    hipLaunchKernelGGL((k_pre_rows_fwd<T, BATCH>), rows, dim3(256), row_lds, s, dev, one);
    hipLaunchKernelGGL((k_pre_cols<T, BATCH, C>), cols, dim3(256), col_lds, s, dev, one);
    hipLaunchKernelGGL((k_pre_rows_inv<T, BATCH>), rows, dim3(256), row_lds, s, dev, one);
}

}  // namespace

template <typename T>
void fill_precond_plan(const dect_plan* p, PrecArgs<T>& a) {
    a.nx = p->nx;
    a.ny = p->ny;
    a.px = p->px;
    a.py = p->py;
    a.lpx = p->lpx;
    a.lpy = p->lpy;
    a.filter = static_cast<const T*>(p->pre_filter);
    a.twx = static_cast<const T*>(p->pre_twx);
    a.twy = static_cast<const T*>(p->pre_twy);
}

template <typename T>
hipError_t launch_precond(const PrecArgs<T>* dev, const PrecArgs<T>& one, int n, hipStream_t s) {
    ProfScope ps("precond", s);
    if (dev)
        precond_launch<T, true>(dev, one, n, s);
    else
        precond_launch<T, false>(dev, one, n, s);
    return hipGetLastError();
}

template void fill_precond_plan<float>(const dect_plan*, PrecArgs<float>&);
template void fill_precond_plan<double>(const dect_plan*, PrecArgs<double>&);
template hipError_t launch_precond<float>(const PrecArgs<float>*, const PrecArgs<float>&, int,
                                          hipStream_t);
template hipError_t launch_precond<double>(const PrecArgs<double>*, const PrecArgs<double>&, int,
                                           hipStream_t);

}  // namespace dect

using namespace dect;

extern "C" {

dect_status dect_precondition(const dect_plan* p, const void* img, void* out, void* stream) {
    if (!p || !img || !out) return fail(DECT_E_ARG, "null argument");
    if (!p->has_precond)
        return fail(DECT_E_SHAPE, "no preconditioner for a %dx%d image (padded side > %d)", p->nx,
                    p->ny, kMaxFft);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (p->dtype == DECT_F32) {
        PrecArgs<float> a{};
        fill_precond_plan<float>(p, a);
        a.W = static_cast<float*>(p->scratch_W);
        a.r = static_cast<const float*>(img);
        a.z = static_cast<float*>(out);
        a.partials = p->scratch_part;
        e = launch_precond<float>(nullptr, a, 1, s);
    } else {
        PrecArgs<double> a{};
        fill_precond_plan<double>(p, a);
        a.W = static_cast<double*>(p->scratch_W);
        a.r = static_cast<const double*>(img);
        a.z = static_cast<double*>(out);
        a.partials = p->scratch_part;
        e = launch_precond<double>(nullptr, a, 1, s);
    }
    if (e != hipSuccess) return fail(DECT_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return DECT_OK;
}

}  // extern "C"
