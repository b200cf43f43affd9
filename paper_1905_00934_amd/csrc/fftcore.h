// Radix-2 FFTs in LDS shared by the preconditioner and the FBP filter.
#pragma once

#include "common.h"

namespace dect {

template <typename T>
struct cx {
    T re, im;
};

__device__ inline int bitrev(int i, int lg) { return (int)(__brev((unsigned)i) >> (32 - lg)); }

// In-place FFTs of `count` sequences of length 2^lg stored back to back in buf,
// each in bit-reversed order on entry and natural order on exit, with the
// twiddles tw[k] = exp(-2 pi i k / 2^lg), k < 2^(lg-1), as (cos, sin) pairs.
// inverse: the conjugate twiddles (no 1/P factor).  Every thread of the block
// must call it.
//
// Radix-2 decimation in time; two consecutive stages (butterfly distances m and
// 2m) are done in registers on groups of four elements (i, i + m, i + 2m, i + 3m),
// with the same operations as the two separate stages, so each pair of stages
// costs one LDS pass and one barrier.  An odd lg starts with one single stage.
template <typename T>
__device__ inline cx<T> twiddled(const T* __restrict__ tw, int k, bool inverse, cx<T> c) {
    const T wr = tw[2 * k];
    const T wi = inverse ? -tw[2 * k + 1] : tw[2 * k + 1];
    return cx<T>{wr * c.re - wi * c.im, wr * c.im + wi * c.re};
}

template <typename T>
__device__ inline void fft_lds(cx<T>* buf, int count, int lg, const T* __restrict__ tw,
                               bool inverse) {
    int s = 0;
    if (lg & 1) {
        __syncthreads();
        const int half = 1 << (lg - 1);
        for (int t = threadIdx.x; t < count * half; t += blockDim.x) {
            cx<T>* x = buf + ((size_t)(t >> (lg - 1)) << lg);
            const int i0 = 2 * (t & (half - 1));
            const cx<T> a = x[i0], b = twiddled(tw, 0, inverse, x[i0 + 1]);
            x[i0] = cx<T>{a.re + b.re, a.im + b.im};
            x[i0 + 1] = cx<T>{a.re - b.re, a.im - b.im};
        }
        s = 1;
    }
    const int quarter = lg >= 2 ? 1 << (lg - 2) : 0;
    for (; s + 1 < lg; s += 2) {
        __syncthreads();
        const int m = 1 << s;
        const int t1 = lg - 1 - s, t2 = lg - 2 - s;  // twiddle index shifts of the two stages
        for (int t = threadIdx.x; t < count * quarter; t += blockDim.x) {
            cx<T>* x = buf + ((size_t)(t >> (lg - 2)) << lg);
            const int b = t & (quarter - 1);
            const int j = b & (m - 1);
            const int i0 = ((b >> s) << (s + 2)) + j;
            const cx<T> x0 = x[i0], x1 = x[i0 + m], x2 = x[i0 + 2 * m], x3 = x[i0 + 3 * m];
            // Stage s: pairs (x0, x1) and (x2, x3), both at position j.
            const cx<T> w1 = twiddled(tw, j << t1, inverse, x1);
            const cx<T> w3 = twiddled(tw, j << t1, inverse, x3);
            const cx<T> y0{x0.re + w1.re, x0.im + w1.im}, y1{x0.re - w1.re, x0.im - w1.im};
            const cx<T> y2{x2.re + w3.re, x2.im + w3.im}, y3{x2.re - w3.re, x2.im - w3.im};
            // Stage s + 1: pairs (y0, y2) at position j and (y1, y3) at j + m.
            const cx<T> v2 = twiddled(tw, j << t2, inverse, y2);
            const cx<T> v3 = twiddled(tw, (j + m) << t2, inverse, y3);
            x[i0] = cx<T>{y0.re + v2.re, y0.im + v2.im};
            x[i0 + 2 * m] = cx<T>{y0.re - v2.re, y0.im - v2.im};
            x[i0 + m] = cx<T>{y1.re + v3.re, y1.im + v3.im};
            x[i0 + 3 * m] = cx<T>{y1.re - v3.re, y1.im - v3.im};
        }
    }
    __syncthreads();
}

}  // namespace dect
