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
template <typename T>
__device__ inline void fft_lds(cx<T>* buf, int count, int lg, const T* __restrict__ tw,
                               bool inverse) {
    const int half = 1 << (lg - 1);
    for (int s = 0; s < lg; ++s) {
        __syncthreads();
        const int m = 1 << s;
        const int ts = lg - 1 - s;  // twiddle index = pos * P / (2m)
        for (int t = threadIdx.x; t < count * half; t += blockDim.x) {
            const int seq = t >> (lg - 1), b = t & (half - 1);
            const int pos = b & (m - 1);
            const int i0 = ((b >> s) << (s + 1)) + pos, i1 = i0 + m;
            const T wr = tw[2 * (pos << ts)];
            const T wi = inverse ? -tw[2 * (pos << ts) + 1] : tw[2 * (pos << ts) + 1];
            cx<T>* x = buf + ((size_t)seq << lg);
            const cx<T> a = x[i0], c = x[i1];
            const T br = wr * c.re - wi * c.im, bi = wr * c.im + wi * c.re;
            x[i0] = cx<T>{a.re + br, a.im + bi};
            x[i1] = cx<T>{a.re - br, a.im - bi};
        }
    }
    __syncthreads();
}

}  // namespace dect
