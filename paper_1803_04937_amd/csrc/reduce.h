// Deterministic block reductions in FP64 (fixed thread-to-value mapping, fixed
// shuffle tree), used for mass / momentum totals, objectives and parameter
// gradients.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

constexpr int kWaves = kBlock / 64;

// Sum (MAX = false) or max of N values over the block; thread 0 writes the
// block's results to out[0..N).  Every thread of the block must call it.
template <int N, bool MAX = false>
__device__ __forceinline__ void block_reduce(double (&v)[N], double *out) {
    __shared__ double sh[N][kWaves];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double y = __shfl_down(x, off, 64);
            x = MAX ? fmax(x, y) : x + y;
        }
        v[k] = x;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) sh[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double r = sh[k][0];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) r = MAX ? fmax(r, sh[k][w]) : r + sh[k][w];
            out[k] = r;
        }
    }
}

}  // namespace lbm
