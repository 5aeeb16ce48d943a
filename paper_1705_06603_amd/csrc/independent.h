// The paper's independent baseline (Section IV, compared methods): every
// tile deblurred on its own, without the consensus step, and the tiles
// blended with the weights omega only in the output (k_assemble).  Run as
// Algorithm 1 with the consensus step replaced by u_t <- x_t, each tile's
// iteration is the proximal-point method on its own f_t, whose limit is
// argmin f_t.
#pragma once

#include "kernels.h"

namespace dbl {

constexpr int kIndThreads = 256;

// u <- x on every support pixel, with per-block partial sums of
// ||x - u||^2 and ||x||^2 (the residual ||u_new - u_old|| / ||u_new||).
// Blocks stride over the (tile, support row) pairs.
__global__ __launch_bounds__(kIndThreads) void k_independent(const float* __restrict__ x, float* __restrict__ u,
                                                            const TileInfo* __restrict__ tiles, int N, int n_tiles,
                                                            float2* __restrict__ part) {
    __shared__ double sa[kIndThreads], sb[kIndThreads];
    double a = 0.0, b = 0.0;
    for (int tr = blockIdx.x; tr < n_tiles * N; tr += gridDim.x) {
        const int t = tr / N, i = tr - t * N;
        const TileInfo ti = tiles[t];
        if (i >= ti.sy) continue;
        const size_t row = (size_t)t * N * N + (size_t)i * N;
        for (int c = threadIdx.x; c < ti.sx; c += kIndThreads) {
            const float xv = x[row + c];
            const float d = xv - u[row + c];
            a += (double)d * d;
            b += (double)xv * xv;
            u[row + c] = xv;
        }
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int o = kIndThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sb[threadIdx.x] += sb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_float2((float)sa[0], (float)sb[0]);
}

}  // namespace dbl
