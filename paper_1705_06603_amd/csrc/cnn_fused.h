// Fused forward pass of the warm-start network: conv1 -> conv2 -> conv3 ->
// conv4 (+ residual) of one output tile in one workgroup, with the 32-channel
// activations in LDS only.  The same arithmetic as the layer-by-layer kernels
// of cnn.h (bf16 rounding at the same points, the same MFMA sequence for the
// 32 -> 32 layers, the same summation order for layers 1 and 4).
//
// A workgroup computes a kTile x kTile block of outputs.  Each 3 x 3 layer
// needs one more pixel of halo, so, around the output block:
//   x   on (kTile + 8)^2  (staged as bf16-rounded fp32, aliasing buffer B)
//   a1  on (kTile + 6)^2  (buffer A)
//   a2  on (kTile + 4)^2  (buffer B)
//   a3  on (kTile + 2)^2  (buffer A again: a1 is dead by then)
// kTile = 28 makes the a2 rows exactly two 16-pixel MFMA row chunks and the
// two buffers 139.5 KB together, one workgroup per CU (160 KB LDS).  Pixels
// outside an image's valid region are zero in every layer (zero padding).
#pragma once

#include "cnn.h"

namespace dbl {
namespace cnn {

constexpr int kTile = 28;
constexpr int kR1 = kTile + 6;            // a1 region side (34)
constexpr int kR2 = kTile + 4;            // a2 region side (32)
constexpr int kR3 = kTile + 2;            // a3 region side (30)
constexpr int kR0 = kTile + 8;            // x region side (36)
constexpr int kFusedThreads = 512;        // 8 waves
constexpr int kBufA = kR1 * kR1 * C;      // bf16 values (a1, later a3)
constexpr int kBufB = kR2 * kR2 * C;      // bf16 values (a2; x staging before)
static_assert(kR2 == 32, "a2 rows must be two 16-pixel chunks");
static_assert(kR3 * kR3 * C <= kBufA, "a3 must fit where a1 was");
static_assert(kR0 * kR0 * 2 <= kBufB, "the x staging must fit in buffer B");

// A operands of one input row for the three horizontal taps of a 16-pixel
// output chunk (output pixel c0 + l reads input columns c0 + l + dx): each
// lane reads its centre column c0 + l + 1 from LDS, the taps dx = 0 and 2 are
// that fragment shifted by one lane inside each 16-lane row (DPP), and the
// edge lanes (l = 0 for dx = 0, l = 15 for dx = 2) read their own column.
// Columns past the region's last one are clamped into it: only lanes whose
// output is discarded read them.
struct RowOps {
    uint4 a[3];
};

__device__ __forceinline__ RowOps row_ops(const unsigned short* __restrict__ rowp, int cc, int ce, int li) {
    RowOps o;
    const uint4 cen = *reinterpret_cast<const uint4*>(rowp + cc * C);
    uint4 edg = make_uint4(0, 0, 0, 0);
    if (li == 0 || li == 15) edg = *reinterpret_cast<const uint4*>(rowp + ce * C);
    const uint4 sl = dpp_row_shift(cen, true);    // lane l gets lane l - 1
    const uint4 sr = dpp_row_shift(cen, false);   // lane l gets lane l + 1
    o.a[0] = li == 0 ? edg : sl;
    o.a[1] = cen;
    o.a[2] = li == 15 ? edg : sr;
    return o;
}

// One 16-pixel x 32-channel output chunk from the operands of its three input
// rows, taps in the order t = 3 dy + dx (the order of the layer-by-layer
// kernel, so the sums round identically).
__device__ __forceinline__ void mid_chunk(const RowOps& r0, const RowOps& r1, const RowOps& r2,
                                          const uint4 (&bw0)[9], const uint4 (&bw1)[9], f32x4& acc0, f32x4& acc1) {
    acc0 = f32x4{0.f, 0.f, 0.f, 0.f};
    acc1 = f32x4{0.f, 0.f, 0.f, 0.f};
    const RowOps* rows[3] = {&r0, &r1, &r2};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const bf16x8 Aop = __builtin_bit_cast(bf16x8, rows[t / 3]->a[t % 3]);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop, __builtin_bit_cast(bf16x8, bw0[t]), acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop, __builtin_bit_cast(bf16x8, bw1[t]), acc1, 0, 0, 0);
    }
}

__global__ __launch_bounds__(kFusedThreads) void k_cnn_fwd(const float* __restrict__ x,
                                                          const ImgDesc* __restrict__ desc, int H, int W,
                                                          const float* __restrict__ w1,
                                                          const unsigned short* __restrict__ wf2,
                                                          const unsigned short* __restrict__ wf3,
                                                          const float* __restrict__ w4,
                                                          const float* __restrict__ master,
                                                          float* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) unsigned short bufA[kBufA];
    __shared__ __attribute__((aligned(16))) unsigned short bufB[kBufB];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int b = blockIdx.z, Y0 = blockIdx.y * kTile, X0 = blockIdx.x * kTile;
    const ImgDesc d = desc[b];
    const float* xi = x + (size_t)b * H * W;
    float* oi = out + (size_t)b * H * W;
    if (Y0 >= d.vh || X0 >= d.vw) {   // no valid output in this block: zeros (uniform per workgroup)
        for (int e = tid; e < kTile * kTile; e += kFusedThreads) {
            const int y = Y0 + e / kTile, xx = X0 + e % kTile;
            if (y < H && xx < W) oi[(size_t)y * W + xx] = 0.f;
        }
        return;
    }
    // x region (bf16-rounded, 0 outside the valid region) into buffer B
    float* xs = reinterpret_cast<float*>(bufB);
    for (int e = tid; e < kR0 * kR0; e += kFusedThreads) {
        const int y = Y0 - 4 + e / kR0, xx = X0 - 4 + e % kR0;
        xs[e] = inside(d, y, xx) ? bf2f(f2bf(xi[(size_t)y * W + xx])) : 0.f;
    }
    __syncthreads();
    // layer 1: a1 = bf16(relu(b1 + sum_t w1[t] x)) on the a1 region
    // the weights of layers 1 and 4 are read from global memory at addresses
    // uniform across the workgroup, so they come in through the scalar cache
    // as SGPR operands
    const float* __restrict__ b1 = master + kB1;
    for (int e = tid; e < kR1 * kR1; e += kFusedThreads) {
        const int r = e / kR1, cc = e % kR1;
        unsigned int* o = reinterpret_cast<unsigned int*>(bufA + e * C);
        if (!inside(d, Y0 - 3 + r, X0 - 3 + cc)) {
            for (int q = 0; q < C / 2; ++q) o[q] = 0u;
            continue;
        }
        float in[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) in[t] = xs[(r + t / 3) * kR0 + cc + t % 3];
#pragma unroll 4
        for (int co = 0; co < C; co += 2) {
            float s0 = b1[co], s1 = b1[co + 1];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                s0 += w1[t * C + co] * in[t];
                s1 += w1[t * C + co + 1] * in[t];
            }
            o[co / 2] = (unsigned int)f2bf(fmaxf(s0, 0.f)) | ((unsigned int)f2bf(fmaxf(s1, 0.f)) << 16);
        }
    }
    __syncthreads();
    // layers 2 and 3 on MFMA: a2 (32 x 32, from a1 in A into B), a3 (30 x 30, from a2 in B into A)
    for (int layer = 0; layer < 2; ++layer) {
        const unsigned short* wq = layer == 0 ? wf2 : wf3;
        const float* bias = master + (layer == 0 ? kB2 : kB3);
        uint4 bw0[9], bw1[9];
        const uint4* wv = reinterpret_cast<const uint4*>(wq);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            bw0[t] = wv[((t * C + li) * C + 8 * lk) / 8];
            bw1[t] = wv[((t * C + 16 + li) * C + 8 * lk) / 8];
        }
        const float b0v = bias[li], b1v = bias[16 + li];
        const unsigned short* src = layer == 0 ? bufA : bufB;
        unsigned short* dst = layer == 0 ? bufB : bufA;
        const int sw = layer == 0 ? kR1 : kR2;        // input region side
        const int side = layer == 0 ? kR2 : kR3;      // output region side
        const int off = layer == 0 ? 2 : 1;           // output region origin: (Y0 - off, X0 - off)
        // wave w: column chunk c0 = 16 (w mod 2) of the output rows of band
        // w / 2 (a quarter of the rows), walked top to bottom with the operands
        // of the three input rows a chunk needs kept in registers, so each
        // input row is read from LDS once per wave
        const int c0 = 16 * (wave & 1), band = wave >> 1;
        const int r_lo = band * side / 4, r_hi = (band + 1) * side / 4;
        const int cc = min(c0 + li + 1, sw - 1);
        const int ce = li == 0 ? c0 : min(c0 + 17, sw - 1);
        const unsigned short* rows = src + 8 * lk;
        auto chunk = [&](int r, const RowOps& q0, const RowOps& q1, const RowOps& q2) {
            f32x4 acc0, acc1;
            mid_chunk(q0, q1, q2, bw0, bw1, acc0, acc1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int cx = c0 + 4 * lk + q;
                if (cx >= side) continue;
                float v0 = fmaxf(acc0[q] + b0v, 0.f), v1 = fmaxf(acc1[q] + b1v, 0.f);
                if (!inside(d, Y0 - off + r, X0 - off + cx)) v0 = v1 = 0.f;
                dst[(r * side + cx) * C + li] = f2bf(v0);
                dst[(r * side + cx) * C + 16 + li] = f2bf(v1);
            }
        };
        RowOps A = row_ops(rows + (size_t)r_lo * sw * C, cc, ce, li);
        RowOps B = row_ops(rows + (size_t)(r_lo + 1) * sw * C, cc, ce, li);
        for (int r = r_lo; r < r_hi; r += 3) {
            RowOps Cn = row_ops(rows + (size_t)(r + 2) * sw * C, cc, ce, li);
            chunk(r, A, B, Cn);
            if (r + 1 >= r_hi) break;
            A = row_ops(rows + (size_t)(r + 3) * sw * C, cc, ce, li);
            chunk(r + 1, B, Cn, A);
            if (r + 2 >= r_hi) break;
            B = row_ops(rows + (size_t)(r + 4) * sw * C, cc, ce, li);
            chunk(r + 2, Cn, A, B);
        }
        __syncthreads();
    }
    // layer 4 and the residual: out = x + b4 + sum_t w4[t] . a3
    for (int e = tid; e < kTile * kTile; e += kFusedThreads) {
        const int r = e / kTile, cc = e % kTile;
        const int y = Y0 + r, xx = X0 + cc;
        if (y >= H || xx >= W) continue;
        if (!inside(d, y, xx)) {
            oi[(size_t)y * W + xx] = 0.f;
            continue;
        }
        float s = master[kB4];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            if (!inside(d, y + t / 3 - 1, xx + t % 3 - 1)) continue;
            const uint4* ap = reinterpret_cast<const uint4*>(bufA + ((r + t / 3) * kR3 + cc + t % 3) * C);
#pragma unroll 2
            for (int q = 0; q < 4; ++q) {
                const uint4 v = ap[q];
                const unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e2 = 0; e2 < 4; ++e2) {
                    const int c = 8 * q + 2 * e2;
                    s += w4[t * C + c] * bf2f((unsigned short)(w[e2] & 0xFFFF)) +
                         w4[t * C + c + 1] * bf2f((unsigned short)(w[e2] >> 16));
                }
            }
        }
        oi[(size_t)y * W + xx] = xi[(size_t)y * W + xx] + s;
    }
}

inline dim3 cnn_fwd_grid(int B, int H, int W) { return dim3((W + kTile - 1) / kTile, (H + kTile - 1) / kTile, B); }

}  // namespace cnn
}  // namespace dbl
