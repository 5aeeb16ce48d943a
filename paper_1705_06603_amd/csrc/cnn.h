// Warm-start network kernels: 3x3 convolutions 1 -> 32 -> 32 -> 32 -> 1 with
// ReLU and a residual output, BF16 weights and activations with FP32
// accumulation, and their backward pass and Adam update.
//
// Images: [B][H][W] fp32 with a per-image valid region (rows < vh[b],
// columns < vw[b]); pixels outside it are zero padding (inputs read as 0,
// outputs written as 0).  Activations: [B][H][W][32] bf16, channel-last.
// Weights: fp32 master [C_out][C_in][3][3] per layer followed by the biases,
// in one flat vector (19,105 values); BF16 working copies:
//   fwd layout  wf[tap][co][ci]                (the conv's B operand)
//   bwd layout  wb[tap][ci][co] with tap = 8 - tap'  (flipped, transposed)
//
// The 32 -> 32 layers run on v_mfma_f32_16x16x32_bf16: one wave computes 16
// consecutive pixels of a row x 32 output channels; for each of the 9 taps
// the 16 x 32 input patch (A, one tap, all 32 input channels) times the
// 32 x 16 weight block (B) accumulates into two 16 x 16 fp32 tiles.
// Operand layout of that instruction: lane l holds A row (l mod 16),
// k = 8 (l / 16) .. + 7; B column (l mod 16), the same k; D column (l mod 16),
// rows 4 (l / 16) .. + 3.
#pragma once

#include <hip/hip_runtime.h>

namespace dbl {
namespace cnn {

constexpr int C = 32;
constexpr int kW1 = 0;                       // layer 1: W 32x1x3x3, b 32
constexpr int kB1 = kW1 + C * 9;
constexpr int kW2 = kB1 + C;                 // layer 2: W 32x32x3x3, b 32
constexpr int kB2 = kW2 + C * C * 9;
constexpr int kW3 = kB2 + C;                 // layer 3
constexpr int kB3 = kW3 + C * C * 9;
constexpr int kW4 = kB3 + C;                 // layer 4: W 1x32x3x3, b 1
constexpr int kB4 = kW4 + C * 9;
constexpr int kNParams = kB4 + 1;            // 19105
constexpr int kMidBf16 = 9 * C * C;          // bf16 values per mid-layer copy

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
    // round to nearest even (finite inputs)
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

struct ImgDesc {          // per image of a batch
    int vh, vw;           // valid rows / columns
};

// ---------------------------------------------------------------------------
// Weight preparation: fp32 master -> bf16 working copies
// ---------------------------------------------------------------------------
// w1 [tap][co] and w4 [tap][ci] are kept in fp32 after bf16 rounding.
__global__ void k_prep_weights(const float* __restrict__ master, unsigned short* __restrict__ wf2,
                               unsigned short* __restrict__ wb2, unsigned short* __restrict__ wf3,
                               unsigned short* __restrict__ wb3, float* __restrict__ w1, float* __restrict__ w4) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMidBf16) {
        // i indexes the fp32 master order [co][ci][tap]
        const int co = i / (C * 9), ci = (i / 9) % C, tap = i % 9;
        const unsigned short a = f2bf(master[kW2 + i]), b = f2bf(master[kW3 + i]);
        wf2[(tap * C + co) * C + ci] = a;
        wf3[(tap * C + co) * C + ci] = b;
        wb2[((8 - tap) * C + ci) * C + co] = a;
        wb3[((8 - tap) * C + ci) * C + co] = b;
    }
    if (i < C * 9) {
        const int c = i / 9, tap = i % 9;
        w1[tap * C + c] = bf2f(f2bf(master[kW1 + i]));
        w4[tap * C + c] = bf2f(f2bf(master[kW4 + i]));
    }
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool inside(const ImgDesc& d, int y, int x) {
    return y >= 0 && x >= 0 && y < d.vh && x < d.vw;
}

// Layer 1 (1 -> 32), thread per pixel: a1 = bf16(relu(conv(bf16(x)) + b1)).
__global__ __launch_bounds__(256) void k_conv_in(const float* __restrict__ x, const ImgDesc* __restrict__ desc,
                                                 int H, int W, const float* __restrict__ w1,
                                                 const float* __restrict__ master, unsigned short* __restrict__ a1) {
    __shared__ float sw[9 * C + C];
    for (int i = threadIdx.x; i < 9 * C; i += 256) sw[i] = w1[i];
    for (int i = threadIdx.x; i < C; i += 256) sw[9 * C + i] = master[kB1 + i];
    __syncthreads();
    const int b = blockIdx.z, y = blockIdx.y, xx = blockIdx.x * 256 + threadIdx.x;
    if (xx >= W) return;
    const ImgDesc d = desc[b];
    const float* xi = x + (size_t)b * H * W;
    uint4* out = reinterpret_cast<uint4*>(a1 + (((size_t)b * H + y) * W + xx) * C);
    if (!inside(d, y, xx)) {
        for (int q = 0; q < 4; ++q) out[q] = make_uint4(0, 0, 0, 0);
        return;
    }
    float in[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y + t / 3 - 1, xs = xx + t % 3 - 1;
        in[t] = inside(d, yy, xs) ? bf2f(f2bf(xi[(size_t)yy * W + xs])) : 0.f;
    }
    unsigned int packed[16];
#pragma unroll
    for (int co = 0; co < C; co += 2) {
        float s0 = sw[9 * C + co], s1 = sw[9 * C + co + 1];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            s0 += sw[t * C + co] * in[t];
            s1 += sw[t * C + co + 1] * in[t];
        }
        packed[co / 2] = (unsigned int)f2bf(fmaxf(s0, 0.f)) | ((unsigned int)f2bf(fmaxf(s1, 0.f)) << 16);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
}

// 32 -> 32 convolution on MFMA.  Epilogue:
//   forward:  out = bf16(relu(acc + bias))
//   backward: out = bf16(acc) where mask[p][c] > 0, else 0   (bias == nullptr)
// Outside the valid region the output is 0.  A wave computes two output rows
// over kMidSeg consecutive pixels, 16 pixels at a time (16 pixels x 32
// channels per row: two 16 x 16 accumulators).  It keeps the B operands of
// all 9 taps (the 18 KB weight block, 72 registers per lane) in registers for
// the whole segment.  Per 16-pixel step it loads the four input rows the two
// output rows need, one 16-byte A fragment per lane and row (pixel x0 + l,
// channels 8k .. 8k + 7), plus the pixel just left or right of the step for
// the edge lanes; the A operands of the taps at dx = -1 and +1 are the same
// fragments shifted by one lane inside each 16-lane row (DPP row_shr:1 and
// row_shl:1).  A workgroup of 4 waves covers 8 rows.
constexpr int kMidSeg = 160;
constexpr int kMidRows = 8;   // output rows per workgroup (2 per wave)

__device__ __forceinline__ uint4 dpp_row_shift(uint4 v, bool right) {
    // right: lane l of each 16-lane row receives lane l - 1's value; else lane l + 1's
    uint4 o;
    if (right) {
        o.x = __builtin_amdgcn_update_dpp(0u, v.x, 0x111, 0xf, 0xf, true);
        o.y = __builtin_amdgcn_update_dpp(0u, v.y, 0x111, 0xf, 0xf, true);
        o.z = __builtin_amdgcn_update_dpp(0u, v.z, 0x111, 0xf, 0xf, true);
        o.w = __builtin_amdgcn_update_dpp(0u, v.w, 0x111, 0xf, 0xf, true);
    } else {
        o.x = __builtin_amdgcn_update_dpp(0u, v.x, 0x101, 0xf, 0xf, true);
        o.y = __builtin_amdgcn_update_dpp(0u, v.y, 0x101, 0xf, 0xf, true);
        o.z = __builtin_amdgcn_update_dpp(0u, v.z, 0x101, 0xf, 0xf, true);
        o.w = __builtin_amdgcn_update_dpp(0u, v.w, 0x101, 0xf, 0xf, true);
    }
    return o;
}

__global__ __launch_bounds__(256) void k_conv_mid(const unsigned short* __restrict__ in,
                                                  const ImgDesc* __restrict__ desc, int H, int W,
                                                  const unsigned short* __restrict__ wgt,
                                                  const float* __restrict__ bias,
                                                  const unsigned short* __restrict__ mask,
                                                  unsigned short* __restrict__ out) {
    __shared__ unsigned short stage[4][16 * C];    // per-wave output staging
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = blockIdx.z, y0 = blockIdx.y * kMidRows + 2 * wave;
    const int xbeg = blockIdx.x * kMidSeg;
    if (y0 >= H) return;   // no workgroup barrier below
    const ImgDesc d = desc[b];
    const int li = lane & 15, lk = lane >> 4;        // row/col index and k group
    uint4 bw0[9], bw1[9];
    const uint4* wq = reinterpret_cast<const uint4*>(wgt);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        bw0[t] = wq[((t * C + li) * C + 8 * lk) / 8];
        bw1[t] = wq[((t * C + 16 + li) * C + 8 * lk) / 8];
    }
    float b0v = 0.f, b1v = 0.f;
    if (bias) {
        b0v = bias[li];
        b1v = bias[16 + li];
    }
    const unsigned short* ib = in + (size_t)b * H * W * C;
    unsigned short* st = stage[wave];
    const int xend = min(W, xbeg + kMidSeg);
    // the pixel an edge lane needs besides its own: x0 - 1 (l = 0) or x0 + 16 (l = 15)
    const int edge_dx = li == 0 ? -1 : (li == 15 ? 16 : li);
    for (int x0 = xbeg; x0 < xend; x0 += 16) {
        uint4 cen[4], edg[4];   // input rows y0 - 1 .. y0 + 2: own pixel, edge pixel
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int yy = y0 - 1 + rr;
            const int xc = x0 + li, xe = x0 + edge_dx;
            cen[rr] = make_uint4(0, 0, 0, 0);
            edg[rr] = make_uint4(0, 0, 0, 0);
            if (inside(d, yy, xc)) cen[rr] = *reinterpret_cast<const uint4*>(ib + ((size_t)yy * W + xc) * C + 8 * lk);
            if ((li == 0 || li == 15) && inside(d, yy, xe))
                edg[rr] = *reinterpret_cast<const uint4*>(ib + ((size_t)yy * W + xe) * C + 8 * lk);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int y = y0 + h;
            if (y >= H) break;
            f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int rr = h + t / 3, dx = t % 3;
                uint4 a = cen[rr];
                if (dx != 1) {
                    // the shift runs on all lanes (a lane reading a masked-off
                    // lane would get 0), then the edge lane takes its own load
                    const uint4 sh = dpp_row_shift(a, dx == 0);
                    a = (dx == 0 ? li == 0 : li == 15) ? edg[rr] : sh;
                }
                const bf16x8 Aop = __builtin_bit_cast(bf16x8, a);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop, __builtin_bit_cast(bf16x8, bw0[t]), acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop, __builtin_bit_cast(bf16x8, bw1[t]), acc1, 0, 0, 0);
            }
            // D: column co = li (+16), rows (pixels) 4 lk .. 4 lk + 3
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int px = 4 * lk + r;
                const int xs = x0 + px;
                float v0 = acc0[r], v1 = acc1[r];
                if (bias) {
                    v0 = fmaxf(v0 + b0v, 0.f);
                    v1 = fmaxf(v1 + b1v, 0.f);
                } else {
                    const size_t mi = (((size_t)b * H + y) * W + (xs < W ? xs : 0)) * C;
                    if (!(xs < W && bf2f(mask[mi + li]) > 0.f)) v0 = 0.f;
                    if (!(xs < W && bf2f(mask[mi + 16 + li]) > 0.f)) v1 = 0.f;
                }
                if (!inside(d, y, xs)) v0 = v1 = 0.f;
                st[px * C + li] = f2bf(v0);
                st[px * C + 16 + li] = f2bf(v1);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // 16 pixels x 64 bytes: 4 lanes per pixel, 16 bytes each
            {
                const int px = lane >> 2, q = lane & 3;
                if (x0 + px < W) {
                    const uint4 v = reinterpret_cast<const uint4*>(st + px * C)[q];
                    reinterpret_cast<uint4*>(out + (((size_t)b * H + y) * W + x0 + px) * C)[q] = v;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

inline dim3 conv_mid_grid(int B, int H, int W) {
    return dim3((W + kMidSeg - 1) / kMidSeg, (H + kMidRows - 1) / kMidRows, B);
}

// Layer 4 (32 -> 1) plus residual, thread per pixel: out = x + conv(a3) + b4.
__global__ __launch_bounds__(256) void k_conv_out(const unsigned short* __restrict__ a3, const float* __restrict__ x,
                                                  const ImgDesc* __restrict__ desc, int H, int W,
                                                  const float* __restrict__ w4, const float* __restrict__ master,
                                                  float* __restrict__ out) {
    __shared__ float sw[9 * C];
    for (int i = threadIdx.x; i < 9 * C; i += 256) sw[i] = w4[i];
    __syncthreads();
    const int b = blockIdx.z, y = blockIdx.y, xx = blockIdx.x * 256 + threadIdx.x;
    if (xx >= W) return;
    const ImgDesc d = desc[b];
    const size_t o = ((size_t)b * H + y) * W + xx;
    if (!inside(d, y, xx)) {
        out[o] = 0.f;
        return;
    }
    float s = master[kB4];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y + t / 3 - 1, xs = xx + t % 3 - 1;
        if (!inside(d, yy, xs)) continue;
        const uint4* ap = reinterpret_cast<const uint4*>(a3 + (((size_t)b * H + yy) * W + xs) * C);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 v = ap[q];
            const unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = 8 * q + 2 * e;
                s += sw[t * C + c] * bf2f((unsigned short)(w[e] & 0xFFFF)) +
                     sw[t * C + c + 1] * bf2f((unsigned short)(w[e] >> 16));
            }
        }
    }
    out[o] = x[o] + s;
}

// ---------------------------------------------------------------------------
// Loss and backward
// ---------------------------------------------------------------------------
// dout = 2 (out - target) / npix (valid pixels only); part[block] = sum (out - target)^2.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ out, const float* __restrict__ target,
                                              const ImgDesc* __restrict__ desc, int H, int W, float inv_npix,
                                              float* __restrict__ dout, double* __restrict__ part) {
    __shared__ double red[256];
    const int b = blockIdx.z, y = blockIdx.y, xx = blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (xx < W) {
        const ImgDesc d = desc[b];
        const size_t o = ((size_t)b * H + y) * W + xx;
        float g = 0.f;
        if (inside(d, y, xx)) {
            const float e = out[o] - target[o];
            s = (double)e * e;
            g = 2.f * e * inv_npix;
        }
        dout[o] = g;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[((size_t)b * gridDim.y + y) * gridDim.x + blockIdx.x] = red[0];
}

// Layer 4 backward-data + ReLU mask of layer 3:
// dp3[p][c] = bf16( (sum_t w4[t][c] dout[p - (t - 1)]) * (a3[p][c] > 0) ).
__global__ __launch_bounds__(256) void k_bwd_out(const float* __restrict__ dout, const unsigned short* __restrict__ a3,
                                                 const ImgDesc* __restrict__ desc, int H, int W,
                                                 const float* __restrict__ w4, unsigned short* __restrict__ dp3) {
    __shared__ float sw[9 * C];
    for (int i = threadIdx.x; i < 9 * C; i += 256) sw[i] = w4[i];
    __syncthreads();
    const int b = blockIdx.z, y = blockIdx.y, xx = blockIdx.x * 256 + threadIdx.x;
    if (xx >= W) return;
    const ImgDesc d = desc[b];
    float g[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y - (t / 3 - 1), xs = xx - (t % 3 - 1);
        g[t] = inside(d, yy, xs) ? dout[((size_t)b * H + yy) * W + xs] : 0.f;
    }
    const size_t o = (((size_t)b * H + y) * W + xx) * C;
    const uint4* ap = reinterpret_cast<const uint4*>(a3 + o);
    uint4* op = reinterpret_cast<uint4*>(dp3 + o);
    const bool in = inside(d, y, xx);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 av = ap[q];
        const unsigned int aw[4] = {av.x, av.y, av.z, av.w};
        unsigned int r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 8 * q + 2 * e;
            float s0 = 0.f, s1 = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                s0 += sw[t * C + c] * g[t];
                s1 += sw[t * C + c + 1] * g[t];
            }
            if (!in || !(bf2f((unsigned short)(aw[e] & 0xFFFF)) > 0.f)) s0 = 0.f;
            if (!in || !(bf2f((unsigned short)(aw[e] >> 16)) > 0.f)) s1 = 0.f;
            r[e] = (unsigned int)f2bf(s0) | ((unsigned int)f2bf(s1) << 16);
        }
        op[q] = make_uint4(r[0], r[1], r[2], r[3]);
    }
}

constexpr int kWgRows = 8, kWgCols = 32;

// Weight gradient of a 32 -> 32 layer over one chunk of kWgRows x kWgCols
// output pixels, on MFMA: for each tap t, dW_t[co][ci] = sum_p dp[p][co]
// a[p + t][ci] is a 32 x 32 x 256 product with K = the chunk's pixels (bf16
// operands, fp32 accumulation), one 32-pixel chunk row per k step.  Wave w
// owns the output block (co half w mod 2, ci half w / 2) for all 9 taps.
// LDS holds dp transposed, [co][p], and three copies of the halo of a
// transposed and pre-shifted by dx, [dx][ci][row][px] = a(row, px + dx), so
// every operand fragment (8 consecutive pixels of one channel) is one
// aligned 16-byte read.  part[chunk] = (dW as [co][ci][t], then sum_p dp[p][co]).
__global__ __launch_bounds__(256) void k_wgrad_mid(const unsigned short* __restrict__ dp,
                                                   const unsigned short* __restrict__ a,
                                                   const ImgDesc* __restrict__ desc, int H, int W,
                                                   float* __restrict__ part) {
    constexpr int P = kWgRows * kWgCols;
    __shared__ __attribute__((aligned(16))) unsigned short sdpT[C][P];
    __shared__ __attribute__((aligned(16))) unsigned short saT[3][C][kWgRows + 2][kWgCols];
    const int b = blockIdx.z, y0 = blockIdx.y * kWgRows, x0 = blockIdx.x * kWgCols;
    const ImgDesc d = desc[b];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    for (int e = tid; e < P * C; e += 256) {
        const int p = e / C, c = e % C;
        const int yy = y0 + p / kWgCols, xs = x0 + p % kWgCols;
        sdpT[c][p] = inside(d, yy, xs) ? dp[(((size_t)b * H + yy) * W + xs) * C + c] : (unsigned short)0;
    }
    for (int e = tid; e < (kWgRows + 2) * (kWgCols + 2) * C; e += 256) {
        const int hp = e / C, c = e % C;
        const int hy = hp / (kWgCols + 2), hx = hp % (kWgCols + 2);
        const int yy = y0 + hy - 1, xs = x0 + hx - 1;
        const unsigned short v = inside(d, yy, xs) ? a[(((size_t)b * H + yy) * W + xs) * C + c] : (unsigned short)0;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int px = hx - dx;
            if (px >= 0 && px < kWgCols) saT[dx][c][hy][px] = v;
        }
    }
    __syncthreads();
    const int co0 = 16 * (wave & 1), ci0 = 16 * (wave >> 1);
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int g = 0; g < kWgRows; ++g) {
        const bf16x8 A = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&sdpT[co0 + li][g * kWgCols + 8 * lk]));
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const uint4 bv = *reinterpret_cast<const uint4*>(&saT[t % 3][ci0 + li][g + t / 3][8 * lk]);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, bv), acc[t], 0, 0, 0);
        }
    }
    const size_t chunk = ((size_t)b * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float* pp = part + chunk * (9 * C * C + C);
    // D: column ci0 + li, rows (co) co0 + 4 lk .. + 3
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int co = co0 + 4 * lk + q, ci = ci0 + li;
#pragma unroll
        for (int t = 0; t < 9; ++t) pp[(co * C + ci) * 9 + t] = acc[t][q];
    }
    if (tid < C) {
        float bsum = 0.f;
        for (int p = 0; p < P; ++p) bsum += bf2f(sdpT[tid][p]);
        pp[9 * C * C + tid] = bsum;
    }
}

// Weight gradients of the 1 -> 32 and 32 -> 1 layers over one chunk:
// mode 0 (layer 1): part[c][t] = sum_p dp1[p][c] bf16(x)[p + t], part[288 + c] = sum_p dp1[p][c]
// mode 1 (layer 4): part[c][t] = sum_p dout[p] a3[p + t][c],     part[288 + c] = sum_p dout[p]
// Thread = (c = tid / 8, taps tid mod 8 and 8).
constexpr int kHalo = (kWgRows + 2) * (kWgCols + 2);
__global__ __launch_bounds__(256) void k_wgrad_edge(int mode, const unsigned short* __restrict__ dpa,
                                                    const float* __restrict__ img,
                                                    const ImgDesc* __restrict__ desc, int H, int W,
                                                    float* __restrict__ part) {
    __shared__ float sc[kHalo][C + 1];   // mode 0: dp1 at the chunk pixels; mode 1: a3 over the halo
    __shared__ float si[kHalo];          // mode 0: bf16(x) over the halo;   mode 1: dout at the chunk pixels
    const int b = blockIdx.z, y0 = blockIdx.y * kWgRows, x0 = blockIdx.x * kWgCols;
    const ImgDesc d = desc[b];
    const int tid = threadIdx.x;
    if (mode == 0) {
        for (int e = tid; e < kWgRows * kWgCols * C; e += 256) {
            const int p = e / C, c = e % C;
            const int yy = y0 + p / kWgCols, xs = x0 + p % kWgCols;
            sc[p][c] = inside(d, yy, xs) ? bf2f(dpa[(((size_t)b * H + yy) * W + xs) * C + c]) : 0.f;
        }
        for (int e = tid; e < kHalo; e += 256) {
            const int yy = y0 + e / (kWgCols + 2) - 1, xs = x0 + e % (kWgCols + 2) - 1;
            si[e] = inside(d, yy, xs) ? bf2f(f2bf(img[((size_t)b * H + yy) * W + xs])) : 0.f;
        }
    } else {
        for (int e = tid; e < kHalo * C; e += 256) {
            const int p = e / C, c = e % C;
            const int yy = y0 + p / (kWgCols + 2) - 1, xs = x0 + p % (kWgCols + 2) - 1;
            sc[p][c] = inside(d, yy, xs) ? bf2f(dpa[(((size_t)b * H + yy) * W + xs) * C + c]) : 0.f;
        }
        for (int e = tid; e < kWgRows * kWgCols; e += 256) {
            const int yy = y0 + e / kWgCols, xs = x0 + e % kWgCols;
            si[e] = inside(d, yy, xs) ? img[((size_t)b * H + yy) * W + xs] : 0.f;
        }
    }
    __syncthreads();
    const int c = tid >> 3, tq = tid & 7;
    float acc0 = 0.f, acc1 = 0.f, bsum = 0.f;
    for (int py = 0; py < kWgRows; ++py) {
        for (int px = 0; px < kWgCols; ++px) {
            const int h0 = (py + tq / 3) * (kWgCols + 2) + px + tq % 3;          // tap tq
            const int h8 = (py + 2) * (kWgCols + 2) + px + 2;                     // tap 8
            if (mode == 0) {
                const float g = sc[py * kWgCols + px][c];
                bsum += g;
                acc0 += g * si[h0];
                acc1 += g * si[h8];
            } else {
                const float g = si[py * kWgCols + px];
                bsum += g;
                acc0 += g * sc[h0][c];
                acc1 += g * sc[h8][c];
            }
        }
    }
    const size_t chunk = ((size_t)b * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float* pp = part + chunk * (9 * C + C);
    pp[c * 9 + tq] = acc0;
    if (tq == 0) {
        pp[c * 9 + 8] = acc1;
        pp[9 * C + c] = bsum;
    }
}

// Deterministic column sums: out[g][i] = sum_{k < rows_per} in[g * rows_per + k][i]
// (rows beyond nrows count as 0).  Repeated by the host until one row is left.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ in, int nrows, int ncols, int rows_per,
                                                float* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y;
    if (i >= ncols) return;
    float s = 0.f;
    const int r0 = g * rows_per, r1 = min(nrows, r0 + rows_per);
    for (int r = r0; r < r1; ++r) s += in[(size_t)r * ncols + i];
    out[(size_t)g * ncols + i] = s;
}

// Scatter one layer's reduced gradient (row 0 of the partials) into the flat
// gradient vector: weights red[0..nw) -> grad[woff..), biases red[bsrc..bsrc+nb) -> grad[boff..).
__global__ void k_scatter_grad(const float* __restrict__ red, int nw, int woff, int nb, int boff, int bsrc,
                               float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) grad[woff + i] = red[i];
    else if (i < nw + nb) grad[boff + (i - nw)] = red[bsrc + (i - nw)];
}

// Adam on the fp32 master vector (bias-corrected), step >= 1.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Tile inputs of the warm start: img[t][m][n] = y(nearest observed pixel) / s_t
// on the support, 0 elsewhere (frames N x N).
__global__ void k_cnn_tile_input(const float* __restrict__ y, const int* __restrict__ sorg,
                                 const int* __restrict__ sdim, const float* __restrict__ scale, int My, int Mx, int N,
                                 float* __restrict__ img) {
    const int t = blockIdx.y;
    const int sy0 = sorg[2 * t], sx0 = sorg[2 * t + 1], sh = sdim[2 * t], swd = sdim[2 * t + 1];
    const float inv = 1.0f / scale[t];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
        const int m = e / N, c = e % N;
        float v = 0.f;
        if (m < sh && c < swd) {
            const int gi = min(max(sy0 + m, 0), My - 1), gj = min(max(sx0 + c, 0), Mx - 1);
            v = y[(size_t)gi * Mx + gj] * inv;
        }
        img[(size_t)t * N * N + e] = v;
    }
}

// x0 = max(0, s_t * net_out) on the support.
__global__ void k_cnn_tile_output(const float* __restrict__ net, const float* __restrict__ scale,
                                  const int* __restrict__ sdim, int N, float* __restrict__ x) {
    const int t = blockIdx.y;
    const int sh = sdim[2 * t], swd = sdim[2 * t + 1];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
        const int m = e / N, c = e % N;
        x[(size_t)t * N * N + e] = (m < sh && c < swd) ? fmaxf(scale[t] * net[(size_t)t * N * N + e], 0.f) : 0.f;
    }
}

// Per-tile input scale of the warm start: s_t = mean over the block of
// max(y, 0), floored at 1e-6 (from the (y, W) frames, block at offset r).
__global__ __launch_bounds__(256) void k_tile_scale(const float2* __restrict__ yw, const int* __restrict__ bdim, int N,
                                                    int r, float* __restrict__ scale) {
    __shared__ double red[256];
    const int t = blockIdx.x;
    const int bh = bdim[2 * t], bw = bdim[2 * t + 1];
    double s = 0.0;
    for (int e = threadIdx.x; e < bh * bw; e += 256) {
        const int m = e / bw + r, c = e % bw + r;
        s += fmaxf(yw[(size_t)t * N * N + (size_t)m * N + c].x, 0.f);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[t] = (float)fmax(red[0] / (double)(bh * bw), 1e-6);
}

// Per-tile squared distance between two frame arrays.
__global__ __launch_bounds__(256) void k_tile_dist2(const float* __restrict__ a, const float* __restrict__ b, int N,
                                                    double* __restrict__ out) {
    __shared__ double red[256];
    const int t = blockIdx.x;
    double s = 0.0;
    for (int e = threadIdx.x; e < N * N; e += 256) {
        const double d = (double)a[(size_t)t * N * N + e] - b[(size_t)t * N * N + e];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[t] = red[0];
}

// x[t] = use_a[t] ? a[t] : b[t]
__global__ void k_tile_select(const float* __restrict__ a, const float* __restrict__ b, const int* __restrict__ use_a,
                              int N, float* __restrict__ x) {
    const int t = blockIdx.y;
    const float* src = use_a[t] ? a : b;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x)
        x[(size_t)t * N * N + e] = src[(size_t)t * N * N + e];
}

}  // namespace cnn
}  // namespace dbl
