// Wave-level Stockham FFT for gfx950 (64-lane wavefronts).
//
// One wavefront owns kPts = 1280 complex points: kV = 20 values per lane, so
// it transforms 1280 / n lines of length n at once.  A transform is a chain
// of radix-R passes (R in {5, 4, 2}; 20 is a multiple of each, so every lane
// does 20/R butterflies per pass and no lane idles).  Between passes the
// values go through the wave's private LDS region; waves never wait on each
// other, only on their own LDS traffic (wave_sync).
//
// Pass p with radix R after sub-length Ns (Stockham autosort, decimation in
// time): butterfly j of a line reads elements j + r n/R, multiplies element r
// by W_{Ns R}^{r (j mod Ns)}, does a length-R DFT and writes element r to
// (j / Ns) Ns R + (j mod Ns) + r Ns.  After the last pass the line is in
// natural order.
//
// Register layout "L_R" (the input layout of a radix-R first pass, which is
// also the output layout of a radix-R last pass): lane l, slot b*R + r holds
// element j + r n/R of line q, where bid = l + 64 b, q = bid / (n/R),
// j = bid mod (n/R).  The forward plan starts with radix 5 and the inverse
// plan is the forward plan reversed, so a forward transform's output layout
// is the inverse transform's input layout and vice versa: a spectrum can be
// multiplied and transformed back without touching LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace dbl {

constexpr int kLanes = 64;
constexpr int kV = 20;
constexpr int kPts = kLanes * kV;

// Forward FFT direction uses exp(-2 pi i ...), inverse exp(+2 pi i ...).
constexpr int kFwd = -1;
constexpr int kInv = +1;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by i (DIR = +1) or -i (DIR = -1)
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
    return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int DIR>
__device__ __forceinline__ void dft2(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2* v) {
    float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    float2 s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    float2 jd13 = mul_i<DIR>(d13);   // DIR * i * (v1 - v3)
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, jd13);
    v[3] = csub(d02, jd13);
}

template <int DIR>
__device__ __forceinline__ void dft5(float2* v) {
    // cos(2 pi/5), cos(4 pi/5), sin(2 pi/5), sin(4 pi/5)
    constexpr float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
    constexpr float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
    float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    float2 b1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    float2 b2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    float2 d1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    float2 d2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    float2 id1 = mul_i<DIR>(d1), id2 = mul_i<DIR>(d2);   // DIR * i * d
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(b1, id1);
    v[4] = csub(b1, id1);
    v[2] = cadd(b2, id2);
    v[3] = csub(b2, id2);
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 2) dft2<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v);
    else dft5<DIR>(v);
}

// Forward radix plans; the inverse runs them in reverse order.
template <int n> struct Plan;
template <> struct Plan<80>  { static constexpr int np = 3; static constexpr int r[5] = {5, 4, 4, 0, 0}; };
template <> struct Plan<160> { static constexpr int np = 4; static constexpr int r[5] = {5, 4, 4, 2, 0}; };
template <> struct Plan<320> { static constexpr int np = 4; static constexpr int r[5] = {5, 4, 4, 4, 0}; };
template <> struct Plan<640> { static constexpr int np = 5; static constexpr int r[5] = {5, 4, 4, 4, 2}; };

template <int n, int DIR, int p>
constexpr int pass_radix() {
    return DIR == kFwd ? Plan<n>::r[p] : Plan<n>::r[Plan<n>::np - 1 - p];
}
// Radix of the first / last pass of a transform.
template <int n, int DIR> constexpr int first_radix() { return pass_radix<n, DIR, 0>(); }
template <int n, int DIR> constexpr int last_radix() { return pass_radix<n, DIR, Plan<n>::np - 1>(); }

// Line stride of the LDS exchange buffers: one padding element per line keeps
// column-wise (transposed) accesses free of bank conflicts.
template <int n> constexpr int line_stride() { return n + 1; }

// Position of register slot s = b*R + r in layout L_R for lines of length n.
template <int n, int R>
__device__ __forceinline__ void slot_pos(int lane, int s, int& line, int& elem) {
    constexpr int nR = n / R;
    const int b = s / R, r = s - (s / R) * R;
    const int bid = lane + kLanes * b;
    line = bid / nR;
    elem = bid - line * nR + r * nR;
}

// Runs passes p..np-1.  v holds the input in layout L_{radix of pass p} (for
// p = 0) and receives the output in layout L_{radix of the last pass}.  sw is
// the wave's LDS region (1280/n lines of stride line_stride<n>()), tw a
// twiddle table with tw[TS * e] = exp(-2 pi i e / n).
// Opaque copy of the lane index: address arithmetic derived from it is redone
// where it is used instead of being hoisted (and kept live) across passes and
// across the callers' loops, which would cost one VGPR per slot and pass.
__device__ __forceinline__ int fresh_lane(int lane) {
    asm volatile("" : "+v"(lane));
    return lane;
}

template <int n, int DIR, int TS, int p = 0, int Ns = 1>
__device__ __forceinline__ void fft_passes(float2 (&v)[kV], float2* __restrict__ sw,
                                           const float2* __restrict__ tw, int lane_in) {
    constexpr int np = Plan<n>::np;
    if constexpr (p < np) {
        const int lane = fresh_lane(lane_in);
        constexpr int R = pass_radix<n, DIR, p>();
        constexpr int NB = kV / R;
        constexpr int nR = n / R;
        constexpr int LS = line_stride<n>();
        if constexpr (p > 0) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int bid = lane + kLanes * b;
                const int q = bid / nR, j = bid - q * nR;
#pragma unroll
                for (int r = 0; r < R; ++r) v[b * R + r] = sw[q * LS + j + r * nR];
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int bid = lane + kLanes * b;
            const int q = bid / nR, j = bid - q * nR;
            if constexpr (Ns > 1) {
                const int k = j % Ns;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[TS * (r * k * (n / (Ns * R)))];
                    if constexpr (DIR == kInv) w.y = -w.y;
                    v[b * R + r] = cmul(v[b * R + r], w);
                }
            }
            dft<R, DIR>(&v[b * R]);
        }
        if constexpr (p + 1 < np) {
            wave_sync();
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int bid = lane + kLanes * b;
                const int q = bid / nR, j = bid - q * nR;
                const int k = j % Ns;
                const int base = (j / Ns) * Ns * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) sw[q * LS + base + r * Ns] = v[b * R + r];
            }
            wave_sync();
        }
        fft_passes<n, DIR, TS, p + 1, Ns * R>(v, sw, tw, lane_in);
    }
}

// Writes v (layout L_R) to the wave's LDS region in natural order.
template <int n, int R>
__device__ __forceinline__ void store_natural(const float2 (&v)[kV], float2* __restrict__ sw, int lane) {
    constexpr int LS = line_stride<n>();
#pragma unroll
    for (int s = 0; s < kV; ++s) {
        int q, e;
        slot_pos<n, R>(lane, s, q, e);
        sw[q * LS + e] = v[s];
    }
}

}  // namespace dbl
