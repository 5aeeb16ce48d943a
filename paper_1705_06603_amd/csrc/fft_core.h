// Wave-level Stockham FFT for gfx950 (64-lane wavefronts).
//
// One wavefront owns kPts = 1280 complex points: kV = 20 values per lane, so
// it transforms 1280 / n lines of length n at once.  A transform is a chain
// of radix-R passes (R in {20, 5, 4, 2}; each divides 20, so every lane does
// 20/R butterflies per pass and no lane idles).  A radix-20 pass is one
// length-20 DFT per lane done in registers (4 x 5 with constant twiddles),
// which saves one LDS exchange over separate radix-5 and radix-4 passes.
// Between passes the values go through the wave's private LDS region; waves
// never wait on each other, only on their own LDS traffic (wave_sync).
//
// Pass p with radix R after sub-length Ns (Stockham autosort, decimation in
// time): butterfly j of a line reads elements j + r n/R, multiplies element r
// by W_{Ns R}^{r (j mod Ns)}, does a length-R DFT and writes element r to
// (j / Ns) Ns R + (j mod Ns) + r Ns.  After the last pass the line is in
// natural order.
//
// Lane mapping: each line is owned by LPL = n / 20 consecutive lanes (a power
// of two for every supported n), so lane l works on line q = l / LPL only and
// its butterflies of a radix-R pass are j = (l mod LPL) + LPL b, b < 20/R.
// Register layout "L_R" (the input layout of a radix-R first pass, which is
// also the output layout of a radix-R last pass): lane l, slot b*R + r holds
// element j + r n/R of line q.  LDS and global addresses of a lane are one
// per-lane base plus compile-time offsets.  The forward plan starts with
// radix 20 and the inverse plan is the forward plan reversed, so a forward transform's output layout
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

// Length-20 DFT in registers, as 4 x 5 (Cooley-Tukey with constant
// twiddles): input index r = 5a + b, output index k = c + 4d, so
//   y[c + 4d] = sum_b w5^{bd} w20^{bc} sum_a x[5a + b] w4^{ac},
// with w_m = exp(DIR 2 pi i / m): five length-4 DFTs, twiddles w20^{bc},
// four length-5 DFTs.
template <int DIR>
__device__ __forceinline__ void dft20(float2* v) {
    // cos and sin of 2 pi m / 20 for the products m = b c (b < 5, c < 4)
    constexpr float kC[13] = {1.f, 0.95105651629515357f, 0.80901699437494742f, 0.58778525229247313f,
                              0.30901699437494742f, 0.f, -0.30901699437494742f, 0.f, -0.80901699437494742f,
                              -0.95105651629515357f, 0.f, 0.f, -0.80901699437494742f};
    constexpr float kS[13] = {0.f, 0.30901699437494742f, 0.58778525229247313f, 0.80901699437494742f,
                              0.95105651629515357f, 1.f, 0.95105651629515357f, 0.f, 0.58778525229247313f,
                              0.30901699437494742f, 0.f, 0.f, -0.58778525229247313f};
    float2 T[5][4];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        float2 u[4] = {v[b], v[5 + b], v[10 + b], v[15 + b]};
        dft4<DIR>(u);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int m = b * c;
            T[b][c] = (m == 0) ? u[c] : cmul(u[c], make_float2(kC[m], DIR * kS[m]));
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float2 w[5] = {T[0][c], T[1][c], T[2][c], T[3][c], T[4][c]};
        dft5<DIR>(w);
#pragma unroll
        for (int d = 0; d < 5; ++d) v[c + 4 * d] = w[d];
    }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 2) dft2<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v);
    else if constexpr (R == 5) dft5<DIR>(v);
    else dft20<DIR>(v);
}

// Forward radix plans; the inverse runs them in reverse order.
template <int n> struct Plan;
template <> struct Plan<80>  { static constexpr int np = 2; static constexpr int r[5] = {20, 4, 0, 0, 0}; };
template <> struct Plan<160> { static constexpr int np = 3; static constexpr int r[5] = {20, 4, 2, 0, 0}; };
template <> struct Plan<320> { static constexpr int np = 3; static constexpr int r[5] = {20, 4, 4, 0, 0}; };
template <> struct Plan<640> { static constexpr int np = 4; static constexpr int r[5] = {20, 4, 4, 2, 0}; };

template <int n, int DIR, int p>
constexpr int pass_radix() {
    return DIR == kFwd ? Plan<n>::r[p] : Plan<n>::r[Plan<n>::np - 1 - p];
}
// Radix of the first / last pass of a transform.
template <int n, int DIR> constexpr int first_radix() { return pass_radix<n, DIR, 0>(); }
template <int n, int DIR> constexpr int last_radix() { return pass_radix<n, DIR, Plan<n>::np - 1>(); }
// Layout of a transform's natural-order side: the forward transform's input
// and the inverse transform's output (the inverse plan is the forward plan
// reversed, so both are L_R of the forward plan's first radix).
template <int n> constexpr int nat_radix() {
    static_assert(first_radix<n, kFwd>() == last_radix<n, kInv>(), "plan is not reversible");
    return first_radix<n, kFwd>();
}

// Padding of the LDS exchange after pass p of a length-n transform: element
// f of the exchange is stored at f + (f / B) P.  LDS serves 16 lanes of a
// 64-bit access per cycle from 32 four-byte banks, so an access is free of
// bank conflicts when its 16 lanes' element positions are distinct mod 16.
// Without padding, the stores of the first pass (stride R) and of the
// inverse plan's middle pass fall on 4 positions mod 16.  B is a multiple of
// the pass's butterfly span Ns R, divides the next pass's stride n / R', and
// is a multiple or a divisor of the lanes per line, so the pad is one
// per-lane value for all of a butterfly's stores and a per-lane value plus a
// compile-time offset for every load.  With 8-lane lines, two lines share an
// access; the odd-line shift below (xline_off) puts them on disjoint banks,
// and the pads only need distinct positions mod 8 within a line.  The
// 80-point rows (4-lane lines) keep the unpadded layout.
template <int n, int DIR, int p> struct XPad { static constexpr int B = n, P = 0; };
template <> struct XPad<320, kFwd, 0> { static constexpr int B = 80, P = 1; };
template <> struct XPad<320, kFwd, 1> { static constexpr int B = 80, P = 4; };
template <> struct XPad<320, kInv, 0> { static constexpr int B = 16, P = 1; };
template <> struct XPad<640, kFwd, 0> { static constexpr int B = 160, P = 1; };
template <> struct XPad<640, kFwd, 1> { static constexpr int B = 160, P = 4; };
template <> struct XPad<640, kInv, 0> { static constexpr int B = 16, P = 1; };
template <> struct XPad<640, kInv, 1> { static constexpr int B = 32, P = 2; };
template <> struct XPad<160, kFwd, 0> { static constexpr int B = 40, P = 1; };
template <> struct XPad<160, kFwd, 1> { static constexpr int B = 80, P = 4; };

// A swizzle instead of a pad, for a pass with power-of-two Ns and R whose
// butterflies lie inside aligned blocks of Z = (lanes per line) elements:
// element Z a + c is stored at Z a + (c ^ Ns (a mod R)), which permutes only
// the R outputs of each butterfly.  Those then land on distinct positions
// across the lanes that share an access, and each load of the next pass is
// the lane index XORed with a compile-time constant.  It needs no extra
// space.
template <int n, int DIR, int p> struct XSwz { static constexpr bool on = false; };
template <> struct XSwz<320, kInv, 1> { static constexpr bool on = true; };
template <> struct XSwz<160, kInv, 0> { static constexpr bool on = true; };
template <> struct XSwz<160, kInv, 1> { static constexpr bool on = true; };
template <> struct XSwz<640, kInv, 2> { static constexpr bool on = true; };
template <int n, int DIR, int p> constexpr int xpad_span() {
    return n + ((n - 1) / XPad<n, DIR, p>::B) * XPad<n, DIR, p>::P;
}
template <int n, int DIR, int p = 0> constexpr int xpad_span_max() {
    if constexpr (p + 1 >= Plan<n>::np) return n;
    else return xpad_span<n, DIR, p>() > xpad_span_max<n, DIR, p + 1>() ? xpad_span<n, DIR, p>()
                                                                         : xpad_span_max<n, DIR, p + 1>();
}

// Line stride (in float2) of the LDS exchange buffers.  It is odd, so the
// column-wise (transposed) accesses of 16 consecutive lines hit distinct
// banks, and it holds the padded exchanges.  When fewer than 16 lanes own a
// line, several lines share one 16-lane LDS access; a stride = 9 (mod 32)
// puts those lines on disjoint banks.
template <int n> constexpr int line_stride() {
    if constexpr (n / kV < 16) return n + 9;
    else {
        constexpr int f = xpad_span_max<n, kFwd>(), i = xpad_span_max<n, kInv>();
        return (f > i ? f : i) | 1;
    }
}
constexpr int kLinePad = 0;
template <int n>
__device__ __forceinline__ int line_off(int q) {
    return q * line_stride<n>();
}

// With 8-lane lines two lines share each 16-lane access.  Their exchanges use
// line bases shifted so that odd lines start 8 positions (mod 16) after the
// even line before them: two lines whose 8 positions are distinct mod 8 then
// fill all 16 positions.  The shift (by at most 8, into the unused tail of
// the neighbouring line) keeps every exchange inside the wave's own lines.
template <int n> constexpr int xline_shift() {
    if constexpr (n / kV != 8) return 0;
    else {
        constexpr int s = ((8 - line_stride<n>()) % 16 + 16) % 16;
        return s > 8 ? s - 16 : s;
    }
}
template <int n>
__device__ __forceinline__ int xline_off(int q) {
    constexpr int sh = xline_shift<n>(), LS = line_stride<n>();
    constexpr int span = xpad_span_max<n, kFwd>() > xpad_span_max<n, kInv>() ? xpad_span_max<n, kFwd>()
                                                                             : xpad_span_max<n, kInv>();
    static_assert(span <= LS + (sh < 0 ? sh : 0) && LS + (sh > 0 ? sh : 0) + span <= 2 * LS,
                  "shifted exchange lines overlap");
    return q * LS + (q & 1) * sh;
}

// Lanes per line: n = 20 * LPL.
template <int n> constexpr int lanes_per_line() { return n / kV; }

// Compile-time part of the element index of slot s = b*R + r in layout L_R.
template <int n, int R> constexpr int slot_const(int s) {
    return lanes_per_line<n>() * (s / R) + (s % R) * (n / R);
}

// Position of register slot s in layout L_R for lines of length n.
template <int n, int R>
__device__ __forceinline__ void slot_pos(int lane, int s, int& line, int& elem) {
    constexpr int LPL = lanes_per_line<n>();
    static_assert((LPL & (LPL - 1)) == 0, "lanes per line must be a power of two");
    line = lane / LPL;
    elem = (lane % LPL) + slot_const<n, R>(s);
}

// Opaque copy of the lane index: address arithmetic derived from it is redone
// where it is used instead of being hoisted (and kept live) across passes and
// across the callers' loops, which would cost registers per slot and pass.
__device__ __forceinline__ int fresh_lane(int lane) {
    asm volatile("" : "+v"(lane));
    // a lane or thread index: non-negative, so divisions and remainders by
    // constants need no sign fix-ups
    __builtin_assume(lane >= 0);
    return lane;
}

// Per-pass twiddle tables.  Pass p (radix R, sub-length Ns > 1) of a length-n
// transform in direction DIR needs W_{Ns R}^{r k} for r in [1, R), k in
// [0, Ns); they are stored at twiddle_offset<n, DIR, p>() + (r - 1) Ns + k, so
// lanes with consecutive k read consecutive entries (no LDS bank conflicts).
// The direction's sign is folded into the table.
template <int n, int DIR, int p>
constexpr int pass_ns() {
    int ns = 1;
    for (int i = 0; i < p; ++i) ns *= (DIR == kFwd ? Plan<n>::r[i] : Plan<n>::r[Plan<n>::np - 1 - i]);
    return ns;
}
template <int n, int DIR, int p>
constexpr int twiddle_offset() {
    int off = 0, ns = 1;
    for (int i = 0; i < p; ++i) {
        const int R = (DIR == kFwd ? Plan<n>::r[i] : Plan<n>::r[Plan<n>::np - 1 - i]);
        if (ns > 1) off += (R - 1) * ns;
        ns *= R;
    }
    return off;
}
template <int n, int DIR>
constexpr int twiddle_count() { return twiddle_offset<n, DIR, Plan<n>::np>(); }

// Fills the tables of one (n, DIR): entry (p, r, k) = exp(DIR 2 pi i r k / (Ns R)), fp64 rounded.
template <int n, int DIR, int p = 0>
__device__ void fill_twiddles(float2* __restrict__ out, int tid, int nthreads) {
    if constexpr (p < Plan<n>::np) {
        constexpr int R = pass_radix<n, DIR, p>();
        constexpr int Ns = pass_ns<n, DIR, p>();
        if constexpr (Ns > 1) {
            constexpr int off = twiddle_offset<n, DIR, p>();
            for (int e = tid; e < (R - 1) * Ns; e += nthreads) {
                const int r = e / Ns + 1, k = e % Ns;
                double sn, cs;
                sincospi((double)DIR * 2.0 * (double)(r * k) / (double)(Ns * R), &sn, &cs);
                out[off + e] = make_float2((float)cs, (float)sn);
            }
        }
        fill_twiddles<n, DIR, p + 1>(out, tid, nthreads);
    }
}

// Runs passes p..np-1.  v holds the input in layout L_{radix of pass p} (for
// p = 0) and receives the output in layout L_{radix of the last pass}.  sw is
// the wave's LDS region (1280/n lines, line_off<n>), tw the per-pass twiddle
// tables of (n, DIR).
template <int n, int DIR, int p = 0, int Ns = 1>
__device__ __forceinline__ void fft_passes(float2 (&v)[kV], float2* __restrict__ sw,
                                           const float2* __restrict__ tw, int lane_in) {
    constexpr int np = Plan<n>::np;
    if constexpr (p < np) {
        const int lane = fresh_lane(lane_in);
        constexpr int R = pass_radix<n, DIR, p>();
        constexpr int NB = kV / R;
        constexpr int nR = n / R;
        constexpr int LPL = lanes_per_line<n>();
        const int l = lane % LPL;
        float2* __restrict__ line = sw + xline_off<n>(lane / LPL);
        if constexpr (p > 0 && XSwz<n, DIR, p - 1>::on) {
            constexpr int SR = pass_radix<n, DIR, p - 1>(), SN = pass_ns<n, DIR, p - 1>();
            static_assert(nR % LPL == 0, "exchange swizzle does not fit the loads");
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int a = b + r * (nR / LPL);   // block of this load (compile-time)
                    v[b * R + r] = line[LPL * a + (l ^ (SN * (a % SR)))];
                }
        } else if constexpr (p > 0) {
            constexpr int PB = XPad<n, DIR, p - 1>::B, PP = XPad<n, DIR, p - 1>::P;
            static_assert(PP == 0 || ((PB % LPL == 0 || LPL % PB == 0) && nR % PB == 0),
                          "exchange padding does not fit the loads");
            // (l + LPL b + r nR) / PB = l / PB + (LPL b) / PB + r nR / PB
            const int lp = (PP != 0 && PB < LPL) ? (l / PB) * PP : 0;
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    v[b * R + r] = line[lp + l + LPL * b + r * nR + ((LPL * b) / PB + r * (nR / PB)) * PP];
        }
        // j = l + LPL b;  k = j mod Ns;  jd = j / Ns
        const int lm = l % Ns, ld = l / Ns;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if constexpr (Ns > 1) {
                const int cb = LPL * b;
                int k = lm + cb % Ns;
                if (k >= Ns) k -= Ns;
                constexpr int off = twiddle_offset<n, DIR, p>();
                const float2* __restrict__ tk = tw + off + k;
#pragma unroll
                for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], tk[(r - 1) * Ns]);
            }
            dft<R, DIR>(&v[b * R]);
        }
        if constexpr (p + 1 < np) {
            constexpr int XB = XPad<n, DIR, p>::B, XP = XPad<n, DIR, p>::P;
            static_assert(XP == 0 || XB % (Ns * R) == 0, "exchange padding splits a butterfly");
            wave_sync();
            if constexpr (XSwz<n, DIR, p>::on) {
                static_assert(LPL % (Ns * R) == 0 && LPL % Ns == 0 && (R & (R - 1)) == 0 && (Ns & (Ns - 1)) == 0,
                              "exchange swizzle does not fit the stores");
                // butterfly jd = ld + b LPL / Ns starts at element jd Ns R + lm, in block
                // a = jd / (LPL / (Ns R)); a mod R is the same for every b
                const int q = (ld / (LPL / (Ns * R))) % R;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    float2* __restrict__ o = line + ld * (Ns * R) + lm + b * (LPL * R);
#pragma unroll
                    for (int r = 0; r < R; ++r) o[Ns * (r ^ q)] = v[b * R + r];
                }
            } else if constexpr (XP != 0 && LPL % Ns == 0 && (LPL * R) % XB == 0) {
                // butterfly jd = ld + b LPL / Ns starts at element ld Ns R + lm + b LPL R,
                // and its pad is the b = 0 pad plus b (LPL R / XB) P
                const int f0 = ld * (Ns * R) + lm;
                float2* __restrict__ o0 = line + f0 + (f0 / XB) * XP;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    float2* __restrict__ o = o0 + b * (LPL * R + (LPL * R / XB) * XP);
#pragma unroll
                    for (int r = 0; r < R; ++r) o[r * Ns] = v[b * R + r];
                }
            } else
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int cb = LPL * b;
                int k = lm + cb % Ns, jd = ld + cb / Ns;
                if (k >= Ns) {
                    k -= Ns;
                    jd += 1;
                }
                const int f = jd * (Ns * R) + k;
                float2* __restrict__ o = line + f + (f / XB) * XP;
#pragma unroll
                for (int r = 0; r < R; ++r) o[r * Ns] = v[b * R + r];
            }
            wave_sync();
        }
        fft_passes<n, DIR, p + 1, Ns * R>(v, sw, tw, lane_in);
    }
}

// Writes v (layout L_R) to the wave's LDS region in natural order.
template <int n, int R>
__device__ __forceinline__ void store_natural(const float2 (&v)[kV], float2* __restrict__ sw, int lane) {
#pragma unroll
    for (int s = 0; s < kV; ++s) {
        int q, e;
        slot_pos<n, R>(lane, s, q, e);
        sw[line_off<n>(q) + e] = v[s];
    }
}

}  // namespace dbl
