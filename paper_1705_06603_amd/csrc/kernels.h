// Device kernels of the batched tile solver.
//
// Every tile t keeps its unknowns in an N x N frame (N in {160, 320, 640}):
// frame pixel (m, c) is the support pixel (m, c) for m < support_h and
// c < support_w, zero elsewhere.  The forward operator of Section II-B is a
// circular convolution on the frame followed by a chop to the block, frame
// rows/columns [r, r + block): any N >= support makes that exact.
//
// Spectra use a packed half-plane stored column-major, [f][g] with
// f in [0, N/2) (row frequency) and g in [0, N) (column frequency): the
// row transform of a real frame is taken as a length-N/2 complex FFT of
// (even + i odd) samples, its DC and Nyquist values (both real) share slot
// f = 0 as DC + i Nyquist, and the column transform runs along g.  The
// column kernels split packed column 0 back into its two real columns (DC
// and Nyquist), each transformed as an ordinary column.  PSF spectra are
// stored with N/2 + 1 columns [node][f][g], f in [0, N/2]: the plain 2-D DFT
// of the wrap-centred PSF scaled by 2/N^2 (the two inverse transforms'
// normalisation and the factor of the half-length row transform).
//
// One Local-Solver step is four kernels:
//   col_H      : sum over terms of column FFT(a_ky . Z_kx) x spectrum, inverse column FFT
//   row_resid  : row C2R -> H x, residual W (H x - y) on the block, its row R2C
//   col_Ht     : column FFT, x conj spectrum per term, inverse column FFT, sum_ky a_ky
//   row_update : row C2R per kx, sum_kx b_kx -> H^T r, + lambda grad phi + alpha (x - u),
//                projected step, then the masked row R2Cs of the new x for the next step
// with a_ky / b_kx the separable PSF-interpolation weights w_k = a_ky(row) b_kx(col).
#pragma once

#include "fft_core.h"

namespace dbl {

constexpr int kMaxK = 3;   // PSF terms per axis and tile

struct TileInfo {
    int ty, tx;        // tile grid position
    int sy, sx;        // support size
    int by, bx;        // block size
    int nky, nkx;      // terms per axis
    int spec[kMaxK * kMaxK];   // spectrum index of term (ky, kx) at ky * 3 + kx
};

constexpr int kMaxCover = 3;   // tiles covering one X row or column (3 in the grid layout, near nodes)
struct Cover {         // tiles covering one X row (or column)
    int n;                 // number of covering tiles, 1 .. kMaxCover
    int a[kMaxCover];      // tile index along the axis
    int m[kMaxCover];      // frame coordinate in that tile
    float w[kMaxCover];    // consensus weight omega there
    int pad[2];
};

struct SolveParams {
    float lambda, reg_param, gamma, rho;
    int reg, bc, positivity, r;
};

// Waves per workgroup a frame kernel may use: the two shapes that split the
// frame evenly (the smaller one doubles the workgroup count).
template <int N> constexpr int waves_hi() { return N == 160 ? 2 : 4; }
template <int N> constexpr int waves_lo() { return waves_hi<N>() / 2; }

template <int N, int WV = waves_hi<N>()> struct Cfg {
    static constexpr int n = N / 2;          // complex length of a row transform
    static constexpr int LwR = kPts / n;     // rows per wave
    static constexpr int LwC = kPts / N;     // columns per wave
    static constexpr int W = WV;             // waves per workgroup
    static constexpr int NT = W * kLanes;
    static constexpr int RB = W * LwR;       // rows per row workgroup
    static constexpr int CB = W * LwC;       // columns per column workgroup
    static constexpr int RG = N / RB;        // row workgroups per tile
    static constexpr int CG = (N / 2) / CB;  // column workgroups per tile
    static constexpr int LSR = line_stride<n>();
    static constexpr int LSC = line_stride<N>();
    // twiddle tables: column transforms (length N) and row transforms (length n)
    static constexpr int TWC_F = twiddle_count<N, kFwd>();
    static constexpr int TWC_I = twiddle_count<N, kInv>();
    static constexpr int TWR_F = twiddle_count<n, kFwd>();
    static constexpr int TWR_I = twiddle_count<n, kInv>();
    static constexpr int TWC = TWC_F + TWC_I;               // column tables, LDS size
    static constexpr int TWR = TWR_F + TWR_I + n;           // row tables + W_N^f, LDS size
    static constexpr int RPOST = TWR_F + TWR_I;             // offset of W_N^f in the row tables
    static constexpr int TW_TOTAL = TWC + TWR;              // global table: [column | row]
    static constexpr size_t SPEC = (size_t)(N / 2) * N;   // complex values of one half-plane
    static constexpr size_t NSPEC = (size_t)(N / 2 + 1) * N;
    static_assert(RG * RB == N && CG * CB == N / 2, "frame does not split into workgroups");
};

// ---------------------------------------------------------------------------
// Row transforms (workgroup level)
// ---------------------------------------------------------------------------

// Row transforms hold slot s of lane l at row l / LPL, complex element
// l mod LPL + slot_const(s) (natural radix layout).  rslot_base is the float
// offset of a lane's first slot in a row-major [rows][N] float frame; slot s
// adds rslot_off(s) floats, a compile-time (immediate) offset.
template <int N>
__device__ __forceinline__ int rslot_base(int lane) {
    constexpr int LPL = lanes_per_line<N / 2>();
    return (lane / LPL) * N + 2 * (lane % LPL);
}
template <int N>
__device__ __forceinline__ int rslot_tent(int lane) {   // the same offset within one row
    return 2 * (lane % lanes_per_line<N / 2>());
}
template <int N>
constexpr int rslot_off(int s) { return 2 * slot_const<N / 2, nat_radix<N / 2>()>(s); }

// Transposed store of the WG's rows (natural-order row FFTs of the packed
// real rows, in sbuf) as packed half-spectra out[f][i0 + row].
template <int N, int WV>
__device__ __forceinline__ void store_spectrum_T(const float2* __restrict__ sbuf, const float2* __restrict__ tw,
                                                 float2* __restrict__ out, int i0, int tid_in) {
    using C = Cfg<N, WV>;
    constexpr int n = C::n;
    // element e = tid + k NT is (row, f) = (e mod RB, e / RB): the row is the
    // thread's own and f advances by FS = NT / RB per step
    static_assert(C::NT % C::RB == 0 && n % (C::NT / C::RB) == 0, "transpose does not tile");
    constexpr int FS = C::NT / C::RB;
    const int tid = fresh_lane(tid_in);
    const int row = tid % C::RB, f0 = tid / C::RB;
    const float2* __restrict__ zl = sbuf + line_off<n>(row);
    float2* __restrict__ ol = out + (size_t)f0 * N + i0 + row;
#pragma unroll 4
    for (int k = 0; k < n / FS; ++k) {
        const int f = f0 + k * FS;
        const float2 Z = zl[f];
        float2 P;
        if (f == 0) {
            P = make_float2(Z.x + Z.y, Z.x - Z.y);
        } else {
            const float2 Zm = zl[n - f];
            // X = (Z + conj Zm)/2 - i W_N^f (Z - conj Zm)/2
            const float2 A = make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
            const float2 B = make_float2(0.5f * (Z.x - Zm.x), 0.5f * (Z.y + Zm.y));
            const float2 wB = cmul(tw[C::RPOST + f], B);
            P = make_float2(A.x + wB.y, A.y - wB.x);
        }
        ol[(size_t)k * FS * N] = P;
    }
}

// Transposed load of packed half-spectra for a row C2R: reads the pair
// (f, n - f) of each row from in[.][i0 + row] and stores the complex
// sequence Z = E + i O whose inverse length-n FFT gives (x[2m], x[2m+1]):
//   E = (X_f + conj X_{n-f}) / 2,  O = (X_f - conj X_{n-f}) W_N^{-f} / 2,
// with X_0 = Re P_0 (DC) and X_{n} = Im P_0 (Nyquist) from the packed slot 0.
template <int N, int WV>
__device__ __forceinline__ void load_c2r_T(float2* __restrict__ sbuf, const float2* __restrict__ in,
                                           const float2* __restrict__ tw, int i0, int tid_in) {
    using C = Cfg<N, WV>;
    constexpr int n = C::n;
    // pair e = tid + k NT is (row, f) = (e mod RB, e / RB), f = f0 + k FS, for
    // f = 0 .. n/2 (see store_spectrum_T)
    static_assert(C::NT % C::RB == 0, "transpose does not tile");
    constexpr int FS = C::NT / C::RB;
    const int tid = fresh_lane(tid_in);
    constexpr int PAIRS = C::RB * (n / 2 + 1);
    constexpr int PER = (PAIRS + C::NT - 1) / C::NT;
    const int row = tid % C::RB, f0 = tid / C::RB;
    const float2* __restrict__ pa = in + (size_t)f0 * N + i0 + row;         // column f
    const float2* __restrict__ pb = in + (size_t)(n - f0) * N + i0 + row;   // column n - f (f >= 1)
    float2 xa[PER], xb[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int f = f0 + k * FS;
        if (f <= n / 2) {
            const float2* qa = pa + (size_t)k * FS * N;
            xa[k] = *qa;
            xb[k] = f == 0 ? *qa : *(pb - (size_t)k * FS * N);   // column (n - f) mod n
        }
    }
    float2* __restrict__ line = sbuf + line_off<n>(row);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int f = f0 + k * FS;
        if (f <= n / 2) {
            if (f == 0) {
                const float2 X = xa[k];
                line[0] = make_float2(0.5f * (X.x + X.y), 0.5f * (X.x - X.y));
            } else {
                const float2 X = xa[k], Xm = xb[k];
                {
                    const float2 E = make_float2(0.5f * (X.x + Xm.x), 0.5f * (X.y - Xm.y));
                    const float2 D = make_float2(0.5f * (X.x - Xm.x), 0.5f * (X.y + Xm.y));
                    const float2 O = cmulc(D, tw[C::RPOST + f]);
                    line[f] = make_float2(E.x - O.y, E.y + O.x);
                }
                if (f != n - f) {
                    const float2 E = make_float2(0.5f * (Xm.x + X.x), 0.5f * (Xm.y - X.y));
                    const float2 D = make_float2(0.5f * (Xm.x - X.x), 0.5f * (Xm.y + X.y));
                    const float2 O = cmulc(D, tw[C::RPOST + (n - f)]);
                    line[n - f] = make_float2(E.x - O.y, E.y + O.x);
                }
            }
        }
    }
}

// Wave-level inverse row FFT of the wave's rows (Z from load_c2r_T).
// Result: v[s] = (x[2m], x[2m+1]) in the natural layout of length n, times N/2
// relative to the normalised inverse (folded into the spectra).
template <int N>
__device__ __forceinline__ void row_c2r_ready(float2 (&v)[kV], float2* __restrict__ sw,
                                              const float2* __restrict__ tw, int lane) {
    using C = Cfg<N>;
    constexpr int n = C::n;
    constexpr int R0 = first_radix<n, kInv>();
#pragma unroll
    for (int s = 0; s < kV; ++s) {
        int q, f;
        slot_pos<n, R0>(lane, s, q, f);
        v[s] = sw[line_off<n>(q) + f];
    }
    wave_sync();
    fft_passes<n, kInv>(v, sw, tw + C::TWR_F, lane);
}

// Wave-level forward row FFT of v (natural layout of length n, packed real pairs)
// into sw in natural order.
template <int N>
__device__ __forceinline__ void row_fft_wave(float2 (&v)[kV], float2* __restrict__ sw,
                                             const float2* __restrict__ tw, int lane) {
    constexpr int n = Cfg<N>::n;
    fft_passes<n, kFwd>(v, sw, tw, lane);
    wave_sync();
    store_natural<n, last_radix<n, kFwd>()>(v, sw, lane);
}

// Copies the column (COL) or row twiddle tables of frame N into LDS.
template <int N, int WV, bool COL>
__device__ __forceinline__ void load_twiddles(float2* __restrict__ tw, const float2* __restrict__ twg, int tid) {
    using C = Cfg<N, WV>;
    constexpr int cnt = COL ? C::TWC : C::TWR;
    const float2* src = twg + (COL ? 0 : C::TWC);
    for (int e = tid; e < cnt; e += C::NT) tw[e] = src[e];
}

// Builds the global twiddle tables of frame N (one workgroup).
template <int N>
__global__ void k_make_twiddles(float2* __restrict__ twg) {
    using C = Cfg<N>;
    const int tid = threadIdx.x, nt = blockDim.x;
    fill_twiddles<N, kFwd>(twg, tid, nt);
    fill_twiddles<N, kInv>(twg + C::TWC_F, tid, nt);
    fill_twiddles<C::n, kFwd>(twg + C::TWC, tid, nt);
    fill_twiddles<C::n, kInv>(twg + C::TWC + C::TWR_F, tid, nt);
    for (int f = tid; f < C::n; f += nt) {
        double sn, cs;
        sincospi(-2.0 * (double)f / (double)N, &sn, &cs);
        twg[C::TWC + C::RPOST + f] = make_float2((float)cs, (float)sn);
    }
}

// Tables the stand-alone FFT stages read: every one of the batch's tiles is
// a full n x n frame with one unmasked term (tent 1 everywhere).
__global__ void k_fill_fft_tables(TileInfo* __restrict__ tiles, int batch, int n, float* __restrict__ tent,
                                  int n_tent) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch) {
        TileInfo t{};
        t.sy = t.sx = t.by = t.bx = n;
        t.nky = t.nkx = 1;
        tiles[i] = t;
    }
    if (i < n_tent) tent[i] = 1.0f;
}

// x (frames) -> packed row half-spectra of b_k . x for each mask k of the
// tile (masked != 0) or of x itself (masked == 0, one output).
template <int N, int WV>
__global__ __launch_bounds__((Cfg<N, WV>::NT)) void k_row_fwd(const float* __restrict__ x, const TileInfo* __restrict__ tiles,
                                                        const float* __restrict__ tentX, const float2* __restrict__ twg,
                                                        float2* __restrict__ out, int masked) {
    using C = Cfg<N, WV>;
    constexpr int n = C::n;
    __shared__ float2 sbuf[C::RB * C::LSR + kLinePad];
    __shared__ float2 tw[C::TWR];
    const int t = blockIdx.y, i0 = blockIdx.x * C::RB;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_twiddles<N, WV, false>(tw, twg, tid);
    const TileInfo ti = tiles[t];
    const int nk = masked ? ti.nkx : 1;
    const int kstride = masked ? kMaxK : 1;
    const float* xt = x + (size_t)t * N * N;
    float2 xv[kV];
    {
        const float* __restrict__ xl = xt + (size_t)(i0 + wave * C::LwR) * N + rslot_base<N>(lane);
#pragma unroll
        for (int s = 0; s < kV; ++s) xv[s] = *reinterpret_cast<const float2*>(xl + rslot_off<N>(s));
    }
    __syncthreads();
    float2* sw = sbuf + line_off<C::n>(wave * C::LwR);
    for (int k = 0; k < nk; ++k) {
        float2 v[kV];
        const float* __restrict__ bl = tentX + ((size_t)ti.tx * kMaxK + k) * N + rslot_tent<N>(lane);
#pragma unroll
        for (int s = 0; s < kV; ++s) {
            const float* b = bl + rslot_off<N>(s);
            v[s] = masked ? make_float2(b[0] * xv[s].x, b[1] * xv[s].y) : xv[s];
        }
        row_fft_wave<N>(v, sw, tw, lane);
        __syncthreads();
        store_spectrum_T<N, WV>(sbuf, tw, out + ((size_t)t * kstride + k) * C::SPEC, i0, tid);
        __syncthreads();
    }
}

// Packed row half-spectra -> real frames: out = sum_k b_k . C2R(in_k)
// (masked != 0) or C2R(in_0) (masked == 0).
template <int N, int WV>
__global__ __launch_bounds__((Cfg<N, WV>::NT)) void k_row_inv(const float2* __restrict__ in, const TileInfo* __restrict__ tiles,
                                                        const float* __restrict__ tentX, const float2* __restrict__ twg,
                                                        float* __restrict__ out, int masked) {
    using C = Cfg<N, WV>;
    constexpr int n = C::n;
    __shared__ float2 sbuf[C::RB * C::LSR + kLinePad];
    __shared__ float2 tw[C::TWR];
    const int t = blockIdx.y, i0 = blockIdx.x * C::RB;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_twiddles<N, WV, false>(tw, twg, tid);
    const TileInfo ti = tiles[t];
    const int nk = masked ? ti.nkx : 1;
    const int kstride = masked ? kMaxK : 1;
    float2* sw = sbuf + line_off<C::n>(wave * C::LwR);
    float2 acc[kV];
#pragma unroll
    for (int s = 0; s < kV; ++s) acc[s] = make_float2(0.f, 0.f);
    for (int k = 0; k < nk; ++k) {
        __syncthreads();
        load_c2r_T<N, WV>(sbuf, in + ((size_t)t * kstride + k) * C::SPEC, tw, i0, tid);
        __syncthreads();
        float2 v[kV];
        row_c2r_ready<N>(v, sw, tw, lane);
        const float* __restrict__ bl = tentX + ((size_t)ti.tx * kMaxK + k) * N + rslot_tent<N>(lane);
#pragma unroll
        for (int s = 0; s < kV; ++s) {
            if (masked) {
                acc[s].x += bl[rslot_off<N>(s)] * v[s].x;
                acc[s].y += bl[rslot_off<N>(s) + 1] * v[s].y;
            } else {
                acc[s] = v[s];
            }
        }
    }
    float* __restrict__ ol = out + (size_t)t * N * N + (size_t)(i0 + wave * C::LwR) * N + rslot_base<N>(lane);
#pragma unroll
    for (int s = 0; s < kV; ++s) *reinterpret_cast<float2*>(ol + rslot_off<N>(s)) = acc[s];
}

// ---------------------------------------------------------------------------
// Column kernels
// ---------------------------------------------------------------------------

// Work items of the column kernels.  Item I < n_tiles * n_cg is one column
// group of one tile; the packed column 0 of a half-plane carries two real
// columns, DC (real part) and Nyquist (imaginary part): the wave owning
// column 0 treats it as the DC column, and n_nyq = ceil(n_tiles / W) extra
// items give every tile one wave for its Nyquist column (wave w of extra
// item j serves tile j W + w).  Both are then ordinary complex columns
// multiplied by their own spectrum column (0 or N/2), so no wave needs the
// g -> -g exchange of the packed form.
//
// XCD-aware mapping: workgroups go to the 8 XCDs round-robin by linear id,
// so workgroup L runs on XCD L mod 8, and item I = (L mod 8) * per + L / 8
// gives every XCD a contiguous range of items.  The tile order decides what
// that range holds:
//   kOrderColumnMajor  items column-group-major: an XCD works on one or two
//                      column groups of all tiles, and that column block of
//                      every PSF spectrum is shared in its L2 by the up-to-9
//                      tiles that use it;
//   kOrderTileMajor    items tile-major: an XCD holds whole tiles, so the
//                      tile's half-planes stay in one L2;
//   kOrderHeavyFirst   column-group-major over the tiles sorted by their
//                      number of PSF terms, most first (perm), so the longest
//                      items start first.
// perm maps the position of a tile in the order to the tile (identity for
// the first two orders).
enum { kOrderColumnMajor = 0, kOrderTileMajor = 1, kOrderHeavyFirst = 2 };

// Per-lane part of a column slot position: element (q, g) of slot s in
// layout L_R lies at slot_base(lane, ls) + slot_const<N, R>(s) for lines of
// stride ls, so a wave's loads and stores of one transform share one lane
// pointer and differ by compile-time (immediate) offsets.
template <int N>
__device__ __forceinline__ int slot_base(int lane, int ls) {
    constexpr int LPL = lanes_per_line<N>();
    return (lane / LPL) * ls + (lane % LPL);
}

struct ColItem {
    int t;        // tile of this wave
    int f0;       // first packed column of this wave (0 for a Nyquist wave)
    bool nyq;     // this wave transforms the Nyquist column of tile t
    bool valid;   // false: padding workgroup or Nyquist slot beyond the last tile
};

template <int N, int WV>
__device__ __forceinline__ ColItem col_item(int n_tiles, const int* __restrict__ perm, int order, int wave) {
    using C = Cfg<N, WV>;
    const int main_items = n_tiles * C::CG;
    const int items = main_items + (n_tiles + C::W - 1) / C::W;
    const int per = (items + 7) / 8;
    const int L = blockIdx.x;
    const int I = (L % 8) * per + L / 8;
    ColItem it;
    if (I < main_items) {
        int cg, pos;
        if (order == kOrderTileMajor) {
            pos = I / C::CG;
            cg = I - pos * C::CG;
        } else {
            cg = I / n_tiles;
            pos = I - cg * n_tiles;
        }
        it.t = perm[pos];
        it.f0 = cg * C::CB + wave * C::LwC;
        it.nyq = false;
        it.valid = true;
    } else {
        const int pos = (I - main_items) * C::W + wave;
        it.valid = I < items && pos < n_tiles;
        it.t = it.valid ? perm[pos] : 0;
        it.f0 = 0;
        it.nyq = true;
    }
    return it;
}

template <int N, int WV>
constexpr int col_grid(int n_tiles) {
    using C = Cfg<N, WV>;
    const int items = n_tiles * C::CG + (n_tiles + C::W - 1) / C::W;
    return 8 * ((items + 7) / 8);
}

// Column modes of a lane: 0 an ordinary packed column, 1 the DC column (real
// part of packed column 0), 2 the Nyquist column (its imaginary part).
__device__ __forceinline__ int col_mode(const ColItem& it, int line) {
    return it.nyq ? 2 : ((it.f0 == 0 && line == 0) ? 1 : 0);
}

__device__ __forceinline__ float2 col_in(float2 z, int mode) {
    return mode == 0 ? z : make_float2(mode == 1 ? z.x : z.y, 0.f);
}

// Stores a column value: the whole complex value for an ordinary column, the
// real part into .x (DC) or .y (Nyquist) of packed column 0 otherwise (the
// transform of a real column's Hermitian product is real).  A Nyquist wave
// stores from its line 0 only.
__device__ __forceinline__ void col_out(float2* __restrict__ p, float2 v, int mode, int line) {
    if (mode == 0) *p = v;
    else if (mode == 1) reinterpret_cast<float*>(p)[0] = v.x;
    else if (line == 0) reinterpret_cast<float*>(p)[1] = v.x;
}

// Stores a wave's transformed columns (layout L_{nat radix}) from the lane
// pointer of slot_base; ordinary waves (special == false, every lane mode 0)
// store whole complex values without selects.
template <int N>
__device__ __forceinline__ void store_col(float2* __restrict__ pl, const float2 (&v)[kV], bool special, int mode,
                                          int line) {
    constexpr int R = nat_radix<N>();
    if (special) {
#pragma unroll
        for (int s = 0; s < kV; ++s) col_out(pl + slot_const<N, R>(s), v[s], mode, line);
    } else {
#pragma unroll
        for (int s = 0; s < kV; ++s) pl[slot_const<N, R>(s)] = v[s];
    }
}

// Loads the spectrum values of one term for the wave's columns, in the
// forward transform's output layout: column f0 + line, or column N/2 on
// every line of a Nyquist wave.
template <int N, int WV>
__device__ __forceinline__ void load_spec(float2 (&sp)[kV], const float2* __restrict__ base, const ColItem& it,
                                          int lane) {
    constexpr int RL = last_radix<N, kFwd>();
    const int c0 = it.nyq ? N / 2 : it.f0, ls = it.nyq ? 0 : N;
    const float2* __restrict__ bl = base + (size_t)c0 * N + slot_base<N>(lane, ls);
#pragma unroll
    for (int s = 0; s < kV; ++s) sp[s] = bl[slot_const<N, RL>(s)];
}

// Loads the y-tent values of the lane's 20 column slots.  The table is kept
// lane-major: row l + LPL s of a tent row is stored at l kV + s, so a lane's
// values are 80 contiguous bytes, five 16-byte loads.
// Q0 .. Q1 - 1 select a part of the five loads (slots 4 Q0 .. 4 Q1 - 1).
template <int N, int Q0 = 0, int Q1 = kV / 4>
__device__ __forceinline__ void load_tent_col(float (&a)[kV], const float* __restrict__ row, int lane) {
    constexpr int LPL = lanes_per_line<N>();
    static_assert(nat_radix<N>() == kV, "the column slots of a lane must be rows l + LPL s");
    const float4* __restrict__ p = reinterpret_cast<const float4*>(row + (lane % LPL) * kV);
#pragma unroll
    for (int q = Q0; q < Q1; ++q) {
        const float4 f = p[q];
        a[4 * q] = f.x;
        a[4 * q + 1] = f.y;
        a[4 * q + 2] = f.z;
        a[4 * q + 3] = f.w;
    }
}

// H: Yc[f][:] = IFFT_col( sum_{ky,kx} spec_k . FFT_col(a_ky . Z_kx[f][:]) )
template <int N, int WV>
__global__ __launch_bounds__((Cfg<N, WV>::NT)) void k_col_H(const float2* __restrict__ Zk, const TileInfo* __restrict__ tiles,
                                                      const float* __restrict__ tentY, const float2* __restrict__ spec,
                                                      const float2* __restrict__ twg, float2* __restrict__ Yc,
                                                      int n_tiles, const int* __restrict__ perm, int order) {
    using C = Cfg<N, WV>;
    constexpr int LPL = lanes_per_line<N>();
    __shared__ float2 lds[C::W * (C::LwC * C::LSC + kLinePad)];
    __shared__ float2 tw[C::TWC];
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const ColItem it = col_item<N, WV>(n_tiles, perm, order, wave);
    load_twiddles<N, WV, true>(tw, twg, tid);
    __syncthreads();
    if (!it.valid) return;
    const int t = it.t, line = lane / LPL, mode = col_mode(it, line);
    const int ls = it.nyq ? 0 : N;    // a Nyquist wave reads column 0 on every line
    const bool special = it.nyq || it.f0 == 0;   // wave-uniform: some lane has mode != 0
    const TileInfo* tp = tiles + t;
    const int nky = tp->nky, nkx = tp->nkx, ty = tp->ty;
    const int nterm = nky * nkx;
    float2* sw = lds + wave * (C::LwC * C::LSC + kLinePad);
    float2 acc[kV];
#pragma unroll
    for (int s = 0; s < kV; ++s) acc[s] = make_float2(0.f, 0.f);
    // terms kx-major: the wave's columns of Z_kx are read once and kept in
    // registers for all k_y terms of that k_x
    for (int kx = 0; kx < nkx; ++kx) {
        float2 z[kV];
        {
            const int ln = fresh_lane(lane);
            const float2* __restrict__ zl =
                Zk + ((size_t)t * kMaxK + kx) * C::SPEC + (size_t)it.f0 * N + slot_base<N>(ln, ls);
#pragma unroll
            for (int s = 0; s < kV; ++s) z[s] = zl[slot_const<N, nat_radix<N>()>(s)];
            if (special) {
#pragma unroll
                for (int s = 0; s < kV; ++s) z[s] = col_in(z[s], mode);
            }
        }
        for (int ky = 0; ky < nky; ++ky) {
            float2 v[kV];
            {
                float a[kV];
                load_tent_col<N>(a, tentY + ((size_t)ty * kMaxK + ky) * N, fresh_lane(lane));
#pragma unroll
                for (int s = 0; s < kV; ++s) v[s] = cscale(z[s], a[s]);
            }
            fft_passes<N, kFwd>(v, sw, tw, lane);
            // the spectrum in two halves, so that Z, v, acc and the
            // spectrum values fit the register budget together
            constexpr int RL = last_radix<N, kFwd>();
            const int c0 = it.nyq ? N / 2 : it.f0;
            const float2* __restrict__ bl = spec + (size_t)tp->spec[ky * kMaxK + kx] * C::NSPEC + (size_t)c0 * N +
                                            slot_base<N>(fresh_lane(lane), ls);
            {
                float2 h[kV / 2];
#pragma unroll
                for (int s = 0; s < kV / 2; ++s) h[s] = bl[slot_const<N, RL>(s)];
#pragma unroll
                for (int s = 0; s < kV / 2; ++s) acc[s] = cadd(acc[s], cmul(h[s], v[s]));
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                float2 h[kV / 2];
#pragma unroll
                for (int s = 0; s < kV / 2; ++s) h[s] = bl[slot_const<N, RL>(kV / 2 + s)];
#pragma unroll
                for (int s = 0; s < kV / 2; ++s) acc[kV / 2 + s] = cadd(acc[kV / 2 + s], cmul(h[s], v[kV / 2 + s]));
            }
        }
    }
    fft_passes<N, kInv>(acc, sw, tw + C::TWC_F, lane);
    float2* __restrict__ yl = Yc + (size_t)t * C::SPEC + (size_t)it.f0 * N + slot_base<N>(lane, ls);
    store_col<N>(yl, acc, special, mode, line);
}

// H^T: Gk[kx][f][:] = sum_ky a_ky . IFFT_col( conj(spec_k) . FFT_col(Rr[f][:]) )
template <int N, int WV>
__global__ __launch_bounds__((Cfg<N, WV>::NT)) void k_col_Ht(const float2* __restrict__ Rr, const TileInfo* __restrict__ tiles,
                                                       const float* __restrict__ tentY, const float2* __restrict__ spec,
                                                       const float2* __restrict__ twg, float2* __restrict__ Gk,
                                                       int n_tiles, const int* __restrict__ perm, int order) {
    using C = Cfg<N, WV>;
    constexpr int LPL = lanes_per_line<N>();
    __shared__ float2 lds[C::W * (C::LwC * C::LSC + kLinePad)];
    __shared__ float2 tw[C::TWC];
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const ColItem it = col_item<N, WV>(n_tiles, perm, order, wave);
    load_twiddles<N, WV, true>(tw, twg, tid);
    __syncthreads();
    if (!it.valid) return;
    const int t = it.t, line = lane / LPL, mode = col_mode(it, line);
    const int ls = it.nyq ? 0 : N;
    const bool special = it.nyq || it.f0 == 0;   // wave-uniform: some lane has mode != 0
    const TileInfo* tp = tiles + t;
    const int nky = tp->nky, nkx = tp->nkx, ty = tp->ty;
    const int nterm = nky * nkx;
    float2* sw = lds + wave * (C::LwC * C::LSC + kLinePad);
    float2 S[kV], sp[kV], acc[kV];
    {
        const float2* __restrict__ rl = Rr + (size_t)t * C::SPEC + (size_t)it.f0 * N + slot_base<N>(lane, ls);
#pragma unroll
        for (int s = 0; s < kV; ++s) S[s] = col_in(rl[slot_const<N, nat_radix<N>()>(s)], mode);
    }
    fft_passes<N, kFwd>(S, sw, tw, lane);
    for (int term = 0; term < nterm; ++term) {
        const int kx = term / nky, ky = term - kx * nky;
        if (ky == 0) {
#pragma unroll
            for (int s = 0; s < kV; ++s) acc[s] = make_float2(0.f, 0.f);
        }
        load_spec<N, WV>(sp, spec + (size_t)tp->spec[ky * kMaxK + kx] * C::NSPEC, it, fresh_lane(lane));
        float2 v[kV];
#pragma unroll
        for (int s = 0; s < kV; ++s) v[s] = cmulc(S[s], sp[s]);
        fft_passes<N, kInv>(v, sw, tw + C::TWC_F, lane);
        const float* am = tentY + ((size_t)ty * kMaxK + ky) * N;
        {
            // in two parts, so that the tents of the second part are loaded
            // into registers the first part's products have freed
            float a[kV];
            load_tent_col<N, 0, 3>(a, am, fresh_lane(lane));
#pragma unroll
            for (int s = 0; s < 12; ++s) acc[s] = cadd(acc[s], cscale(v[s], a[s]));
            __builtin_amdgcn_sched_barrier(0);
            load_tent_col<N, 3, 5>(a, am, fresh_lane(lane));
#pragma unroll
            for (int s = 12; s < kV; ++s) acc[s] = cadd(acc[s], cscale(v[s], a[s]));
        }
        if (ky == nky - 1) {
            const int ln = fresh_lane(lane);
            float2* __restrict__ gl = Gk + ((size_t)t * kMaxK + kx) * C::SPEC + (size_t)it.f0 * N + slot_base<N>(ln, ls);
            store_col<N>(gl, acc, special, mode, line);
        }
    }
}

// Diagnostic: forward (dir < 0) or unnormalised inverse (dir > 0) FFT of every
// column in[t][f][:] of packed half-planes.
template <int N, int WV>
__global__ __launch_bounds__((Cfg<N, WV>::NT)) void k_col_fft_dbg(const float2* __restrict__ in, const float2* __restrict__ twg,
                                                            float2* __restrict__ out, int dir) {
    using C = Cfg<N, WV>;
    __shared__ float2 lds[C::W * (C::LwC * C::LSC + kLinePad)];
    __shared__ float2 tw[C::TWC];
    const int t = blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int f0 = blockIdx.x * C::CB + wave * C::LwC;
    load_twiddles<N, WV, true>(tw, twg, tid);
    __syncthreads();
    float2* sw = lds + wave * (C::LwC * C::LSC + kLinePad);
    const float2* it = in + (size_t)t * C::SPEC + (size_t)f0 * N;
    float2* ot = out + (size_t)t * C::SPEC + (size_t)f0 * N;
    float2 v[kV];
    if (dir < 0) {
#pragma unroll
        for (int s = 0; s < kV; ++s) {
            int q, g;
            slot_pos<N, first_radix<N, kFwd>()>(lane, s, q, g);
            v[s] = it[(size_t)q * N + g];
        }
        fft_passes<N, kFwd>(v, sw, tw, lane);
#pragma unroll
        for (int s = 0; s < kV; ++s) {
            int q, g;
            slot_pos<N, last_radix<N, kFwd>()>(lane, s, q, g);
            ot[(size_t)q * N + g] = v[s];
        }
    } else {
#pragma unroll
        for (int s = 0; s < kV; ++s) {
            int q, g;
            slot_pos<N, first_radix<N, kInv>()>(lane, s, q, g);
            v[s] = it[(size_t)q * N + g];
        }
        fft_passes<N, kInv>(v, sw, tw + C::TWC_F, lane);
#pragma unroll
        for (int s = 0; s < kV; ++s) {
            int q, g;
            slot_pos<N, last_radix<N, kInv>()>(lane, s, q, g);
            ot[(size_t)q * N + g] = v[s];
        }
    }
}

// ---------------------------------------------------------------------------
// Fused row kernels of the Local-Solver step
// ---------------------------------------------------------------------------

template <int N, int WV>
__device__ __forceinline__ float block_sum(float v, float* red, int tid) {
    using C = Cfg<N, WV>;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    float s = 0.f;
    if (tid == 0) {
        for (int w = 0; w < C::W; ++w) s += red[w];
    }
    return s;   // valid in thread 0
}

// H x (from Yc) -> residual W (H x - y) on the block -> its packed row spectra.
// obj_part[t * RG + rg] = 1/2 sum W (H x - y)^2 over the workgroup's rows.
template <int N, int WV>
__global__ __launch_bounds__((Cfg<N, WV>::NT)) void k_row_resid(const float2* __restrict__ Yc, const float2* __restrict__ yw,
                                                          const float2* __restrict__ twg, float2* __restrict__ Rr,
                                                          float* __restrict__ obj_part, int t0) {
    using C = Cfg<N, WV>;
    constexpr int n = C::n;
    __shared__ float2 sbuf[C::RB * C::LSR + kLinePad];
    __shared__ float2 tw[C::TWR];
    __shared__ float red[C::W];
    const int t = t0 + blockIdx.y, i0 = blockIdx.x * C::RB;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_twiddles<N, WV, false>(tw, twg, tid);
    __syncthreads();
    load_c2r_T<N, WV>(sbuf, Yc + (size_t)t * C::SPEC, tw, i0, tid);
    __syncthreads();
    float2* sw = sbuf + line_off<C::n>(wave * C::LwR);
    float2 v[kV];
    row_c2r_ready<N>(v, sw, tw, lane);
    // (y, W) pairs of pixels (2m, 2m + 1) as one float4, at float2 offset row N + 2m
    const float2* __restrict__ yl = yw + (size_t)t * N * N + (size_t)(i0 + wave * C::LwR) * N + rslot_base<N>(lane);
    float obj = 0.f;
#pragma unroll
    for (int s = 0; s < kV; ++s) {
        const float4 o = *reinterpret_cast<const float4*>(yl + rslot_off<N>(s));   // (y0, W0, y1, W1)
        const float d0 = v[s].x - o.x, d1 = v[s].y - o.z;
        const float r0 = o.y * d0, r1 = o.w * d1;
        obj += r0 * d0 + r1 * d1;
        v[s] = make_float2(r0, r1);
    }
    wave_sync();
    row_fft_wave<N>(v, sw, tw, lane);
    __syncthreads();
    store_spectrum_T<N, WV>(sbuf, tw, Rr + (size_t)t * C::SPEC, i0, tid);
    const float tot = block_sum<N, WV>(obj, red, tid);
    if (tid == 0) obj_part[t * C::RG + blockIdx.x] = 0.5f * tot;
}

// Projection onto the non-negative orthant. Written as a compare rather than
// fmaxf so that a NaN (a diverged step) stays NaN, as max(0, NaN) does in the
// definition, and the non-finite check sees it instead of a clamped 0.
__device__ __forceinline__ float project_nonneg(float v) { return v < 0.f ? 0.f : v; }

// Scale of the regulariser's derivative for a forward-difference vector g:
// d phi / d g = s(g) g with s = 1/sqrt(|g|^2 + eps^2) (smoothed TV) or
// delta / max(|g|, delta) (Huber).
// REG is the regulariser kind (0: smoothed TV, 1: Huber) and rp its eps or
// delta.  For smoothed TV the argument of the reciprocal square root is at
// least eps^2, a normal number (eps >= 2^-63 is required at creation), where
// the hardware's reciprocal square root equals rsqrtf (whose extra steps
// only rescale subnormal arguments).
template <int REG>
__device__ __forceinline__ float reg_scale_k(float gh, float gv, float rp) {
    const float n2 = gh * gh + gv * gv;
    if constexpr (REG == 0) return __builtin_amdgcn_rsqf(n2 + rp * rp);
    else return rp * __frcp_rn(fmaxf(sqrtf(n2), rp));
}
__device__ __forceinline__ float reg_scale(float gh, float gv, const SolveParams& P) {
    return P.reg == 0 ? reg_scale_k<0>(gh, gv, P.reg_param) : reg_scale_k<1>(gh, gv, P.reg_param);
}
template <int V> struct IntC { static constexpr int value = V; };

// Value of v in the next (lane + 1) and previous (lane - 1) lane of the wave,
// by a whole-wave DPP shift (a VALU operation, no LDS traffic); lane 63
// resp. lane 0 receive 0.  Every lane must execute the call.
__device__ __forceinline__ float from_next_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_prev_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}

// Tasks of the column-strip update phase: every column split into segments
// of kSeg rows, (N / RB-row workgroup) -> N * RB / kSeg tasks, a multiple of NT.
constexpr int kSeg = 8;
static_assert((kSeg & (kSeg - 1)) == 0, "the strip rows are picked by lane mod kSeg");

// H^T r (from Gk), regulariser and metric terms, projected step; then the
// masked row spectra of the new iterate for the next step.
//
// Phase 1: per mask k, transposed load of G_k, row C2R, accumulate b_k . (.)
//          into the data gradient (registers), then park it in LDS as
//          natural [row][col] floats.
// Phase 2: strips of 8 rows walked top to bottom, carrying the vertical flux
//          of the row above: with Neumann differences a wave owns 62
//          columns of a strip and takes horizontal neighbours from adjacent
//          lanes (one regulariser scale per pixel); with circular
//          differences a thread owns one column and loads x at c - 1, c and
//          c + 1.  Writes the new x frame, and the new value of each pixel
//          over its gradient in LDS.
// Phase 3: each wave reads its rows of the new x from LDS and, per mask k,
//          does the forward row FFT and the transposed store of Z_k.
//
// FISTA (accelerated Local-Solver): xc holds the gradient point y_j, the
// projected step gives w_j, which is stored in wb, and the next gradient
// point y_{j+1} = w_j + beta (w_j - w_{j-1}) (w_{j-1} read from wb) is
// written to xn and transformed in phase 3.  beta = 0 makes y_{j+1} = w_j.
template <int N, int WV, bool FISTA = false>
__global__ __launch_bounds__((Cfg<N, WV>::NT)) void k_row_update(
        const float2* __restrict__ Gk, const float* __restrict__ xc, const float* __restrict__ u,
        const TileInfo* __restrict__ tiles, const float* __restrict__ tentX, const float* __restrict__ omY,
        const float* __restrict__ omX, const float* __restrict__ tau, SolveParams P,
        const float2* __restrict__ twg, float* __restrict__ xn, float2* __restrict__ Zk, int t0,
        float beta, float* __restrict__ wb) {
    using C = Cfg<N, WV>;
    constexpr int n = C::n;
    static_assert(C::RB * N * sizeof(float) <= C::RB * C::LSR * sizeof(float2), "LDS view too small");
    static_assert((N * (C::RB / kSeg)) % C::NT == 0, "update tasks do not divide the workgroup");
    __shared__ float2 sbuf[C::RB * C::LSR + kLinePad];
    __shared__ float2 tw[C::TWR];
    float* sg = reinterpret_cast<float*>(sbuf);   // [RB][N] natural view
    const int t = t0 + blockIdx.y, i0 = blockIdx.x * C::RB;
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    load_twiddles<N, WV, false>(tw, twg, tid);
    const TileInfo ti = tiles[t];
    float2* sw = sbuf + line_off<C::n>(wave * C::LwR);

    // ---- phase 1: data gradient H^T r
    {
        float2 gd[kV];
#pragma unroll
        for (int s = 0; s < kV; ++s) gd[s] = make_float2(0.f, 0.f);
        for (int kx = 0; kx < ti.nkx; ++kx) {
            __syncthreads();
            load_c2r_T<N, WV>(sbuf, Gk + ((size_t)t * kMaxK + kx) * C::SPEC, tw, i0, tid);
            __syncthreads();
            float2 v[kV];
            row_c2r_ready<N>(v, sw, tw, lane);
            const float* __restrict__ bl = tentX + ((size_t)ti.tx * kMaxK + kx) * N + rslot_tent<N>(lane);
#pragma unroll
            for (int s = 0; s < kV; ++s) {
                const float2 b = *reinterpret_cast<const float2*>(bl + rslot_off<N>(s));
                gd[s].x += b.x * v[s].x;
                gd[s].y += b.y * v[s].y;
            }
        }
        __syncthreads();
        {
            float* gl = sg + wave * C::LwR * N + rslot_base<N>(lane);
#pragma unroll
            for (int s = 0; s < kV; ++s) *reinterpret_cast<float2*>(gl + rslot_off<N>(s)) = gd[s];
        }
        __syncthreads();
    }

    // ---- phase 2: regulariser, metric term, projected step (column strips)
    {
        const float* xt = xc + (size_t)t * N * N;
        const float* ut = u + (size_t)t * N * N;
        float* xo = xn + (size_t)t * N * N;
        float* wt = nullptr;
        if constexpr (FISTA) wt = wb + (size_t)t * N * N;
        const float tt = tau[t];
        const float* oy = omY + (size_t)ti.ty * N;
        const float* ox = omX + (size_t)ti.tx * N;
        const int sy = ti.sy, sx = ti.sx;
        const bool circ = P.bc != 0;
        constexpr int SEGS = C::RB / kSeg;
        constexpr int TASKS = N * SEGS / C::NT;   // per thread (5 for every frame size)
        if (!circ) {
            // Neumann differences: wave-wide strips.  A task is kSeg rows of
            // 64 consecutive columns c0 - 1 .. c0 + 62; lanes 1..62 own their
            // column, lanes 0 and 63 are halo.  Each lane evaluates the
            // regulariser scale of its own pixel once; x(i, c + 1) and the
            // left neighbour's horizontal flux s gh come from the adjacent
            // lanes.  The loads of a wave's next two tasks are in flight while
            // the current task is computed (three register buffers).
            constexpr int OWN = kLanes - 2;
            constexpr int NCG = (N + OWN - 1) / OWN;
            constexpr int NTASK = NCG * SEGS;
            // U holds u on the task's rows, then (FISTA) the previous w_{j-1}
            constexpr int UN = FISTA ? 2 * kSeg : kSeg;
            // O[0] = omega_x of the lane's column, O[1] = omega_y of the
            // strip's row ia + (lane mod kSeg), read per row by readlane: the
            // update issues no global load of its own, so its waits never
            // reach the later strips' loads (the load counter drains in order)
            auto load = [&](int task, float (&X)[kSeg + 2], float (&U)[UN], float (&O)[2]) {
                const int c = (task % NCG) * OWN - 1 + lane;
                const int ia = i0 + (task / NCG) * kSeg;
                // Every load is unconditional, from the column and the halo
                // rows clamped into the frame (rows ia .. ia + kSeg - 1 lie
                // in it); the update replaces a value outside the support by
                // 0 when it uses it, so no exec-mask branch guards a load and
                // no wait for these loads is taken before that use.
                const int cc = min(max(c, 0), N - 1);
                const size_t o = (size_t)ia * N + cc;
                const float* __restrict__ xs = xt + o;
                const float* __restrict__ us = ut + o;
                X[0] = xt[(size_t)max(ia - 1, 0) * N + cc];
#pragma unroll
                for (int j = 1; j <= kSeg; ++j) X[j] = xs[(j - 1) * N];
                X[kSeg + 1] = xt[(size_t)min(ia + kSeg, N - 1) * N + cc];
#pragma unroll
                for (int k = 0; k < kSeg; ++k) U[k] = us[k * N];
                if constexpr (FISTA) {
                    const float* __restrict__ ws = wt + o;
#pragma unroll
                    for (int k = 0; k < kSeg; ++k) U[kSeg + k] = ws[k * N];
                }
                O[0] = ox[cc];
                O[1] = oy[min(ia + (lane & (kSeg - 1)), N - 1)];
            };
            // the regulariser kind is a compile-time constant of each strip
            // loop, so its scale takes no per-pixel branch
            auto update = [&](auto regc, int task, const float (&XL)[kSeg + 2], const float (&UL)[UN],
                              const float (&O)[2]) {
                constexpr int REG = decltype(regc)::value;
                const int c = (task % NCG) * OWN - 1 + lane;
                const int ia = i0 + (task / NCG) * kSeg;
                // the loaded values, 0 outside the support
                float X[kSeg + 2], U[UN];
                {
                    const bool cin = c >= 0 && c < sx;
#pragma unroll
                    for (int j = 0; j < kSeg + 2; ++j) {
                        const int rr = ia - 1 + j;
                        X[j] = (cin && rr >= 0 && rr < sy) ? XL[j] : 0.f;
                    }
#pragma unroll
                    for (int k = 0; k < UN; ++k) U[k] = (cin && ia + k % kSeg < sy) ? UL[k] : 0.f;
                }
                // pixel (ia, c) in the frame and in sg; row ia + k at offset k N
                const size_t o = (size_t)ia * N + c;
                const float* sgs = sg + (ia - i0) * N + c;
                float* sgw = sg + (ia - i0) * N + c;   // the same pixel: its new value
                float* __restrict__ xos = xo + o;
                const bool colin = c >= 0 && c < sx;
                const bool rin = c + 1 < sx;   // the right neighbour is in the support
                // lanes 1..OWN own their column; the halo lanes only supply
                // neighbour values and never touch the LDS frame, whose
                // pixels their neighbouring tasks overwrite
                const bool own = lane >= 1 && lane <= OWN && c < N;
                // vertical flux of the row above the strip
                float qv_up = 0.f;
                {
                    const float xr = from_next_lane(X[0]);
                    if (colin && ia >= 1 && ia < sy) {
                        const float gh = rin ? xr - X[0] : 0.f;
                        const float gv = X[1] - X[0];
                        qv_up = reg_scale_k<REG>(gh, gv, P.reg_param) * gv;
                    }
                }
                const float oxc = colin ? O[0] : 0.f;
#pragma unroll
                for (int k = 0; k < kSeg; ++k) {
                    const int i = ia + k;
                    const float oyi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(O[1]), k));
                    const bool pin = colin && i < sy;
                    const float xm = X[k + 1];
                    const float xr = from_next_lane(xm);
                    const float gh = (pin && rin) ? xr - xm : 0.f;
                    const float gv = (pin && i + 1 < sy) ? X[k + 2] - xm : 0.f;
                    const float sc = reg_scale_k<REG>(gh, gv, P.reg_param);
                    const float qh = sc * gh, qv = sc * gv;
                    const float qh_l = from_prev_lane(qh);
                    float val = 0.f;
                    if (pin && own) {
                        // -div of the flux (s gh, s gv): backward differences
                        const float g = (qh_l - qh) + (qv_up - qv);
                        const float alpha = P.gamma * oyi * oxc;
                        const float grad = sgs[k * N] + P.lambda * g + alpha * (xm - U[k]);
                        val = xm - tt * grad;
                        if (P.positivity) val = project_nonneg(val);
                    }
                    qv_up = qv;
                    if (own) {
                        float xv = val;
                        if constexpr (FISTA) {
                            wt[o + (size_t)k * N] = val;
                            if (beta != 0.f) xv = val + beta * (val - U[kSeg + k]);
                        }
                        xos[k * N] = xv;
                        sgw[k * N] = xv;
                    }
                }
            };
            auto strips = [&](auto regc) {
                float XA[kSeg + 2], UA[UN], XB[kSeg + 2], UB[UN], XC[kSeg + 2], UC[UN];
                float OA[2], OB[2], OC[2];
                constexpr int S = C::W;   // task stride of a wave
                // loads are issued unconditionally (a task past the last one
                // reloads the last task's strip, unused), so the load counter
                // sees the same sequence on every path and each update waits
                // only for its own strip
                const auto ld = [&](int task, float (&X)[kSeg + 2], float (&U)[UN], float (&O)[2]) {
                    load(min(task, NTASK - 1), X, U, O);
                };
                ld(wave, XA, UA, OA);
                ld(wave + S, XB, UB, OB);
                for (int task = wave; task < NTASK; task += 3 * S) {
                    ld(task + 2 * S, XC, UC, OC);
                    update(regc, task, XA, UA, OA);
                    if (task + S >= NTASK) break;
                    ld(task + 3 * S, XA, UA, OA);
                    update(regc, task + S, XB, UB, OB);
                    if (task + 2 * S >= NTASK) break;
                    ld(task + 4 * S, XB, UB, OB);
                    update(regc, task + 2 * S, XC, UC, OC);
                }
            };
            if (P.reg == 0) strips(IntC<0>{});
            else strips(IntC<1>{});
        } else {
            // Circular differences (this branch runs only for them): one thread
            // per (column, kSeg rows), x at c - 1, c and c + 1 (wrapping around
            // the support) per row.  Two tasks per step.  All their loads, with
            // omega_x, omega_y and (FISTA) w_{j-1}, are issued together and
            // unconditionally (every index lies in the frame), and a value
            // outside the support is replaced by 0 where it is used, so the
            // update issues no global load of its own (a wait for one would
            // drain every load issued before it).
            constexpr int UN = FISTA ? 2 * kSeg : kSeg;   // u, then (FISTA) w_{j-1}
            auto circ_strips = [&](auto regc) {
                constexpr int REG = decltype(regc)::value;
                for (int t2 = 0; t2 < TASKS; t2 += 2) {
                    float X[2][kSeg + 2][3];
                    float U[2][UN], OY[2][kSeg], OX[2];
                    int cc[2], iaa[2];
                    bool act[2];
    #pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        act[h] = t2 + h < TASKS;
                        // an inactive slot loads the last task again (unused)
                        const int task = tid + min(t2 + h, TASKS - 1) * C::NT;
                        const int c = task % N;
                        const int ia = i0 + (task / N) * kSeg;
                        cc[h] = c;
                        iaa[h] = ia;
                        const int cl = c >= 1 ? c - 1 : sx - 1, cr = c + 1 < sx ? c + 1 : 0;
    #pragma unroll
                        for (int j = 0; j < kSeg + 2; ++j) {
                            int rr = ia - 1 + j;
                            if (rr < 0) rr = sy - 1;
                            else if (rr >= sy) rr = 0;   // row sy wraps to 0; rows past it are masked
                            const float* rowp = xt + (size_t)rr * N;
                            X[h][j][0] = rowp[cl];
                            X[h][j][1] = rowp[c];
                            X[h][j][2] = rowp[cr];
                        }
    #pragma unroll
                        for (int k = 0; k < kSeg; ++k) U[h][k] = ut[(size_t)(ia + k) * N + c];
                        if constexpr (FISTA) {
    #pragma unroll
                            for (int k = 0; k < kSeg; ++k) U[h][kSeg + k] = wt[(size_t)(ia + k) * N + c];
                        }
                        OX[h] = ox[c];
    #pragma unroll
                        for (int k = 0; k < kSeg; ++k) OY[h][k] = oy[ia + k];
                    }
    #pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (!act[h]) continue;
                        const int c = cc[h], ia = iaa[h];
                        const bool colin = c < sx;
                        // the loaded rows, 0 where the row lies outside the support
                        // (rows past the wrapped row sy) or the column does
                        float Xv[kSeg + 2][3];
    #pragma unroll
                        for (int j = 0; j < kSeg + 2; ++j) {
                            const int rr = ia - 1 + j;
                            const bool ok = colin && rr <= sy;
    #pragma unroll
                            for (int m = 0; m < 3; ++m) Xv[j][m] = ok ? X[h][j][m] : 0.f;
                        }
                        const float oxc = colin ? OX[h] : 0.f;
                        // vertical term of the row above the segment: qv(ia-1, c)
                        float qv_up = 0.f;
                        if (colin && ia < sy) {
                            const float gh = Xv[0][2] - Xv[0][1];
                            const float gv = Xv[1][1] - Xv[0][1];
                            qv_up = reg_scale_k<REG>(gh, gv, P.reg_param) * gv;
                        }
    #pragma unroll
                        for (int k = 0; k < kSeg; ++k) {
                            const int i = ia + k;
                            float val = 0.f;
                            if (colin && i < sy) {
                                const float xm = Xv[k + 1][1];
                                const float gh = Xv[k + 1][2] - xm;
                                const float gv = Xv[k + 2][1] - xm;
                                const float sc = reg_scale_k<REG>(gh, gv, P.reg_param);
                                float g = qv_up - sc * (gh + gv);
                                {
                                    const float xl = Xv[k + 1][0];
                                    const float ghl = xm - xl;   // column c is the right neighbour of c-1
                                    const float gvl = Xv[k + 2][0] - xl;
                                    g += reg_scale_k<REG>(ghl, gvl, P.reg_param) * ghl;
                                }
                                qv_up = sc * gv;
                                const float alpha = P.gamma * OY[h][k] * oxc;
                                const float grad = sg[(i - i0) * N + c] + P.lambda * g + alpha * (xm - U[h][k]);
                                val = xm - tt * grad;
                                if (P.positivity) val = project_nonneg(val);
                            }
                            float xv = val;
                            if constexpr (FISTA) {
                                const float wp = U[h][kSeg + k];   // w_{j-1}: 0 outside the support
                                wt[(size_t)i * N + c] = val;
                                if (beta != 0.f) xv = val + beta * (val - wp);
                            }
                            xo[(size_t)i * N + c] = xv;
                            sg[(i - i0) * N + c] = xv;
                        }
                    }
                }
            };
            if (P.reg == 0) circ_strips(IntC<0>{});
            else circ_strips(IntC<1>{});
        }
        __syncthreads();
    }

    // ---- phase 3: forward row spectra of b_k . x_new.  Phase 2 left x_new
    // in the LDS frame (each pixel's gradient replaced by its new value);
    // the wave's rows are read from there once and kept in registers for
    // every k_x.
    float2 xr[kV];
    {
        const float* __restrict__ xl = sg + wave * C::LwR * N + rslot_base<N>(fresh_lane(lane));
#pragma unroll
        for (int s = 0; s < kV; ++s) xr[s] = *reinterpret_cast<const float2*>(xl + rslot_off<N>(s));
    }
    for (int kx = 0; kx < ti.nkx; ++kx) {
        const float* bm = tentX + ((size_t)ti.tx * kMaxK + kx) * N;
        float2 v[kV];
        const int ln = fresh_lane(lane);
        const float* __restrict__ bl = bm + rslot_tent<N>(ln);
#pragma unroll
        for (int s = 0; s < kV; ++s) {
            const float2 b = *reinterpret_cast<const float2*>(bl + rslot_off<N>(s));
            v[s] = make_float2(b.x * xr[s].x, b.y * xr[s].y);
        }
        __syncthreads();
        row_fft_wave<N>(v, sw, tw, lane);
        __syncthreads();
        store_spectrum_T<N, WV>(sbuf, tw, Zk + ((size_t)t * kMaxK + kx) * C::SPEC, i0, tid);
    }
}

// ---------------------------------------------------------------------------
// Consensus, assembly and bookkeeping (one thread per pixel of X)
// ---------------------------------------------------------------------------

constexpr int kPixBlock = 256;

__device__ __forceinline__ float2 block_sum2(float2 v, float2* red, int tid) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    float2 s = make_float2(0.f, 0.f);
    if (tid == 0) {
        for (int w = 0; w < kPixBlock / 64; ++w) {
            s.x += red[w].x;
            s.y += red[w].y;
        }
    }
    return s;
}

// zbar = sum omega (2x - u) / sum omega over covering tiles; u += rho (zbar - x).
// part[block] = (sum (u_new - u_old)^2, sum u_new^2) over the pixels' tile copies.
// MAXC: the most tiles covering an X row or column (2 in the pitch layout,
// 3 in the grid layout), a compile-time bound for the per-pixel arrays.
template <int MAXC>
__global__ __launch_bounds__(kPixBlock) void k_consensus(const float* __restrict__ x, float* __restrict__ u,
                                                        const Cover* __restrict__ cy, const Cover* __restrict__ cx,
                                                        int Xy, int Xx, int Tx, int N, float rho,
                                                        float2* __restrict__ part) {
    __shared__ float2 red[kPixBlock / 64];
    const int tid = threadIdx.x;
    const int J = blockIdx.x * kPixBlock + tid, I = blockIdx.y;
    float du2 = 0.f, un2 = 0.f;
    if (J < Xx) {
        const Cover a = cy[I], b = cx[J];
        size_t idx[MAXC * MAXC];
        float xv[MAXC * MAXC], uv[MAXC * MAXC];
        float num = 0.f, den = 0.f;
        int k = 0;
#pragma unroll
        for (int ia = 0; ia < MAXC; ++ia) {
            if (ia >= a.n) break;
#pragma unroll
            for (int ib = 0; ib < MAXC; ++ib) {
                if (ib >= b.n) break;
                const float w = a.w[ia] * b.w[ib];
                idx[k] = ((size_t)(a.a[ia] * Tx + b.a[ib]) * N + a.m[ia]) * N + b.m[ib];
                xv[k] = x[idx[k]];
                uv[k] = u[idx[k]];
                num += w * (2.f * xv[k] - uv[k]);
                den += w;
                ++k;
            }
        }
        const float zb = num / den;
#pragma unroll
        for (int j = 0; j < MAXC * MAXC; ++j) {
            if (j >= k) break;
            const float un = uv[j] + rho * (zb - xv[j]);
            u[idx[j]] = un;
            du2 += (un - uv[j]) * (un - uv[j]);
            un2 += un * un;
        }
    }
    const float2 s = block_sum2(make_float2(du2, un2), red, tid);
    if (tid == 0) part[(size_t)I * gridDim.x + blockIdx.x] = s;
}

// Fixed-order reduction of the consensus partials into the residual
// ||u_new - u_old|| / ||u_new||, written to hist[*counter] and *last.
// Thread t sums partials t, t + 1024, ... in that order; the 1024 sums are
// combined by a fixed butterfly in each wave and then wave by wave.
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void k_finalize_residual(const float2* __restrict__ part, int np,
                                                                  double* __restrict__ hist,
                                                                  int* __restrict__ counter,
                                                                  double* __restrict__ last, int cap) {
    __shared__ double sa[kFinThreads / 64], sb[kFinThreads / 64];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0;
#pragma unroll 8
    for (int i = tid; i < np; i += kFinThreads) {
        const float2 p = part[i];
        a += (double)p.x;
        b += (double)p.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if ((tid & 63) == 0) {
        sa[tid >> 6] = a;
        sb[tid >> 6] = b;
    }
    __syncthreads();
    if (tid == 0) {
        double A = 0.0, B = 0.0;
        for (int w = 0; w < kFinThreads / 64; ++w) {
            A += sa[w];
            B += sb[w];
        }
        const double res = B > 0.0 ? sqrt(A / B) : 0.0;
        const double out = (isfinite(A) && isfinite(B)) ? res : (double)NAN;
        *last = out;
        const int k = *counter;
        if (k < cap) hist[k] = out;
        *counter = k + 1;
    }
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// x_hat = sum omega x / sum omega on X.
__global__ __launch_bounds__(kPixBlock) void k_assemble(const float* __restrict__ x, const Cover* __restrict__ cy,
                                                       const Cover* __restrict__ cx, int Xx, int Tx, int N,
                                                       float* __restrict__ out) {
    const int J = blockIdx.x * kPixBlock + threadIdx.x, I = blockIdx.y;
    if (J >= Xx) return;
    const Cover a = cy[I], b = cx[J];
    float num = 0.f, den = 0.f;
    for (int ia = 0; ia < a.n; ++ia) {
        for (int ib = 0; ib < b.n; ++ib) {
            const float w = a.w[ia] * b.w[ib];
            num += w * x[((size_t)(a.a[ia] * Tx + b.a[ib]) * N + a.m[ia]) * N + b.m[ib]];
            den += w;
        }
    }
    out[(size_t)I * Xx + J] = num / den;
}

// ---------------------------------------------------------------------------
// Packing between user layouts and frames
// ---------------------------------------------------------------------------

struct PackDesc {        // per tile
    int y0, x0;          // frame coordinate of the region's first pixel
    int h, w;            // region size
    long long off;       // float offset in the packed array
};

// frames[t] = region from packed (zero elsewhere in the frame)
__global__ void k_pack(const float* __restrict__ packed, const PackDesc* __restrict__ d, int N,
                       float* __restrict__ frames) {
    const int t = blockIdx.y;
    const PackDesc pd = d[t];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
        const int m = e / N - pd.y0, c = e % N - pd.x0;
        float v = 0.f;
        if (m >= 0 && m < pd.h && c >= 0 && c < pd.w) v = packed[pd.off + (long long)m * pd.w + c];
        frames[(size_t)t * N * N + e] = v;
    }
}

__global__ void k_unpack(const float* __restrict__ frames, const PackDesc* __restrict__ d, int N,
                         float* __restrict__ packed) {
    const int t = blockIdx.y;
    const PackDesc pd = d[t];
    const int tot = pd.h * pd.w;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
        const int m = e / pd.w, c = e % pd.w;
        packed[pd.off + e] = frames[(size_t)t * N * N + (size_t)(m + pd.y0) * N + (c + pd.x0)];
    }
}

// Global image on X -> support frames (zero outside supports).
__global__ void k_scatter_X(const float* __restrict__ xg, const TileInfo* __restrict__ tiles,
                            const int* __restrict__ org, int Xx, int N, float* __restrict__ frames) {
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const int oy = org[2 * t], ox = org[2 * t + 1];   // X index of the support origin
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
        const int m = e / N, c = e % N;
        float v = 0.f;
        if (m < ti.sy && c < ti.sx) v = xg[(size_t)(oy + m) * Xx + ox + c];
        frames[(size_t)t * N * N + e] = v;
    }
}

// Observed y (global) <- frames' block regions, each pixel from its owner tile.
__global__ void k_gather_owner(const float* __restrict__ frames, int My, int Mx, int pitch, int Ty, int Tx, int N,
                               int r, float* __restrict__ y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= Mx) return;
    const int a = min(i / pitch, Ty - 1), b = min(j / pitch, Tx - 1);
    const int m = i - a * pitch + r, c = j - b * pitch + r;
    y[(size_t)i * Mx + j] = frames[((size_t)(a * Tx + b) * N + m) * N + c];
}

// (y, W) frames on the block region from the global observation.
__global__ void k_set_obs(const float* __restrict__ y, const float* __restrict__ w, const TileInfo* __restrict__ tiles,
                          const int* __restrict__ borg, int Mx, int N, int r, float2* __restrict__ yw) {
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const int by0 = borg[2 * t], bx0 = borg[2 * t + 1];   // observed coordinate of the block origin
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
        const int m = e / N - r, c = e % N - r;
        float2 v = make_float2(0.f, 0.f);
        if (m >= 0 && m < ti.by && c >= 0 && c < ti.bx) {
            const size_t g = (size_t)(by0 + m) * Mx + (bx0 + c);
            v = make_float2(y[g], w ? w[g] : 1.0f);
        }
        yw[(size_t)t * N * N + e] = v;
    }
}

// x0 = max(y, 0) at the nearest observed pixel, on the supports; u0 = x0.
__global__ void k_init_observed(const float* __restrict__ y, const TileInfo* __restrict__ tiles,
                                const int* __restrict__ sorg, int My, int Mx, int N, float* __restrict__ x,
                                float* __restrict__ u) {
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const int sy0 = sorg[2 * t], sx0 = sorg[2 * t + 1];   // observed coordinate of the support origin
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
        const int m = e / N, c = e % N;
        float v = 0.f;
        if (m < ti.sy && c < ti.sx) {
            const int gi = min(max(sy0 + m, 0), My - 1), gj = min(max(sx0 + c, 0), Mx - 1);
            v = fmaxf(y[(size_t)gi * Mx + gj], 0.f);
        }
        x[(size_t)t * N * N + e] = v;
        u[(size_t)t * N * N + e] = v;
    }
}

__global__ void k_copy(const float* __restrict__ a, float* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void k_fill(float* __restrict__ a, float v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// Per-tile maximum over the block region of a frame array (stride 1) or of the
// W component of the (y, W) frames (stride 2, offset 1).
// Per tile: the maximum over the block of a frame component, or NaN if a
// value there is not finite (or, with nonneg, negative).
__global__ __launch_bounds__(256) void k_block_max(const float* __restrict__ fr, int stride, int off,
                                                  const TileInfo* __restrict__ tiles, int N, int r,
                                                  float* __restrict__ out, int nonneg) {
    __shared__ float red[256];
    const int t = blockIdx.x;
    const TileInfo ti = tiles[t];
    float m = -INFINITY;
    int bad = 0;
    for (int e = threadIdx.x; e < ti.by * ti.bx; e += 256) {
        const int i = e / ti.bx + r, c = e % ti.bx + r;
        const float v = fr[((size_t)t * N * N + (size_t)i * N + c) * stride + off];
        bad |= !isfinite(v) || (nonneg && v < 0.f);
        m = fmaxf(m, v);
    }
    bad = __syncthreads_or(bad);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[t] = bad ? NAN : red[0];
}

// flag[t] = (1 if frame t of x holds a non-finite value) + (2 if frame t of
// u does) (one workgroup per tile; an error path only).
__global__ __launch_bounds__(256) void k_tile_nonfinite(const float* __restrict__ x, const float* __restrict__ u,
                                                       int N, int* __restrict__ flag) {
    const int t = blockIdx.x;
    const size_t base = (size_t)t * N * N;
    int bx = 0, bu = 0;
    for (int e = threadIdx.x; e < N * N; e += 256) {
        bx |= !isfinite(x[base + e]);
        bu |= !isfinite(u[base + e]);
    }
    bx = __syncthreads_or(bx);
    bu = __syncthreads_or(bu);
    if (threadIdx.x == 0) flag[t] = (bx ? 1 : 0) + (bu ? 2 : 0);
}

// Regulariser value and metric term per tile and row block:
// part[t * gridDim.x + blk] = (sum phi(D x), sum 1/2 alpha (x - u)^2).
__global__ __launch_bounds__(256) void k_reg_terms(const float* __restrict__ x, const float* __restrict__ u,
                                                  const TileInfo* __restrict__ tiles, const float* __restrict__ omY,
                                                  const float* __restrict__ omX, int N, SolveParams P,
                                                  double* __restrict__ part) {
    __shared__ double ra[256], rb[256];
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const float* xt = x + (size_t)t * N * N;
    const float* ut = u + (size_t)t * N * N;
    double sa = 0.0, sb = 0.0;
    const int rows_per = (ti.sy + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * rows_per, r1 = min(ti.sy, r0 + rows_per);
    for (int e = threadIdx.x; e < (r1 - r0) * ti.sx; e += 256) {
        const int i = r0 + e / ti.sx, c = e % ti.sx;
        const float x0 = xt[(size_t)i * N + c];
        float gh, gv;
        if (P.bc) {
            gh = xt[(size_t)i * N + (c + 1 < ti.sx ? c + 1 : 0)] - x0;
            gv = xt[(size_t)(i + 1 < ti.sy ? i + 1 : 0) * N + c] - x0;
        } else {
            gh = c + 1 < ti.sx ? xt[(size_t)i * N + c + 1] - x0 : 0.f;
            gv = i + 1 < ti.sy ? xt[(size_t)(i + 1) * N + c] - x0 : 0.f;
        }
        const double n2 = (double)gh * gh + (double)gv * gv;
        const double p = P.reg_param;
        double phi;
        if (P.reg == 0) {
            phi = sqrt(n2 + p * p) - p;
        } else {
            const double nn = sqrt(n2);
            phi = nn <= p ? 0.5 * n2 : p * (nn - 0.5 * p);
        }
        sa += phi;
        const double d = (double)x0 - ut[(size_t)i * N + c];
        sb += 0.5 * (double)P.gamma * omY[(size_t)ti.ty * N + i] * omX[(size_t)ti.tx * N + c] * d * d;
    }
    ra[threadIdx.x] = sa;
    rb[threadIdx.x] = sb;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            ra[threadIdx.x] += ra[threadIdx.x + o];
            rb[threadIdx.x] += rb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * ((size_t)t * gridDim.x + blockIdx.x)] = ra[0];
        part[2 * ((size_t)t * gridDim.x + blockIdx.x) + 1] = rb[0];
    }
}

// PSF spectra by a direct 2-D DFT in fp64 (setup only).  For each node and
// each stored column f in [0, N/2] and row frequency g:
//   H(g, f) = sum_q h(q) exp(-2 pi i (g qy + f qx) / N), scaled by 2/N^2,
// stored as described at the top of this file.  twd[k] = exp(-2 pi i k / N)
// in fp64; dynamic LDS holds a copy (N double2).
__global__ void k_psf_spectra(const float* __restrict__ psf, int P, int N, const double2* __restrict__ twd,
                              float2* __restrict__ spec) {
    extern __shared__ double2 tws[];
    for (int e = threadIdx.x; e < N; e += blockDim.x) tws[e] = twd[e];
    __syncthreads();
    const int node = blockIdx.y;
    const int r = P / 2;
    const int nf = N / 2 + 1;
    const float* h = psf + (size_t)node * P * P;
    const double scale = 2.0 / ((double)N * N);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nf * N; e += gridDim.x * blockDim.x) {
        const int f = e / N, g = e % N;
        auto dft = [&](int ff) {
            double re = 0.0, im = 0.0;
            for (int a = 0; a < P; ++a) {
                const int qy = a - r;
                int ph = (int)(((long long)g * qy) % N);
                if (ph < 0) ph += N;
                int phx = (int)(((long long)ff * (-r)) % N);
                if (phx < 0) phx += N;
                int p0 = ph + phx;
                if (p0 >= N) p0 -= N;
                for (int b = 0; b < P; ++b) {
                    const double2 w = tws[p0];
                    const double hv = h[a * P + b];
                    re += hv * w.x;
                    im += hv * w.y;
                    p0 += ff;
                    if (p0 >= N) p0 -= N;
                }
            }
            return make_double2(re * scale, im * scale);
        };
        const double2 v = dft(f);
        const float2 out = make_float2((float)v.x, (float)v.y);
        spec[(size_t)node * nf * N + (size_t)f * N + g] = out;
    }
}

}  // namespace dbl
