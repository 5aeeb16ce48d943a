// VMLM-B Local-Solver (Section IV-B): limited-memory variable metric (BFGS)
// with the bound x >= 0, batched over all tiles, each tile with its own
// memory of pairs and its own line search.
//
// One iteration of tile t, from w with prox gradient g (f_t plus the metric
// term 1/2 ||w - u_t||^2_alpha):
//   F  = free variables: all but w_i <= 0 with g_i > 0 (all without positivity)
//   d  = -F . B (F . g), B the inverse BFGS matrix of the last kVmMem pairs
//        (s_i, y_i) by the two-loop recursion, initial scaling <s,y>/<y,y> of
//        the newest pair (1 with no pair)
//   w(a) = P(w + a d), a = tau_t with no pair, else 1, halved until the
//        objective change f(w(a)) - f(w) <= c1 <g, w(a) - w> (Armijo, c1 = 1e-4)
//   s = w(a) - w, y = g(w(a)) - g, kept if <s, y> > 0, else the memory is
//        cleared; after kVmMaxTrials halvings the tile takes no step and
//        clears its memory.
// The objective change is evaluated through its exact expansion in
// D = w(a) - w, with r = H w - y:
//   sum W e (r + e/2) with e = H D,  lambda sum (phi(D(w + D)) - phi(D w))
//   per pixel in a cancellation-free form, sum alpha D (w - u + D/2),
// so the line search keeps its relative accuracy for steps whose decrease is
// far below the rounding of the objective itself (fp32 here).
//
// Device data per tile: the unweighted residual r on the frame (double
// buffered), the gradient (double buffered), the direction (the two-loop's
// q and r in place), the trial step D, kVmMem s and y frames (a ring), and a
// VmTile record.  Reductions: per-block partial sums in fp64, summed per tile
// in a fixed order.
#pragma once

#include "kernels.h"

namespace dbl {

constexpr int kVmMem = 5;          // pairs kept (m)
constexpr int kVmBlocks = 16;      // blocks per tile of the vector kernels
constexpr int kVmThreads = 256;
constexpr int kVmMaxTrials = 30;   // halvings before a tile gives up the step
constexpr double kVmC1 = 1e-4;     // Armijo constant

struct VmTile {
    float alpha;        // step length of the current trial
    int done;           // line search finished (accepted or given up)
    int count;          // pairs in memory
    int head;           // ring slot of the newest pair
    double gamma;       // initial scaling <s, y> / <y, y> of the newest pair
    double coef;        // coefficient of the current two-loop update
    double rho[kVmMem]; // 1 / <s_i, y_i> per ring slot
    double a[kVmMem];   // first-loop coefficients by position (0 = newest)
};

// Ring slot of the pair at position j (0 = newest) of tile v.
__device__ __forceinline__ int vm_slot(const VmTile& v, int j) { return (v.head - j + 2 * kVmMem) % kVmMem; }

__device__ __forceinline__ double vm_block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kVmThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Rows [r0, r1) of tile t's support handled by this block of the vector grid.
__device__ __forceinline__ void vm_rows(const TileInfo& ti, int& r0, int& r1) {
    const int per = (ti.sy + gridDim.x - 1) / gridDim.x;
    r0 = blockIdx.x * per;
    r1 = min(ti.sy, r0 + per);
}

// Regulariser flux (s g_h, s g_v) of x at support pixel (i, c): forward
// differences, 0 at the last row/column (Neumann) or wrapped (circular).
__device__ __forceinline__ float2 vm_flux(const float* __restrict__ xt, int N, int sy, int sx, int i, int c,
                                          const SolveParams& P) {
    const float x0 = xt[(size_t)i * N + c];
    float gh, gv;
    if (P.bc) {
        gh = xt[(size_t)i * N + (c + 1 < sx ? c + 1 : 0)] - x0;
        gv = xt[(size_t)(i + 1 < sy ? i + 1 : 0) * N + c] - x0;
    } else {
        gh = c + 1 < sx ? xt[(size_t)i * N + c + 1] - x0 : 0.f;
        gv = i + 1 < sy ? xt[(size_t)(i + 1) * N + c] - x0 : 0.f;
    }
    const float s = reg_scale(gh, gv, P);
    return make_float2(s * gh, s * gv);
}

// g = H^T W r (hr) + lambda grad phi(x) + alpha (x - u) on the support.
__global__ __launch_bounds__(kVmThreads) void k_vm_grad(const float* __restrict__ hr, const float* __restrict__ x,
                                                       const float* __restrict__ u, const TileInfo* __restrict__ tiles,
                                                       const float* __restrict__ omY, const float* __restrict__ omX,
                                                       int N, SolveParams P, float* __restrict__ g) {
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const size_t base = (size_t)t * N * N;
    const float* xt = x + base;
    int r0, r1;
    vm_rows(ti, r0, r1);
    for (int e = threadIdx.x; e < (r1 - r0) * ti.sx; e += kVmThreads) {
        const int i = r0 + e / ti.sx, c = e % ti.sx;
        const size_t o = (size_t)i * N + c;
        const float2 f = vm_flux(xt, N, ti.sy, ti.sx, i, c, P);
        float div = -f.x - f.y;
        if (c > 0 || P.bc) div += vm_flux(xt, N, ti.sy, ti.sx, i, c > 0 ? c - 1 : ti.sx - 1, P).x;
        if (i > 0 || P.bc) div += vm_flux(xt, N, ti.sy, ti.sx, i > 0 ? i - 1 : ti.sy - 1, c, P).y;
        const float alpha = P.gamma * omY[(size_t)ti.ty * N + i] * omX[(size_t)ti.tx * N + c];
        g[base + o] = hr[base + o] + P.lambda * div + alpha * (xt[o] - u[base + o]);
    }
}

__device__ __forceinline__ bool vm_active(float w, float g, const SolveParams& P) {
    return P.positivity && w <= 0.f && g > 0.f;
}

// Empty memory for every tile.
__global__ void k_vm_reset(VmTile* __restrict__ vt, int n_tiles) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    vt[t].count = 0;
    vt[t].head = kVmMem - 1;
    vt[t].gamma = 1.0;
}

// q = F . g (into q); partial <s_{pos 0}, q>.
__global__ __launch_bounds__(kVmThreads) void k_vm_free(const float* __restrict__ x, const float* __restrict__ g,
                                                       const TileInfo* __restrict__ tiles, int N, SolveParams P,
                                                       const float* __restrict__ S, size_t fe,
                                                       const VmTile* __restrict__ vt, float* __restrict__ q,
                                                       double* __restrict__ part) {
    __shared__ double sh[kVmThreads];
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const size_t base = (size_t)t * N * N;
    const float* sl = S + (size_t)vm_slot(vt[t], 0) * fe + base;
    int r0, r1;
    vm_rows(ti, r0, r1);
    double acc = 0.0;
    for (int e = threadIdx.x; e < (r1 - r0) * ti.sx; e += kVmThreads) {
        const size_t o = base + (size_t)(r0 + e / ti.sx) * N + e % ti.sx;
        const float gv = g[o];
        const float qv = vm_active(x[o], gv, P) ? 0.f : gv;
        q[o] = qv;
        acc += (double)sl[o - base] * qv;
    }
    const double tot = vm_block_sum(acc, sh);
    if (threadIdx.x == 0) part[(size_t)t * gridDim.x + blockIdx.x] = tot;
}

// Per tile: the two-loop coefficient at position j from the partial sums of
// <s_j, q> (first loop: a_j = rho_j <s_j, q>, update q -= a_j y_j) or of
// <y_j, r> (second loop: b_j = rho_j <y_j, r>, update r += (a_j - b_j) s_j).
// Positions beyond the tile's memory get coefficient 0 (no update).
__global__ void k_vm_coef(VmTile* __restrict__ vt, const double* __restrict__ part, int nb, int n_tiles, int j,
                          int second) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    VmTile& v = vt[t];
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)t * nb + b];
    if (j >= v.count) {
        v.coef = 0.0;
        if (!second) v.a[j] = 0.0;
        return;
    }
    const double c = v.rho[vm_slot(v, j)] * s;
    if (second) {
        v.coef = v.a[j] - c;
    } else {
        v.a[j] = c;
        v.coef = -c;
    }
}

// v += coef . src_{pos j} (skipped where the coefficient is 0), then the
// partial <dot_{pos jn}, v> (jn < 0: none).  In the scale form (scale != 0)
// the update is v *= gamma (1 with no pair) instead.
__global__ __launch_bounds__(kVmThreads) void k_vm_axpy_dot(float* __restrict__ v, const float* __restrict__ src, int j,
                                                           const float* __restrict__ dot, int jn, int scale,
                                                           const TileInfo* __restrict__ tiles, int N, size_t fe,
                                                           const VmTile* __restrict__ vt, double* __restrict__ part) {
    __shared__ double sh[kVmThreads];
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const VmTile vv = vt[t];
    const size_t base = (size_t)t * N * N;
    float c = 0.f;
    bool upd;
    if (scale) {
        c = vv.count > 0 ? (float)vv.gamma : 1.f;
        upd = true;
    } else {
        c = (float)vv.coef;
        upd = j < vv.count;
    }
    const float* sl = upd && !scale ? src + (size_t)vm_slot(vv, j) * fe + base : nullptr;
    const float* dl = jn >= 0 ? dot + (size_t)vm_slot(vv, jn) * fe + base : nullptr;
    int r0, r1;
    vm_rows(ti, r0, r1);
    double acc = 0.0;
    for (int e = threadIdx.x; e < (r1 - r0) * ti.sx; e += kVmThreads) {
        const size_t o = (size_t)(r0 + e / ti.sx) * N + e % ti.sx;
        float w = v[base + o];
        if (scale) w *= c;
        else if (upd) w += c * sl[o];
        if (upd) v[base + o] = w;
        if (dl) acc += (double)dl[o] * w;
    }
    if (jn >= 0) {
        const double tot = vm_block_sum(acc, sh);
        if (threadIdx.x == 0) part[(size_t)t * gridDim.x + blockIdx.x] = tot;
    }
}

// d = -F . r (in place) and the line search's first trial length.
__global__ __launch_bounds__(kVmThreads) void k_vm_direction(const float* __restrict__ x, const float* __restrict__ g,
                                                            const TileInfo* __restrict__ tiles, int N, SolveParams P,
                                                            float* __restrict__ d) {
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const size_t base = (size_t)t * N * N;
    int r0, r1;
    vm_rows(ti, r0, r1);
    for (int e = threadIdx.x; e < (r1 - r0) * ti.sx; e += kVmThreads) {
        const size_t o = base + (size_t)(r0 + e / ti.sx) * N + e % ti.sx;
        d[o] = vm_active(x[o], g[o], P) ? 0.f : -d[o];
    }
}

__global__ void k_vm_ls_init(VmTile* __restrict__ vt, const float* __restrict__ tau, int n_tiles) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    vt[t].alpha = vt[t].count == 0 ? tau[t] : 1.f;
    vt[t].done = 0;
}

// Trial point of the step: w(a) = P(w + a d) (into xt), D = w(a) - w (into
// dl), and per block the partial sums of <g, D>, sum alpha D (w - u + D/2)
// and the regulariser's change (cancellation-free, per pixel).
__device__ __forceinline__ float vm_step(const float* __restrict__ x, const float* __restrict__ d, size_t o, float a,
                                         const SolveParams& P, float* xnew) {
    float w = x[o] + a * d[o];
    if (P.positivity) w = project_nonneg(w);
    *xnew = w;
    return w - x[o];
}

__device__ __forceinline__ float vm_reg_change(float ah, float av, float dh, float dv, const SolveParams& P) {
    const float bh = ah + dh, bv = av + dv;
    const float na2 = ah * ah + av * av, nb2 = bh * bh + bv * bv;
    const float diff = dh * (ah + bh) + dv * (av + bv);
    const float p = P.reg_param;
    if (P.reg == 0) return diff / (sqrtf(nb2 + p * p) + sqrtf(na2 + p * p));
    const float na = sqrtf(na2), nb = sqrtf(nb2);
    if (na <= p && nb <= p) return 0.5f * diff;
    if (na > p && nb > p) return p * diff / (na + nb);
    const float ha = na <= p ? 0.5f * na2 : p * (na - 0.5f * p);
    const float hb = nb <= p ? 0.5f * nb2 : p * (nb - 0.5f * p);
    return hb - ha;
}

__global__ __launch_bounds__(kVmThreads) void k_vm_trial(const float* __restrict__ x, const float* __restrict__ d,
                                                        const float* __restrict__ g, const float* __restrict__ u,
                                                        const TileInfo* __restrict__ tiles,
                                                        const float* __restrict__ omY, const float* __restrict__ omX,
                                                        int N, SolveParams P, const VmTile* __restrict__ vt,
                                                        float* __restrict__ xt, float* __restrict__ dl,
                                                        double* __restrict__ part) {
    __shared__ double sh[kVmThreads];
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const float a = vt[t].alpha;
    const size_t base = (size_t)t * N * N;
    int r0, r1;
    vm_rows(ti, r0, r1);
    double s_gd = 0.0, s_met = 0.0, s_reg = 0.0;
    for (int e = threadIdx.x; e < (r1 - r0) * ti.sx; e += kVmThreads) {
        const int i = r0 + e / ti.sx, c = e % ti.sx;
        const size_t o = base + (size_t)i * N + c;
        float w0;
        const float D0 = vm_step(x, d, o, a, P, &w0);
        xt[o] = w0;
        dl[o] = D0;
        // forward differences of w and of D at (i, c)
        float ah = 0.f, av = 0.f, dh = 0.f, dv = 0.f, wn;
        const bool has_h = c + 1 < ti.sx || P.bc, has_v = i + 1 < ti.sy || P.bc;
        if (has_h) {
            const size_t on = base + (size_t)i * N + (c + 1 < ti.sx ? c + 1 : 0);
            ah = x[on] - x[o];
            dh = vm_step(x, d, on, a, P, &wn) - D0;
        }
        if (has_v) {
            const size_t on = base + (size_t)(i + 1 < ti.sy ? i + 1 : 0) * N + c;
            av = x[on] - x[o];
            dv = vm_step(x, d, on, a, P, &wn) - D0;
        }
        s_reg += vm_reg_change(ah, av, dh, dv, P);
        s_gd += (double)g[o] * D0;
        const float alpha = P.gamma * omY[(size_t)ti.ty * N + i] * omX[(size_t)ti.tx * N + c];
        s_met += (double)alpha * D0 * ((double)x[o] - u[o] + 0.5 * D0);
    }
    const double t_gd = vm_block_sum(s_gd, sh);
    const double t_met = vm_block_sum(s_met, sh);
    const double t_reg = vm_block_sum(s_reg, sh);
    if (threadIdx.x == 0) {
        double* p = part + 3 * ((size_t)t * gridDim.x + blockIdx.x);
        p[0] = t_gd;
        p[1] = t_met;
        p[2] = t_reg;
    }
}

// Armijo test per tile still searching: the data change (obj_part, per row
// workgroup of k_row_resid_vm) plus lambda times the regulariser change plus
// the metric change against c1 <g, D>.  Accept, else halve; on the last trial
// give up (length 0).  Counts the tiles still searching or just given up.
__global__ void k_vm_armijo(VmTile* __restrict__ vt, const float* __restrict__ obj_part, int rg,
                            const double* __restrict__ part, int nb, int n_tiles, float lambda, int last,
                            int* __restrict__ searching) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    VmTile& v = vt[t];
    if (v.done) return;
    double data = 0.0, gd = 0.0, met = 0.0, reg = 0.0;
    for (int b = 0; b < rg; ++b) data += obj_part[(size_t)t * rg + b];
    for (int b = 0; b < nb; ++b) {
        const double* p = part + 3 * ((size_t)t * nb + b);
        gd += p[0];
        met += p[1];
        reg += p[2];
    }
    const double df = data + (double)lambda * reg + met;
    if (df <= kVmC1 * gd) {
        v.done = 1;
    } else if (last) {
        v.alpha = 0.f;   // gives up: the step is recomputed with length 0
        v.done = 1;
        atomicAdd(searching, 1);
    } else {
        v.alpha *= 0.5f;
        atomicAdd(searching, 1);
    }
}

// The new pair into the next ring slot: s = D, y = g_new - g; partial sums
// of <s, y> and <y, y>.
__global__ __launch_bounds__(kVmThreads) void k_vm_pair(const float* __restrict__ dl, const float* __restrict__ gn,
                                                       const float* __restrict__ g, const TileInfo* __restrict__ tiles,
                                                       int N, size_t fe, const VmTile* __restrict__ vt,
                                                       float* __restrict__ S, float* __restrict__ Y,
                                                       double* __restrict__ part) {
    __shared__ double sh[kVmThreads];
    const int t = blockIdx.y;
    const TileInfo ti = tiles[t];
    const size_t base = (size_t)t * N * N;
    const size_t slot = (size_t)((vt[t].head + 1) % kVmMem) * fe;
    int r0, r1;
    vm_rows(ti, r0, r1);
    double sy = 0.0, yy = 0.0;
    for (int e = threadIdx.x; e < (r1 - r0) * ti.sx; e += kVmThreads) {
        const size_t o = base + (size_t)(r0 + e / ti.sx) * N + e % ti.sx;
        const float s = dl[o], y = gn[o] - g[o];
        S[slot + o] = s;
        Y[slot + o] = y;
        sy += (double)s * y;
        yy += (double)y * y;
    }
    const double a = vm_block_sum(sy, sh);
    const double b = vm_block_sum(yy, sh);
    if (threadIdx.x == 0) {
        part[2 * ((size_t)t * gridDim.x + blockIdx.x)] = a;
        part[2 * ((size_t)t * gridDim.x + blockIdx.x) + 1] = b;
    }
}

// Keep the pair if <s, y> > 0 (it becomes the newest), else clear the memory.
__global__ void k_vm_memory(VmTile* __restrict__ vt, const double* __restrict__ part, int nb, int n_tiles) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    VmTile& v = vt[t];
    double sy = 0.0, yy = 0.0;
    for (int b = 0; b < nb; ++b) {
        sy += part[2 * ((size_t)t * nb + b)];
        yy += part[2 * ((size_t)t * nb + b) + 1];
    }
    if (sy > 0.0) {
        v.head = (v.head + 1) % kVmMem;
        v.rho[v.head] = 1.0 / sy;
        v.gamma = sy / yy;
        v.count = min(v.count + 1, kVmMem);
    } else {
        v.count = 0;
        v.gamma = 1.0;
    }
}

// Row pass of the data term for the line search (the structure of
// k_row_resid).  Yc holds the column-transformed spectrum of H v.
//   MODE 0 (start): v = H w; r_out = v - y (unweighted residual);
//                   obj = 1/2 sum W r^2; Rr = row spectrum of W r.
//   MODE 1 (trial): v = e = H D; r_out = r_in + e (the trial's residual);
//                   obj = sum W e (r_in + e/2) (the data change);
//                   Rr = row spectrum of W r_out.
template <int N, int WV, int MODE>
__global__ __launch_bounds__((Cfg<N, WV>::NT)) void k_row_resid_vm(const float2* __restrict__ Yc,
                                                                 const float2* __restrict__ yw,
                                                                 const float2* __restrict__ twg,
                                                                 const float* __restrict__ r_in,
                                                                 float* __restrict__ r_out, float2* __restrict__ Rr,
                                                                 float* __restrict__ obj_part) {
    using C = Cfg<N, WV>;
    __shared__ float2 sbuf[C::RB * C::LSR + kLinePad];
    __shared__ float2 tw[C::TWR];
    __shared__ float red[C::W];
    const int t = blockIdx.y, i0 = blockIdx.x * C::RB;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_twiddles<N, WV, false>(tw, twg, tid);
    __syncthreads();
    load_c2r_T<N, WV>(sbuf, Yc + (size_t)t * C::SPEC, tw, i0, tid);
    __syncthreads();
    float2* sw = sbuf + line_off<C::n>(wave * C::LwR);
    float2 v[kV];
    row_c2r_ready<N>(v, sw, tw, lane);
    const size_t row0 = (size_t)t * N * N + (size_t)(i0 + wave * C::LwR) * N + rslot_base<N>(lane);
    const float2* __restrict__ yl = yw + row0;
    float obj = 0.f;
#pragma unroll
    for (int s = 0; s < kV; ++s) {
        const float4 o = *reinterpret_cast<const float4*>(yl + rslot_off<N>(s));   // (y0, W0, y1, W1)
        float2 r;
        if constexpr (MODE == 0) {
            r = make_float2(v[s].x - o.x, v[s].y - o.z);
            obj += 0.5f * (o.y * r.x * r.x + o.w * r.y * r.y);
        } else {
            const float2 ri = *reinterpret_cast<const float2*>(r_in + row0 + rslot_off<N>(s));
            obj += o.y * v[s].x * (ri.x + 0.5f * v[s].x) + o.w * v[s].y * (ri.y + 0.5f * v[s].y);
            r = make_float2(ri.x + v[s].x, ri.y + v[s].y);
        }
        *reinterpret_cast<float2*>(r_out + row0 + rslot_off<N>(s)) = r;
        v[s] = make_float2(o.y * r.x, o.w * r.y);
    }
    wave_sync();
    row_fft_wave<N>(v, sw, tw, lane);
    __syncthreads();
    store_spectrum_T<N, WV>(sbuf, tw, Rr + (size_t)t * C::SPEC, i0, tid);
    const float tot = block_sum<N, WV>(obj, red, tid);
    if (tid == 0) obj_part[t * C::RG + blockIdx.x] = tot;
}

}  // namespace dbl
