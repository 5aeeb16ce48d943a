// Host side of the MI355X tile solver: context, layout tables, launches,
// HIP-graph capture of the D-R rounds and the C ABI declared in deblur.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/deblur.h"
#include "kernels.h"
#include "cnn.h"
#include "cnn_fused.h"
#include "vmlmb.h"
#include "independent.h"

using dbl::Cover;
using dbl::PackDesc;
using dbl::SolveParams;
using dbl::TileInfo;

namespace {

thread_local std::string g_create_error;

constexpr int kFrames[3] = {160, 320, 640};
constexpr int kResCap = 4096;
constexpr int kMaxGroups = 4;   // tile groups of a launch plan (concurrent branches)
constexpr double kPsfSumTol = 1e-4;   // accepted |sum of a PSF - 1| (fp32 rounding of a normalised PSF)

// One axis of the tiling and of the PSF grid (Section III-A, Fig. 1).
struct Axis {
    int M, T, p, o, r, G;
    int kind = DEBLUR_LAYOUT_PITCH;

    void block(int a, int& s, int& e) const {
        if (kind == DEBLUR_LAYOUT_GRID) {   // the pixels strictly between nodes a - 1 and a + 1
            s = a == 0 ? 0 : (int)std::floor(centre(a - 1)) + 1;
            e = a == T - 1 ? M : (int)std::ceil(centre(a + 1));
            return;
        }
        s = a * p;
        e = (a == T - 1) ? M : std::min(a * p + p + o, M);
    }
    void support(int a, int& s, int& e) const {
        block(a, s, e);
        s -= r;
        e += r;
    }
    int support_len(int a) const {
        int s, e;
        support(a, s, e);
        return e - s;
    }
    // grid layout: node a's tent widened to reach over its support
    double grid_phi(int a, int coord) const {
        const double h = (double)M / G + r + 0.5;
        return std::max(0.0, 1.0 - std::fabs(coord - centre(a)) / h);
    }
    // consensus weight of tile a at support offset m
    double omega(int a, int m) const {
        int s0, s1;
        support(a, s0, s1);
        if (kind == DEBLUR_LAYOUT_GRID) {   // normalised over the supports holding the pixel
            const int coord = s0 + m;
            double den = 0.0;
            for (int b = 0; b < T; ++b) {
                int b0, b1;
                support(b, b0, b1);
                if (coord >= b0 && coord < b1) den += grid_phi(b, coord);
            }
            return grid_phi(a, coord) / den;
        }
        double w = 1.0;
        if (a > 0) {
            int ps, pe;
            support(a - 1, ps, pe);
            const int L = pe - s0;
            if (m < L) w = (m + 0.5) / L;
        }
        if (a < T - 1) {
            int ns, ne;
            support(a + 1, ns, ne);
            const int L = s1 - ns;
            const int s = (s0 + m) - ns;
            if (s >= 0) w = (L - s - 0.5) / L;
        }
        return w;
    }
    double centre(int k) const { return (k + 0.5) * ((double)M / G) - 0.5; }
    // first-order interpolation weight of node k at observed coordinate c
    double tent(int k, double c) const {
        const double q = (double)M / G, ck = centre(k);
        if (k == 0 && c <= ck) return 1.0;
        if (k == G - 1 && c >= ck) return 1.0;
        return std::max(0.0, 1.0 - std::fabs(c - ck) / q);
    }
    std::vector<int> nodes(int a) const {
        int s0, s1;
        support(a, s0, s1);
        std::vector<int> out;
        for (int k = 0; k < G; ++k) {
            bool any = false;
            for (int c = s0; c < s1 && !any; ++c) any = tent(k, c) > 0.0;
            if (any) out.push_back(k);
        }
        return out;
    }
    std::string validate() const {
        if (kind == DEBLUR_LAYOUT_GRID) {
            if (M < 1 || T < 1 || G < 1 || r < 0) return "non-positive size";
            if (T != G) return "the grid layout has one tile per PSF node (T = G)";
            if (G > 1 && 2.0 * r > (double)M / G) return "the grid layout needs 2r <= the node spacing M / G";
        } else if (kind != DEBLUR_LAYOUT_PITCH) {
            return "unknown layout";
        }
        if (kind == DEBLUR_LAYOUT_PITCH && (M < 1 || T < 1 || G < 1 || p < 1 || o < 0 || r < 0))
            return "non-positive size";
        if (kind == DEBLUR_LAYOUT_PITCH && T > 1) {
            if (o + 2 * r > p) return "overlap + 2r exceeds the pitch";
            if (M - (T - 1) * p <= o) return "last block does not extend past the previous one";
        } else if (p < M && T == 1) {
            // a single tile always covers the whole axis
        }
        for (int a = 0; a < T; ++a) {
            int s, e;
            block(a, s, e);
            if (e - s < 2 * r + 1) return "a block is smaller than the PSF";
        }
        return "";
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free FFT stages (deblur_debug_fft_noalloc):
// the twiddle table of the largest frame, a tile table for up to
// kNoAllocMaxBatch frames and one tent row. Each GPU holds its own copy until
// the process ends. In host code `scratch` names a host-side stand-in, never
// the device memory: host code uses the address hipGetSymbolAddress returns.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocMaxBatch = 4096;
constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kNoAllocTwBytes = round256((size_t)dbl::Cfg<640>::TW_TOTAL * sizeof(float2));
constexpr size_t kNoAllocTileBytes = round256((size_t)kNoAllocMaxBatch * sizeof(TileInfo));
constexpr size_t kNoAllocTentBytes = round256((size_t)dbl::kMaxK * 640 * sizeof(float));
constexpr size_t kNoAllocScratchBytes = kNoAllocTwBytes + kNoAllocTileBytes + kNoAllocTentBytes;
static_assert(dbl::Cfg<160>::TW_TOTAL <= dbl::Cfg<640>::TW_TOTAL &&
                  dbl::Cfg<320>::TW_TOTAL <= dbl::Cfg<640>::TW_TOTAL,
              "the scratch twiddle region holds the largest frame's table");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct deblur_ctx {
    deblur_params p{};
    int r = 0, N = 0, nt = 0, nodes = 0, Xy = 0, Xx = 0;
    Axis ay{}, ax{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::string err;

    std::vector<TileInfo> tiles_h;
    std::vector<deblur_tile_desc> desc;
    std::vector<float> omega_max;
    int64_t support_total = 0, block_total = 0;

    TileInfo* tiles = nullptr;
    float *tentY = nullptr, *tentX = nullptr, *omY = nullptr, *omX = nullptr;
    Cover *covY = nullptr, *covX = nullptr;
    int *sorg = nullptr, *borg = nullptr, *xorg = nullptr;
    PackDesc *pd_support = nullptr, *pd_block = nullptr;
    float2* tw = nullptr;
    float2* spec = nullptr;
    float* x[2] = {nullptr, nullptr};
    int cur = 0;
    float* u = nullptr;
    float2* yw = nullptr;
    float* frame_tmp = nullptr;
    float* frame_tmp2 = nullptr;
    float2 *Zk = nullptr, *Yc = nullptr, *Rr = nullptr, *Gk = nullptr;
    float* obj_part = nullptr;
    float2* cons_part = nullptr;
    int cons_nparts = 0;
    double* res_hist = nullptr;
    int* res_counter = nullptr;
    double* res_last = nullptr;
    double* reg_part = nullptr;
    int reg_blocks = 8;
    float* tau = nullptr;
    float* maxW = nullptr;
    float* rowsum = nullptr;
    float* y_glob = nullptr;
    double* h_pinned = nullptr;
    bool have_obs = false;
    bool have_state = false;
    int32_t round = 0;            // consensus steps (D-R rounds) since the state was set
    int* tile_flag = nullptr;     // per-tile scratch flags (non-finite search)
    // warm-start bookkeeping
    float* tile_scale = nullptr;
    int* sdim = nullptr;
    int* bdim = nullptr;
    double* gmap = nullptr;
    int* use_cnn = nullptr;
    bool fista = false;           // Local-Solver: FISTA (else projected gradient)
    float* wbuf = nullptr;        // FISTA: the last projected-gradient point w_j per tile frame
    bool vmlmb = false;           // Local-Solver: VMLM-B (limited-memory BFGS with bounds)
    float* vm_g[2] = {nullptr, nullptr};   // VMLM-B: prox gradient frames (current, next)
    float* vm_r[2] = {nullptr, nullptr};   // VMLM-B: unweighted residual H w - y frames
    float* vm_d = nullptr;        // VMLM-B: direction (the two-loop's q and r)
    float* vm_delta = nullptr;    // VMLM-B: trial step D
    float* vm_S = nullptr;        // VMLM-B: kVmMem s frames (ring)
    float* vm_Y = nullptr;        // VMLM-B: kVmMem y frames (ring)
    dbl::VmTile* vm_tile = nullptr;
    double* vm_part = nullptr;    // VMLM-B: per-block partial sums
    int* vm_search = nullptr;     // VMLM-B: tiles still searching
    int vm_gc = 0, vm_rc = 0;     // current gradient / residual buffer
    int max_cover = 2;            // the most tiles covering an X row or column
    std::vector<void*> allocs;
    // captured rounds, keyed by (col waves, row waves, tile order, tile
    // groups, steps, parity, with consensus); kept until deblur_destroy
    std::map<std::tuple<int, int, int, int, int, int, int>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
    // launch plan (frame fixed at creation; the rest set by deblur_set_plan)
    deblur_plan plan{};
    int* perm_id = nullptr;      // tile order tables of the column kernels
    int* perm_heavy = nullptr;   // all tiles by term count
    int* perm_heavy_g[kMaxGroups + 1] = {};   // [G]: each of G tile groups by term count
    hipStream_t aux_stream[kMaxGroups - 1] = {};   // further branches of a round with G > 1 tile groups
    hipStream_t cap_aux[kMaxGroups - 1] = {};      // their counterparts during graph capture
    hipEvent_t ev_fork = nullptr, ev_join[kMaxGroups - 1] = {};
};

namespace {

int fail(deblur_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIP_TRY(ctx, call)                                                                         \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((ctx), DEBLUR_E_HIP, std::string(#call ": ") + hipGetErrorString(e_));     \
    } while (0)

int check_launch(deblur_ctx* c, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, DEBLUR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return DEBLUR_OK;
}

template <class T>
int dev_alloc(deblur_ctx* c, T** ptr, size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, DEBLUR_E_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    c->allocs.push_back(p);
    *ptr = static_cast<T*>(p);
    return DEBLUR_OK;
}

// A device buffer used only during setup, freed on every return path.
template <class T>
struct ScratchBuf {
    T* p = nullptr;
    ~ScratchBuf() {
        if (p) (void)hipFree(p);
    }
};

size_t frame_elems(const deblur_ctx* c) { return (size_t)c->nt * c->N * c->N; }
size_t half_elems(const deblur_ctx* c) { return (size_t)c->nt * (c->N / 2) * c->N; }

// ---------------------------------------------------------------------------
// Launch helpers (dispatch on the frame size)
// ---------------------------------------------------------------------------

template <int N, int WV>
void launch_row_fwd(deblur_ctx* c, hipStream_t s, const float* x, float2* out, int masked) {
    using C = dbl::Cfg<N, WV>;
    hipLaunchKernelGGL((dbl::k_row_fwd<N, WV>), dim3(C::RG, c->nt), dim3(C::NT), 0, s, x, c->tiles, c->tentX, c->tw,
                       out, masked);
}
template <int N, int WV>
void launch_row_inv(deblur_ctx* c, hipStream_t s, const float2* in, float* out, int masked) {
    using C = dbl::Cfg<N, WV>;
    hipLaunchKernelGGL((dbl::k_row_inv<N, WV>), dim3(C::RG, c->nt), dim3(C::NT), 0, s, in, c->tiles, c->tentX, c->tw,
                       out, masked);
}
// A contiguous range of tiles [t0, t0 + cnt) and the column kernels' order
// of it (perm[0 .. cnt) are tile indices).
struct TileRange {
    int t0, cnt;
    const int* perm;
};
TileRange all_tiles(const deblur_ctx* c) {
    return {0, c->nt, c->plan.tile_order == DEBLUR_ORDER_HEAVY_FIRST ? c->perm_heavy : c->perm_id};
}
// Tile group g of G: contiguous ranges of tiles, the first T mod G of them
// one tile longer.
void group_bounds(int nt, int G, int g, int& t0, int& cnt) {
    const int q = nt / G, r = nt % G;
    t0 = g * q + std::min(g, r);
    cnt = q + (g < r ? 1 : 0);
}
TileRange tile_group(const deblur_ctx* c, int g) {
    const int G = c->plan.tile_groups;
    int t0, cnt;
    group_bounds(c->nt, G, g, t0, cnt);
    return {t0, cnt, (c->plan.tile_order == DEBLUR_ORDER_HEAVY_FIRST ? c->perm_heavy_g[G] : c->perm_id) + t0};
}
template <int N, int WV>
void launch_col_H(deblur_ctx* c, hipStream_t s, TileRange r) {
    using C = dbl::Cfg<N, WV>;
    hipLaunchKernelGGL((dbl::k_col_H<N, WV>), dim3(dbl::col_grid<N, WV>(r.cnt)), dim3(C::NT), 0, s, c->Zk, c->tiles,
                       c->tentY, c->spec, c->tw, c->Yc, r.cnt, r.perm, c->plan.tile_order);
}
template <int N, int WV>
void launch_row_resid(deblur_ctx* c, hipStream_t s, TileRange r) {
    using C = dbl::Cfg<N, WV>;
    hipLaunchKernelGGL((dbl::k_row_resid<N, WV>), dim3(C::RG, r.cnt), dim3(C::NT), 0, s, c->Yc, c->yw, c->tw, c->Rr,
                       c->obj_part, r.t0);
}
template <int N, int WV>
void launch_row_resid_vm(deblur_ctx* c, hipStream_t s, int mode, const float* r_in, float* r_out) {
    using C = dbl::Cfg<N, WV>;
    if (mode == 0)
        hipLaunchKernelGGL((dbl::k_row_resid_vm<N, WV, 0>), dim3(C::RG, c->nt), dim3(C::NT), 0, s, c->Yc, c->yw,
                           c->tw, r_in, r_out, c->Rr, c->obj_part);
    else
        hipLaunchKernelGGL((dbl::k_row_resid_vm<N, WV, 1>), dim3(C::RG, c->nt), dim3(C::NT), 0, s, c->Yc, c->yw,
                           c->tw, r_in, r_out, c->Rr, c->obj_part);
}
template <int N, int WV>
void launch_col_Ht(deblur_ctx* c, hipStream_t s, TileRange r) {
    using C = dbl::Cfg<N, WV>;
    hipLaunchKernelGGL((dbl::k_col_Ht<N, WV>), dim3(dbl::col_grid<N, WV>(r.cnt)), dim3(C::NT), 0, s, c->Rr, c->tiles,
                       c->tentY, c->spec, c->tw, c->Gk, r.cnt, r.perm, c->plan.tile_order);
}
SolveParams solve_params(const deblur_ctx* c) {
    SolveParams P;
    P.lambda = c->p.lambda;
    P.reg_param = c->p.reg_param;
    P.gamma = c->p.gamma;
    P.rho = c->p.rho;
    P.reg = c->p.reg;
    P.bc = c->p.bc;
    P.positivity = c->p.positivity;
    P.r = c->r;
    return P;
}
template <int N, int WV>
void launch_row_update(deblur_ctx* c, hipStream_t s, const float* xc, float* xn, TileRange r, float beta) {
    using C = dbl::Cfg<N, WV>;
    if (c->fista)
        hipLaunchKernelGGL((dbl::k_row_update<N, WV, true>), dim3(C::RG, r.cnt), dim3(C::NT), 0, s, c->Gk, xc, c->u,
                           c->tiles, c->tentX, c->omY, c->omX, c->tau, solve_params(c), c->tw, xn, c->Zk, r.t0, beta,
                           c->wbuf);
    else
        hipLaunchKernelGGL((dbl::k_row_update<N, WV, false>), dim3(C::RG, r.cnt), dim3(C::NT), 0, s, c->Gk, xc, c->u,
                           c->tiles, c->tentX, c->omY, c->omX, c->tau, solve_params(c), c->tw, xn, c->Zk, r.t0, 0.f,
                           nullptr);
}

// Momentum factor of step j (0-based) of an n-step FISTA run: with s_1 = 1,
// s_{i+1} = (1 + sqrt(1 + 4 s_i^2)) / 2, step j uses (s_{j+1} - 1) / s_{j+2};
// the last step uses 0, so the run ends on its projected-gradient point.
float fista_beta(int j, int n) {
    if (j + 1 >= n) return 0.f;
    double s = 1.0;
    for (int i = 0; i < j; ++i) s = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * s * s));
    const double s_next = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * s * s));
    return (float)((s - 1.0) / s_next);
}

template <int N, int WV>
void launch_col_fft_dbg(deblur_ctx* c, hipStream_t s, const float2* in, float2* out, int dir) {
    using C = dbl::Cfg<N, WV>;
    hipLaunchKernelGGL((dbl::k_col_fft_dbg<N, WV>), dim3(C::CG, c->nt), dim3(C::NT), 0, s, in, c->tw, out, dir);
}

template <int N>
int make_twiddles_n(deblur_ctx* c, hipStream_t s) {
    int rc = dev_alloc(c, &c->tw, dbl::Cfg<N>::TW_TOTAL);
    if (rc) return rc;
    hipLaunchKernelGGL(dbl::k_make_twiddles<N>, dim3(1), dim3(256), 0, s, c->tw);
    return check_launch(c, "k_make_twiddles");
}

int make_twiddles(deblur_ctx* c, hipStream_t s) {
    switch (c->N) {
        case 160: return make_twiddles_n<160>(c, s);
        case 320: return make_twiddles_n<320>(c, s);
        default: return make_twiddles_n<640>(c, s);
    }
}

// Dispatch on the frame size and on the plan's waves per workgroup (W is
// the column kernels' or the row kernels' count, one of the two shapes the
// frame allows).
#define DISPATCH_NW(c, W, fn, ...)                                                              \
    do {                                                                                        \
        switch ((c)->N) {                                                                       \
            case 160:                                                                           \
                if ((W) == dbl::waves_lo<160>()) fn<160, dbl::waves_lo<160>()>(c, __VA_ARGS__); \
                else fn<160, dbl::waves_hi<160>()>(c, __VA_ARGS__);                             \
                break;                                                                          \
            case 320:                                                                           \
                if ((W) == dbl::waves_lo<320>()) fn<320, dbl::waves_lo<320>()>(c, __VA_ARGS__);                         \
                else fn<320, dbl::waves_hi<320>()>(c, __VA_ARGS__);                             \
                break;                                                                          \
            default:                                                                            \
                if ((W) == dbl::waves_lo<640>()) fn<640, dbl::waves_lo<640>()>(c, __VA_ARGS__);                         \
                else fn<640, dbl::waves_hi<640>()>(c, __VA_ARGS__);                             \
                break;                                                                          \
        }                                                                                       \
    } while (0)

void row_fwd(deblur_ctx* c, hipStream_t s, const float* x, float2* out, int masked) {
    DISPATCH_NW(c, c->plan.row_waves, launch_row_fwd, s, x, out, masked);
}
void row_inv(deblur_ctx* c, hipStream_t s, const float2* in, float* out, int masked) {
    DISPATCH_NW(c, c->plan.row_waves, launch_row_inv, s, in, out, masked);
}
void col_H(deblur_ctx* c, hipStream_t s, TileRange r) { DISPATCH_NW(c, c->plan.col_waves, launch_col_H, s, r); }
void row_resid(deblur_ctx* c, hipStream_t s, TileRange r) {
    DISPATCH_NW(c, c->plan.row_waves, launch_row_resid, s, r);
}
void col_Ht(deblur_ctx* c, hipStream_t s, TileRange r) { DISPATCH_NW(c, c->plan.col_waves, launch_col_Ht, s, r); }
void row_update(deblur_ctx* c, hipStream_t s, const float* xc, float* xn, TileRange r, float beta = 0.f) {
    DISPATCH_NW(c, c->plan.row_waves, launch_row_update, s, xc, xn, r, beta);
}
void col_H(deblur_ctx* c, hipStream_t s) { col_H(c, s, all_tiles(c)); }
void row_resid(deblur_ctx* c, hipStream_t s) { row_resid(c, s, all_tiles(c)); }
void col_Ht(deblur_ctx* c, hipStream_t s) { col_Ht(c, s, all_tiles(c)); }
void row_update(deblur_ctx* c, hipStream_t s, const float* xc, float* xn, float beta = 0.f) {
    row_update(c, s, xc, xn, all_tiles(c), beta);
}

// Resolves the frame kernels of a plan's shapes (loading their code) outside
// any stream capture, so that a graph capture never makes a first use.
template <int N, int WV>
hipError_t preload_row(deblur_ctx*) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&dbl::k_row_resid<N, WV>));
    if (e == hipSuccess) e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&dbl::k_row_update<N, WV, false>));
    if (e == hipSuccess) e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&dbl::k_row_update<N, WV, true>));
    if (e == hipSuccess) e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&dbl::k_row_fwd<N, WV>));
    if (e == hipSuccess) e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&dbl::k_row_inv<N, WV>));
    return e;
}
template <int N, int WV>
hipError_t preload_col(deblur_ctx*) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&dbl::k_col_H<N, WV>));
    if (e == hipSuccess) e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&dbl::k_col_Ht<N, WV>));
    return e;
}

int waves_hi(int N) { return N == 160 ? dbl::waves_hi<160>() : dbl::waves_hi<320>(); }
int waves_lo(int N) { return waves_hi(N) / 2; }

// Launch shapes the autotuner measures: all of them, except the one-wave
// workgroups at frame 160.  A plan sweep over that frame once ended the test
// process inside a round (an abort with no fault message) while a variant of
// the row-update kernel was under test, and no cause was found; the shapes
// stay selectable with deblur_set_plan but are never picked automatically.
bool autotune_candidate(int N, int col_waves, int row_waves) {
    return !(N == 160 && (col_waves == 1 || row_waves == 1));
}

template <int N, int WV>
void preload_row_v(deblur_ctx* c, hipError_t* e) { *e = preload_row<N, WV>(c); }
template <int N, int WV>
void preload_col_v(deblur_ctx* c, hipError_t* e) { *e = preload_col<N, WV>(c); }
hipError_t preload_plan(deblur_ctx* c) {
    hipError_t e1 = hipSuccess, e2 = hipSuccess;
    DISPATCH_NW(c, c->plan.row_waves, preload_row_v, &e1);
    DISPATCH_NW(c, c->plan.col_waves, preload_col_v, &e2);
    return e1 != hipSuccess ? e1 : e2;
}

// Row workgroups per tile under the current plan, and the most any plan uses.
int row_groups(const deblur_ctx* c) { return c->N / (c->plan.row_waves * (dbl::kPts / (c->N / 2))); }
int row_groups_max(const deblur_ctx* c) { return c->N / (waves_lo(c->N) * (dbl::kPts / (c->N / 2))); }

dim3 pix_grid(const deblur_ctx* c) {
    return dim3((c->Xx + dbl::kPixBlock - 1) / dbl::kPixBlock, c->Xy);
}

dim3 frame_grid(const deblur_ctx* c) {
    const int per = (c->N * c->N + 255) / 256;
    return dim3(std::min(per, 64), c->nt);
}

// One Local-Solver step on the tiles of r: x[cur] -> x[1 - cur] (with FISTA,
// from the gradient point y_j to y_{j+1}, with momentum beta).
void inner_step(deblur_ctx* c, hipStream_t s, int parity, TileRange r, float beta = 0.f) {
    col_H(c, s, r);
    row_resid(c, s, r);
    col_Ht(c, s, r);
    row_update(c, s, c->x[parity], c->x[1 - parity], r, beta);
}
void inner_step(deblur_ctx* c, hipStream_t s, int parity, float beta = 0.f) {
    inner_step(c, s, parity, all_tiles(c), beta);
}
float step_beta(const deblur_ctx* c, int i, int n) { return c->fista ? fista_beta(i, n) : 0.f; }

// n Local-Solver steps on every tile starting from x[parity].  With G > 1
// tile groups the groups run as G independent chains, on s and on aux[0 ..
// G-2] (forked and joined with events; under graph capture this makes G
// branches).
hipError_t local_steps(deblur_ctx* c, hipStream_t s, hipStream_t* aux, int n, int parity) {
    if (n == 0) return hipSuccess;
    const int G = std::min(c->plan.tile_groups, c->nt);
    if (G <= 1) {
        for (int i = 0; i < n; ++i, parity = 1 - parity) inner_step(c, s, parity, step_beta(c, i, n));
        return hipGetLastError();
    }
    hipError_t e = hipEventRecord(c->ev_fork, s);
    for (int g = 1; g < G && e == hipSuccess; ++g) e = hipStreamWaitEvent(aux[g - 1], c->ev_fork, 0);
    if (e != hipSuccess) return e;
    TileRange rg[kMaxGroups];
    for (int g = 0; g < G; ++g) rg[g] = tile_group(c, g);
    for (int i = 0, p = parity; i < n; ++i, p = 1 - p)
        for (int g = 0; g < G; ++g) inner_step(c, g ? aux[g - 1] : s, p, rg[g], step_beta(c, i, n));
    for (int g = 1; g < G && e == hipSuccess; ++g) {
        e = hipEventRecord(c->ev_join[g - 1], aux[g - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, c->ev_join[g - 1], 0);
    }
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}

void consensus_launch(deblur_ctx* c, hipStream_t s, int parity) {
    if (c->p.independent)   // the independent baseline: u <- x, no exchange between tiles
        hipLaunchKernelGGL(dbl::k_independent, dim3(c->cons_nparts), dim3(dbl::kIndThreads), 0, s, c->x[parity],
                           c->u, c->tiles, c->N, c->nt, c->cons_part);
    else
        hipLaunchKernelGGL(c->max_cover > 2 ? dbl::k_consensus<3> : dbl::k_consensus<2>, pix_grid(c), dim3(dbl::kPixBlock), 0, s, c->x[parity], c->u, c->covY,
                           c->covX, c->Xy, c->Xx, c->p.T_x, c->N, c->p.rho, c->cons_part);
    hipLaunchKernelGGL(dbl::k_finalize_residual, dim3(1), dim3(dbl::kFinThreads), 0, s, c->cons_part, c->cons_nparts,
                       c->res_hist, c->res_counter, c->res_last, kResCap);
}

// Forward row transforms of the current iterate (start of the next step).
void refresh_spectra(deblur_ctx* c, hipStream_t s) { row_fwd(c, s, c->x[c->cur], c->Zk, 1); }

// ---------------------------------------------------------------------------
// VMLM-B Local-Solver (vmlmb.h): n iterations on every tile from the current
// x, with an empty memory at the start.  Each line-search trial ends with a
// readback of the number of tiles still searching, so this path runs eagerly
// (no graph capture).
// ---------------------------------------------------------------------------

void row_resid_vm(deblur_ctx* c, hipStream_t s, int mode, const float* r_in, float* r_out) {
    DISPATCH_NW(c, c->plan.row_waves, launch_row_resid_vm, s, mode, r_in, r_out);
}

// Residual, data spectrum and objective change of the trial step in vm_delta.
void vm_trial_data(deblur_ctx* c, hipStream_t s, const float* r, float* rt) {
    row_fwd(c, s, c->vm_delta, c->Zk, 1);
    col_H(c, s);
    row_resid_vm(c, s, 1, r, rt);
}

int vmlmb_steps(deblur_ctx* c, int n) {
    if (n <= 0) return DEBLUR_OK;
    using namespace dbl;
    hipStream_t s = c->stream;
    const size_t fe = frame_elems(c);
    const SolveParams P = solve_params(c);
    const dim3 vg(kVmBlocks, c->nt), vb(kVmThreads), tg((c->nt + 255) / 256), tb(256);
    int* h_search = reinterpret_cast<int*>(c->h_pinned + 32);
    // residual, row spectrum of W r and prox gradient at the start point
    row_fwd(c, s, c->x[c->cur], c->Zk, 1);
    col_H(c, s);
    row_resid_vm(c, s, 0, nullptr, c->vm_r[c->vm_rc]);
    col_Ht(c, s);
    row_inv(c, s, c->Gk, c->frame_tmp, 1);
    hipLaunchKernelGGL(k_vm_grad, vg, vb, 0, s, c->frame_tmp, c->x[c->cur], c->u, c->tiles, c->omY, c->omX, c->N, P,
                       c->vm_g[c->vm_gc]);
    hipLaunchKernelGGL(k_vm_reset, tg, tb, 0, s, c->vm_tile, c->nt);
    for (int it = 0; it < n; ++it) {
        float *x = c->x[c->cur], *xt = c->x[1 - c->cur];
        float *g = c->vm_g[c->vm_gc], *gn = c->vm_g[1 - c->vm_gc];
        float *r = c->vm_r[c->vm_rc], *rt = c->vm_r[1 - c->vm_rc];
        // d = -F B (F g) by the two-loop recursion, newest pair first, then
        // the initial scaling, then oldest first
        hipLaunchKernelGGL(k_vm_free, vg, vb, 0, s, x, g, c->tiles, c->N, P, c->vm_S, fe, c->vm_tile, c->vm_d,
                           c->vm_part);
        for (int j = 0; j < kVmMem; ++j) {
            hipLaunchKernelGGL(k_vm_coef, tg, tb, 0, s, c->vm_tile, c->vm_part, kVmBlocks, c->nt, j, 0);
            hipLaunchKernelGGL(k_vm_axpy_dot, vg, vb, 0, s, c->vm_d, c->vm_Y, j, c->vm_S, j + 1 < kVmMem ? j + 1 : -1,
                               0, c->tiles, c->N, fe, c->vm_tile, c->vm_part);
        }
        hipLaunchKernelGGL(k_vm_axpy_dot, vg, vb, 0, s, c->vm_d, c->vm_S, -1, c->vm_Y, kVmMem - 1, 1, c->tiles,
                           c->N, fe, c->vm_tile, c->vm_part);
        for (int j = kVmMem - 1; j >= 0; --j) {
            hipLaunchKernelGGL(k_vm_coef, tg, tb, 0, s, c->vm_tile, c->vm_part, kVmBlocks, c->nt, j, 1);
            hipLaunchKernelGGL(k_vm_axpy_dot, vg, vb, 0, s, c->vm_d, c->vm_S, j, c->vm_Y, j - 1, 0, c->tiles, c->N,
                               fe, c->vm_tile, c->vm_part);
        }
        hipLaunchKernelGGL(k_vm_direction, vg, vb, 0, s, x, g, c->tiles, c->N, P, c->vm_d);
        // projected Armijo search, all tiles at once (a tile that is done
        // recomputes its accepted trial unchanged)
        hipLaunchKernelGGL(k_vm_ls_init, tg, tb, 0, s, c->vm_tile, c->tau, c->nt);
        for (int trial = 0; trial < kVmMaxTrials; ++trial) {
            const int last = trial == kVmMaxTrials - 1;
            hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->vm_search, 0);
            hipLaunchKernelGGL(k_vm_trial, vg, vb, 0, s, x, c->vm_d, g, c->u, c->tiles, c->omY, c->omX, c->N, P,
                               c->vm_tile, xt, c->vm_delta, c->vm_part);
            vm_trial_data(c, s, r, rt);
            hipLaunchKernelGGL(k_vm_armijo, tg, tb, 0, s, c->vm_tile, c->obj_part, row_groups(c), c->vm_part,
                               kVmBlocks, c->nt, c->p.lambda, last, c->vm_search);
            HIP_TRY(c, hipMemcpyAsync(h_search, c->vm_search, sizeof(int), hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipStreamSynchronize(s));
            if (*h_search == 0) break;
            if (last) {   // the tiles that gave up: their step of length 0
                hipLaunchKernelGGL(k_vm_trial, vg, vb, 0, s, x, c->vm_d, g, c->u, c->tiles, c->omY, c->omX, c->N,
                                   P, c->vm_tile, xt, c->vm_delta, c->vm_part);
                vm_trial_data(c, s, r, rt);
            }
        }
        // gradient at the accepted point, the new pair, the memory
        col_Ht(c, s);
        row_inv(c, s, c->Gk, c->frame_tmp, 1);
        hipLaunchKernelGGL(k_vm_grad, vg, vb, 0, s, c->frame_tmp, xt, c->u, c->tiles, c->omY, c->omX, c->N, P, gn);
        hipLaunchKernelGGL(k_vm_pair, vg, vb, 0, s, c->vm_delta, gn, g, c->tiles, c->N, fe, c->vm_tile, c->vm_S,
                           c->vm_Y, c->vm_part);
        hipLaunchKernelGGL(k_vm_memory, tg, tb, 0, s, c->vm_tile, c->vm_part, kVmBlocks, c->nt);
        c->cur = 1 - c->cur;
        c->vm_gc ^= 1;
        c->vm_rc ^= 1;
    }
    refresh_spectra(c, s);
    return check_launch(c, "vmlmb");
}

// ---------------------------------------------------------------------------
// Layout tables
// ---------------------------------------------------------------------------

int build_layout(deblur_ctx* c, const float* psfs_host) {
    const deblur_params& p = c->p;
    c->r = p.P / 2;
    c->ay = Axis{p.M_y, p.T_y, p.pitch, p.overlap, c->r, p.G_y, p.layout};
    c->ax = Axis{p.M_x, p.T_x, p.pitch, p.overlap, c->r, p.G_x, p.layout};
    std::string e = c->ay.validate();
    if (e.empty()) e = c->ax.validate();
    if (!e.empty()) return fail(nullptr, DEBLUR_E_SHAPE, "geometry: " + e);
    if (p.model == DEBLUR_MODEL_LOCAL && (p.G_y != p.T_y || p.G_x != p.T_x))
        return fail(nullptr, DEBLUR_E_SHAPE, "local model needs one PSF node per tile");
    if (p.layout == DEBLUR_LAYOUT_GRID && p.model != DEBLUR_MODEL_LOCAL)
        return fail(nullptr, DEBLUR_E_SHAPE, "the grid layout uses each block's own PSF (DEBLUR_MODEL_LOCAL)");
    c->nt = p.T_y * p.T_x;
    c->nodes = p.G_y * p.G_x;
    c->Xy = p.M_y + 2 * c->r;
    c->Xx = p.M_x + 2 * c->r;
    int smax = 0;
    for (int a = 0; a < p.T_y; ++a) smax = std::max(smax, c->ay.support_len(a));
    for (int b = 0; b < p.T_x; ++b) smax = std::max(smax, c->ax.support_len(b));
    if (p.fft_size) {
        if (p.fft_size != 160 && p.fft_size != 320 && p.fft_size != 640)
            return fail(nullptr, DEBLUR_E_ARG, "fft_size must be 0, 160, 320 or 640");
        if (p.fft_size < smax) return fail(nullptr, DEBLUR_E_SHAPE, "fft_size smaller than a tile support");
        c->N = p.fft_size;
    } else {
        c->N = 0;
        for (int f : kFrames)
            if (f >= smax) {
                c->N = f;
                break;
            }
        if (!c->N) return fail(nullptr, DEBLUR_E_SHAPE, "tile support larger than the largest frame (640)");
    }
    const int N = c->N;
    c->plan = deblur_plan{N, waves_hi(N), waves_hi(N), DEBLUR_ORDER_COLUMN_MAJOR, 1, 0.f};
    // PSF contract: finite, non-negative, unit sum per node.  The step size
    // tau_t = 1/L_t bounds ||H_t||^2 by the largest row sum of H_t, which is
    // valid because every column sum of H_t is at most 1 -- true exactly for
    // non-negative unit-sum PSFs blended by tents summing to one.
    const int PP = p.P * p.P;
    for (int k = 0; k < c->nodes; ++k) {
        const float* h = psfs_host + (size_t)k * PP;
        double sum = 0.0;
        for (int i = 0; i < PP; ++i) {
            if (!std::isfinite(h[i])) return fail(nullptr, DEBLUR_E_ARG, "non-finite PSF value");
            if (h[i] < 0.f)
                return fail(nullptr, DEBLUR_E_ARG,
                            "PSF of node " + std::to_string(k) + " has a negative value (PSFs must be >= 0)");
            sum += h[i];
        }
        if (std::fabs(sum - 1.0) > kPsfSumTol)
            return fail(nullptr, DEBLUR_E_ARG,
                        "PSF of node " + std::to_string(k) + " sums to " + std::to_string(sum) +
                            ", not 1 (normalise the PSFs: the step sizes assume unit-sum PSFs)");
    }

    std::vector<std::vector<int>> ny(p.T_y), nx(p.T_x);
    for (int a = 0; a < p.T_y; ++a)
        ny[a] = (p.model == DEBLUR_MODEL_LOCAL) ? std::vector<int>{a} : c->ay.nodes(a);
    for (int b = 0; b < p.T_x; ++b)
        nx[b] = (p.model == DEBLUR_MODEL_LOCAL) ? std::vector<int>{b} : c->ax.nodes(b);
    for (auto& v : ny)
        if (v.size() > (size_t)dbl::kMaxK) return fail(nullptr, DEBLUR_E_SHAPE, "more than 3 PSF nodes per tile axis");
    for (auto& v : nx)
        if (v.size() > (size_t)dbl::kMaxK) return fail(nullptr, DEBLUR_E_SHAPE, "more than 3 PSF nodes per tile axis");

    c->tiles_h.resize(c->nt);
    c->desc.resize(c->nt);
    c->omega_max.resize(c->nt);
    int64_t xo = 0, yo = 0;
    for (int a = 0; a < p.T_y; ++a)
        for (int b = 0; b < p.T_x; ++b) {
            const int t = a * p.T_x + b;
            TileInfo& ti = c->tiles_h[t];
            int bs0, be0, bs1, be1, ss0, se0, ss1, se1;
            c->ay.block(a, bs0, be0);
            c->ax.block(b, bs1, be1);
            c->ay.support(a, ss0, se0);
            c->ax.support(b, ss1, se1);
            ti.ty = a;
            ti.tx = b;
            ti.sy = se0 - ss0;
            ti.sx = se1 - ss1;
            ti.by = be0 - bs0;
            ti.bx = be1 - bs1;
            ti.nky = (int)ny[a].size();
            ti.nkx = (int)nx[b].size();
            for (int k = 0; k < dbl::kMaxK * dbl::kMaxK; ++k) ti.spec[k] = 0;
            for (int ky = 0; ky < ti.nky; ++ky)
                for (int kx = 0; kx < ti.nkx; ++kx) ti.spec[ky * dbl::kMaxK + kx] = ny[a][ky] * p.G_x + nx[b][kx];
            deblur_tile_desc& d = c->desc[t];
            d.support_y0 = ss0;
            d.support_x0 = ss1;
            d.support_h = ti.sy;
            d.support_w = ti.sx;
            d.block_y0 = bs0;
            d.block_x0 = bs1;
            d.block_h = ti.by;
            d.block_w = ti.bx;
            d.x_offset = xo;
            d.y_offset = yo;
            d.n_terms = ti.nky * ti.nkx;
            d.frame = N;
            d.n_terms_y = ti.nky;
            d.n_terms_x = ti.nkx;
            xo += (int64_t)ti.sy * ti.sx;
            yo += (int64_t)ti.by * ti.bx;
            double om = 0.0;
            for (int m = 0; m < ti.sy; ++m) om = std::max(om, c->ay.omega(a, m));
            double omx = 0.0;
            for (int m = 0; m < ti.sx; ++m) omx = std::max(omx, c->ax.omega(b, m));
            c->omega_max[t] = (float)(om * omx);
        }
    c->support_total = xo;
    c->block_total = yo;
    return DEBLUR_OK;
}

int upload_tables(deblur_ctx* c, const float* psfs_host) {
    const deblur_params& p = c->p;
    const int N = c->N, r = c->r;
    // tents and omegas per tile row / column
    std::vector<float> tY((size_t)p.T_y * dbl::kMaxK * N, 0.f), tX((size_t)p.T_x * dbl::kMaxK * N, 0.f);
    std::vector<float> oY((size_t)p.T_y * N, 0.f), oX((size_t)p.T_x * N, 0.f);
    auto fill_axis = [&](const Axis& A, int T, std::vector<float>& tent, std::vector<float>& om) {
        for (int a = 0; a < T; ++a) {
            int s0, s1;
            A.support(a, s0, s1);
            std::vector<int> nodes = (p.model == DEBLUR_MODEL_LOCAL) ? std::vector<int>{a} : A.nodes(a);
            for (size_t k = 0; k < nodes.size(); ++k)
                for (int m = 0; m < s1 - s0; ++m)
                    tent[((size_t)a * dbl::kMaxK + k) * N + m] =
                        (p.model == DEBLUR_MODEL_LOCAL) ? 1.0f : (float)A.tent(nodes[k], s0 + m);
            for (int m = 0; m < s1 - s0; ++m) om[(size_t)a * N + m] = (float)A.omega(a, m);
        }
    };
    fill_axis(c->ay, p.T_y, tY, oY);
    fill_axis(c->ax, p.T_x, tX, oX);
    // the column kernels read the y tents lane-major: row l + LPL s of a
    // tent row (LPL = N / 20 lanes per column, s < 20) at l * 20 + s
    {
        const int LPL = N / dbl::kV;
        std::vector<float> row(N);
        for (size_t base = 0; base < tY.size(); base += N) {
            for (int l = 0; l < LPL; ++l)
                for (int s = 0; s < dbl::kV; ++s) row[(size_t)l * dbl::kV + s] = tY[base + l + (size_t)LPL * s];
            std::copy(row.begin(), row.end(), tY.begin() + base);
        }
    }
    // coverage of X rows / columns
    auto cover_axis = [&](const Axis& A, int T, int Xn) {
        std::vector<Cover> cv(Xn);
        for (int I = 0; I < Xn; ++I) {
            const int coord = I - r;
            Cover cc{};
            for (int a = 0; a < T; ++a) {
                int s0, s1;
                A.support(a, s0, s1);
                if (coord >= s0 && coord < s1) {
                    if (cc.n < dbl::kMaxCover) {
                        cc.a[cc.n] = a;
                        cc.m[cc.n] = coord - s0;
                        cc.w[cc.n] = (float)A.omega(a, coord - s0);
                    }
                    ++cc.n;
                }
            }
            cv[I] = cc;
        }
        return cv;
    };
    std::vector<Cover> cY = cover_axis(c->ay, p.T_y, c->Xy), cX = cover_axis(c->ax, p.T_x, c->Xx);
    for (const std::vector<Cover>* cv : {&cY, &cX})
        for (const Cover& cc : *cv) {
            if (cc.n < 1) return fail(c, DEBLUR_E_SHAPE, "an X row or column is covered by no tile");
            if (cc.n > dbl::kMaxCover)
                return fail(c, DEBLUR_E_SHAPE, "an X row or column is covered by more than three tiles");
            c->max_cover = std::max(c->max_cover, cc.n);
        }

    std::vector<int> so(2 * c->nt), bo(2 * c->nt), xo(2 * c->nt);
    std::vector<PackDesc> pds(c->nt), pdb(c->nt);
    for (int t = 0; t < c->nt; ++t) {
        const deblur_tile_desc& d = c->desc[t];
        so[2 * t] = d.support_y0;
        so[2 * t + 1] = d.support_x0;
        bo[2 * t] = d.block_y0;
        bo[2 * t + 1] = d.block_x0;
        xo[2 * t] = d.support_y0 + r;
        xo[2 * t + 1] = d.support_x0 + r;
        pds[t] = PackDesc{0, 0, d.support_h, d.support_w, (long long)d.x_offset};
        pdb[t] = PackDesc{r, r, d.block_h, d.block_w, (long long)d.y_offset};
    }
    std::vector<double2> twd(N);
    for (int e = 0; e < N; ++e) {
        const double a = -2.0 * M_PI * (double)e / N;
        twd[e] = make_double2(std::cos(a), std::sin(a));
    }

    int rc;
    if ((rc = dev_alloc(c, &c->tiles, c->nt))) return rc;
    if ((rc = dev_alloc(c, &c->tentY, tY.size()))) return rc;
    if ((rc = dev_alloc(c, &c->tentX, tX.size()))) return rc;
    if ((rc = dev_alloc(c, &c->omY, oY.size()))) return rc;
    if ((rc = dev_alloc(c, &c->omX, oX.size()))) return rc;
    if ((rc = dev_alloc(c, &c->covY, cY.size()))) return rc;
    if ((rc = dev_alloc(c, &c->covX, cX.size()))) return rc;
    if ((rc = dev_alloc(c, &c->sorg, so.size()))) return rc;
    if ((rc = dev_alloc(c, &c->borg, bo.size()))) return rc;
    if ((rc = dev_alloc(c, &c->xorg, xo.size()))) return rc;
    std::vector<int> sd(2 * c->nt), bd(2 * c->nt);
    for (int t = 0; t < c->nt; ++t) {
        sd[2 * t] = c->desc[t].support_h;
        sd[2 * t + 1] = c->desc[t].support_w;
        bd[2 * t] = c->desc[t].block_h;
        bd[2 * t + 1] = c->desc[t].block_w;
    }
    if ((rc = dev_alloc(c, &c->sdim, sd.size()))) return rc;
    if ((rc = dev_alloc(c, &c->bdim, bd.size()))) return rc;
    HIP_TRY(c, hipMemcpy(c->sdim, sd.data(), sd.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->bdim, bd.data(), bd.size() * 4, hipMemcpyHostToDevice));
    // tile orders of the column kernels: identity, and by PSF term count (most first)
    std::vector<int> pid(c->nt), phv(c->nt);
    for (int t = 0; t < c->nt; ++t) pid[t] = phv[t] = t;
    std::stable_sort(phv.begin(), phv.end(), [&](int a, int b) {
        return c->desc[a].n_terms > c->desc[b].n_terms;
    });
    if ((rc = dev_alloc(c, &c->perm_id, c->nt))) return rc;
    if ((rc = dev_alloc(c, &c->perm_heavy, c->nt))) return rc;
    HIP_TRY(c, hipMemcpy(c->perm_id, pid.data(), c->nt * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->perm_heavy, phv.data(), c->nt * 4, hipMemcpyHostToDevice));
    // the same order within each group of a split into G tile groups
    c->perm_heavy_g[1] = c->perm_heavy;
    for (int G = 2; G <= kMaxGroups; ++G) {
        std::vector<int> pg(pid);
        for (int g = 0; g < G; ++g) {
            int t0, cnt;
            group_bounds(c->nt, G, g, t0, cnt);
            std::stable_sort(pg.begin() + t0, pg.begin() + t0 + cnt,
                             [&](int a, int b) { return c->desc[a].n_terms > c->desc[b].n_terms; });
        }
        if ((rc = dev_alloc(c, &c->perm_heavy_g[G], c->nt))) return rc;
        HIP_TRY(c, hipMemcpy(c->perm_heavy_g[G], pg.data(), c->nt * 4, hipMemcpyHostToDevice));
    }
    if ((rc = dev_alloc(c, &c->pd_support, pds.size()))) return rc;
    if ((rc = dev_alloc(c, &c->pd_block, pdb.size()))) return rc;
    if ((rc = make_twiddles(c, c->stream))) return rc;
    HIP_TRY(c, hipMemcpy(c->tiles, c->tiles_h.data(), c->nt * sizeof(TileInfo), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->tentY, tY.data(), tY.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->tentX, tX.data(), tX.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->omY, oY.data(), oY.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->omX, oX.data(), oX.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->covY, cY.data(), cY.size() * sizeof(Cover), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->covX, cX.data(), cX.size() * sizeof(Cover), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->sorg, so.data(), so.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->borg, bo.data(), bo.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->xorg, xo.data(), xo.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->pd_support, pds.data(), pds.size() * sizeof(PackDesc), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->pd_block, pdb.data(), pdb.size() * sizeof(PackDesc), hipMemcpyHostToDevice));

    // PSF spectra
    ScratchBuf<float> psf_buf;
    ScratchBuf<double2> twd_buf;
    const size_t npsf = (size_t)c->nodes * p.P * p.P;
    HIP_TRY(c, hipMalloc(&psf_buf.p, npsf * sizeof(float)));
    HIP_TRY(c, hipMalloc(&twd_buf.p, N * sizeof(double2)));
    float* psf_d = psf_buf.p;
    double2* twd_d = twd_buf.p;
    if ((rc = dev_alloc(c, &c->spec, (size_t)c->nodes * (N / 2 + 1) * N))) return rc;
    HIP_TRY(c, hipMemcpy(psf_d, psfs_host, npsf * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(twd_d, twd.data(), N * sizeof(double2), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(dbl::k_psf_spectra, dim3(std::min(((N / 2 + 1) * N + 255) / 256, 1024), c->nodes),
                       dim3(256), N * sizeof(double2), c->stream, psf_d, p.P, N, twd_d, c->spec);
    if ((rc = check_launch(c, "k_psf_spectra"))) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DEBLUR_OK;
}

int alloc_state(deblur_ctx* c) {
    int rc;
    const size_t fe = frame_elems(c), he = half_elems(c);
    if ((rc = dev_alloc(c, &c->x[0], fe))) return rc;
    if ((rc = dev_alloc(c, &c->x[1], fe))) return rc;
    if ((rc = dev_alloc(c, &c->u, fe))) return rc;
    if ((rc = dev_alloc(c, &c->frame_tmp, fe))) return rc;
    if ((rc = dev_alloc(c, &c->frame_tmp2, fe))) return rc;
    if ((rc = dev_alloc(c, &c->yw, fe))) return rc;
    if ((rc = dev_alloc(c, &c->Zk, he * dbl::kMaxK))) return rc;
    if ((rc = dev_alloc(c, &c->Gk, he * dbl::kMaxK))) return rc;
    if ((rc = dev_alloc(c, &c->Yc, he))) return rc;
    if ((rc = dev_alloc(c, &c->Rr, he))) return rc;
    if ((rc = dev_alloc(c, &c->obj_part, (size_t)c->nt * row_groups_max(c)))) return rc;
    const dim3 pg = pix_grid(c);
    c->cons_nparts = (int)(pg.x * pg.y);
    if ((rc = dev_alloc(c, &c->cons_part, c->cons_nparts))) return rc;
    if ((rc = dev_alloc(c, &c->res_hist, kResCap))) return rc;
    if ((rc = dev_alloc(c, &c->res_counter, 1))) return rc;
    if ((rc = dev_alloc(c, &c->res_last, 1))) return rc;
    if ((rc = dev_alloc(c, &c->reg_part, (size_t)2 * c->nt * c->reg_blocks))) return rc;
    if ((rc = dev_alloc(c, &c->tau, c->nt))) return rc;
    if ((rc = dev_alloc(c, &c->maxW, c->nt))) return rc;
    if ((rc = dev_alloc(c, &c->rowsum, c->nt))) return rc;
    if ((rc = dev_alloc(c, &c->y_glob, (size_t)c->p.M_y * c->p.M_x))) return rc;
    if ((rc = dev_alloc(c, &c->tile_scale, c->nt))) return rc;
    if ((rc = dev_alloc(c, &c->gmap, 2 * (size_t)c->nt))) return rc;
    if ((rc = dev_alloc(c, &c->use_cnn, c->nt))) return rc;
    if ((rc = dev_alloc(c, &c->tile_flag, c->nt))) return rc;
    if (c->fista) {
        if ((rc = dev_alloc(c, &c->wbuf, fe))) return rc;
        HIP_TRY(c, hipMemsetAsync(c->wbuf, 0, fe * sizeof(float), c->stream));
    }
    if (c->vmlmb) {
        // frames are written on the supports only: the rest stays zero
        for (float** f : {&c->vm_g[0], &c->vm_g[1], &c->vm_r[0], &c->vm_r[1], &c->vm_d, &c->vm_delta}) {
            if ((rc = dev_alloc(c, f, fe))) return rc;
            HIP_TRY(c, hipMemsetAsync(*f, 0, fe * sizeof(float), c->stream));
        }
        for (float** f : {&c->vm_S, &c->vm_Y}) {
            if ((rc = dev_alloc(c, f, fe * dbl::kVmMem))) return rc;
            HIP_TRY(c, hipMemsetAsync(*f, 0, fe * dbl::kVmMem * sizeof(float), c->stream));
        }
        if ((rc = dev_alloc(c, &c->vm_tile, c->nt))) return rc;
        HIP_TRY(c, hipMemsetAsync(c->vm_tile, 0, c->nt * sizeof(dbl::VmTile), c->stream));
        if ((rc = dev_alloc(c, &c->vm_part, (size_t)3 * c->nt * dbl::kVmBlocks))) return rc;
        if ((rc = dev_alloc(c, &c->vm_search, 1))) return rc;
    }
    HIP_TRY(c, hipHostMalloc((void**)&c->h_pinned, 64 * sizeof(double), hipHostMallocDefault));
    // zero everything that is read before being written
    for (float* f : {c->x[0], c->x[1], c->u, c->frame_tmp, c->frame_tmp2})
        HIP_TRY(c, hipMemsetAsync(f, 0, fe * sizeof(float), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->yw, 0, fe * sizeof(float2), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->Zk, 0, he * dbl::kMaxK * sizeof(float2), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->Gk, 0, he * dbl::kMaxK * sizeof(float2), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->Yc, 0, he * sizeof(float2), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->Rr, 0, he * sizeof(float2), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DEBLUR_OK;
}

// H applied to the frames in src (support frames) -> Hx frames in dst.
void apply_H_frames(deblur_ctx* c, hipStream_t s, const float* src, float* dst) {
    row_fwd(c, s, src, c->Zk, 1);
    col_H(c, s);
    row_inv(c, s, c->Yc, dst, 0);
}

// Row sums max_Bt (H_t 1) per tile (for the step sizes).
int compute_rowsums(deblur_ctx* c) {
    hipLaunchKernelGGL(dbl::k_fill, dim3(1024), dim3(256), 0, c->stream, c->frame_tmp2, 1.0f, frame_elems(c));
    // ones on the supports only
    std::vector<float> ones((size_t)c->support_total, 1.0f);
    ScratchBuf<float> ones_buf;
    HIP_TRY(c, hipMalloc(&ones_buf.p, std::max<size_t>(ones.size(), 1) * sizeof(float)));
    float* ones_d = ones_buf.p;
    HIP_TRY(c, hipMemcpy(ones_d, ones.data(), ones.size() * sizeof(float), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(dbl::k_pack, frame_grid(c), dim3(256), 0, c->stream, ones_d, c->pd_support, c->N,
                       c->frame_tmp2);
    apply_H_frames(c, c->stream, c->frame_tmp2, c->frame_tmp);
    hipLaunchKernelGGL(dbl::k_block_max, dim3(c->nt), dim3(256), 0, c->stream, c->frame_tmp, 1, 0, c->tiles, c->N,
                       c->r, c->rowsum, 0);
    int rc = check_launch(c, "row sums");
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DEBLUR_OK;
}

// The captured graph of n_inner Local-Solver steps from x[parity], followed
// by the consensus step when with_consensus (one D-R round), under the
// current launch plan; cached per plan and key for the context's lifetime,
// so a change of plan captures the new plan's rounds (once) and leaves the
// earlier ones in place.
int ensure_graph(deblur_ctx* c, int n_inner, int parity, bool with_consensus, hipGraphExec_t* out) {
    const deblur_plan& pl = c->plan;
    const auto key = std::make_tuple(pl.col_waves, pl.row_waves, pl.tile_order, pl.tile_groups, n_inner, parity,
                                     with_consensus ? 1 : 0);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return DEBLUR_OK;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = local_steps(c, c->cap_stream, c->cap_aux, n_inner, parity);
    const int par = (n_inner & 1) ? 1 - parity : parity;
    if (with_consensus) consensus_launch(c, c->cap_stream, par);
    if (e1 == hipSuccess) e1 = hipGetLastError();
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(c, DEBLUR_E_HIP, std::string("graph capture: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    hipGraphExec_t ex = nullptr;
    HIP_TRY(c, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    c->graph_defs.push_back(g);
    c->graphs[key] = ex;
    *out = ex;
    return DEBLUR_OK;
}

void drop_graphs(deblur_ctx* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t g : c->graph_defs) (void)hipGraphDestroy(g);
    c->graphs.clear();
    c->graph_defs.clear();
}

// DEBLUR_E_NONFINITE naming the tiles whose current x holds a non-finite
// value (where a local solve diverged), else those whose u does (searched on
// the device), so the caller can see where a solve broke down.
int nonfinite_fail(deblur_ctx* c, const std::string& what) {
    hipLaunchKernelGGL(dbl::k_tile_nonfinite, dim3(c->nt), dim3(256), 0, c->stream, c->x[c->cur], c->u, c->N,
                       c->tile_flag);
    std::vector<int> flag(c->nt, 0);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(flag.data(), c->tile_flag, c->nt * sizeof(int), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, DEBLUR_E_NONFINITE, what + "; the non-finite tile search failed");
    for (int bit : {1, 2}) {
        std::string list;
        int n = 0;
        for (int t = 0; t < c->nt; ++t)
            if (flag[t] & bit) {
                if (n < 8)
                    list += (n ? ", " : "") + std::to_string(t) + " (row " + std::to_string(t / c->p.T_x) +
                            ", column " + std::to_string(t % c->p.T_x) + ")";
                ++n;
            }
        if (n)
            return fail(c, DEBLUR_E_NONFINITE,
                        what + "; non-finite " + (bit == 1 ? "x" : "u") + " in " + std::to_string(n) +
                            " tile(s): " + list + (n > 8 ? ", ..." : ""));
    }
    return fail(c, DEBLUR_E_NONFINITE, what + "; x and u are finite on every tile");
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char* deblur_last_error(const deblur_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

void deblur_destroy(deblur_ctx* c) {
    if (!c) return;
    // every stream that may still run this context's kernels drains before
    // any of its memory is released
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipStream_t a : c->aux_stream)
        if (a) (void)hipStreamSynchronize(a);
    drop_graphs(c);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (int g = 0; g < kMaxGroups - 1; ++g) {
        if (c->cap_aux[g]) (void)hipStreamDestroy(c->cap_aux[g]);
        if (c->aux_stream[g]) (void)hipStreamDestroy(c->aux_stream[g]);
        if (c->ev_join[g]) (void)hipEventDestroy(c->ev_join[g]);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    delete c;
}

int deblur_create(const deblur_params* params, const float* psfs_host, void* stream, deblur_ctx** out) {
    if (!params || !psfs_host || !out) return fail(nullptr, DEBLUR_E_ARG, "null argument");
    *out = nullptr;
    const deblur_params& p = *params;
    if (p.P < 1 || p.P % 2 == 0) return fail(nullptr, DEBLUR_E_ARG, "P must be odd and positive");
    if (p.model != DEBLUR_MODEL_INTERP && p.model != DEBLUR_MODEL_LOCAL) return fail(nullptr, DEBLUR_E_ARG, "model");
    if (p.reg != DEBLUR_REG_SMOOTH_TV && p.reg != DEBLUR_REG_HUBER) return fail(nullptr, DEBLUR_E_ARG, "reg");
    if (p.bc != DEBLUR_BC_NEUMANN && p.bc != DEBLUR_BC_CIRCULAR) return fail(nullptr, DEBLUR_E_ARG, "bc");
    if (!(p.reg_param > 0.f) || !(p.gamma > 0.f) || !(p.lambda >= 0.f) || !(p.rho > 0.f && p.rho < 2.f))
        return fail(nullptr, DEBLUR_E_ARG, "need reg_param > 0, gamma > 0, lambda >= 0, 0 < rho < 2");
    if (p.reg == DEBLUR_REG_SMOOTH_TV && !(p.reg_param >= 0x1p-63f))   // eps^2 a normal float
        return fail(nullptr, DEBLUR_E_ARG, "smoothed TV needs eps >= 2^-63 (eps^2 must be a normal float)");
    if (p.local_solver != DEBLUR_SOLVER_PG && p.local_solver != DEBLUR_SOLVER_FISTA &&
        p.local_solver != DEBLUR_SOLVER_VMLMB)
        return fail(nullptr, DEBLUR_E_ARG, "local_solver");
    if (p.independent != 0 && p.independent != 1) return fail(nullptr, DEBLUR_E_ARG, "independent must be 0 or 1");
    deblur_ctx* c = new deblur_ctx();
    c->p = p;
    c->fista = p.local_solver == DEBLUR_SOLVER_FISTA;
    c->vmlmb = p.local_solver == DEBLUR_SOLVER_VMLMB;
    c->stream = static_cast<hipStream_t>(stream);
    int rc = build_layout(c, psfs_host);
    if (rc) {
        delete c;
        return rc;
    }
    bool ok = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int g = 0; ok && g < kMaxGroups - 1; ++g)
        ok = hipStreamCreateWithFlags(&c->cap_aux[g], hipStreamNonBlocking) == hipSuccess &&
             hipStreamCreateWithFlags(&c->aux_stream[g], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&c->ev_join[g], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        deblur_destroy(c);
        return fail(nullptr, DEBLUR_E_HIP, "hipStreamCreate / hipEventCreate failed");
    }
    rc = upload_tables(c, psfs_host);
    if (!rc && preload_plan(c) != hipSuccess) rc = fail(c, DEBLUR_E_HIP, "kernel code could not be loaded");
    if (!rc) rc = alloc_state(c);
    if (!rc) rc = compute_rowsums(c);
    if (rc) {
        g_create_error = c->err;
        deblur_destroy(c);
        return rc;
    }
    *out = c;
    return DEBLUR_OK;
}

int deblur_tile_layout(const deblur_ctx* c, deblur_tile_desc* desc, int32_t cap, int64_t* support_total,
                       int64_t* block_total) {
    if (!c) return DEBLUR_E_ARG;
    if (desc)
        for (int t = 0; t < std::min<int>(cap, c->nt); ++t) desc[t] = c->desc[t];
    if (support_total) *support_total = c->support_total;
    if (block_total) *block_total = c->block_total;
    return c->nt;
}

int deblur_set_observation(deblur_ctx* c, const float* y, const float* w) {
    if (!c || !y) return fail(c, DEBLUR_E_ARG, "null argument");
    // a failed call leaves neither an observation nor a state to iterate on
    const bool had_state = c->have_state;
    c->have_obs = false;
    c->have_state = false;
    hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, c->stream, y, c->y_glob,
                       (size_t)c->p.M_y * c->p.M_x);
    hipLaunchKernelGGL(dbl::k_set_obs, frame_grid(c), dim3(256), 0, c->stream, y, w, c->tiles, c->borg, c->p.M_x,
                       c->N, c->r, c->yw);
    hipLaunchKernelGGL(dbl::k_block_max, dim3(c->nt), dim3(256), 0, c->stream, reinterpret_cast<float*>(c->yw), 2, 1,
                       c->tiles, c->N, c->r, c->maxW, 1);
    // y checked for finiteness the same way (frame_tmp is free scratch here)
    hipLaunchKernelGGL(dbl::k_block_max, dim3(c->nt), dim3(256), 0, c->stream, reinterpret_cast<float*>(c->yw), 2, 0,
                       c->tiles, c->N, c->r, c->frame_tmp, 0);
    int rc = check_launch(c, "set_observation");
    if (rc) return rc;
    std::vector<float> mw(c->nt), my(c->nt), rs(c->nt), tau(c->nt);
    HIP_TRY(c, hipMemcpyAsync(mw.data(), c->maxW, c->nt * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(my.data(), c->frame_tmp, c->nt * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(rs.data(), c->rowsum, c->nt * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const double Lphi = (c->p.reg == DEBLUR_REG_SMOOTH_TV) ? 8.0 / c->p.reg_param : 8.0;
    for (int t = 0; t < c->nt; ++t) {
        if (!std::isfinite(my[t])) return fail(c, DEBLUR_E_ARG, "y must be finite");
        if (!std::isfinite(mw[t]) || mw[t] < 0.f) return fail(c, DEBLUR_E_ARG, "W must be finite and >= 0");
        const double L = (double)mw[t] * rs[t] + (double)c->p.lambda * Lphi + (double)c->p.gamma * c->omega_max[t];
        tau[t] = (float)(1.0 / L);
    }
    HIP_TRY(c, hipMemcpyAsync(c->tau, tau.data(), c->nt * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->have_obs = true;
    c->have_state = had_state;
    return DEBLUR_OK;
}

int deblur_apply_H(deblur_ctx* c, const float* x_tiles, float* y_tiles) {
    if (!c || !x_tiles || !y_tiles) return fail(c, DEBLUR_E_ARG, "null argument");
    hipLaunchKernelGGL(dbl::k_pack, frame_grid(c), dim3(256), 0, c->stream, x_tiles, c->pd_support, c->N,
                       c->frame_tmp2);
    apply_H_frames(c, c->stream, c->frame_tmp2, c->frame_tmp);
    hipLaunchKernelGGL(dbl::k_unpack, frame_grid(c), dim3(256), 0, c->stream, c->frame_tmp, c->pd_block, c->N,
                       y_tiles);
    int rc = check_launch(c, "apply_H");
    if (rc) return rc;
    if (c->have_state) refresh_spectra(c, c->stream);
    return check_launch(c, "apply_H");
}

int deblur_apply_Ht(deblur_ctx* c, const float* s_tiles, float* x_tiles) {
    if (!c || !s_tiles || !x_tiles) return fail(c, DEBLUR_E_ARG, "null argument");
    hipLaunchKernelGGL(dbl::k_pack, frame_grid(c), dim3(256), 0, c->stream, s_tiles, c->pd_block, c->N,
                       c->frame_tmp2);
    row_fwd(c, c->stream, c->frame_tmp2, c->Rr, 0);
    col_Ht(c, c->stream);
    row_inv(c, c->stream, c->Gk, c->frame_tmp, 1);
    hipLaunchKernelGGL(dbl::k_unpack, frame_grid(c), dim3(256), 0, c->stream, c->frame_tmp, c->pd_support, c->N,
                       x_tiles);
    return check_launch(c, "apply_Ht");
}

int deblur_init(deblur_ctx* c, int32_t mode, const float* x0) {
    if (!c) return DEBLUR_E_ARG;
    if (!c->have_obs) return fail(c, DEBLUR_E_STATE, "deblur_set_observation must come first");
    c->cur = 0;
    if (mode == DEBLUR_INIT_ZERO) {
        hipLaunchKernelGGL(dbl::k_fill, dim3(1024), dim3(256), 0, c->stream, c->x[0], 0.0f, frame_elems(c));
        hipLaunchKernelGGL(dbl::k_fill, dim3(1024), dim3(256), 0, c->stream, c->u, 0.0f, frame_elems(c));
    } else if (mode == DEBLUR_INIT_OBSERVED) {
        hipLaunchKernelGGL(dbl::k_init_observed, frame_grid(c), dim3(256), 0, c->stream, c->y_glob, c->tiles,
                           c->sorg, c->p.M_y, c->p.M_x, c->N, c->x[0], c->u);
    } else if (mode == DEBLUR_INIT_GIVEN) {
        if (!x0) return fail(c, DEBLUR_E_ARG, "x0 required for DEBLUR_INIT_GIVEN");
        hipLaunchKernelGGL(dbl::k_pack, frame_grid(c), dim3(256), 0, c->stream, x0, c->pd_support, c->N, c->x[0]);
        hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, c->stream, c->x[0], c->u, frame_elems(c));
    } else {
        return fail(c, DEBLUR_E_ARG, "unknown init mode");
    }
    refresh_spectra(c, c->stream);
    c->have_state = true;
    c->round = 0;
    return check_launch(c, "init");
}

int deblur_solve_tiles(deblur_ctx* c, int32_t n_inner) {
    if (!c || n_inner < 0) return fail(c, DEBLUR_E_ARG, "bad argument");
    if (!c->have_state) return fail(c, DEBLUR_E_STATE, "deblur_init must come first");
    if (c->vmlmb) return vmlmb_steps(c, n_inner);
    const hipError_t e = local_steps(c, c->stream, c->aux_stream, n_inner, c->cur);
    if (e != hipSuccess) return fail(c, DEBLUR_E_HIP, std::string("solve_tiles: ") + hipGetErrorString(e));
    if (n_inner & 1) c->cur = 1 - c->cur;
    return check_launch(c, "solve_tiles");
}

int deblur_consensus(deblur_ctx* c, double* residual) {
    if (!c) return DEBLUR_E_ARG;
    if (!c->have_state) return fail(c, DEBLUR_E_STATE, "deblur_init must come first");
    hipLaunchKernelGGL(dbl::k_set_int, dim3(1), dim3(1), 0, c->stream, c->res_counter, 0);
    consensus_launch(c, c->stream, c->cur);
    int rc = check_launch(c, "consensus");
    if (rc) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->h_pinned, c->res_last, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (residual) *residual = c->h_pinned[0];
    c->round += 1;
    if (!std::isfinite(c->h_pinned[0])) return nonfinite_fail(c, "non-finite consensus residual");
    return DEBLUR_OK;
}

// D-R rounds with the VMLM-B Local-Solver, launched eagerly: round k runs
// n_inner + growth (first_round + k) VMLM-B iterations, then the consensus
// step.
int vmlmb_run(deblur_ctx* c, int n_outer, int n_inner, int growth, int first_round, double tol, double* residuals,
              int32_t* done) {
    hipLaunchKernelGGL(dbl::k_set_int, dim3(1), dim3(1), 0, c->stream, c->res_counter, 0);
    int k = 0;
    bool nonfinite = false;
    for (; k < n_outer;) {
        int rc = vmlmb_steps(c, n_inner + growth * (first_round + k));
        if (rc) return rc;
        consensus_launch(c, c->stream, c->cur);
        if ((rc = check_launch(c, "consensus"))) return rc;
        ++k;
        if (tol > 0.0) {
            HIP_TRY(c, hipMemcpyAsync(c->h_pinned, c->res_last, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (!std::isfinite(c->h_pinned[0])) {
                nonfinite = true;
                break;
            }
            if (c->h_pinned[0] <= tol) break;
        }
    }
    if (residuals && k > 0)
        HIP_TRY(c, hipMemcpyAsync(residuals, c->res_hist, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (done) *done = k;
    c->round += k;
    if (nonfinite) return nonfinite_fail(c, "non-finite consensus residual");
    if (residuals)
        for (int i = 0; i < k; ++i)
            if (!std::isfinite(residuals[i]))
                return nonfinite_fail(c, "non-finite consensus residual in round " + std::to_string(c->round - k + i));
    return DEBLUR_OK;
}

int deblur_run(deblur_ctx* c, int32_t n_outer, int32_t n_inner, double tol, double* residuals, int32_t* done) {
    if (!c || n_outer < 0 || n_inner < 0) return fail(c, DEBLUR_E_ARG, "bad argument");
    if (n_outer > kResCap) return fail(c, DEBLUR_E_ARG, "n_outer exceeds 4096");
    if (!c->have_state) return fail(c, DEBLUR_E_STATE, "deblur_init must come first");
    if (c->vmlmb) return vmlmb_run(c, n_outer, n_inner, 0, 0, tol, residuals, done);
    hipGraphExec_t g[2] = {nullptr, nullptr};
    int rc = ensure_graph(c, n_inner, c->cur, true, &g[c->cur]);
    if (!rc && (n_inner & 1)) rc = ensure_graph(c, n_inner, 1 - c->cur, true, &g[1 - c->cur]);
    if (rc) return rc;
    hipLaunchKernelGGL(dbl::k_set_int, dim3(1), dim3(1), 0, c->stream, c->res_counter, 0);
    int k = 0;
    bool nonfinite = false;
    for (; k < n_outer;) {
        HIP_TRY(c, hipGraphLaunch(g[c->cur], c->stream));
        if (n_inner & 1) c->cur = 1 - c->cur;
        ++k;
        if (tol > 0.0) {
            HIP_TRY(c, hipMemcpyAsync(c->h_pinned, c->res_last, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (!std::isfinite(c->h_pinned[0])) {
                nonfinite = true;
                break;
            }
            if (c->h_pinned[0] <= tol) break;
        }
    }
    if (residuals && k > 0)
        HIP_TRY(c, hipMemcpyAsync(residuals, c->res_hist, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (done) *done = k;
    c->round += k;
    if (nonfinite) return nonfinite_fail(c, "non-finite consensus residual");
    if (residuals)
        for (int i = 0; i < k; ++i)
            if (!std::isfinite(residuals[i]))
                return nonfinite_fail(c, "non-finite consensus residual in round " + std::to_string(c->round - k + i));
    return DEBLUR_OK;
}

int deblur_run_schedule(deblur_ctx* c, int32_t n_outer, int32_t n_inner, int32_t growth, int32_t first_round,
                        double tol, double* residuals, int32_t* done) {
    if (!c || n_outer < 0 || n_inner < 1 || growth < 0 || first_round < 0)
        return fail(c, DEBLUR_E_ARG, "bad argument");
    if (growth % n_inner) return fail(c, DEBLUR_E_ARG, "growth must be a multiple of n_inner");
    if (growth > 0 && c->fista)
        return fail(c, DEBLUR_E_ARG, "the growing schedule runs projected-gradient steps only");
    if (growth == 0) return deblur_run(c, n_outer, n_inner, tol, residuals, done);
    if (n_outer > kResCap) return fail(c, DEBLUR_E_ARG, "n_outer exceeds 4096");
    if (!c->have_state) return fail(c, DEBLUR_E_STATE, "deblur_init must come first");
    if (c->vmlmb) return vmlmb_run(c, n_outer, n_inner, growth, first_round, tol, residuals, done);
    // one graph of n_inner steps and one of the consensus step alone, per parity
    hipGraphExec_t steps[2] = {nullptr, nullptr}, cons[2] = {nullptr, nullptr};
    int rc = 0;
    for (int p = 0; p < 2 && !rc; ++p) {
        if ((n_inner & 1) || p == c->cur) rc = ensure_graph(c, n_inner, p, false, &steps[p]);
        if (!rc) rc = ensure_graph(c, 0, p, true, &cons[p]);
    }
    if (rc) return rc;
    hipLaunchKernelGGL(dbl::k_set_int, dim3(1), dim3(1), 0, c->stream, c->res_counter, 0);
    int k = 0;
    bool nonfinite = false;
    for (; k < n_outer;) {
        const long long m = 1 + (long long)(growth / n_inner) * (first_round + k);
        for (long long i = 0; i < m; ++i) {
            HIP_TRY(c, hipGraphLaunch(steps[c->cur], c->stream));
            if (n_inner & 1) c->cur = 1 - c->cur;
        }
        HIP_TRY(c, hipGraphLaunch(cons[c->cur], c->stream));
        ++k;
        if (tol > 0.0) {
            HIP_TRY(c, hipMemcpyAsync(c->h_pinned, c->res_last, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (!std::isfinite(c->h_pinned[0])) {
                nonfinite = true;
                break;
            }
            if (c->h_pinned[0] <= tol) break;
        }
    }
    if (residuals && k > 0)
        HIP_TRY(c, hipMemcpyAsync(residuals, c->res_hist, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (done) *done = k;
    c->round += k;
    if (nonfinite) return nonfinite_fail(c, "non-finite consensus residual");
    if (residuals)
        for (int i = 0; i < k; ++i)
            if (!std::isfinite(residuals[i]))
                return nonfinite_fail(c, "non-finite consensus residual in round " + std::to_string(c->round - k + i));
    return DEBLUR_OK;
}

int deblur_get_state(deblur_ctx* c, float* x_tiles, float* u_tiles, int32_t* round_host) {
    if (!c) return DEBLUR_E_ARG;
    if (!c->have_state) return fail(c, DEBLUR_E_STATE, "no state yet");
    if (round_host) *round_host = c->round;
    if (x_tiles)
        hipLaunchKernelGGL(dbl::k_unpack, frame_grid(c), dim3(256), 0, c->stream, c->x[c->cur], c->pd_support, c->N,
                           x_tiles);
    if (u_tiles)
        hipLaunchKernelGGL(dbl::k_unpack, frame_grid(c), dim3(256), 0, c->stream, c->u, c->pd_support, c->N,
                           u_tiles);
    return check_launch(c, "get_state");
}

int deblur_set_state(deblur_ctx* c, const float* x_tiles, const float* u_tiles, int32_t round) {
    if (!c || !x_tiles || !u_tiles) return fail(c, DEBLUR_E_ARG, "null argument");
    if (round < 0) return fail(c, DEBLUR_E_ARG, "round must be >= 0");
    if (!c->have_obs) return fail(c, DEBLUR_E_STATE, "deblur_set_observation must come first");
    c->round = round;
    c->cur = 0;
    hipLaunchKernelGGL(dbl::k_pack, frame_grid(c), dim3(256), 0, c->stream, x_tiles, c->pd_support, c->N, c->x[0]);
    hipLaunchKernelGGL(dbl::k_pack, frame_grid(c), dim3(256), 0, c->stream, u_tiles, c->pd_support, c->N, c->u);
    refresh_spectra(c, c->stream);
    c->have_state = true;
    return check_launch(c, "set_state");
}

int deblur_assemble(deblur_ctx* c, float* xg) {
    if (!c || !xg) return fail(c, DEBLUR_E_ARG, "null argument");
    if (!c->have_state) return fail(c, DEBLUR_E_STATE, "no state yet");
    hipLaunchKernelGGL(dbl::k_assemble, pix_grid(c), dim3(dbl::kPixBlock), 0, c->stream, c->x[c->cur], c->covY,
                       c->covX, c->Xx, c->p.T_x, c->N, xg);
    return check_launch(c, "assemble");
}

int deblur_objective(deblur_ctx* c, double* out) {
    if (!c || !out) return fail(c, DEBLUR_E_ARG, "null argument");
    if (!c->have_state) return fail(c, DEBLUR_E_STATE, "no state yet");
    // data term through the same kernels as the solver (Zk holds the current x)
    col_H(c, c->stream);
    row_resid(c, c->stream);
    hipLaunchKernelGGL(dbl::k_reg_terms, dim3(c->reg_blocks, c->nt), dim3(256), 0, c->stream, c->x[c->cur], c->u,
                       c->tiles, c->omY, c->omX, c->N, solve_params(c), c->reg_part);
    int rc = check_launch(c, "objective");
    if (rc) return rc;
    const int ng = c->nt * row_groups(c);
    std::vector<float> op(ng);
    std::vector<double> rp((size_t)2 * c->nt * c->reg_blocks);
    HIP_TRY(c, hipMemcpyAsync(op.data(), c->obj_part, ng * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(rp.data(), c->reg_part, rp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double d = 0.0, a = 0.0, b = 0.0;
    for (float v : op) d += v;
    for (size_t i = 0; i < rp.size(); i += 2) {
        a += rp[i];
        b += rp[i + 1];
    }
    out[0] = d;
    out[1] = (double)c->p.lambda * a;
    out[2] = b;
    if (!std::isfinite(d) || !std::isfinite(a) || !std::isfinite(b)) return nonfinite_fail(c, "non-finite objective");
    return DEBLUR_OK;
}

int deblur_step_sizes(deblur_ctx* c, float* tau_host) {
    if (!c || !tau_host) return fail(c, DEBLUR_E_ARG, "null argument");
    if (!c->have_obs) return fail(c, DEBLUR_E_STATE, "deblur_set_observation must come first");
    HIP_TRY(c, hipMemcpyAsync(tau_host, c->tau, c->nt * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DEBLUR_OK;
}

int deblur_blur_global(deblur_ctx* c, const float* xg, float* yg) {
    if (!c || !xg || !yg) return fail(c, DEBLUR_E_ARG, "null argument");
    if (c->p.layout != DEBLUR_LAYOUT_PITCH)
        return fail(c, DEBLUR_E_STATE, "deblur_blur_global needs the pitch layout (its blocks own the pixels)");
    hipLaunchKernelGGL(dbl::k_scatter_X, frame_grid(c), dim3(256), 0, c->stream, xg, c->tiles, c->xorg, c->Xx, c->N,
                       c->frame_tmp2);
    apply_H_frames(c, c->stream, c->frame_tmp2, c->frame_tmp);
    hipLaunchKernelGGL(dbl::k_gather_owner, dim3((c->p.M_x + 255) / 256, c->p.M_y), dim3(256), 0, c->stream,
                       c->frame_tmp, c->p.M_y, c->p.M_x, c->p.pitch, c->p.T_y, c->p.T_x, c->N, c->r, yg);
    int rc = check_launch(c, "blur_global");
    if (rc) return rc;
    if (c->have_state) refresh_spectra(c, c->stream);
    return check_launch(c, "blur_global");
}

int deblur_time_kernels(deblur_ctx* c, int32_t reps, float* ms) {
    if (!c || !ms || reps < 1) return fail(c, DEBLUR_E_ARG, "bad argument");
    if (!c->have_state) return fail(c, DEBLUR_E_STATE, "deblur_init must come first");
    constexpr int K = 4;   // kernels of one Local-Solver step
    hipEvent_t ev[K + 1];
    for (hipEvent_t& e : ev) HIP_TRY(c, hipEventCreate(&e));
    const int cur = c->cur;
    // the steps overwrite x[cur] (every second one) and the consensus step u: keep copies
    hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, c->stream, c->u, c->frame_tmp, frame_elems(c));
    hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, c->stream, c->x[cur], c->frame_tmp2, frame_elems(c));
    // Local-Solver kernels, timed one by one inside consecutive steps, as in a D-R round
    double acc[K] = {0, 0, 0, 0};
    int par = cur;
    for (int i = 0; i <= reps; ++i) {   // step 0 is a warm-up
        HIP_TRY(c, hipEventRecord(ev[0], c->stream));
        col_H(c, c->stream);
        HIP_TRY(c, hipEventRecord(ev[1], c->stream));
        row_resid(c, c->stream);
        HIP_TRY(c, hipEventRecord(ev[2], c->stream));
        col_Ht(c, c->stream);
        HIP_TRY(c, hipEventRecord(ev[3], c->stream));
        row_update(c, c->stream, c->x[par], c->x[1 - par], step_beta(c, 1, 10));
        HIP_TRY(c, hipEventRecord(ev[4], c->stream));
        HIP_TRY(c, hipEventSynchronize(ev[4]));
        par = 1 - par;
        if (i == 0) continue;
        for (int k = 0; k < K; ++k) {
            float t = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&t, ev[k], ev[k + 1]));
            acc[k] += t;
        }
    }
    for (int k = 0; k < K; ++k) ms[k] = (float)(acc[k] / reps);
    hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, c->stream, c->frame_tmp2, c->x[cur], frame_elems(c));
    // consensus step, repeated on the same (x, u)
    auto cons = [&]() {
        hipLaunchKernelGGL(c->max_cover > 2 ? dbl::k_consensus<3> : dbl::k_consensus<2>, pix_grid(c), dim3(dbl::kPixBlock), 0, c->stream, c->x[cur], c->u, c->covY,
                           c->covX, c->Xy, c->Xx, c->p.T_x, c->N, c->p.rho, c->cons_part);
    };
    cons();
    HIP_TRY(c, hipEventRecord(ev[0], c->stream));
    for (int i = 0; i < reps; ++i) cons();
    HIP_TRY(c, hipEventRecord(ev[1], c->stream));
    HIP_TRY(c, hipEventSynchronize(ev[1]));
    float t = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&t, ev[0], ev[1]));
    ms[K] = t / reps;
    hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, c->stream, c->frame_tmp, c->u, frame_elems(c));
    refresh_spectra(c, c->stream);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
    return check_launch(c, "time_kernels");
}

int deblur_get_plan(const deblur_ctx* c, deblur_plan* out) {
    if (!c || !out) return DEBLUR_E_ARG;
    *out = c->plan;
    return DEBLUR_OK;
}

int deblur_set_plan(deblur_ctx* c, const deblur_plan* pl) {
    if (!c || !pl) return fail(c, DEBLUR_E_ARG, "null argument");
    const int lo = waves_lo(c->N), hi = waves_hi(c->N);
    if (pl->frame != 0 && pl->frame != c->N)
        return fail(c, DEBLUR_E_ARG, "plan frame differs from the context's (" + std::to_string(c->N) + ")");
    if ((pl->col_waves != lo && pl->col_waves != hi) || (pl->row_waves != lo && pl->row_waves != hi))
        return fail(c, DEBLUR_E_ARG,
                    "waves per workgroup must be " + std::to_string(lo) + " or " + std::to_string(hi));
    if (pl->tile_order < DEBLUR_ORDER_COLUMN_MAJOR || pl->tile_order > DEBLUR_ORDER_HEAVY_FIRST)
        return fail(c, DEBLUR_E_ARG, "unknown tile order");
    if (pl->tile_groups != 1 && pl->tile_groups != 2 && pl->tile_groups != 4)
        return fail(c, DEBLUR_E_ARG, "tile_groups must be 1, 2 or 4");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (hipStream_t a : c->aux_stream) HIP_TRY(c, hipStreamSynchronize(a));
    c->plan = *pl;
    c->plan.frame = c->N;
    HIP_TRY(c, preload_plan(c));
    return DEBLUR_OK;
}

int deblur_autotune(const deblur_params* params, const float* psfs_host, void* stream, int32_t n_inner,
                    int32_t reps, deblur_plan* best, deblur_plan* trials, int32_t cap, int32_t* n_trials) {
    if (!params || !psfs_host || !best || reps < 1 || n_inner < 1 || (trials && cap < 0))
        return fail(nullptr, DEBLUR_E_ARG, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // candidate frames: the smallest supported frame that holds every support, and the next one
    std::vector<int> frames;
    if (params->fft_size) {
        frames.push_back(params->fft_size);
    } else {
        const int r = params->P / 2;
        const Axis ay{params->M_y, params->T_y, params->pitch, params->overlap, r, params->G_y, params->layout};
        const Axis ax{params->M_x, params->T_x, params->pitch, params->overlap, r, params->G_x, params->layout};
        int smax = 0;
        for (int a = 0; a < params->T_y; ++a) smax = std::max(smax, ay.support_len(a));
        for (int b = 0; b < params->T_x; ++b) smax = std::max(smax, ax.support_len(b));
        for (int f : kFrames)
            if (f >= smax && frames.size() < 2) frames.push_back(f);
        if (frames.empty()) return fail(nullptr, DEBLUR_E_SHAPE, "tile support larger than the largest frame (640)");
    }
    int count = 0;
    bool have = false;
    deblur_plan top{};
    for (size_t fi = 0; fi < frames.size(); ++fi) {
        deblur_params q = *params;
        q.fft_size = frames[fi];
        deblur_ctx* c = nullptr;
        int rc = deblur_create(&q, psfs_host, stream, &c);
        if (rc) {
            if (fi > 0 && rc == DEBLUR_E_OOM) break;   // the larger frame does not fit: keep what we have
            return rc;
        }
        float* y = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const size_t npix = (size_t)q.M_y * q.M_x;
        auto cleanup = [&]() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (y) (void)hipFree(y);
            deblur_destroy(c);
        };
        auto hip_fail = [&](hipError_t e, const char* what) {
            std::string m = std::string("autotune: ") + what + ": " + hipGetErrorString(e);
            cleanup();
            return fail(nullptr, DEBLUR_E_HIP, m);
        };
        hipError_t e = hipMalloc(&y, npix * sizeof(float));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            cleanup();
            if (fi > 0) break;
            return fail(nullptr, DEBLUR_E_OOM, "autotune: observation buffer");
        }
        hipLaunchKernelGGL(dbl::k_fill, dim3(1024), dim3(256), 0, s, y, 0.1f, npix);
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
            return hip_fail(e, "hipEventCreate");
        rc = deblur_set_observation(c, y, nullptr);
        if (!rc) rc = deblur_init(c, DEBLUR_INIT_OBSERVED, nullptr);
        const int lo = waves_lo(c->N), hi = waves_hi(c->N);
        for (int groups : {1, 2, 4})
        for (int cw : {hi, lo})
            for (int rw : {hi, lo})
                for (int order : {DEBLUR_ORDER_COLUMN_MAJOR, DEBLUR_ORDER_TILE_MAJOR, DEBLUR_ORDER_HEAVY_FIRST}) {
                    if (rc) break;
                    if (groups > c->nt) break;
                    if (!autotune_candidate(c->N, cw, rw)) continue;
                    deblur_plan pl{c->N, cw, rw, order, groups, 0.f};
                    rc = deblur_set_plan(c, &pl);
                    if (!rc) rc = deblur_run(c, 1, n_inner, 0.0, nullptr, nullptr);   // capture + warm
                    if (rc) break;
                    if ((e = hipEventRecord(e0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
                    rc = deblur_run(c, reps, n_inner, 0.0, nullptr, nullptr);
                    if (rc) break;
                    if ((e = hipEventRecord(e1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
                    if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
                    float ms = 0.f;
                    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
                    pl.us_per_iter = 1000.f * ms / ((float)reps * n_inner);
                    if (trials && count < cap) trials[count] = pl;
                    ++count;
                    if (!have || pl.us_per_iter < top.us_per_iter) {
                        top = pl;
                        have = true;
                    }
                }
        if (rc) {
            const std::string m = "autotune: " + c->err;
            cleanup();
            return fail(nullptr, rc, m);
        }
        cleanup();
    }
    if (!have) return fail(nullptr, DEBLUR_E_STATE, "autotune measured no plan");
    *best = top;
    if (n_trials) *n_trials = count;
    return DEBLUR_OK;
}

int deblur_debug_fft(int32_t n, int32_t batch, int32_t which, const float* in, float* out, void* stream) {
    if (n != 160 && n != 320 && n != 640) return fail(nullptr, DEBLUR_E_ARG, "n must be 160, 320 or 640");
    if (batch < 1 || !in || !out || which < 0 || which > 3) return fail(nullptr, DEBLUR_E_ARG, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // A throw-away context with the tables the row kernels read (unmasked).
    deblur_ctx tmp;
    tmp.N = n;
    tmp.nt = batch;
    tmp.plan = deblur_plan{n, waves_hi(n), waves_hi(n), DEBLUR_ORDER_COLUMN_MAJOR, 1, 0.f};
    std::vector<TileInfo> ti(batch);
    for (int t = 0; t < batch; ++t) {
        ti[t] = TileInfo{};
        ti[t].sy = ti[t].sx = ti[t].by = ti[t].bx = n;
        ti[t].nky = ti[t].nkx = 1;
    }
    std::vector<float> ones((size_t)dbl::kMaxK * n, 1.0f);
    int rc = dev_alloc(&tmp, &tmp.tiles, batch);
    if (!rc) rc = dev_alloc(&tmp, &tmp.tentX, ones.size());
    if (!rc) rc = make_twiddles(&tmp, s);
    hipError_t e = hipSuccess;
    if (!rc) {
        e = hipMemcpy(tmp.tiles, ti.data(), batch * sizeof(TileInfo), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(tmp.tentX, ones.data(), ones.size() * 4, hipMemcpyHostToDevice);
    }
    if (!rc && e == hipSuccess) {
        if (which == 0) {
            row_fwd(&tmp, s, in, reinterpret_cast<float2*>(out), 0);
        } else if (which == 3) {
            row_inv(&tmp, s, reinterpret_cast<const float2*>(in), out, 0);
        } else {
            DISPATCH_NW(&tmp, tmp.plan.col_waves, launch_col_fft_dbg, s, reinterpret_cast<const float2*>(in),
                        reinterpret_cast<float2*>(out), which == 1 ? -1 : 1);
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    for (void* p : tmp.allocs) (void)hipFree(p);
    tmp.allocs.clear();
    if (rc) return fail(nullptr, rc, tmp.err);
    if (e != hipSuccess) return fail(nullptr, DEBLUR_E_HIP, hipGetErrorString(e));
    return DEBLUR_OK;
}

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

// This GPU's copy of `scratch`: its device address is looked up once per
// device, with that device current, and kept.
int scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, DEBLUR_E_ARG, "device index " + std::to_string(dev) + " is beyond the " +
                                               std::to_string(kMaxDevices) + " devices the scratch table tracks");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, DEBLUR_E_HIP,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_dev[dev];
    return DEBLUR_OK;
}

}  // namespace

extern "C" {

int deblur_debug_fft_noalloc(int32_t n, int32_t batch, int32_t which, const float* in, float* out, void* stream) {
    if (n != 160 && n != 320 && n != 640) return fail(nullptr, DEBLUR_E_ARG, "n must be 160, 320 or 640");
    if (batch < 1 || !in || !out || which < 0 || which > 3) return fail(nullptr, DEBLUR_E_ARG, "bad argument");
    if (batch > kNoAllocMaxBatch)
        return fail(nullptr, DEBLUR_E_ARG, "batch " + std::to_string(batch) + " exceeds the allocation-free limit of " +
                                               std::to_string(kNoAllocMaxBatch) + " frames");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, DEBLUR_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (s) {
        hipDevice_t sdev = -1;
        e = hipStreamGetDevice(s, &sdev);
        if (e != hipSuccess)
            return fail(nullptr, DEBLUR_E_HIP, std::string("hipStreamGetDevice: ") + hipGetErrorString(e));
        if (sdev != dev)
            return fail(nullptr, DEBLUR_E_ARG, "the stream belongs to device " + std::to_string(sdev) + ", device " +
                                                   std::to_string(dev) + " is current");
    }
    unsigned char* base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;
    // The same launches as deblur_debug_fft, with the tables in scratch.
    deblur_ctx tmp;
    tmp.N = n;
    tmp.nt = batch;
    tmp.plan = deblur_plan{n, waves_hi(n), waves_hi(n), DEBLUR_ORDER_COLUMN_MAJOR, 1, 0.f};
    tmp.tw = reinterpret_cast<float2*>(base);
    tmp.tiles = reinterpret_cast<TileInfo*>(base + kNoAllocTwBytes);
    tmp.tentX = reinterpret_cast<float*>(base + kNoAllocTwBytes + kNoAllocTileBytes);
    const int n_tent = dbl::kMaxK * n;
    const int fill = std::max(batch, n_tent);
    hipLaunchKernelGGL(dbl::k_fill_fft_tables, dim3((fill + 255) / 256), dim3(256), 0, s, tmp.tiles, batch, n,
                       tmp.tentX, n_tent);
    switch (n) {
        case 160: hipLaunchKernelGGL(dbl::k_make_twiddles<160>, dim3(1), dim3(256), 0, s, tmp.tw); break;
        case 320: hipLaunchKernelGGL(dbl::k_make_twiddles<320>, dim3(1), dim3(256), 0, s, tmp.tw); break;
        default: hipLaunchKernelGGL(dbl::k_make_twiddles<640>, dim3(1), dim3(256), 0, s, tmp.tw); break;
    }
    if (which == 0) {
        row_fwd(&tmp, s, in, reinterpret_cast<float2*>(out), 0);
    } else if (which == 3) {
        row_inv(&tmp, s, reinterpret_cast<const float2*>(in), out, 0);
    } else {
        DISPATCH_NW(&tmp, tmp.plan.col_waves, launch_col_fft_dbg, s, reinterpret_cast<const float2*>(in),
                    reinterpret_cast<float2*>(out), which == 1 ? -1 : 1);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, DEBLUR_E_HIP, hipGetErrorString(e));
    return DEBLUR_OK;
}

}  // extern "C"

// ===========================================================================
// Warm-start network (host side)
// ===========================================================================

struct deblur_cnn {
    hipStream_t stream = nullptr;
    int maxB = 0, maxH = 0, maxW = 0;
    bool trainable = true;   // false: forward buffers only (deblur_cnn_create_inference)
    std::string err;
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    unsigned short *wf2 = nullptr, *wb2 = nullptr, *wf3 = nullptr, *wb3 = nullptr;
    float *w1 = nullptr, *w4 = nullptr;
    dbl::cnn::ImgDesc* desc = nullptr;
    unsigned short *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *dpA = nullptr, *dpB = nullptr;
    float *out = nullptr, *dout = nullptr;
    float *part = nullptr, *red0 = nullptr, *red1 = nullptr;
    size_t max_chunks = 0;
    double* loss_part = nullptr;
    size_t max_loss_parts = 0;
    int step = 0;
    std::vector<void*> allocs;
};

namespace {

int cfail(deblur_cnn* n, int code, const std::string& msg) {
    if (n) n->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIP_TRY_N(net, call)                                                                       \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return cfail((net), DEBLUR_E_HIP, std::string(#call ": ") + hipGetErrorString(e_));    \
    } while (0)

template <class T>
int net_alloc(deblur_cnn* n, T** ptr, size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return cfail(n, DEBLUR_E_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n->allocs.push_back(p);
    *ptr = static_cast<T*>(p);
    return DEBLUR_OK;
}

int net_check(deblur_cnn* n, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cfail(n, DEBLUR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return DEBLUR_OK;
}

namespace K = dbl::cnn;

dim3 pix_grid_cnn(int B, int H, int W) { return dim3((W + 255) / 256, H, B); }

int net_set_desc(deblur_cnn* n, int B, int H, int W, const int32_t* valid) {
    std::vector<K::ImgDesc> d(B);
    for (int b = 0; b < B; ++b) {
        d[b].vh = valid ? std::min<int>(valid[2 * b], H) : H;
        d[b].vw = valid ? std::min<int>(valid[2 * b + 1], W) : W;
    }
    HIP_TRY_N(n, hipMemcpyAsync(n->desc, d.data(), B * sizeof(K::ImgDesc), hipMemcpyHostToDevice, n->stream));
    HIP_TRY_N(n, hipStreamSynchronize(n->stream));   // d is a temporary
    return DEBLUR_OK;
}

void net_prep(deblur_cnn* n) {
    hipLaunchKernelGGL(K::k_prep_weights, dim3((K::kMidBf16 + 255) / 256), dim3(256), 0, n->stream, n->master, n->wf2,
                       n->wb2, n->wf3, n->wb3, n->w1, n->w4);
}

// Forward of B images [B][H][W] (device) -> n->out; activations kept.
void net_forward(deblur_cnn* n, const float* img, int B, int H, int W) {
    hipLaunchKernelGGL(K::k_conv_in, pix_grid_cnn(B, H, W), dim3(256), 0, n->stream, img, n->desc, H, W, n->w1,
                       n->master, n->a1);
    const dim3 mg = K::conv_mid_grid(B, H, W);
    hipLaunchKernelGGL(K::k_conv_mid, mg, dim3(256), 0, n->stream, n->a1, n->desc, H, W, n->wf2, n->master + K::kB2,
                       nullptr, n->a2);
    hipLaunchKernelGGL(K::k_conv_mid, mg, dim3(256), 0, n->stream, n->a2, n->desc, H, W, n->wf3, n->master + K::kB3,
                       nullptr, n->a3);
    hipLaunchKernelGGL(K::k_conv_out, pix_grid_cnn(B, H, W), dim3(256), 0, n->stream, n->a3, img, n->desc, H, W, n->w4,
                       n->master, n->out);
}

// Forward for inference: the fused kernel (activations in LDS only) for an
// inference-only network, the layer-by-layer kernels (activations kept for
// the backward pass) for a trainable one.  Both compute the same values.
void net_infer(deblur_cnn* n, const float* img, int B, int H, int W) {
    if (n->trainable) {
        net_forward(n, img, B, H, W);
        return;
    }
    hipLaunchKernelGGL(K::k_cnn_fwd, K::cnn_fwd_grid(B, H, W), dim3(K::kFusedThreads), 0, n->stream, img, n->desc, H,
                       W, n->w1, n->wf2, n->wf3, n->w4, n->master, n->out);
}

// Reduces n->part ([nchunk][ncols]) to one row and scatters it into n->grad.
void net_reduce(deblur_cnn* n, size_t nchunk, int ncols, int nw, int woff, int nb, int boff, int bsrc) {
    const float* src = n->part;
    float* bufs[2] = {n->red0, n->red1};
    int which = 0;
    size_t rows = nchunk;
    do {
        const size_t G = (rows + 63) / 64;
        hipLaunchKernelGGL(K::k_colsum, dim3((ncols + 255) / 256, (unsigned)G), dim3(256), 0, n->stream, src, (int)rows,
                           ncols, 64, bufs[which]);
        src = bufs[which];
        which ^= 1;
        rows = G;
    } while (rows > 1);
    hipLaunchKernelGGL(K::k_scatter_grad, dim3((nw + nb + 255) / 256), dim3(256), 0, n->stream, src, nw, woff, nb,
                       boff, bsrc, n->grad);
}

// Loss and gradients into n->grad for images / targets [B][H][W].
int net_loss_grad(deblur_cnn* n, const float* img, const float* target, int B, int H, int W, const int32_t* valid,
                  double* loss) {
    int rc = net_set_desc(n, B, H, W, valid);
    if (rc) return rc;
    net_prep(n);
    net_forward(n, img, B, H, W);
    long long npix = 0;
    for (int b = 0; b < B; ++b)
        npix += (long long)(valid ? std::min<int>(valid[2 * b], H) : H) * (valid ? std::min<int>(valid[2 * b + 1], W) : W);
    const dim3 pg = pix_grid_cnn(B, H, W);
    const size_t nlp = (size_t)pg.x * pg.y * pg.z;
    hipLaunchKernelGGL(K::k_loss, pg, dim3(256), 0, n->stream, n->out, target, n->desc, H, W, 1.0f / (float)npix,
                       n->dout, n->loss_part);
    const dim3 wg(W / K::kWgCols, H / K::kWgRows, B);
    const size_t nchunk = (size_t)wg.x * wg.y * wg.z;
    // layer 4
    hipLaunchKernelGGL(K::k_wgrad_edge, wg, dim3(256), 0, n->stream, 1, n->a3, n->dout, n->desc, H, W, n->part);
    net_reduce(n, nchunk, 9 * K::C + K::C, 9 * K::C, K::kW4, 1, K::kB4, 9 * K::C);
    hipLaunchKernelGGL(K::k_bwd_out, pg, dim3(256), 0, n->stream, n->dout, n->a3, n->desc, H, W, n->w4, n->dpA);
    // layer 3
    hipLaunchKernelGGL(K::k_wgrad_mid, wg, dim3(256), 0, n->stream, n->dpA, n->a2, n->desc, H, W, n->part);
    net_reduce(n, nchunk, 9 * K::C * K::C + K::C, 9 * K::C * K::C, K::kW3, K::C, K::kB3, 9 * K::C * K::C);
    const dim3 mg = K::conv_mid_grid(B, H, W);
    hipLaunchKernelGGL(K::k_conv_mid, mg, dim3(256), 0, n->stream, n->dpA, n->desc, H, W, n->wb3, nullptr, n->a2,
                       n->dpB);
    // layer 2
    hipLaunchKernelGGL(K::k_wgrad_mid, wg, dim3(256), 0, n->stream, n->dpB, n->a1, n->desc, H, W, n->part);
    net_reduce(n, nchunk, 9 * K::C * K::C + K::C, 9 * K::C * K::C, K::kW2, K::C, K::kB2, 9 * K::C * K::C);
    hipLaunchKernelGGL(K::k_conv_mid, mg, dim3(256), 0, n->stream, n->dpB, n->desc, H, W, n->wb2, nullptr, n->a1,
                       n->dpA);
    // layer 1
    hipLaunchKernelGGL(K::k_wgrad_edge, wg, dim3(256), 0, n->stream, 0, n->dpA, img, n->desc, H, W, n->part);
    net_reduce(n, nchunk, 9 * K::C + K::C, 9 * K::C, K::kW1, K::C, K::kB1, 9 * K::C);
    rc = net_check(n, "cnn backward");
    if (rc) return rc;
    if (loss) {
        std::vector<double> lp(nlp);
        HIP_TRY_N(n, hipMemcpyAsync(lp.data(), n->loss_part, nlp * sizeof(double), hipMemcpyDeviceToHost, n->stream));
        HIP_TRY_N(n, hipStreamSynchronize(n->stream));
        double s = 0.0;
        for (double v : lp) s += v;
        *loss = s / (double)npix;
        if (!std::isfinite(*loss)) return cfail(n, DEBLUR_E_NONFINITE, "non-finite loss");
    }
    return DEBLUR_OK;
}

int net_shape_ok(deblur_cnn* n, int B, int H, int W) {
    if (B < 1 || B > n->maxB || H < 1 || H > n->maxH || W < 1 || W > n->maxW)
        return cfail(n, DEBLUR_E_SHAPE, "batch or image larger than the network was created for");
    if (H % K::kWgRows || W % K::kWgCols) return cfail(n, DEBLUR_E_SHAPE, "H must be a multiple of 8 and W of 32");
    return DEBLUR_OK;
}

}  // namespace

extern "C" {

static int cnn_create(const float* params, int32_t seed, int32_t maxB, int32_t maxH, int32_t maxW, void* stream,
                      bool trainable, deblur_cnn** out) {
    if (!out || maxB < 1 || maxH < 8 || maxW < 32) return cfail(nullptr, DEBLUR_E_ARG, "bad argument");
    *out = nullptr;
    deblur_cnn* n = new deblur_cnn();
    n->trainable = trainable;
    n->stream = static_cast<hipStream_t>(stream);
    n->maxB = maxB;
    n->maxH = maxH;
    n->maxW = maxW;
    const size_t px = (size_t)maxB * maxH * maxW;
    n->max_chunks = (size_t)maxB * (maxH / K::kWgRows) * ((maxW + K::kWgCols - 1) / K::kWgCols);
    const size_t ncol = 9 * K::C * K::C + K::C;
    n->max_loss_parts = (size_t)maxB * maxH * ((maxW + 255) / 256);
    int rc = 0;
    if (!rc) rc = net_alloc(n, &n->master, K::kNParams);
    if (!rc) rc = net_alloc(n, &n->m, K::kNParams);
    if (!rc) rc = net_alloc(n, &n->v, K::kNParams);
    if (!rc) rc = net_alloc(n, &n->grad, K::kNParams);
    if (!rc) rc = net_alloc(n, &n->wf2, K::kMidBf16);
    if (!rc) rc = net_alloc(n, &n->wb2, K::kMidBf16);
    if (!rc) rc = net_alloc(n, &n->wf3, K::kMidBf16);
    if (!rc) rc = net_alloc(n, &n->wb3, K::kMidBf16);
    if (!rc) rc = net_alloc(n, &n->w1, 9 * K::C);
    if (!rc) rc = net_alloc(n, &n->w4, 9 * K::C);
    if (!rc) rc = net_alloc(n, &n->desc, maxB);
    if (!rc) rc = net_alloc(n, &n->out, px);
    if (trainable) {   // activations, backward activations, weight-gradient partials, loss partials
        if (!rc) rc = net_alloc(n, &n->a1, px * K::C);
        if (!rc) rc = net_alloc(n, &n->a2, px * K::C);
        if (!rc) rc = net_alloc(n, &n->a3, px * K::C);
        if (!rc) rc = net_alloc(n, &n->dpA, px * K::C);
        if (!rc) rc = net_alloc(n, &n->dpB, px * K::C);
        if (!rc) rc = net_alloc(n, &n->dout, px);
        if (!rc) rc = net_alloc(n, &n->part, n->max_chunks * ncol);
        if (!rc) rc = net_alloc(n, &n->red0, ((n->max_chunks + 63) / 64) * ncol);
        if (!rc) rc = net_alloc(n, &n->red1, ((n->max_chunks + 4095) / 4096 + 1) * ncol);
        if (!rc) rc = net_alloc(n, &n->loss_part, n->max_loss_parts);
    }
    if (rc) {
        g_create_error = n->err;
        for (void* p : n->allocs) (void)hipFree(p);
        delete n;
        return rc;
    }
    std::vector<float> w(K::kNParams, 0.f);
    if (params) {
        for (int i = 0; i < K::kNParams; ++i) w[i] = params[i];
    } else {
        // He initialisation from a counter-free LCG + Box-Muller (deterministic per seed)
        unsigned long long st = 0x9E3779B97F4A7C15ull ^ (unsigned long long)(uint32_t)seed;
        auto uni = [&]() {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            return ((st >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        };
        auto gauss = [&]() { return std::sqrt(-2.0 * std::log(uni())) * std::cos(2.0 * M_PI * uni()); };
        const int offs[4] = {K::kW1, K::kW2, K::kW3, K::kW4}, fan[4] = {9, 9 * K::C, 9 * K::C, 9 * K::C};
        const int cnt[4] = {9 * K::C, 9 * K::C * K::C, 9 * K::C * K::C, 9 * K::C};
        for (int l = 0; l < 4; ++l)
            for (int i = 0; i < cnt[l]; ++i) w[offs[l] + i] = (float)(gauss() * std::sqrt(2.0 / fan[l]) * (l == 3 ? 0.1 : 1.0));
    }
    hipError_t e = hipMemcpy(n->master, w.data(), K::kNParams * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->m, 0, K::kNParams * 4);
    if (e == hipSuccess) e = hipMemset(n->v, 0, K::kNParams * 4);
    if (e != hipSuccess) {
        g_create_error = hipGetErrorString(e);
        for (void* p : n->allocs) (void)hipFree(p);
        delete n;
        return DEBLUR_E_HIP;
    }
    *out = n;
    return DEBLUR_OK;
}

int deblur_cnn_create(const float* params, int32_t seed, int32_t maxB, int32_t maxH, int32_t maxW, void* stream,
                      deblur_cnn** out) {
    return cnn_create(params, seed, maxB, maxH, maxW, stream, true, out);
}

int deblur_cnn_create_inference(const float* params, int32_t seed, int32_t maxB, int32_t maxH, int32_t maxW,
                                void* stream, deblur_cnn** out) {
    return cnn_create(params, seed, maxB, maxH, maxW, stream, false, out);
}

void deblur_cnn_destroy(deblur_cnn* n) {
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    for (void* p : n->allocs) (void)hipFree(p);
    delete n;
}

const char* deblur_cnn_last_error(const deblur_cnn* n) { return n ? n->err.c_str() : g_create_error.c_str(); }

int deblur_cnn_get_params(deblur_cnn* n, float* params_host) {
    if (!n || !params_host) return cfail(n, DEBLUR_E_ARG, "null argument");
    HIP_TRY_N(n, hipMemcpyAsync(params_host, n->master, K::kNParams * 4, hipMemcpyDeviceToHost, n->stream));
    HIP_TRY_N(n, hipStreamSynchronize(n->stream));
    return DEBLUR_OK;
}

int deblur_cnn_set_params(deblur_cnn* n, const float* params_host) {
    if (!n || !params_host) return cfail(n, DEBLUR_E_ARG, "null argument");
    HIP_TRY_N(n, hipMemcpyAsync(n->master, params_host, K::kNParams * 4, hipMemcpyHostToDevice, n->stream));
    HIP_TRY_N(n, hipMemsetAsync(n->m, 0, K::kNParams * 4, n->stream));
    HIP_TRY_N(n, hipMemsetAsync(n->v, 0, K::kNParams * 4, n->stream));
    HIP_TRY_N(n, hipStreamSynchronize(n->stream));
    n->step = 0;
    return DEBLUR_OK;
}

int deblur_cnn_forward(deblur_cnn* n, const float* img, const int32_t* valid_host, int32_t B, int32_t H, int32_t W,
                       float* out) {
    if (!n || !img || !out) return cfail(n, DEBLUR_E_ARG, "null argument");
    int rc = net_shape_ok(n, B, H, W);
    if (!rc) rc = net_set_desc(n, B, H, W, valid_host);
    if (rc) return rc;
    net_prep(n);
    net_infer(n, img, B, H, W);
    HIP_TRY_N(n, hipMemcpyAsync(out, n->out, (size_t)B * H * W * 4, hipMemcpyDeviceToDevice, n->stream));
    return net_check(n, "cnn forward");
}

int deblur_cnn_loss_grad(deblur_cnn* n, const float* img, const float* target, int32_t B, int32_t H, int32_t W,
                         double* loss_host, float* grad_host) {
    if (!n || !img || !target) return cfail(n, DEBLUR_E_ARG, "null argument");
    if (!n->trainable) return cfail(n, DEBLUR_E_STATE, "inference-only network");
    int rc = net_shape_ok(n, B, H, W);
    if (!rc) rc = net_loss_grad(n, img, target, B, H, W, nullptr, loss_host);
    if (rc) return rc;
    if (grad_host) {
        HIP_TRY_N(n, hipMemcpyAsync(grad_host, n->grad, K::kNParams * 4, hipMemcpyDeviceToHost, n->stream));
        HIP_TRY_N(n, hipStreamSynchronize(n->stream));
    }
    return DEBLUR_OK;
}

int deblur_cnn_train_step(deblur_cnn* n, const float* img, const float* target, int32_t B, int32_t H, int32_t W,
                          float lr, double* loss_host) {
    if (!n || !img || !target || !(lr > 0.f)) return cfail(n, DEBLUR_E_ARG, "bad argument");
    if (!n->trainable) return cfail(n, DEBLUR_E_STATE, "inference-only network");
    int rc = net_shape_ok(n, B, H, W);
    if (!rc) rc = net_loss_grad(n, img, target, B, H, W, nullptr, loss_host);
    if (rc) return rc;
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow((double)b1, n->step)), c2 = (float)(1.0 - std::pow((double)b2, n->step));
    hipLaunchKernelGGL(K::k_adam, dim3((K::kNParams + 255) / 256), dim3(256), 0, n->stream, n->master, n->m, n->v,
                       n->grad, K::kNParams, lr, b1, b2, 1e-8f, c1, c2);
    return net_check(n, "adam");
}

int deblur_cnn_time_forward(deblur_cnn* n, const float* img, int32_t B, int32_t H, int32_t W, int32_t reps,
                            float* ms_host) {
    if (!n || !img || !ms_host || reps < 1) return cfail(n, DEBLUR_E_ARG, "bad argument");
    int rc = net_shape_ok(n, B, H, W);
    if (!rc) rc = net_set_desc(n, B, H, W, nullptr);
    if (rc) return rc;
    net_prep(n);
    hipEvent_t e0, e1, e2;
    HIP_TRY_N(n, hipEventCreate(&e0));
    HIP_TRY_N(n, hipEventCreate(&e1));
    HIP_TRY_N(n, hipEventCreate(&e2));
    net_infer(n, img, B, H, W);
    HIP_TRY_N(n, hipEventRecord(e0, n->stream));
    for (int i = 0; i < reps; ++i) net_infer(n, img, B, H, W);
    HIP_TRY_N(n, hipEventRecord(e1, n->stream));
    const dim3 mg = K::conv_mid_grid(B, H, W);
    if (n->trainable)   // the layer-by-layer 32 -> 32 layer alone
        for (int i = 0; i < reps; ++i)
            hipLaunchKernelGGL(K::k_conv_mid, mg, dim3(256), 0, n->stream, n->a1, n->desc, H, W, n->wf2,
                               n->master + K::kB2, nullptr, n->a2);
    HIP_TRY_N(n, hipEventRecord(e2, n->stream));
    HIP_TRY_N(n, hipEventSynchronize(e2));
    float t0 = 0.f, t1 = 0.f;
    HIP_TRY_N(n, hipEventElapsedTime(&t0, e0, e1));
    HIP_TRY_N(n, hipEventElapsedTime(&t1, e1, e2));
    ms_host[0] = t0 / reps;
    ms_host[1] = n->trainable ? t1 / reps : 0.f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    return net_check(n, "cnn timing");
}

int deblur_warm_inputs(deblur_ctx* c, float* frames, float* scale_host) {
    if (!c || !frames) return fail(c, DEBLUR_E_ARG, "null argument");
    if (!c->have_obs) return fail(c, DEBLUR_E_STATE, "deblur_set_observation must come first");
    hipLaunchKernelGGL(K::k_tile_scale, dim3(c->nt), dim3(256), 0, c->stream, c->yw, c->bdim, c->N, c->r,
                       c->tile_scale);
    hipLaunchKernelGGL(K::k_cnn_tile_input, frame_grid(c), dim3(256), 0, c->stream, c->y_glob, c->sorg, c->sdim,
                       c->tile_scale, c->p.M_y, c->p.M_x, c->N, frames);
    if (scale_host) {
        HIP_TRY(c, hipMemcpyAsync(scale_host, c->tile_scale, c->nt * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return check_launch(c, "warm_inputs");
}

int deblur_init_cnn(deblur_ctx* c, deblur_cnn* n, int32_t* use_cnn_host, int32_t* n_fallback) {
    if (!c || !n) return fail(c, DEBLUR_E_ARG, "null argument");
    if (!c->have_obs) return fail(c, DEBLUR_E_STATE, "deblur_set_observation must come first");
    const int N = c->N;
    if (n->maxH < N || n->maxW < N) return fail(c, DEBLUR_E_SHAPE, "network buffers smaller than the FFT frame");
    if (n->stream != c->stream) return fail(c, DEBLUR_E_ARG, "network and context must share a stream");
    hipStream_t s = c->stream;
    const size_t NN = (size_t)N * N;
    // network input: y at the nearest observed pixel / s_t on each support
    hipLaunchKernelGGL(K::k_tile_scale, dim3(c->nt), dim3(256), 0, s, c->yw, c->bdim, N, c->r, c->tile_scale);
    hipLaunchKernelGGL(K::k_cnn_tile_input, frame_grid(c), dim3(256), 0, s, c->y_glob, c->sorg, c->sdim,
                       c->tile_scale, c->p.M_y, c->p.M_x, N, c->frame_tmp2);
    net_prep(n);
    std::vector<int32_t> valid(2 * (size_t)c->nt);
    for (int t = 0; t < c->nt; ++t) {
        valid[2 * t] = c->desc[t].support_h;
        valid[2 * t + 1] = c->desc[t].support_w;
    }
    for (int t0 = 0; t0 < c->nt; t0 += n->maxB) {
        const int B = std::min(n->maxB, c->nt - t0);
        int rc = net_set_desc(n, B, N, N, valid.data() + 2 * t0);
        if (rc) return fail(c, rc, n->err);
        net_infer(n, c->frame_tmp2 + t0 * NN, B, N, N);
        hipLaunchKernelGGL(K::k_cnn_tile_output, dim3(std::min<int>((int)((NN + 255) / 256), 64), B), dim3(256), 0, s,
                           n->out, c->tile_scale + t0, c->sdim + 2 * t0, N, c->frame_tmp + t0 * NN);
    }
    // plain init (the fallback) into frame_tmp2
    hipLaunchKernelGGL(dbl::k_init_observed, frame_grid(c), dim3(256), 0, s, c->y_glob, c->tiles, c->sorg, c->p.M_y,
                       c->p.M_x, N, c->frame_tmp2, c->u);
    // projected-gradient map norm ||x0 - P(x0 - tau grad f_t(x0))|| per tile for both
    float* cand[2] = {c->frame_tmp, c->frame_tmp2};
    for (int k = 0; k < 2; ++k) {
        hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, s, cand[k], c->x[0], frame_elems(c));
        hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, s, cand[k], c->u, frame_elems(c));
        row_fwd(c, s, c->x[0], c->Zk, 1);
        inner_step(c, s, 0);
        hipLaunchKernelGGL(K::k_tile_dist2, dim3(c->nt), dim3(256), 0, s, c->x[1], c->x[0], N, c->gmap + k * c->nt);
    }
    std::vector<double> gm(2 * (size_t)c->nt);
    HIP_TRY(c, hipMemcpyAsync(gm.data(), c->gmap, gm.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    std::vector<int> use(c->nt);
    int nf = 0;
    for (int t = 0; t < c->nt; ++t) {
        if (!std::isfinite(gm[t]) || !std::isfinite(gm[c->nt + t])) {
            use[t] = 0;
        } else {
            // keep the network's start only if its map norm is >= 0.1% smaller
            use[t] = std::sqrt(gm[t]) <= 0.999 * std::sqrt(gm[c->nt + t]) ? 1 : 0;
        }
        nf += 1 - use[t];
        if (use_cnn_host) use_cnn_host[t] = use[t];
    }
    if (n_fallback) *n_fallback = nf;
    HIP_TRY(c, hipMemcpyAsync(c->use_cnn, use.data(), c->nt * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(K::k_tile_select, frame_grid(c), dim3(256), 0, s, c->frame_tmp, c->frame_tmp2, c->use_cnn, N,
                       c->x[0]);
    hipLaunchKernelGGL(dbl::k_copy, dim3(1024), dim3(256), 0, s, c->x[0], c->u, frame_elems(c));
    c->cur = 0;
    refresh_spectra(c, s);
    c->have_state = true;
    c->round = 0;
    HIP_TRY(c, hipStreamSynchronize(s));
    return check_launch(c, "init_cnn");
}

}  // extern "C"
