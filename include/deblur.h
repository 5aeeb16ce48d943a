/*
 * deblur.h -- C ABI of the MI355X tile solver for distributed non-blind
 * deblurring (Mourya, Ferrari, Flamary, Bianchi, Richard: "Distributed
 * Deblurring of Large Images of Wide Field-Of-View").
 *
 * All tiles of the paper's distributed formulation (Section III-A) live on
 * one GPU as a single batch.  The library owns every device buffer it needs;
 * after deblur_create() no call allocates memory.  Every call is ordered on
 * the HIP stream given at creation and is not thread-safe for one context
 * (several contexts may coexist).
 *
 * Pointers: "device" arguments are HIP device pointers that must stay valid
 * until the context stream has finished the call's work; "host" arguments
 * are ordinary host memory read or written before the call returns.
 * All floating-point data are IEEE fp32, row-major, no padding.
 *
 * Return values: DEBLUR_OK (0) or a negative DEBLUR_E_* code.  A failing
 * call leaves a message retrievable with deblur_last_error(ctx); failures of
 * deblur_create are reported by deblur_last_error(NULL).  No C++ exception
 * crosses this interface.
 *
 * Geometry (Section III-A, Fig. 1).  The observed image y is M_y x M_x.  The
 * unknown image x lives on X = [-r, M_y + r) x [-r, M_x + r), r = P/2.
 * Along one axis, block a covers observed pixels [a*pitch, min(a*pitch +
 * pitch + overlap, M)) for a < T-1 and [(T-1)*pitch, M) for the last block;
 * its support (the unknowns the tile estimates) is the block dilated by r.
 * Tile t = a * T_x + b.  Consensus weights omega_t are 1 inside a support
 * and ramp linearly, (s + 1/2)/L, across each overlap of length
 * L = overlap + 2r, so they sum to one over the tiles covering a pixel.
 *
 * Packed tile layouts used by apply_H / apply_Ht / get_state / set_state:
 *   "support-packed": tile after tile, each tile's support_h x support_w
 *                     pixels row-major, starting at desc.x_offset floats;
 *   "block-packed":   tile after tile, each block_h x block_w observed
 *                     pixels row-major, starting at desc.y_offset floats.
 */
#ifndef DEBLUR_H
#define DEBLUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct deblur_ctx deblur_ctx;

enum {
    DEBLUR_OK = 0,
    DEBLUR_E_ARG = -1,       /* bad pointer or parameter value            */
    DEBLUR_E_SHAPE = -2,     /* geometry the library cannot tile          */
    DEBLUR_E_OOM = -3,       /* device allocation failed (create only)    */
    DEBLUR_E_HIP = -4,       /* a HIP runtime call failed                 */
    DEBLUR_E_STATE = -5,     /* call out of order (e.g. no observation)   */
    DEBLUR_E_NONFINITE = -6  /* a residual or objective was not finite; the
                                message lists the tiles whose x (else u)
                                holds a non-finite value                   */
};

/* Blur model of a tile (Section II-B). */
enum {
    DEBLUR_MODEL_INTERP = 0, /* sum_k h_k * (w_k . x) over the PSF nodes whose first-order
                                interpolation weight w_k touches the tile */
    DEBLUR_MODEL_LOCAL = 1   /* the tile's own PSF only, H_i = C_i calH_i (needs G = T)   */
};

/* Regulariser phi(D x) (Section IV-A), D = forward differences. */
enum {
    DEBLUR_REG_SMOOTH_TV = 0, /* sum sqrt(|Dx|^2 + eps^2) - eps            */
    DEBLUR_REG_HUBER = 1      /* per-pixel Huber of |Dx| with threshold delta */
};

/* Block layout (Section III-A, Fig. 1; Section III-C).  PITCH: block a is
 * [a p, min(a p + p + o, M)), the last one [(T-1) p, M); supports of
 * neighbours overlap by o + 2r <= p; consensus weights 1 inside a support
 * and ramps (s + 1/2)/L across each overlap of length L = o + 2r.  GRID (the
 * smooth shift-variant layout of Section III-C): one block per PSF node
 * (T = G), spanning the grid points a - 1 .. a + 1 (the pixels strictly
 * between the node centres c_{a-1} and c_{a+1}, the first block from 0 and
 * the last to M), so neighbouring blocks overlap by half an interior block
 * and a pixel lies in two blocks per axis; pitch and overlap are unused;
 * the operator is each block's own PSF (DEBLUR_MODEL_LOCAL); needs
 * 2r <= M / G.  Consensus weights: node a's tent widened to reach over its
 * support, max(0, 1 - |i - c_a| / (M/G + r + 1/2)), normalised over the
 * (at most three) supports holding pixel i. */
enum {
    DEBLUR_LAYOUT_PITCH = 0,
    DEBLUR_LAYOUT_GRID = 1
};

enum {
    DEBLUR_BC_NEUMANN = 0,    /* difference 0 at the support's last row/column */
    DEBLUR_BC_CIRCULAR = 1    /* difference wraps within the support           */
};

/* Local-Solver of Algorithm 1 (Section III-B; Section IV-B allows any fast
 * first-order method).  Both take steps of length tau_t = 1/L_t on the prox
 * objective f_t(w) + 1/2 ||w - u_t||^2_alpha with projection onto w >= 0.
 * FISTA adds Nesterov momentum (Beck-Teboulle): w_j = P(y_j - tau g(y_j)),
 * y_{j+1} = w_j + beta_j (w_j - w_{j-1}), beta_j = (s_j - 1)/s_{j+1}, s_1 = 1,
 * s_{j+1} = (1 + sqrt(1 + 4 s_j^2))/2, restarted at every run of n steps
 * (each D-R round, each deblur_solve_tiles call) from y_1 = the current x, and
 * ending on w_n (the last step's beta is 0).  It keeps one more frame per tile
 * and is not available with the growing schedule. */
/* VMLM-B (Section IV-B: the paper's Local-Solver, a limited-memory
 * variable-metric BFGS method with bound constraints whose step comes from
 * a line search).  Per tile and iteration, from w with prox gradient g:
 * free variables F = all but w_i <= 0 with g_i > 0; d = -F B (F g) with B the
 * inverse BFGS matrix of the last 5 pairs (s, y) (two-loop recursion, initial
 * scaling <s,y>/<y,y> of the newest pair); w(a) = P(w + a d) with a = tau_t
 * when the memory is empty, else 1, halved until the prox objective's change
 * (evaluated through its exact expansion in w(a) - w) is at most
 * 1e-4 <g, w(a) - w>; the pair (w(a) - w, g(w(a)) - g) is kept if its inner
 * product is positive, else the memory is cleared; after 30 trials the tile
 * takes no step and clears its memory.  The memory starts empty at every run
 * of n iterations (each D-R round, each deblur_solve_tiles call).  Every
 * line-search trial ends with a 4-byte readback, so runs with this solver are
 * launched eagerly (no HIP graph); it keeps 16 more frames per tile. */
enum {
    DEBLUR_SOLVER_PG = 0,     /* projected gradient                              */
    DEBLUR_SOLVER_FISTA = 1,  /* accelerated projected gradient (FISTA)          */
    DEBLUR_SOLVER_VMLMB = 2   /* limited-memory BFGS with bounds (VMLM-B)        */
};

enum {
    DEBLUR_INIT_ZERO = 0,     /* x0 = 0                                          */
    DEBLUR_INIT_OBSERVED = 1, /* x0 = max(y, 0) at the nearest observed pixel     */
    DEBLUR_INIT_GIVEN = 2     /* x0 from a support-packed device array             */
};

typedef struct deblur_params {
    int32_t M_y, M_x;     /* observed image size                          */
    int32_t T_y, T_x;     /* tiles per axis                               */
    int32_t pitch;        /* tile pitch p                                 */
    int32_t overlap;      /* block overlap o (overlap + 2r <= pitch)      */
    int32_t G_y, G_x;     /* PSF grid nodes per axis                      */
    int32_t P;            /* PSF size, odd; r = P / 2                     */
    int32_t model;        /* DEBLUR_MODEL_*                               */
    int32_t reg;          /* DEBLUR_REG_*                                 */
    int32_t bc;           /* DEBLUR_BC_*                                  */
    int32_t positivity;   /* 1: x >= 0 constraint of Eq. (3), 0: none     */
    int32_t fft_size;     /* 0: chosen by the library; else 160/320/640   */
    float lambda;         /* regularisation weight                        */
    float reg_param;      /* eps (smoothed TV, >= 2^-63 so that eps^2 is a
                             normal float) or delta (Huber), > 0          */
    float gamma;          /* metric alpha_t = gamma * omega_t, > 0        */
    float rho;            /* D-R relaxation, in (0, 2)                    */
    int32_t local_solver; /* DEBLUR_SOLVER_*                              */
    int32_t independent;  /* 1: the paper's independent baseline (Section IV):
                             no consensus; each round sets u_t <- x_t, so
                             every tile runs the proximal-point method on its
                             own f_t; deblur_consensus and the rounds of
                             deblur_run report ||u_new - u_old|| / ||u_new||
                             and deblur_assemble blends with omega as usual.
                             0: Algorithm 1 (consensus)                   */
    int32_t layout;       /* DEBLUR_LAYOUT_* (0: pitch / overlap blocks)   */
} deblur_params;

typedef struct deblur_tile_desc {
    int32_t support_y0, support_x0; /* observed coordinate of the first support pixel (>= -r) */
    int32_t support_h, support_w;
    int32_t block_y0, block_x0;     /* observed coordinate of the first block pixel          */
    int32_t block_h, block_w;
    int64_t x_offset;               /* float offset of the tile in support-packed arrays     */
    int64_t y_offset;               /* float offset of the tile in block-packed arrays       */
    int32_t n_terms;                /* PSF terms K_t = n_terms_y * n_terms_x of the operator  */
    int32_t frame;                  /* FFT frame size used for the tile                      */
    int32_t n_terms_y, n_terms_x;   /* PSF nodes per axis whose weight touches the support  */
} deblur_tile_desc;

/* Create a context for the distributed problem of Section III-A: the image
 * split into overlapping blocks (Fig. 1), one local cost f_i per block with
 * the shift-variant blur of Section II-B (PSFs sampled on a regular grid and
 * blended by first-order interpolation weights, Eq. (2)).
 * psfs_host: host [G_y][G_x][P][P] fp32, PSF of node (ky, kx) sampled at
 * offsets q in [-r, r]^2 (index q + r); the operator is the true convolution
 * (H x)(j) = sum_q h(q) x(j - q).  Every PSF must be finite, non-negative and
 * sum to 1 within 1e-4 (the normalised PSFs of Section IV), else DEBLUR_E_ARG
 * with the offending node in deblur_last_error(NULL): the step sizes below
 * bound ||H_t||^2 by the largest row sum of H_t, which holds because the
 * column sums of H_t are at most 1 for such PSFs.  stream: a hipStream_t
 * (NULL = default stream).  Validates the geometry (overlap + 2r <= pitch,
 * every block >= P, supports fit the largest frame 640), allocates all
 * device memory, computes the PSF spectra.  *out receives the context, owned
 * by the caller until deblur_destroy.  On failure nothing stays allocated. */
int deblur_create(const deblur_params* params, const float* psfs_host, void* stream,
                  deblur_ctx** out);

void deblur_destroy(deblur_ctx* ctx);

/* Message of the last failing call on ctx (ctx == NULL: last failing create
 * on this thread).  Valid until the next call on the same context. */
const char* deblur_last_error(const deblur_ctx* ctx);

/* The blocks y_i and the supports of the unknowns x_i of Section III-A
 * (Fig. 1: each x_i extends its block by the PSF half-width r on every side).
 * Copies up to cap tile descriptors to host memory desc_host (may be NULL);
 * writes the total float counts of support- and block-packed arrays to
 * *support_total and *block_total (either may be NULL).  Returns the number
 * of tiles, or DEBLUR_E_ARG for a NULL context. */
int deblur_tile_layout(const deblur_ctx* ctx, deblur_tile_desc* desc_host, int32_t cap,
                       int64_t* support_total, int64_t* block_total);

/* Set the observation: y and w are device [M_y][M_x]; w = NULL means W = 1.
 * W is the inverse-variance weight of Eq. (3) (0 marks unmeasured pixels).
 * y must be finite and W finite and >= 0 on every block, else DEBLUR_E_ARG
 * (the context then keeps neither an observation nor a state: set a valid
 * observation and call deblur_init again).  A successful call keeps the
 * current state (x, u), so a solve can be resumed on new data.  Computes each tile's step size
 * tau_t = 1 / (max_Bt W * max_Bt (H_t 1) + lambda * L_phi + gamma * max omega_t),
 * with L_phi = 8/eps (TV) or 8 (Huber). */
int deblur_set_observation(deblur_ctx* ctx, const float* y, const float* w);

/* Forward operator of every tile (Section II-B):
 * y_t(j) = sum_k sum_q h_k(q) w_k(j - q) x_t(j - q) for j in block B_t.
 * x_tiles: device, support-packed; y_tiles: device, block-packed. */
int deblur_apply_H(deblur_ctx* ctx, const float* x_tiles, float* y_tiles);

/* Adjoint of deblur_apply_H: x_t(i) = sum_k w_k(i) sum_q h_k(q) s_t(i + q).
 * s_tiles: device, block-packed; x_tiles: device, support-packed. */
int deblur_apply_Ht(deblur_ctx* ctx, const float* s_tiles, float* x_tiles);

/* Set x^0 and u^0 = x^0 (Algorithm 1's initialisation).  x0_tiles (device,
 * support-packed) is read only for DEBLUR_INIT_GIVEN.  Needs an observation. */
int deblur_init(deblur_ctx* ctx, int32_t mode, const float* x0_tiles);

/* n_inner Local-Solver steps on every tile (Algorithm 1, first loop):
 * projected gradient on f_t(w) + 1/2 ||w - u_t||^2_alpha,
 *   w <- max(0, w - tau_t (H^T W (H w - y) + lambda grad phi(w) + alpha (w - u))),
 * warm-started from the current x (Section IV-B). */
int deblur_solve_tiles(deblur_ctx* ctx, int32_t n_inner);

/* Consensus and dual update (Lemma of Section III-B and Algorithm 1):
 * zbar = sum_t omega_t (2 x_t - u_t) / sum_t omega_t over the tiles covering
 * each pixel, u_t <- u_t + rho (zbar - x_t).  With params.independent = 1
 * (the independent baseline) the step is u_t <- x_t instead.  *residual_host
 * (may be NULL) receives ||u_new - u_old|| / ||u_new|| over all tiles. */
int deblur_consensus(deblur_ctx* ctx, double* residual_host);

/* Algorithm 1: up to n_outer rounds of (n_inner Local-Solver steps +
 * consensus), each round one captured HIP graph.  Stops after the first
 * round whose residual is <= tol (tol <= 0: run all rounds without host
 * synchronisation in between).  residuals_host (may be NULL) receives one
 * value per round run; *rounds_done the number of rounds. */
int deblur_run(deblur_ctx* ctx, int32_t n_outer, int32_t n_inner, double tol,
               double* residuals_host, int32_t* rounds_done);

/* Algorithm 1 with the growing inexact schedule of Section IV-B: round k
 * (k = first_round, first_round + 1, ...) runs n_inner + growth * k
 * Local-Solver steps, then the consensus step (growth 10 with n_inner 10 is
 * the paper's 10 + 10k).  growth must be a multiple of n_inner (the rounds
 * are replays of one captured n_inner-step graph and a consensus graph);
 * growth = 0 is deblur_run.  first_round lets a caller continue a schedule
 * over several calls.  tol, residuals_host and rounds_done as deblur_run. */
int deblur_run_schedule(deblur_ctx* ctx, int32_t n_outer, int32_t n_inner, int32_t growth, int32_t first_round,
                        double tol, double* residuals_host, int32_t* rounds_done);

/* Checkpoint / restore of Algorithm 1's iterate: the local estimates x_i
 * and the dual variables u_i (device, support-packed), and the round index k
 * of the outer loop (the number of consensus steps since the state was set
 * by deblur_init, deblur_init_cnn or deblur_set_state; deblur_run,
 * deblur_run_schedule and deblur_consensus advance it).  get: x_tiles,
 * u_tiles and round_host may each be NULL (only the others are written);
 * needs a state (DEBLUR_E_STATE).  set: round >= 0 becomes the context's
 * round index (a caller continuing a growing schedule passes it back as
 * first_round); needs an observation.  The state fully determines the next
 * rounds: FISTA restarts its momentum at every round, so nothing else is
 * carried across a round boundary. */
int deblur_get_state(deblur_ctx* ctx, float* x_tiles, float* u_tiles, int32_t* round_host);
int deblur_set_state(deblur_ctx* ctx, const float* x_tiles, const float* u_tiles, int32_t round);

/* Output of Algorithm 1, returned as the local estimates x_1 ... x_N, merged
 * into one image with the consensus weights: x_hat = sum_t omega_t x_t on X
 * (equal to the consensus image zbar at convergence): device
 * [M_y + 2r][M_x + 2r], written on the context stream.  Needs a state. */
int deblur_assemble(deblur_ctx* ctx, float* x_global);

/* Objective terms summed over tiles at the current (x, u), host doubles:
 * out[0] = sum 1/2 ||y_t - H_t x_t||^2_W, out[1] = sum lambda phi(D x_t),
 * out[2] = sum 1/2 ||x_t - u_t||^2_alpha. */
int deblur_objective(deblur_ctx* ctx, double* out_host);

/* Per-tile step sizes tau_t (host float[n_tiles]); needs an observation. */
int deblur_step_sizes(deblur_ctx* ctx, float* tau_host);

/* Image formation without noise (Eq. (2)): y = R sum_k Z_k H_k W_k C_k x for a
 * device image x_global on X, written to device y_global [M_y][M_x].  Each
 * observed pixel is taken from the tile whose block owns it (pitch layout
 * only: DEBLUR_E_STATE for the grid layout). */
int deblur_blur_global(deblur_ctx* ctx, const float* x_global, float* y_global);

/* Kernel timing on the context stream: reps Local-Solver steps (after one
 * warm-up step) with a HIP event between consecutive kernels, so each of the
 * four kernels is timed where it runs in a D-R round, then reps launches of
 * the consensus kernel.  Writes the mean milliseconds per launch to
 * ms_host[DEBLUR_N_KERNELS] in the order col_H, row_resid, col_Ht,
 * row_update, consensus.  The state (x, u) is saved and restored around the
 * measurement.  With the FISTA Local-Solver the steps use the momentum of a
 * step inside a 10-step run, so row_update is timed with its extra frame
 * traffic. */
enum { DEBLUR_N_KERNELS = 5 };
int deblur_time_kernels(deblur_ctx* ctx, int32_t reps, float* ms_host);

/* ---------------------------------------------------------------------------
 * Launch plans and the autotuner.  The per-iteration work of Algorithm 1
 * (all tiles' Local-Solver steps, then the consensus step) is the same
 * whatever the plan; the plan only decides how it is laid onto the GPU:
 *   frame       FFT frame N (any supported N >= the largest support gives
 *               the same operator, Section II-B's circular embedding);
 *               fixed when the context is created (params.fft_size);
 *   col_waves   waves per workgroup of the column-transform kernels;
 *   row_waves   waves per workgroup of the row-transform kernels;
 *               each one of two shapes the frame allows: {1, 2} for N = 160,
 *               {2, 4} for N = 320 and 640;
 *   tile_order  order in which the column kernels' work items (tiles x
 *               column groups) are laid over the GPU's 8 XCDs:
 *               DEBLUR_ORDER_COLUMN_MAJOR  a column group of all tiles per
 *                                          XCD (PSF spectra shared in L2),
 *               DEBLUR_ORDER_TILE_MAJOR    whole tiles per XCD,
 *               DEBLUR_ORDER_HEAVY_FIRST   column-group-major over the tiles
 *                                          sorted by PSF term count, most
 *                                          first.
 *   tile_groups 1: every kernel launch covers all tiles; 2 or 4: the tiles
 *               are split into that many contiguous groups (sizes differing
 *               by at most one) whose Local-Solver steps run as independent
 *               chains of launches on their own streams, joined before each
 *               consensus step (branches of the captured graph), so the
 *               kernels of one group fill the GPU while another's drain.
 * The iterates are bitwise identical under every plan: each pixel goes
 * through the same operations in the same order.  Only the grouping of the
 * partial sums of deblur_objective follows row_waves. */
enum {
    DEBLUR_ORDER_COLUMN_MAJOR = 0,
    DEBLUR_ORDER_TILE_MAJOR = 1,
    DEBLUR_ORDER_HEAVY_FIRST = 2
};
typedef struct deblur_plan {
    int32_t frame;
    int32_t col_waves;
    int32_t row_waves;
    int32_t tile_order;
    int32_t tile_groups;
    float us_per_iter;    /* measured microseconds per iteration (all tiles'
                             Local-Solver step + 1/n_inner of a consensus
                             step) when the plan comes from deblur_autotune;
                             0 otherwise                                   */
} deblur_plan;

/* The context's plan (host out).  A new context starts with the frame it
 * chose, the larger workgroup shape for both kernel families,
 * DEBLUR_ORDER_COLUMN_MAJOR and one tile group. */
int deblur_get_plan(const deblur_ctx* ctx, deblur_plan* plan_host);

/* Replaces the context's plan (host in).  plan.frame must equal the
 * context's frame (0 is taken as that frame); waves, order and tile_groups
 * must be among the values above, else DEBLUR_E_ARG.  Synchronises the
 * context's streams.  The graphs deblur_run captures are kept per plan until
 * deblur_destroy: the new plan's rounds are captured on their first use and
 * reused when the plan is set again.  State and observation are kept. */
int deblur_set_plan(deblur_ctx* ctx, const deblur_plan* plan_host);

/* Autotuner.  For the problem (params, psfs_host as for deblur_create) it
 * creates a scratch context per candidate frame (each supported N >= the
 * largest support, at most two, the smallest first; params.fft_size, if not
 * 0, is the only candidate), with a synthetic flat observation, and times
 * every plan of that frame: reps graph-captured D-R rounds of n_inner
 * Local-Solver steps each, after one untimed round, between HIP events on
 * stream.  best_host receives the fastest plan; trials_host (may be NULL),
 * of capacity cap, receives every plan measured, in the order measured, and
 * *n_trials_host their number.  All scratch memory is freed before return.
 * Errors as deblur_create (the scratch contexts' allocations) or
 * DEBLUR_E_ARG for reps < 1 or n_inner < 1. */
int deblur_autotune(const deblur_params* params, const float* psfs_host, void* stream, int32_t n_inner,
                    int32_t reps, deblur_plan* best_host, deblur_plan* trials_host, int32_t cap,
                    int32_t* n_trials_host);

/* Diagnostic access to the FFT core, one stage at a time (synchronous on
 * stream).  n in {160, 320, 640}; batch frames; all data device fp32,
 * complex values as interleaved (re, im) pairs:
 *   which = 0: row R2C.  in [batch][n][n] real -> out [batch][n/2][n]
 *              complex, out[b][f][i] = sum_c in[b][i][c] e^{-2 pi i f c/n}
 *              for 1 <= f < n/2 and out[b][0][i] = DC + i Nyquist of row i;
 *   which = 1: forward column FFT.  in, out [batch][n/2][n] complex,
 *              out[b][f][g] = sum_m in[b][f][m] e^{-2 pi i g m/n};
 *   which = 2: unnormalised inverse column FFT (e^{+2 pi i g m/n});
 *   which = 3: row C2R, the inverse of which = 0 times n/2:
 *              in [batch][n/2][n] complex -> out [batch][n][n] real. */
int deblur_debug_fft(int32_t n, int32_t batch, int32_t which, const float* in, float* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * FFT stages as deblur_debug_fft, with the same arguments and results, that
 * allocate nothing.  The stage tables (twiddles, tile table, tent row) live
 * in a fixed library-owned device array of 303,872 bytes per GPU, set up on
 * the first call on each device and held until the process ends; batch is
 * limited to 4096 frames (larger: DEBLUR_E_ARG, message in
 * deblur_last_error(NULL)).  The work is enqueued on stream, which must
 * belong to the current device (else DEBLUR_E_ARG); the call does not wait
 * for it.  Every call on one GPU rewrites that GPU's array: calls that
 * overlap on one GPU (different streams, or threads racing on one stream)
 * race.  Errors: DEBLUR_E_ARG as above, DEBLUR_E_HIP for a failed launch or
 * symbol lookup. */
int deblur_debug_fft_noalloc(int32_t n, int32_t batch, int32_t which, const float* in, float* out, void* stream);


/* ---------------------------------------------------------------------------
 * Learned warm start.  A 4-layer 3x3 convolutional network (1 -> 32 -> 32 ->
 * 32 -> 1 channels, ReLU, residual output, 19,105 parameters) predicts a
 * tile's solution from its normalised blurred input; it only sets the
 * starting point x^0 = u^0 of Algorithm 1, which then runs unchanged.
 * Weights and activations are BF16 with FP32 accumulation (MFMA for the
 * 32 -> 32 layers); the master weights and the Adam state are FP32.
 * Parameter vector layout: per layer W[C_out][C_in][3][3] then b[C_out].
 * Images are device [B][H][W] fp32, row-major; H a multiple of 8, W of 32.
 * ------------------------------------------------------------------------- */
typedef struct deblur_cnn deblur_cnn;

/* Create a network with buffers for up to max_batch images of
 * max_h x max_w.  params_host: 19,105 floats, or NULL for a seeded He
 * initialisation (last layer scaled by 0.1).  stream as for deblur_create. */
int deblur_cnn_create(const float* params_host, int32_t seed, int32_t max_batch, int32_t max_h, int32_t max_w,
                      void* stream, deblur_cnn** out);
/* The same for inference only: its forward pass is one fused launch (all
 * four layers of a 28 x 28 output block in one workgroup, the activations in
 * LDS only; the same values as the layer-by-layer kernels), so it holds the
 * output alone (4 bytes per pixel of max_batch x max_h x max_w) and
 * warm-starts many large tiles in one launch; loss_grad and train_step
 * return DEBLUR_E_STATE on it.  Weights come from params_host (e.g.
 * deblur_cnn_get_params of a trained network). */
int deblur_cnn_create_inference(const float* params_host, int32_t seed, int32_t max_batch, int32_t max_h,
                                int32_t max_w, void* stream, deblur_cnn** out);
void deblur_cnn_destroy(deblur_cnn* net);
const char* deblur_cnn_last_error(const deblur_cnn* net);
int deblur_cnn_get_params(deblur_cnn* net, float* params_host);
/* Replaces the weights and resets the optimiser state. */
int deblur_cnn_set_params(deblur_cnn* net, const float* params_host);

/* out = img + conv4(relu(conv3(relu(conv2(relu(conv1(img))))))) with zero
 * padding outside each image's valid region (valid_host: host [B][2] rows,
 * columns, or NULL for the whole image); out is 0 outside it. */
int deblur_cnn_forward(deblur_cnn* net, const float* img, const int32_t* valid_host, int32_t B, int32_t H,
                       int32_t W, float* out);

/* Loss mean((out - target)^2) over all pixels and its gradient w.r.t. the
 * parameters (grad_host: 19,105 floats, may be NULL; loss_host may be NULL). */
int deblur_cnn_loss_grad(deblur_cnn* net, const float* img, const float* target, int32_t B, int32_t H, int32_t W,
                         double* loss_host, float* grad_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss. */
int deblur_cnn_train_step(deblur_cnn* net, const float* img, const float* target, int32_t B, int32_t H, int32_t W,
                          float lr, double* loss_host);

/* Mean milliseconds over reps launches (HIP events on the network stream):
 * ms_host[0] of the network's forward pass (fused for an inference-only
 * network, layer by layer otherwise), ms_host[1] of one layer-by-layer
 * 32 -> 32 MFMA layer (0 for an inference-only network). */
int deblur_cnn_time_forward(deblur_cnn* net, const float* img, int32_t B, int32_t H, int32_t W, int32_t reps,
                            float* ms_host);

/* The network input of every tile as the warm start computes it: device
 * frames [n_tiles][frame][frame] = y (nearest observed pixel) / s_t on the
 * support, 0 elsewhere, with s_t = mean over the block of max(y, 0) (floored
 * at 1e-6) written to scale_host (host float[n_tiles], may be NULL). */
int deblur_warm_inputs(deblur_ctx* ctx, float* frames, float* scale_host);

/* Warm start of every tile: input y (nearest observed pixel) / s_t on the
 * support, s_t = mean over the block of max(y, 0); x^0 = max(0, s_t * net).
 * Per tile the network's start is kept only if its projected-gradient map
 * ||x0 - max(0, x0 - tau_t grad f_t(x0))|| is at least 0.1% smaller than that
 * of the plain start (DEBLUR_INIT_OBSERVED); otherwise the tile falls back to
 * the plain start, so the network never starts a tile worse by that measure.  use_cnn_host (may be NULL): host int32[n_tiles], 1 where
 * the network's start was kept; *n_fallback: tiles that fell back.  The
 * network must share the context's stream and have max_h, max_w >= frame. */
int deblur_init_cnn(deblur_ctx* ctx, deblur_cnn* net, int32_t* use_cnn_host, int32_t* n_fallback);

#ifdef __cplusplus
}
#endif

#endif /* DEBLUR_H */
