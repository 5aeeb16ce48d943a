"""ctypes binding of libdeblur.so (declared in include/deblur.h).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch provides device memory and the stream.  Importing this
module fails loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdeblur.so")

MODEL_INTERP, MODEL_LOCAL = 0, 1
REG_SMOOTH_TV, REG_HUBER = 0, 1
BC_NEUMANN, BC_CIRCULAR = 0, 1
INIT_ZERO, INIT_OBSERVED, INIT_GIVEN = 0, 1, 2
SOLVER_PG, SOLVER_FISTA, SOLVER_VMLMB = 0, 1, 2
LAYOUT_PITCH, LAYOUT_GRID = 0, 1
N_KERNELS = 5
KERNEL_NAMES = ("col_H", "row_resid", "col_Ht", "row_update", "consensus")

ORDER_COLUMN_MAJOR, ORDER_TILE_MAJOR, ORDER_HEAVY_FIRST = 0, 1, 2
ORDER_NAMES = {0: "column_major", 1: "tile_major", 2: "heavy_first"}

ERRORS = {-1: "E_ARG", -2: "E_SHAPE", -3: "E_OOM", -4: "E_HIP", -5: "E_STATE", -6: "E_NONFINITE"}


class DeblurError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("M_y", ctypes.c_int32), ("M_x", ctypes.c_int32),
        ("T_y", ctypes.c_int32), ("T_x", ctypes.c_int32),
        ("pitch", ctypes.c_int32), ("overlap", ctypes.c_int32),
        ("G_y", ctypes.c_int32), ("G_x", ctypes.c_int32),
        ("P", ctypes.c_int32), ("model", ctypes.c_int32),
        ("reg", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("positivity", ctypes.c_int32), ("fft_size", ctypes.c_int32),
        ("lambda_", ctypes.c_float), ("reg_param", ctypes.c_float),
        ("gamma", ctypes.c_float), ("rho", ctypes.c_float),
        ("local_solver", ctypes.c_int32), ("independent", ctypes.c_int32),
        ("layout", ctypes.c_int32),
    ]


class TileDesc(ctypes.Structure):
    _fields_ = [
        ("support_y0", ctypes.c_int32), ("support_x0", ctypes.c_int32),
        ("support_h", ctypes.c_int32), ("support_w", ctypes.c_int32),
        ("block_y0", ctypes.c_int32), ("block_x0", ctypes.c_int32),
        ("block_h", ctypes.c_int32), ("block_w", ctypes.c_int32),
        ("x_offset", ctypes.c_int64), ("y_offset", ctypes.c_int64),
        ("n_terms", ctypes.c_int32), ("frame", ctypes.c_int32),
        ("n_terms_y", ctypes.c_int32), ("n_terms_x", ctypes.c_int32),
    ]


class Plan(ctypes.Structure):
    _fields_ = [
        ("frame", ctypes.c_int32), ("col_waves", ctypes.c_int32), ("row_waves", ctypes.c_int32),
        ("tile_order", ctypes.c_int32), ("tile_groups", ctypes.c_int32), ("us_per_iter", ctypes.c_float),
    ]

    def as_dict(self):
        return {"frame": self.frame, "col_waves": self.col_waves, "row_waves": self.row_waves,
                "tile_order": ORDER_NAMES.get(self.tile_order, self.tile_order), "tile_groups": self.tile_groups,
                "us_per_iter": round(float(self.us_per_iter), 2)}


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1705_06603_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, f32p, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    sig = {
        "deblur_create": ([ctypes.POINTER(Params), vp, vp, ctypes.POINTER(vp)], i32),
        "deblur_destroy": ([vp], None),
        "deblur_last_error": ([vp], ctypes.c_char_p),
        "deblur_tile_layout": ([vp, ctypes.POINTER(TileDesc), i32, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64)], i32),
        "deblur_set_observation": ([vp, f32p, f32p], i32),
        "deblur_apply_H": ([vp, f32p, f32p], i32),
        "deblur_apply_Ht": ([vp, f32p, f32p], i32),
        "deblur_init": ([vp, i32, f32p], i32),
        "deblur_solve_tiles": ([vp, i32], i32),
        "deblur_consensus": ([vp, dp], i32),
        "deblur_run": ([vp, i32, i32, ctypes.c_double, dp, ctypes.POINTER(i32)], i32),
        "deblur_run_schedule": ([vp, i32, i32, i32, i32, ctypes.c_double, dp, ctypes.POINTER(i32)], i32),
        "deblur_get_state": ([vp, f32p, f32p, ctypes.POINTER(i32)], i32),
        "deblur_set_state": ([vp, f32p, f32p, i32], i32),
        "deblur_assemble": ([vp, f32p], i32),
        "deblur_objective": ([vp, dp], i32),
        "deblur_step_sizes": ([vp, ctypes.POINTER(ctypes.c_float)], i32),
        "deblur_blur_global": ([vp, f32p, f32p], i32),
        "deblur_time_kernels": ([vp, i32, ctypes.POINTER(ctypes.c_float)], i32),
        "deblur_debug_fft": ([i32, i32, i32, f32p, f32p, vp], i32),
        "deblur_debug_fft_noalloc": ([i32, i32, i32, f32p, f32p, vp], i32),
        "deblur_cnn_create": ([vp, i32, i32, i32, i32, vp, ctypes.POINTER(vp)], i32),
        "deblur_cnn_create_inference": ([vp, i32, i32, i32, i32, vp, ctypes.POINTER(vp)], i32),
        "deblur_cnn_destroy": ([vp], None),
        "deblur_cnn_last_error": ([vp], ctypes.c_char_p),
        "deblur_cnn_get_params": ([vp, vp], i32),
        "deblur_cnn_set_params": ([vp, vp], i32),
        "deblur_cnn_forward": ([vp, f32p, vp, i32, i32, i32, f32p], i32),
        "deblur_cnn_loss_grad": ([vp, f32p, f32p, i32, i32, i32, dp, vp], i32),
        "deblur_cnn_train_step": ([vp, f32p, f32p, i32, i32, i32, ctypes.c_float, dp], i32),
        "deblur_cnn_time_forward": ([vp, f32p, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_float)], i32),
        "deblur_init_cnn": ([vp, vp, vp, ctypes.POINTER(i32)], i32),
        "deblur_warm_inputs": ([vp, f32p, ctypes.POINTER(ctypes.c_float)], i32),
        "deblur_get_plan": ([vp, ctypes.POINTER(Plan)], i32),
        "deblur_set_plan": ([vp, ctypes.POINTER(Plan)], i32),
        "deblur_autotune": ([ctypes.POINTER(Params), vp, vp, i32, i32, ctypes.POINTER(Plan), ctypes.POINTER(Plan),
                             i32, ctypes.POINTER(i32)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def exported_symbols():
    """Names of the C entry points the binding declares."""
    return [
        "deblur_create", "deblur_destroy", "deblur_last_error", "deblur_tile_layout",
        "deblur_set_observation", "deblur_apply_H", "deblur_apply_Ht", "deblur_init",
        "deblur_solve_tiles", "deblur_consensus", "deblur_run", "deblur_run_schedule", "deblur_get_state",
        "deblur_set_state", "deblur_assemble", "deblur_objective", "deblur_step_sizes",
        "deblur_blur_global", "deblur_time_kernels", "deblur_debug_fft", "deblur_debug_fft_noalloc",
        "deblur_cnn_create", "deblur_cnn_create_inference", "deblur_cnn_destroy", "deblur_cnn_last_error", "deblur_cnn_get_params",
        "deblur_cnn_set_params", "deblur_cnn_forward", "deblur_cnn_loss_grad", "deblur_cnn_train_step",
        "deblur_cnn_time_forward", "deblur_init_cnn", "deblur_warm_inputs",
        "deblur_get_plan", "deblur_set_plan", "deblur_autotune",
    ]


def _ptr(t):
    """Device pointer of a contiguous float32 CUDA tensor (or None)."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def make_params(M, T, pitch, overlap, G, P, *, model=MODEL_INTERP, reg=REG_SMOOTH_TV, bc=BC_NEUMANN,
                positivity=True, fft_size=0, lam=1e-3, reg_param=1e-3, gamma=0.4, rho=1.0,
                M_x=None, T_x=None, G_x=None, local_solver=SOLVER_PG, independent=False, layout=0):
    p = Params()
    p.M_y, p.M_x = M, M if M_x is None else M_x
    p.T_y, p.T_x = T, T if T_x is None else T_x
    p.pitch, p.overlap = pitch, overlap
    p.G_y, p.G_x = G, G if G_x is None else G_x
    p.P, p.model, p.reg, p.bc = P, model, reg, bc
    p.positivity, p.fft_size = int(bool(positivity)), fft_size
    p.lambda_, p.reg_param, p.gamma, p.rho = lam, reg_param, gamma, rho
    p.local_solver = local_solver
    p.independent = int(bool(independent))
    p.layout = layout
    return p


class Context:
    """One deblurring problem on the GPU (all tiles as one batch)."""

    def __init__(self, params: Params, psfs, stream=None):
        import torch
        self._torch = torch
        self._L = lib()
        self.params = params
        psf = np.ascontiguousarray(np.asarray(psfs, dtype=np.float32))
        self._stream = _stream_handle(stream)
        self._stream_obj = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self._L.deblur_create(ctypes.byref(params), psf.ctypes.data_as(ctypes.c_void_p), self._stream,
                                   ctypes.byref(h))
        if rc != 0:
            raise DeblurError(rc, self._L.deblur_last_error(None).decode())
        self._h = h
        n = self._L.deblur_tile_layout(self._h, None, 0, None, None)
        descs = (TileDesc * n)()
        st, bt = ctypes.c_int64(), ctypes.c_int64()
        self._L.deblur_tile_layout(self._h, descs, n, ctypes.byref(st), ctypes.byref(bt))
        self.tiles = list(descs)
        self.support_total, self.block_total = st.value, bt.value
        self.r = params.P // 2
        self.X_shape = (params.M_y + 2 * self.r, params.M_x + 2 * self.r)

    # -- helpers -------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise DeblurError(rc, self._L.deblur_last_error(self._h).decode())

    def _empty(self, n):
        return self._torch.empty(n, dtype=self._torch.float32, device="cuda")

    @property
    def n_tiles(self):
        return len(self.tiles)

    def close(self):
        if getattr(self, "_h", None):
            self._L.deblur_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI calls ------------------------------------------------------------
    def set_observation(self, y, w=None):
        self._y_keep, self._w_keep = y, w
        self._check(self._L.deblur_set_observation(self._h, _ptr(y), _ptr(w)))

    def apply_H(self, x_tiles, out=None):
        out = self._empty(self.block_total) if out is None else out
        self._check(self._L.deblur_apply_H(self._h, _ptr(x_tiles), _ptr(out)))
        return out

    def apply_Ht(self, s_tiles, out=None):
        out = self._empty(self.support_total) if out is None else out
        self._check(self._L.deblur_apply_Ht(self._h, _ptr(s_tiles), _ptr(out)))
        return out

    def init(self, mode=INIT_OBSERVED, x0=None):
        self._check(self._L.deblur_init(self._h, mode, _ptr(x0)))

    def solve_tiles(self, n_inner):
        self._check(self._L.deblur_solve_tiles(self._h, n_inner))

    def consensus(self):
        r = ctypes.c_double()
        self._check(self._L.deblur_consensus(self._h, ctypes.byref(r)))
        return r.value

    def run(self, n_outer, n_inner=10, tol=0.0, growth=0, first_round=0):
        """D-R rounds; with growth > 0 round k runs n_inner + growth * k steps."""
        res = (ctypes.c_double * max(n_outer, 1))()
        done = ctypes.c_int32()
        if growth:
            self._check(self._L.deblur_run_schedule(self._h, n_outer, n_inner, growth, first_round, tol, res,
                                                    ctypes.byref(done)))
        else:
            self._check(self._L.deblur_run(self._h, n_outer, n_inner, tol, res, ctypes.byref(done)))
        return [res[i] for i in range(done.value)]

    def get_state(self):
        """(x, u) support-packed device arrays of the current iterate."""
        x, u = self._empty(self.support_total), self._empty(self.support_total)
        self._check(self._L.deblur_get_state(self._h, _ptr(x), _ptr(u), None))
        return x, u

    def state_round(self):
        """Round index k of the current state (consensus steps since it was set)."""
        k = ctypes.c_int32()
        self._check(self._L.deblur_get_state(self._h, None, None, ctypes.byref(k)))
        return k.value

    def set_state(self, x, u, round=0):
        self._check(self._L.deblur_set_state(self._h, _ptr(x), _ptr(u), round))

    def assemble(self):
        out = self._empty(self.X_shape[0] * self.X_shape[1])
        self._check(self._L.deblur_assemble(self._h, _ptr(out)))
        return out.view(self.X_shape)

    def objective(self):
        out = (ctypes.c_double * 3)()
        self._check(self._L.deblur_objective(self._h, out))
        return tuple(out)

    def step_sizes(self):
        out = (ctypes.c_float * self.n_tiles)()
        self._check(self._L.deblur_step_sizes(self._h, out))
        return np.array(out[:], dtype=np.float64)

    def blur_global(self, x_global):
        out = self._empty(self.params.M_y * self.params.M_x)
        self._check(self._L.deblur_blur_global(self._h, _ptr(x_global), _ptr(out)))
        return out.view(self.params.M_y, self.params.M_x)

    def time_kernels(self, reps=20):
        out = (ctypes.c_float * N_KERNELS)()
        self._check(self._L.deblur_time_kernels(self._h, reps, out))
        return dict(zip(KERNEL_NAMES, out[:]))

    def init_cnn(self, net):
        """Warm start from the network with per-tile fallback; returns the
        host array of per-tile flags (1: network start kept) and the number
        of tiles that fell back."""
        use = (ctypes.c_int32 * self.n_tiles)()
        nf = ctypes.c_int32()
        self._check(self._L.deblur_init_cnn(self._h, net._h, use, ctypes.byref(nf)))
        return np.array(use[:], dtype=np.int32), nf.value

    def warm_inputs(self):
        """Network inputs [n_tiles, N, N] (device) and per-tile scales (host)."""
        N = self.tiles[0].frame
        frames = self._torch.empty((self.n_tiles, N, N), dtype=self._torch.float32, device="cuda")
        sc = (ctypes.c_float * self.n_tiles)()
        self._check(self._L.deblur_warm_inputs(self._h, _ptr(frames), sc))
        return frames, np.array(sc[:], dtype=np.float64)

    def plan(self):
        pl = Plan()
        self._check(self._L.deblur_get_plan(self._h, ctypes.byref(pl)))
        return pl

    def set_plan(self, plan=None, **fields):
        """Replace the launch plan (a Plan, or fields changed from the current one)."""
        pl = self.plan() if plan is None else plan
        for k, v in fields.items():
            setattr(pl, k, v)
        self._check(self._L.deblur_set_plan(self._h, ctypes.byref(pl)))
        return pl

    # -- host-side layout helpers (no method arithmetic) ------------------------
    def pack_support(self, x_global):
        """Support-packed float32 host array from a host image on X."""
        r = self.r
        out = np.empty(self.support_total, dtype=np.float32)
        for d in self.tiles:
            sl = x_global[d.support_y0 + r:d.support_y0 + r + d.support_h,
                          d.support_x0 + r:d.support_x0 + r + d.support_w]
            out[d.x_offset:d.x_offset + d.support_h * d.support_w] = sl.ravel()
        return out

    def unpack_support(self, packed):
        """List of per-tile support arrays from a support-packed host array."""
        return [np.asarray(packed[d.x_offset:d.x_offset + d.support_h * d.support_w]).reshape(d.support_h, d.support_w)
                for d in self.tiles]

    def unpack_block(self, packed):
        return [np.asarray(packed[d.y_offset:d.y_offset + d.block_h * d.block_w]).reshape(d.block_h, d.block_w)
                for d in self.tiles]

    def pack_list_support(self, tiles):
        return np.concatenate([np.asarray(a, dtype=np.float32).ravel() for a in tiles])

    def pack_list_block(self, tiles):
        return np.concatenate([np.asarray(a, dtype=np.float32).ravel() for a in tiles])


def autotune(params: Params, psfs, n_inner=10, reps=3, stream=None):
    """Fastest launch plan for the problem and every plan measured (the
    library's autotuner, on scratch contexts it creates and frees)."""
    L = lib()
    psf = np.ascontiguousarray(np.asarray(psfs, dtype=np.float32))
    best = Plan()
    cap = 128
    trials = (Plan * cap)()
    n = ctypes.c_int32()
    rc = L.deblur_autotune(ctypes.byref(params), psf.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream),
                           n_inner, reps, ctypes.byref(best), trials, cap, ctypes.byref(n))
    if rc != 0:
        raise DeblurError(rc, L.deblur_last_error(None).decode())
    return best, [trials[i] for i in range(min(n.value, cap))]


def debug_fft(n, which, data, stream=None, out=None, noalloc=False):
    """Runs one FFT stage of the library on a CUDA float32 tensor (see deblur.h).
    noalloc=True calls deblur_debug_fft_noalloc, which takes its tables from
    the library's fixed device scratch and does not wait for the stream; out
    may then be a caller-owned tensor of the stage's output shape."""
    import torch
    L = lib()
    batch = data.shape[0]
    shape = (batch, n, n) if which == 3 else (batch, n // 2, n, 2)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device="cuda")
    elif tuple(out.shape) != shape:
        raise ValueError(f"out must have shape {shape}")
    fn = L.deblur_debug_fft_noalloc if noalloc else L.deblur_debug_fft
    rc = fn(n, batch, which, _ptr(data.contiguous()), _ptr(out), _stream_handle(stream))
    if rc != 0:
        raise DeblurError(rc, L.deblur_last_error(None).decode())
    return out


N_CNN_PARAMS = 19105


class Net:
    """The warm-start network on the GPU (weights, Adam state, buffers)."""

    def __init__(self, max_batch, max_h, max_w, params=None, seed=0, stream=None, inference_only=False):
        import torch
        self._torch = torch
        self._L = lib()
        h = ctypes.c_void_p()
        p = None
        if params is not None:
            p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
            if p.size != N_CNN_PARAMS:
                raise ValueError("expected 19105 parameters")
        create = self._L.deblur_cnn_create_inference if inference_only else self._L.deblur_cnn_create
        rc = create(p.ctypes.data_as(ctypes.c_void_p) if p is not None else None, seed,
                    max_batch, max_h, max_w, _stream_handle(stream), ctypes.byref(h))
        if rc != 0:
            raise DeblurError(rc, self._L.deblur_cnn_last_error(None).decode())
        self._h = h
        self.max_batch, self.max_h, self.max_w = max_batch, max_h, max_w

    def _check(self, rc):
        if rc != 0:
            raise DeblurError(rc, self._L.deblur_cnn_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.deblur_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(N_CNN_PARAMS, dtype=np.float32)
        self._check(self._L.deblur_cnn_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        self._check(self._L.deblur_cnn_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)))

    def forward(self, img, valid=None):
        B, H, W = img.shape
        out = self._torch.empty_like(img)
        v = None
        if valid is not None:
            v = np.ascontiguousarray(np.asarray(valid, dtype=np.int32))
        self._check(self._L.deblur_cnn_forward(self._h, _ptr(img), v.ctypes.data_as(ctypes.c_void_p) if v is not None
                                               else None, B, H, W, _ptr(out)))
        return out

    def loss_grad(self, img, target):
        B, H, W = img.shape
        loss = ctypes.c_double()
        g = np.empty(N_CNN_PARAMS, dtype=np.float32)
        self._check(self._L.deblur_cnn_loss_grad(self._h, _ptr(img), _ptr(target), B, H, W, ctypes.byref(loss),
                                                 g.ctypes.data_as(ctypes.c_void_p)))
        return loss.value, g

    def train_step(self, img, target, lr):
        B, H, W = img.shape
        loss = ctypes.c_double()
        self._check(self._L.deblur_cnn_train_step(self._h, _ptr(img), _ptr(target), B, H, W, lr, ctypes.byref(loss)))
        return loss.value

    def time_forward(self, img, reps=10):
        B, H, W = img.shape
        ms = (ctypes.c_float * 2)()
        self._check(self._L.deblur_cnn_time_forward(self._h, _ptr(img), B, H, W, reps, ms))
        return ms[0], ms[1]
