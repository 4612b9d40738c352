"""Thin Python binding of libboxfmm.so (argument marshalling only).

Every step of the evaluation runs in the library's HIP kernels; torch is used
for device memory and streams.  Importing this module does not load the
library; the first call does, and raises if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BOXFMM_LIB names another build of the same library (side-by-side builds)
LIB_PATH = os.environ.get("BOXFMM_LIB") or os.path.join(HERE, "libboxfmm.so")

BX_OK = 0
BX_E_ARG, BX_E_NOT_BALANCED, BX_E_INVALID_TREE, BX_E_UNSUPPORTED, BX_E_HIP, BX_E_OOM, BX_E_NO_TABLES = (
    -1, -2, -3, -4, -5, -6, -7)
BX_FP64, BX_SPLIT_INT8, BX_HOST_ONLY = 0, 1, 0x100
Q = dict(n_leaves=0, n_boxes=1, n_levels=2, nodes=3, order=4, near_pairs=5, v_pairs=6, w_pairs=7,
         x_pairs=8, near_flops=9, far_flops=10, near_tiles=11, near_slots=12, upload_ms=13,
         split_products=14)
TABLES = dict(near=0, p2m=1, m2m=2, l2l=3, m2l_core=4, m2l_src_pow=5, m2l_tgt_pow=6, logd=7, l2t=8,
              m2t=9, p2l=10, weights=11, split_slices=12, split_row_scale=13,
              split_err=14)
PHASES = ["p2m", "m2m", "m2l", "p2l", "l2l", "leaf"]
SYMBOLS = ["bx_create", "bx_build_tables", "bx_tree_upload", "bx_volume_eval_grad", "bx_volume_eval",
           "bx_volume_grad", "bx_query", "bx_tree_list", "bx_table_copy", "bx_split_tolerance", "bx_profile",
           "bx_interpolate", "bx_tree_tuning", "bx_tree_tuning_get", "bx_autotune",
           "bx_profile_read", "bx_expansion_read", "bx_mlp_features", "bx_mlp_create", "bx_mlp_set_params", "bx_mlp_forward",
           "bx_mlp_grad", "bx_mlp_adam", "bx_mlp_read", "bx_mlp_destroy",
           "bx_tree_destroy", "bx_destroy", "bx_last_error"]

_lib = None


class BoxFMMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"boxfmm error {code}: {msg}")
        self.code = code


class _TreeDesc(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_double), ("cy", ctypes.c_double), ("width", ctypes.c_double),
                ("n_leaves", ctypes.c_int32), ("level", ctypes.c_void_p), ("ix", ctypes.c_void_p),
                ("iy", ctypes.c_void_p)]


def lib():
    """Load libboxfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1610_00823_amd.build_lib.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, i64, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double
        L.bx_create.argtypes = [ctypes.POINTER(vp), i32, i32, u32]
        L.bx_build_tables.argtypes = [vp, dp, ctypes.c_char_p]
        L.bx_tree_upload.argtypes = [vp, ctypes.POINTER(_TreeDesc), i32, ctypes.POINTER(vp), vp]
        L.bx_volume_eval_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.bx_volume_eval.argtypes = [vp, vp, vp, i32, vp, vp]
        L.bx_volume_grad.argtypes = [vp, vp, vp, i32, vp, vp]
        L.bx_query.argtypes = [vp, vp, i32, ctypes.POINTER(dp)]
        L.bx_tree_list.argtypes = [vp, i32, vp, i64, ctypes.POINTER(i64)]
        L.bx_table_copy.argtypes = [vp, i32, vp, i64, ctypes.POINTER(i64)]
        L.bx_interpolate.argtypes = [vp, vp, vp, vp, i32, vp, i64, vp, vp, vp]
        L.bx_split_tolerance.argtypes = [vp, dp]
        L.bx_tree_tuning.argtypes = [vp, vp, vp, vp]
        L.bx_expansion_read.argtypes = [vp, vp, i32, i64, i32, vp, vp]
        L.bx_tree_tuning_get.argtypes = [vp, vp]
        L.bx_autotune.argtypes = [vp, vp, vp, i32, vp, vp, i32, vp, vp]
        L.bx_profile.argtypes = [vp, i32]
        L.bx_profile_read.argtypes = [vp, ctypes.POINTER(dp), ctypes.POINTER(i32)]
        L.bx_mlp_features.argtypes = [vp, vp, i64, vp, vp]
        L.bx_mlp_create.argtypes = [ctypes.POINTER(vp), vp, vp]
        L.bx_mlp_set_params.argtypes = [vp, vp, vp]
        L.bx_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.bx_mlp_grad.argtypes = [vp, vp, vp, i64, vp]
        L.bx_mlp_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
        L.bx_mlp_read.argtypes = [vp, i32, vp, i64, vp]
        L.bx_mlp_destroy.argtypes = [vp]
        L.bx_tree_destroy.argtypes = [vp]
        L.bx_destroy.argtypes = [vp]
        L.bx_last_error.restype = ctypes.c_char_p
        for name in SYMBOLS:
            if name not in ("bx_tree_destroy", "bx_destroy", "bx_last_error"):
                getattr(L, name).restype = i32
        L.bx_tree_destroy.restype = None
        L.bx_destroy.restype = None
        L.bx_mlp_destroy.restype = None
        _lib = L
    return _lib


def _check(rc):
    if rc != BX_OK:
        raise BoxFMMError(rc, lib().bx_last_error().decode())


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Context:
    """bx_create + bx_build_tables."""

    def __init__(self, n: int = 8, p: int = 30, flags: int = BX_FP64, cache_dir=None, quad_tol: float = 0.0,
                 build: bool = True):
        self._h = ctypes.c_void_p()
        _check(lib().bx_create(ctypes.byref(self._h), int(n), int(p), int(flags)))
        self.n, self.p, self.flags = n, p, flags
        if build:
            self.build_tables(quad_tol, cache_dir)

    def build_tables(self, quad_tol=0.0, cache_dir=None):
        cd = cache_dir.encode() if cache_dir else None
        _check(lib().bx_build_tables(self._h, float(quad_tol), cd))

    def table(self, name: str) -> np.ndarray:
        cnt = ctypes.c_int64()
        _check(lib().bx_table_copy(self._h, TABLES[name], None, 0, ctypes.byref(cnt)))
        out = np.zeros(cnt.value)
        _check(lib().bx_table_copy(self._h, TABLES[name], out.ctypes.data, cnt.value, ctypes.byref(cnt)))
        return out

    def split_tolerance(self, tol: float):
        _check(lib().bx_split_tolerance(self._h, float(tol)))

    def profile(self, enable: bool = True):
        _check(lib().bx_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """{phase: total ms} and the number of timed evaluations since the last read."""
        ms = (ctypes.c_double * len(PHASES))()
        nev = ctypes.c_int()
        _check(lib().bx_profile_read(self._h, ms, ctypes.byref(nev)))
        return dict(zip(PHASES, list(ms))), nev.value

    def close(self):
        if self._h:
            lib().bx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """bx_tree_upload of one leaf set (level, ix, iy arrays) on a root box."""

    def __init__(self, ctx: Context, level, ix, iy, cx=0.0, cy=0.0, width=1.0, stream=None):
        self.ctx = ctx
        self._lv = np.ascontiguousarray(level, np.int8)
        self._ix = np.ascontiguousarray(ix, np.int32)
        self._iy = np.ascontiguousarray(iy, np.int32)
        d = _TreeDesc(float(cx), float(cy), float(width), int(self._lv.size), self._lv.ctypes.data,
                      self._ix.ctypes.data, self._iy.ctypes.data)
        self._h = ctypes.c_void_p()
        _check(lib().bx_tree_upload(ctx._h, ctypes.byref(d), 1, ctypes.byref(self._h), _stream_ptr(stream)))
        self.n_leaves = int(self._lv.size)

    @classmethod
    def from_inputs(cls, ctx, tree, stream=None):
        return cls(ctx, tree.level, tree.ix, tree.iy, tree.cx, tree.cy, tree.width, stream)

    @classmethod
    def forest(cls, ctx, trees, stream=None):
        """One bx_tree of several trees (objects with level, ix, iy, cx, cy, width):
        leaves numbered tree after tree; the trees must share the root width."""
        self = cls.__new__(cls)
        self.ctx = ctx
        self._keep = []
        descs = (_TreeDesc * len(trees))()
        for k, t in enumerate(trees):
            lv = np.ascontiguousarray(t.level, np.int8)
            ix = np.ascontiguousarray(t.ix, np.int32)
            iy = np.ascontiguousarray(t.iy, np.int32)
            self._keep += [lv, ix, iy]
            descs[k] = _TreeDesc(float(t.cx), float(t.cy), float(t.width), int(lv.size), lv.ctypes.data,
                                 ix.ctypes.data, iy.ctypes.data)
        self._h = ctypes.c_void_p()
        _check(lib().bx_tree_upload(ctx._h, descs, len(trees), ctypes.byref(self._h), _stream_ptr(stream)))
        self.n_leaves = int(sum(np.asarray(t.level).size for t in trees))
        return self

    def query(self, what: str) -> float:
        v = ctypes.c_double()
        _check(lib().bx_query(self.ctx._h, self._h, Q[what], ctypes.byref(v)))
        return v.value

    def phase_cost(self, phase: str):
        """(algorithmic flops, algorithmic bytes) of one evaluation phase for one RHS."""
        k = PHASES.index(phase)
        fl, by = ctypes.c_double(), ctypes.c_double()
        _check(lib().bx_query(self.ctx._h, self._h, 20 + k, ctypes.byref(fl)))
        _check(lib().bx_query(self.ctx._h, self._h, 40 + k, ctypes.byref(by)))
        return fl.value, by.value

    def tuning(self):
        """(heavy-tile threshold, FP64 slot weight, M2L blocks, two-level threshold) of this tree's schedule."""
        t = np.zeros(4)
        _check(lib().bx_tree_tuning_get(self._h, t.ctypes.data))
        return float(t[0]), float(t[1]), int(t[2]), int(t[3])

    def set_tuning(self, heavy=0.0, f64_weight=0.0, m2l_blocks=0, fuse=-1, stream=None):
        """Set scheduling parameters (0, or -1 for fuse, keeps one); results do not change."""
        t = np.array([heavy, f64_weight, m2l_blocks, fuse], np.float64)
        _check(lib().bx_tree_tuning(self.ctx._h, self._h, t.ctypes.data, _stream_ptr(stream)))

    def expansion(self, which: str = "multipole", box: int = 0, rhs: int = 0, stream=None) -> np.ndarray:
        """Complex coefficients (k = 0..p) of a box's multipole or local expansion
        from the last evaluation, unscaled, about the box centre."""
        out = np.zeros(2 * (self.ctx.p + 1))
        _check(lib().bx_expansion_read(self.ctx._h, self._h, 0 if which == "multipole" else 1, int(box), int(rhs),
                                       out.ctypes.data, _stream_ptr(stream)))
        return out[0::2] + 1j * out[1::2]

    def lists(self, kind: int) -> np.ndarray:
        cnt = ctypes.c_int64()
        _check(lib().bx_tree_list(self._h, int(kind), None, 0, ctypes.byref(cnt)))
        out = np.zeros((cnt.value, 3), np.int64)
        _check(lib().bx_tree_list(self._h, int(kind), out.ctypes.data, cnt.value, ctypes.byref(cnt)))
        return out

    def close(self):
        if self._h:
            lib().bx_tree_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_check(t, shape, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 tensor on the GPU")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def volume_eval_grad(ctx: Context, tree: Tree, f, V=None, G=None, stream=None):
    """V[n_rhs, N_L, n, n] and G[n_rhs, N_L, 2, n, n] for f[n_rhs, N_L, n, n] (torch, on the GPU)."""
    import torch
    if f.dim() == 3:
        f = f.unsqueeze(0)
    nrhs, n = f.shape[0], ctx.n
    _dev_check(f, (nrhs, tree.n_leaves, n, n), "f")
    if V is None:
        V = torch.empty_like(f)
    if G is None:
        G = torch.empty((nrhs, tree.n_leaves, 2, n, n), dtype=f.dtype, device=f.device)
    _dev_check(V, (nrhs, tree.n_leaves, n, n), "V")
    _dev_check(G, (nrhs, tree.n_leaves, 2, n, n), "G")
    if stream is None:
        stream = torch.cuda.current_stream(f.device)
    _check(lib().bx_volume_eval_grad(ctx._h, tree._h, ctypes.c_void_p(f.data_ptr()), int(nrhs),
                                     ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                     _stream_ptr(stream)))
    return V, G


def autotune(ctx: Context, tree: Tree, f, V=None, G=None, reps: int = 5, stream=None):
    """Time candidate schedules of tree for f [n_rhs, N_L, n, n] and keep the fastest;
    returns (V, G, (heavy, f64_weight, m2l_blocks, fuse, ms per evaluation))."""
    import torch
    if f.dim() == 3:
        f = f.unsqueeze(0)
    nrhs, n = f.shape[0], ctx.n
    _dev_check(f, (nrhs, tree.n_leaves, n, n), "f")
    V = torch.empty_like(f) if V is None else V
    G = torch.empty((nrhs, tree.n_leaves, 2, n, n), dtype=f.dtype, device=f.device) if G is None else G
    _dev_check(V, (nrhs, tree.n_leaves, n, n), "V")
    _dev_check(G, (nrhs, tree.n_leaves, 2, n, n), "G")
    if stream is None:
        stream = torch.cuda.current_stream(f.device)
    best = np.zeros(5)
    _check(lib().bx_autotune(ctx._h, tree._h, ctypes.c_void_p(f.data_ptr()), int(nrhs),
                             ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(G.data_ptr()), int(reps),
                             best.ctypes.data, _stream_ptr(stream)))
    return V, G, (float(best[0]), float(best[1]), int(best[2]), int(best[3]), float(best[4]))


def interpolate(ctx: Context, tree: Tree, xy, V=None, G=None, stream=None):
    """The per-leaf interpolants of V [n_rhs, N_L, n, n] and/or G [n_rhs, N_L, 2, n, n]
    at points xy [m, 2] (torch, on the GPU): (v [n_rhs, m] or None, g [n_rhs, m, 2] or None)."""
    import torch
    if V is None and G is None:
        raise ValueError("interpolate: give V or G")
    ref = V if V is not None else G
    nrhs, n, m = ref.shape[0], ctx.n, xy.shape[0]
    _dev_check(xy, (m, 2), "xy")
    if V is not None:
        _dev_check(V, (nrhs, tree.n_leaves, n, n), "V")
    if G is not None:
        _dev_check(G, (nrhs, tree.n_leaves, 2, n, n), "G")
    v = torch.empty((nrhs, m), dtype=torch.float64, device=xy.device) if V is not None else None
    g = torch.empty((nrhs, m, 2), dtype=torch.float64, device=xy.device) if G is not None else None
    if stream is None:
        stream = torch.cuda.current_stream(xy.device)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)
    _check(lib().bx_interpolate(ctx._h, tree._h, ptr(V), ptr(G), int(nrhs), ptr(xy), int(m), ptr(v), ptr(g),
                                _stream_ptr(stream)))
    return v, g


def volume_eval(ctx, tree, f, V=None, stream=None):
    import torch
    if f.dim() == 3:
        f = f.unsqueeze(0)
    _dev_check(f, (f.shape[0], tree.n_leaves, ctx.n, ctx.n), "f")
    V = torch.empty_like(f) if V is None else V
    _dev_check(V, tuple(f.shape), "V")
    stream = torch.cuda.current_stream(f.device) if stream is None else stream
    _check(lib().bx_volume_eval(ctx._h, tree._h, ctypes.c_void_p(f.data_ptr()), int(f.shape[0]),
                                ctypes.c_void_p(V.data_ptr()), _stream_ptr(stream)))
    return V


def volume_grad(ctx, tree, f, G=None, stream=None):
    import torch
    if f.dim() == 3:
        f = f.unsqueeze(0)
    nrhs, n = f.shape[0], ctx.n
    _dev_check(f, (nrhs, tree.n_leaves, n, n), "f")
    G = torch.empty((nrhs, tree.n_leaves, 2, n, n), dtype=f.dtype, device=f.device) if G is None else G
    _dev_check(G, (nrhs, tree.n_leaves, 2, n, n), "G")
    stream = torch.cuda.current_stream(f.device) if stream is None else stream
    _check(lib().bx_volume_grad(ctx._h, tree._h, ctypes.c_void_p(f.data_ptr()), int(nrhs),
                                ctypes.c_void_p(G.data_ptr()), _stream_ptr(stream)))
    return G


# ------------------------------------------------------------ refinement network
MLP_IN, MLP_NPARAMS = 288, 53633


def mlp_features(samples, level, stream=None):
    """Features [B, 288] (torch.bfloat16, on the GPU) of boxes with samples
    [B, 16, 16] (float64, GPU) on their 16 x 16 first-kind grids and levels [B] (int8, GPU)."""
    import torch
    B_ = samples.shape[0]
    if not (samples.is_cuda and samples.dtype == torch.float64 and samples.is_contiguous()
            and tuple(samples.shape[1:]) == (16, 16)):
        raise ValueError("samples must be a contiguous float64 [B, 16, 16] GPU tensor")
    if not (level.is_cuda and level.dtype == torch.int8 and level.shape == (B_,)):
        raise ValueError("level must be an int8 [B] GPU tensor")
    x = torch.empty((B_, MLP_IN), dtype=torch.bfloat16, device=samples.device)
    stream = torch.cuda.current_stream(samples.device) if stream is None else stream
    _check(lib().bx_mlp_features(ctypes.c_void_p(samples.data_ptr()), ctypes.c_void_p(level.data_ptr()), int(B_),
                                 ctypes.c_void_p(x.data_ptr()), _stream_ptr(stream)))
    return x


class RefineNet:
    """The refinement network on the GPU (BF16 products, FP32 parameters)."""

    def __init__(self, params=None, stream=None):
        self._h = ctypes.c_void_p()
        p = None if params is None else np.ascontiguousarray(params, np.float32)
        if p is not None and p.size != MLP_NPARAMS:
            raise ValueError(f"expected {MLP_NPARAMS} parameters")
        _check(lib().bx_mlp_create(ctypes.byref(self._h), None if p is None else p.ctypes.data, _stream_ptr(stream)))

    def set_params(self, params, stream=None):
        p = np.ascontiguousarray(params, np.float32)
        if p.size != MLP_NPARAMS:
            raise ValueError(f"expected {MLP_NPARAMS} parameters")
        _check(lib().bx_mlp_set_params(self._h, p.ctypes.data, _stream_ptr(stream)))

    def read(self, what: str = "params", stream=None) -> np.ndarray:
        k = ["params", "grad", "adam_m", "adam_v", "loss"].index(what)
        out = np.zeros(1 if k == 4 else MLP_NPARAMS, np.float32)
        _check(lib().bx_mlp_read(self._h, k, out.ctypes.data, out.size, _stream_ptr(stream)))
        return out

    @staticmethod
    def _x(x):
        import torch
        if not (x.is_cuda and x.dtype == torch.bfloat16 and x.is_contiguous() and x.dim() == 2
                and x.shape[1] == MLP_IN and x.data_ptr() % 16 == 0):
            raise ValueError("x must be a contiguous, 16-byte aligned bfloat16 [B, 288] GPU tensor")

    def forward(self, x, stream=None):
        """Logits [B] (float32, GPU) of features x [B, 288]."""
        import torch
        self._x(x)
        out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        stream = torch.cuda.current_stream(x.device) if stream is None else stream
        _check(lib().bx_mlp_forward(self._h, ctypes.c_void_p(x.data_ptr()), int(x.shape[0]),
                                    ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def grad(self, x, y, stream=None):
        """Gradient of the mean BCE against labels y [B] (float32, GPU), held in the network."""
        import torch
        self._x(x)
        if not (y.is_cuda and y.dtype == torch.float32 and y.is_contiguous() and y.shape == (x.shape[0],)):
            raise ValueError("y must be a contiguous float32 [B] GPU tensor")
        stream = torch.cuda.current_stream(x.device) if stream is None else stream
        _check(lib().bx_mlp_grad(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                 int(x.shape[0]), _stream_ptr(stream)))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        import torch
        stream = torch.cuda.current_stream() if stream is None else stream
        _check(lib().bx_mlp_adam(self._h, lr, beta1, beta2, eps, _stream_ptr(stream)))

    def close(self):
        if self._h:
            lib().bx_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
