"""ctypes binding of the C ABI in include/lse.h (argument marshalling only).

Every computation runs in the HIP library ``liblse.so``; this module only
loads it, converts arguments and raises on error codes.  PyTorch supplies the
device memory (the workspace and the I/O tensors) and the stream.  There is no
fallback: if the library is missing, ``load()`` raises.

Low-level functions carry the C names (``lse_init``, ``lse_step``, ...);
``LSE`` wraps one context.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblse.so")

LSE_OK = 0
LSE_ERR_INVALID_ARG = -1
LSE_ERR_BAD_VALUE = -2
LSE_ERR_WORKSPACE = -3
LSE_ERR_DEVICE = -4
LSE_ERR_STATE = -5
LSE_ERR_UNSUPPORTED = -6

TERMS = {"region": 0, "edge": 1, "region_intensity": 2}
ORDERS = {"table1": 0, "listing": 1}
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}

# Every function the header declares; tests check that the library exports them.
EXPORTS = (
    "lse_params_default", "lse_workspace_bytes", "lse_init", "lse_step", "lse_run", "lse_mask",
    "lse_lsf", "lse_set_mask", "lse_set_lsf", "lse_edge_map", "lse_stats", "lse_check", "lse_profile", "lse_profile_read",
    "lse_step_bytes_per_pixel", "lse_destroy", "lse_batch_bytes", "lse_batch_create", "lse_batch_update",
    "lse_batch_run", "lse_autotune", "lse_tuning_lookup", "lse_ctx_tuning", "lse_tuning_set", "lse_tuning_clear",
    "lse_batch_destroy", "lse_solve_static", "lse_status_str", "lse_version",
)

# Size of the library-owned workspace of lse_solve_static (per GPU).
STATIC_WORKSPACE_BYTES = 64 << 20


class lse_params(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("bands", ctypes.c_int32),
        ("term", ctypes.c_int32), ("order", ctypes.c_int32), ("image_dtype", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("dt", ctypes.c_float), ("sigma", ctypes.c_float),
        ("ksize", ctypes.c_int32), ("sigma_img", ctypes.c_float), ("ksize_img", ctypes.c_int32),
        ("edge_scale", ctypes.c_float), ("reinit_every", ctypes.c_int32),
    ]


class lse_stats_t(ctypes.Structure):
    _fields_ = [
        ("n_plus", ctypes.c_uint64), ("flips", ctypes.c_uint64), ("iters_done", ctypes.c_int32),
        ("converged", ctypes.c_int32), ("bad_value", ctypes.c_int32), ("lsf_overflow", ctypes.c_int32),
        ("c_plus", ctypes.c_float * 4), ("c_minus", ctypes.c_float * 4), ("M", ctypes.c_float),
        ("pad", ctypes.c_float * 3),
    ]


class lse_profile_t(ctypes.Structure):
    _fields_ = [
        ("step_ms", ctypes.c_double), ("mpass_ms", ctypes.c_double),
        ("step_launches", ctypes.c_int64), ("mpass_launches", ctypes.c_int64),
        ("needed_pixels", ctypes.c_int64), ("counted_steps", ctypes.c_int64),
        ("visited_tiles", ctypes.c_int64), ("heavy_tiles", ctypes.c_int64), ("tiles", ctypes.c_int64),
    ]


class lse_tuning_t(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32), ("tile_rows", ctypes.c_int32), ("tile_cols", ctypes.c_int32),
        ("waves_per_simd", ctypes.c_int32), ("size_class", ctypes.c_int32), ("candidates", ctypes.c_int32),
        ("ms", ctypes.c_float * 4),
    ]

    def as_dict(self) -> dict:
        return {"variant": self.variant, "tile_rows": self.tile_rows, "tile_cols": self.tile_cols,
                "waves_per_simd": self.waves_per_simd, "size_class": self.size_class,
                "candidates": self.candidates, "ms": [round(float(x), 4) for x in self.ms[:self.candidates]]}


PROFILE_TIMING = 1
PROFILE_COUNT = 2


def PROFILE_SAMPLE(k: int) -> int:
    """With PROFILE_TIMING: time one launch in 2**k of each kernel."""
    return (int(k) & 15) << 8
BATCH_GRAPH = 1


class LSEError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} ({status})")


_lib = None


def load() -> ctypes.CDLL:
    """Load liblse.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH} (build it with `python __graft_entry__.py`)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    P = ctypes.POINTER
    lib.lse_params_default.argtypes = [P(lse_params), i32, i32, i32]
    lib.lse_params_default.restype = None
    lib.lse_workspace_bytes.argtypes = [P(lse_params)]
    lib.lse_workspace_bytes.restype = ctypes.c_size_t
    lib.lse_init.argtypes = [P(lse_params), vp, vp, vp, ctypes.c_size_t, vp, P(vp)]
    lib.lse_init.restype = st
    lib.lse_step.argtypes = [vp, vp]
    lib.lse_step.restype = st
    lib.lse_run.argtypes = [vp, i32, i32, vp]
    lib.lse_run.restype = st
    lib.lse_mask.argtypes = [vp, vp, vp]
    lib.lse_mask.restype = st
    lib.lse_lsf.argtypes = [vp, vp, vp]
    lib.lse_lsf.restype = st
    lib.lse_set_mask.argtypes = [vp, vp, i32, i32, vp]
    lib.lse_set_mask.restype = st
    lib.lse_set_lsf.argtypes = [vp, vp, vp, i32, vp]
    lib.lse_set_lsf.restype = st
    lib.lse_edge_map.argtypes = [vp, vp, vp]
    lib.lse_edge_map.restype = st
    lib.lse_stats.argtypes = [vp, P(lse_stats_t), vp]
    lib.lse_stats.restype = st
    lib.lse_check.argtypes = [vp, vp]
    lib.lse_check.restype = st
    lib.lse_profile.argtypes = [vp, i32]
    lib.lse_profile.restype = st
    lib.lse_profile_read.argtypes = [vp, P(lse_profile_t)]
    lib.lse_profile_read.restype = st
    lib.lse_step_bytes_per_pixel.argtypes = [vp]
    lib.lse_step_bytes_per_pixel.restype = ctypes.c_double
    lib.lse_destroy.argtypes = [vp]
    lib.lse_destroy.restype = None
    lib.lse_batch_bytes.argtypes = [P(vp), i32]
    lib.lse_batch_bytes.restype = ctypes.c_size_t
    lib.lse_batch_create.argtypes = [P(vp), i32, P(i32), vp, ctypes.c_size_t, vp, P(vp)]
    lib.lse_batch_create.restype = st
    lib.lse_batch_update.argtypes = [vp, P(vp), i32, P(i32), vp, ctypes.c_size_t, vp]
    lib.lse_batch_update.restype = st
    lib.lse_batch_run.argtypes = [vp, i32, i32, i32, vp]
    lib.lse_batch_run.restype = st
    lib.lse_batch_destroy.argtypes = [vp]
    lib.lse_batch_destroy.restype = None
    lib.lse_solve_static.argtypes = [P(lse_params), vp, vp, i32, i32, vp, vp, vp]
    lib.lse_solve_static.restype = st
    lib.lse_autotune.argtypes = [P(lse_params), vp, vp, vp, ctypes.c_size_t, i32, vp, P(lse_tuning_t)]
    lib.lse_autotune.restype = st
    lib.lse_tuning_lookup.argtypes = [P(lse_params), P(lse_tuning_t)]
    lib.lse_tuning_lookup.restype = st
    lib.lse_ctx_tuning.argtypes = [vp, P(lse_tuning_t)]
    lib.lse_ctx_tuning.restype = st
    lib.lse_tuning_set.argtypes = [P(lse_params), i32]
    lib.lse_tuning_set.restype = st
    lib.lse_tuning_clear.argtypes = []
    lib.lse_tuning_clear.restype = None
    lib.lse_status_str.argtypes = [st]
    lib.lse_status_str.restype = ctypes.c_char_p
    lib.lse_version.argtypes = []
    lib.lse_version.restype = i32
    _lib = lib
    return lib


def status_str(status: int) -> str:
    return load().lse_status_str(int(status)).decode()


def _check(status: int, where: str) -> None:
    if status != LSE_OK:
        raise LSEError(status, where)


# ----------------------------------------------------------- C-named calls

def lse_params_default(height: int, width: int, bands: int) -> lse_params:
    p = lse_params()
    load().lse_params_default(ctypes.byref(p), int(height), int(width), int(bands))
    return p


def lse_workspace_bytes(p: lse_params) -> int:
    return int(load().lse_workspace_bytes(ctypes.byref(p)))


def lse_init(p: lse_params, image_ptr: int, mask_ptr: int, workspace_ptr: int, workspace_bytes: int,
             stream: int = 0) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(load().lse_init(ctypes.byref(p), image_ptr, mask_ptr, workspace_ptr, workspace_bytes, stream,
                           ctypes.byref(ctx)), "lse_init")
    return ctx


def lse_step(ctx, stream: int = 0) -> None:
    _check(load().lse_step(ctx, stream), "lse_step")


def lse_run(ctx, max_iters: int, stop_when_unchanged: bool = False, stream: int = 0) -> None:
    _check(load().lse_run(ctx, int(max_iters), int(bool(stop_when_unchanged)), stream), "lse_run")


def lse_mask(ctx, mask_ptr: int, stream: int = 0) -> None:
    _check(load().lse_mask(ctx, mask_ptr, stream), "lse_mask")


def lse_lsf(ctx, lsf_ptr: int, stream: int = 0) -> None:
    _check(load().lse_lsf(ctx, lsf_ptr, stream), "lse_lsf")


def lse_set_mask(ctx, mask_ptr: int, smoothed: bool, iteration: int = 0, stream: int = 0) -> None:
    _check(load().lse_set_mask(ctx, mask_ptr, int(bool(smoothed)), int(iteration), stream), "lse_set_mask")


def lse_set_lsf(ctx, lsf_ptr: int, mask_ptr, iteration: int = 0, stream: int = 0) -> None:
    _check(load().lse_set_lsf(ctx, lsf_ptr, mask_ptr, int(iteration), stream), "lse_set_lsf")


def lse_edge_map(ctx, g_ptr: int, stream: int = 0) -> None:
    _check(load().lse_edge_map(ctx, g_ptr, stream), "lse_edge_map")


def lse_stats(ctx, stream: int = 0) -> lse_stats_t:
    out = lse_stats_t()
    _check(load().lse_stats(ctx, ctypes.byref(out), stream), "lse_stats")
    return out


def lse_check(ctx, stream: int = 0) -> int:
    return int(load().lse_check(ctx, stream))


def lse_profile(ctx, flags: int) -> None:
    """flags: 0 off, PROFILE_TIMING (1), PROFILE_COUNT (2), or both; with
    PROFILE_TIMING, PROFILE_SAMPLE(k) times one launch in 2**k."""
    _check(load().lse_profile(ctx, int(flags)), "lse_profile")


def lse_profile_read(ctx) -> lse_profile_t:
    out = lse_profile_t()
    _check(load().lse_profile_read(ctx, ctypes.byref(out)), "lse_profile_read")
    return out


def lse_step_bytes_per_pixel(ctx) -> float:
    return float(load().lse_step_bytes_per_pixel(ctx))


def lse_destroy(ctx) -> None:
    load().lse_destroy(ctx)


def lse_version() -> int:
    return int(load().lse_version())


def _ctx_array(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))()
    for i, c in enumerate(ctxs):
        arr[i] = c.value if isinstance(c, ctypes.c_void_p) else c
    return arr


def lse_batch_bytes(ctxs) -> int:
    return int(load().lse_batch_bytes(_ctx_array(ctxs), len(ctxs)))


def lse_batch_create(ctxs, targets, table_ptr: int, table_bytes: int, stream: int = 0) -> ctypes.c_void_p:
    b = ctypes.c_void_p()
    tg = None
    if targets is not None:
        tg = (ctypes.c_int32 * len(ctxs))(*[int(t) for t in targets])
    _check(load().lse_batch_create(_ctx_array(ctxs), len(ctxs), tg, table_ptr, table_bytes, stream,
                                   ctypes.byref(b)), "lse_batch_create")
    return b


def lse_batch_update(batch, ctxs, targets, table_ptr: int, table_bytes: int, stream: int = 0) -> None:
    tg = None
    if targets is not None:
        tg = (ctypes.c_int32 * len(ctxs))(*[int(t) for t in targets])
    _check(load().lse_batch_update(batch, _ctx_array(ctxs), len(ctxs), tg, table_ptr, table_bytes, stream),
           "lse_batch_update")


def lse_batch_run(batch, iters: int, stop_when_unchanged: bool = False, flags: int = 0, stream: int = 0) -> None:
    _check(load().lse_batch_run(batch, int(iters), int(bool(stop_when_unchanged)), int(flags), stream),
           "lse_batch_run")


def lse_batch_destroy(batch) -> None:
    load().lse_batch_destroy(batch)


def lse_solve_static(p: lse_params, image_ptr: int, mask_ptr: int, max_iters: int, stop_when_unchanged: bool,
                     mask_out_ptr: int, lsf_out_ptr=None, stream: int = 0) -> None:
    """One whole solve in the library's own per-GPU workspace (no allocation)."""
    _check(load().lse_solve_static(ctypes.byref(p), image_ptr, mask_ptr, int(max_iters),
                                   int(bool(stop_when_unchanged)), mask_out_ptr, lsf_out_ptr, stream),
           "lse_solve_static")


def lse_autotune(p: lse_params, image_ptr: int, mask_ptr: int, workspace_ptr: int, workspace_bytes: int,
                 iters: int, stream: int = 0) -> lse_tuning_t:
    out = lse_tuning_t()
    _check(load().lse_autotune(ctypes.byref(p), image_ptr, mask_ptr, workspace_ptr, workspace_bytes, int(iters),
                               stream, ctypes.byref(out)), "lse_autotune")
    return out


def lse_tuning_lookup(p: lse_params) -> lse_tuning_t:
    out = lse_tuning_t()
    _check(load().lse_tuning_lookup(ctypes.byref(p), ctypes.byref(out)), "lse_tuning_lookup")
    return out


def lse_ctx_tuning(ctx) -> lse_tuning_t:
    out = lse_tuning_t()
    _check(load().lse_ctx_tuning(ctx, ctypes.byref(out)), "lse_ctx_tuning")
    return out


def lse_tuning_set(p: lse_params, variant: int) -> None:
    _check(load().lse_tuning_set(ctypes.byref(p), int(variant)), "lse_tuning_set")


def lse_tuning_clear() -> None:
    load().lse_tuning_clear()


# ------------------------------------------------------------ torch wrapper

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}
    if t.dtype not in m:
        raise TypeError(f"image dtype {t.dtype} not supported (float32, float16, bfloat16)")
    return m[t.dtype]


def make_params(height: int, width: int, bands: int, *, term: str = "region", order: str = "table1",
                dt: float = 15.0, sigma: float = 1.0, ksize: int = 0, sigma_img: float = 1.0,
                ksize_img: int = 9, edge_scale: float = 255.0, storage: str = "f32",
                image_dtype: str = "f32", reinit_every: int = 1) -> lse_params:
    p = lse_params_default(height, width, bands)
    p.term = TERMS[term]
    p.order = ORDERS[order]
    p.dt = dt
    p.sigma = sigma
    p.ksize = ksize
    p.sigma_img = sigma_img
    p.ksize_img = ksize_img
    p.edge_scale = edge_scale
    p.storage = DTYPES[storage]
    p.image_dtype = DTYPES[image_dtype]
    p.reinit_every = reinit_every
    return p


class LSE:
    """One evolution (one image) on the current CUDA/HIP device.

    image: H x W or H x W x B tensor on the GPU (float32 / float16 / bfloat16),
    init_mask: H x W uint8 tensor on the GPU (nonzero = inside the initial curve).
    The workspace is a torch uint8 tensor owned by this object.
    """

    def __init__(self, image, init_mask, *, term: str = "region", order: str = "table1", dt: float = 15.0,
                 sigma: float = 1.0, ksize: int = 0, sigma_img: float = 1.0, ksize_img: int = 9,
                 edge_scale: float = 255.0, storage: str = "f32", reinit_every: int = 1, stream=None):
        torch = _torch()
        if image.dim() == 2:
            image = image.unsqueeze(-1)
        if image.dim() != 3 or not image.is_cuda:
            raise ValueError("image must be an H x W [x B] GPU tensor")
        image = image.contiguous()
        init_mask = init_mask.to(torch.uint8).contiguous()
        h, w, b = image.shape
        if tuple(init_mask.shape) != (h, w) or not init_mask.is_cuda:
            raise ValueError("init_mask must be an H x W GPU tensor")
        self.device = image.device
        self.shape = (h, w, b)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = make_params(h, w, b, term=term, order=order, dt=dt, sigma=sigma, ksize=ksize,
                                  sigma_img=sigma_img, ksize_img=ksize_img, edge_scale=edge_scale,
                                  storage=storage, reinit_every=reinit_every)
        self.params.image_dtype = _dtype_code(image)
        nbytes = lse_workspace_bytes(self.params)
        if nbytes == 0:
            raise LSEError(LSE_ERR_INVALID_ARG, "lse_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self._ws_bytes = nbytes
        self._keep = (image, init_mask)
        self.ctx = lse_init(self.params, image.data_ptr(), init_mask.data_ptr(), self._ws_ptr, nbytes,
                            self._s())

    def _s(self) -> int:
        return int(self.stream.cuda_stream)

    def _handoff(self, out):
        # `out` is written on this job's stream; order the caller's current
        # stream after it so that torch work there sees the result.
        cur = _torch().cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)
        return out

    def step(self) -> None:
        lse_step(self.ctx, self._s())

    def run(self, iters: int, stop_when_unchanged: bool = False) -> None:
        lse_run(self.ctx, iters, stop_when_unchanged, self._s())

    def mask(self, out=None):
        torch = _torch()
        h, w, _ = self.shape
        out = out if out is not None else torch.empty((h, w), dtype=torch.uint8, device=self.device)
        lse_mask(self.ctx, out.data_ptr(), self._s())
        return self._handoff(out)

    def lsf(self, out=None):
        torch = _torch()
        h, w, _ = self.shape
        out = out if out is not None else torch.empty((h, w), dtype=torch.float32, device=self.device)
        lse_lsf(self.ctx, out.data_ptr(), self._s())
        return self._handoff(out)

    def set_mask(self, mask, smoothed: bool, iteration: int = 0) -> None:
        mask = mask.to(_torch().uint8).contiguous()
        self._keep_mask = mask
        lse_set_mask(self.ctx, mask.data_ptr(), smoothed, iteration, self._s())

    def set_lsf(self, lsf, mask=None, iteration: int = 0) -> None:
        """Continuous-LSF modes: load a checkpoint (lsf(), mask(), iters_done)."""
        torch = _torch()
        lsf = lsf.to(torch.float32).contiguous()
        h, w, _ = self.shape
        if tuple(lsf.shape) != (h, w) or not lsf.is_cuda:
            raise ValueError("lsf must be an H x W GPU tensor")
        mptr = None
        if mask is not None:
            mask = mask.to(torch.uint8).contiguous()
            if tuple(mask.shape) != (h, w) or not mask.is_cuda:
                raise ValueError("mask must be an H x W GPU tensor")
            mptr = mask.data_ptr()
        self._keep_state = (lsf, mask)
        lse_set_lsf(self.ctx, lsf.data_ptr(), mptr, iteration, self._s())

    def edge_map(self, out=None):
        """The edge map g of eq. (14) as stored (edge term only)."""
        torch = _torch()
        h, w, _ = self.shape
        out = out if out is not None else torch.empty((h, w), dtype=torch.float32, device=self.device)
        lse_edge_map(self.ctx, out.data_ptr(), self._s())
        return self._handoff(out)

    def stats(self) -> dict:
        s = lse_stats(self.ctx, self._s())
        nb = 1 if self.params.term == TERMS["region_intensity"] else self.shape[2]
        return {"n_plus": int(s.n_plus), "flips": int(s.flips), "iters_done": int(s.iters_done),
                "converged": bool(s.converged), "bad_value": bool(s.bad_value),
                "lsf_overflow": bool(s.lsf_overflow),
                "c_plus": list(s.c_plus)[:nb], "c_minus": list(s.c_minus)[:nb], "M": float(s.M)}

    def check(self) -> int:
        return lse_check(self.ctx, self._s())

    def profile(self, flags: int = PROFILE_TIMING) -> None:
        lse_profile(self.ctx, flags)

    def profile_read(self) -> dict:
        p = lse_profile_read(self.ctx)
        return {"step_ms": p.step_ms, "mpass_ms": p.mpass_ms, "step_launches": int(p.step_launches),
                "mpass_launches": int(p.mpass_launches), "needed_pixels": int(p.needed_pixels),
                "counted_steps": int(p.counted_steps), "visited_tiles": int(p.visited_tiles),
                "heavy_tiles": int(p.heavy_tiles), "tiles": int(p.tiles)}

    def step_bytes_per_pixel(self) -> float:
        return lse_step_bytes_per_pixel(self.ctx)

    def tuning(self) -> dict:
        """The step-kernel variant this job runs (lse_ctx_tuning)."""
        return lse_ctx_tuning(self.ctx).as_dict()

    def close(self) -> None:
        if getattr(self, "ctx", None):
            lse_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(image, init_mask, iters: int = 30, stream=None, **kw) -> dict:
    """lse_autotune on this job (image / init_mask as for LSE, keyword
    parameters as for make_params) with a temporary workspace; the choice is
    entered in the library's table for the job's family and size class."""
    torch = _torch()
    if image.dim() == 2:
        image = image.unsqueeze(-1)
    image = image.contiguous()
    init_mask = init_mask.to(torch.uint8).contiguous()
    h, w, b = image.shape
    p = make_params(h, w, b, **kw)
    p.image_dtype = _dtype_code(image)
    nbytes = lse_workspace_bytes(p)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=image.device)
    ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    s = stream if stream is not None else torch.cuda.current_stream(image.device)
    return lse_autotune(p, image.data_ptr(), init_mask.data_ptr(), ptr, nbytes, iters, int(s.cuda_stream)).as_dict()


class Batch:
    """Several LSE jobs advanced together (lse_batch_*).  The table memory is a
    torch uint8 tensor owned by this object; the jobs must outlive it."""

    def __init__(self, jobs, targets=None, stream=None):
        torch = _torch()
        if not jobs:
            raise ValueError("empty batch")
        self.jobs = list(jobs)
        self.device = self.jobs[0].device
        self.stream = stream if stream is not None else self.jobs[0].stream
        ctxs = [j.ctx for j in self.jobs]
        self.table, ptr, nbytes = self._table(ctxs)
        if nbytes == 0:
            self.batch = lse_batch_create(ctxs, targets, 0, 0, self._s())  # raises with the reason
        self.batch = lse_batch_create(ctxs, targets, ptr, nbytes, self._s())

    def _table(self, ctxs):
        nbytes = lse_batch_bytes(ctxs)
        table = _torch().empty(max(nbytes, 1) + 256, dtype=_torch().uint8, device=self.device)
        base = table.data_ptr()
        return table, base + (-base) % 256, nbytes

    @property
    def table_bytes(self) -> int:
        return int(self.table.numel())

    def update(self, jobs, targets=None):
        """Re-plan for a new member list (lse_batch_update) on a new table;
        returns the previous table tensor, which the caller keeps alive until
        the runs enqueued on it have completed."""
        jobs = list(jobs)
        ctxs = [j.ctx for j in jobs]
        table, ptr, nbytes = self._table(ctxs)
        if nbytes == 0:
            lse_batch_update(self.batch, ctxs, targets, 0, 0, self._s())  # raises with the reason
        lse_batch_update(self.batch, ctxs, targets, ptr, nbytes, self._s())
        old, self.table, self.jobs = self.table, table, jobs
        return old

    def _s(self) -> int:
        return int(self.stream.cuda_stream)

    def run(self, iters: int, stop_when_unchanged: bool = False, graph: bool = False) -> None:
        lse_batch_run(self.batch, iters, stop_when_unchanged, BATCH_GRAPH if graph else 0, self._s())

    def close(self) -> None:
        if getattr(self, "batch", None):
            lse_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
