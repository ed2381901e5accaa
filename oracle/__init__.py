"""FP64 CPU oracle of the fast level set evolutions (arXiv 1409.7474).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
imports, links or calls it, and the two share no code.

The arithmetic lives in ``lse_oracle.c`` (plain C, double precision, direct 2-D
template convolution); this module only builds it with gcc when needed and
marshals numpy arrays through ctypes.  Every function cites the passage of the
paper it follows:

* ``template2d``      -- normalised Gaussian template (Table I step 4, Table III TS)
* ``conv2_same``      -- direct 2-D convolution, zero padding, same size (step 4)
* ``gradient``        -- first differences, one-sided at borders (appendix listing)
* ``region_means``    -- c+ / c- of eq. (15)
* ``region_term``     -- normalised region term of eq. (17)
* ``edge_map``        -- g(I) of eq. (14)
* ``step``            -- one iteration, Table I steps 2-4 with eq. (18)
* ``run``             -- Table I steps 1-6
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lse_oracle.c")
_LIB = os.path.join(_HERE, "liblse_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over rows).  Returns the .so path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i8p = ctypes.POINTER(ctypes.c_int8)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    c_int, c_double = ctypes.c_int, ctypes.c_double
    lib.lseo_template2d.argtypes = [c_double, c_int, dp]
    lib.lseo_conv2_same.argtypes = [dp, c_int, c_int, dp, c_int, dp]
    lib.lseo_gradient.argtypes = [dp, c_int, c_int, dp, dp]
    lib.lseo_grad_mag.argtypes = [dp, c_int, c_int, dp]
    lib.lseo_region_means.argtypes = [dp, c_int, c_int, c_int, dp, dp, dp, i64p]
    lib.lseo_region_term.argtypes = [dp, c_int, c_int, c_int, dp, dp, dp, dp]
    lib.lseo_edge_map.argtypes = [dp, c_int, c_int, c_int, c_double, c_int, c_double, dp]
    lib.lseo_step.argtypes = [dp, c_int, c_int, c_int, dp, c_int, c_int, c_int, c_double, dp,
                              c_int, dp, dp, dp, dp, i8p, dp]
    lib.lseo_run.argtypes = [dp, c_int, c_int, c_int, dp, c_int, c_int, c_int, c_double, dp,
                             c_int, u8p, c_int, c_int, dp, i8p, ip, i64p]
    lib.lseo_run.restype = c_int
    lib.lseo_num_threads.restype = c_int
    lib.lseo_set_threads.argtypes = [c_int]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _image3(img):
    """Accept H x W or H x W x B; return contiguous float64 H x W x B."""
    img = _f64(img)
    if img.ndim == 2:
        img = img[:, :, None]
    if img.ndim != 3 or not 1 <= img.shape[2] <= 4:
        raise ValueError("image must be H x W or H x W x B with 1 <= B <= 4")
    return np.ascontiguousarray(img)


def num_threads() -> int:
    return _load().lseo_num_threads()


def set_threads(n: int) -> None:
    _load().lseo_set_threads(int(n))


def template2d(sigma: float, ts: int) -> np.ndarray:
    """Normalised ts x ts Gaussian template (Table I step 4; Table III 'TS')."""
    if ts < 1 or ts % 2 == 0:
        raise ValueError("ts must be odd and positive")
    K = np.empty((ts, ts), np.float64)
    _load().lseo_template2d(float(sigma), int(ts), _dp(K))
    return K


def conv2_same(f: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Direct 2-D convolution of f with K, zero padding, same-size output."""
    f = _f64(f)
    K = _f64(K)
    out = np.empty_like(f)
    _load().lseo_conv2_same(_dp(f), f.shape[0], f.shape[1], _dp(K), K.shape[0], _dp(out))
    return out


def gradient(f: np.ndarray):
    """(fx, fy): central differences inside, one-sided at the border."""
    f = _f64(f)
    fx = np.empty_like(f)
    fy = np.empty_like(f)
    _load().lseo_gradient(_dp(f), f.shape[0], f.shape[1], _dp(fx), _dp(fy))
    return fx, fy


def grad_mag(f: np.ndarray) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    _load().lseo_grad_mag(_dp(f), f.shape[0], f.shape[1], _dp(out))
    return out


def region_means(img: np.ndarray, phi: np.ndarray):
    """(c_plus, c_minus, n_plus) of eq. (15): means over phi >= 0 / phi < 0."""
    img = _image3(img)
    phi = _f64(phi)
    h, w, nb = img.shape
    cp = np.zeros(4)
    cm = np.zeros(4)
    npl = ctypes.c_int64(0)
    _load().lseo_region_means(_dp(img), h, w, nb, _dp(phi), _dp(cp), _dp(cm), ctypes.byref(npl))
    return cp[:nb].copy(), cm[:nb].copy(), int(npl.value)


def region_term(img: np.ndarray, c_plus, c_minus):
    """(R, M): normalised region data term of eq. (17) and its normaliser."""
    img = _image3(img)
    h, w, nb = img.shape
    cp = np.zeros(4)
    cm = np.zeros(4)
    cp[:nb] = c_plus
    cm[:nb] = c_minus
    R = np.empty((h, w))
    M = ctypes.c_double(0.0)
    _load().lseo_region_term(_dp(img), h, w, nb, _dp(cp), _dp(cm), _dp(R), ctypes.byref(M))
    return R, float(M.value)


def edge_map(img: np.ndarray, sigma1: float = 1.0, ts1: int = 9, scale: float = 255.0) -> np.ndarray:
    """g(I) of eq. (14) on the band mean times `scale` (listing: 8-bit numbers)."""
    img = _image3(img)
    h, w, nb = img.shape
    g = np.empty((h, w))
    _load().lseo_edge_map(_dp(img), h, w, nb, float(sigma1), int(ts1), float(scale), _dp(g))
    return g


@dataclass
class StepResult:
    phi: np.ndarray          # LSF after the iteration
    u: np.ndarray            # phi + dt * R * |grad phi|
    psi: np.ndarray | None   # listing order: G * u
    b: np.ndarray            # int8 +1/-1 binary of this iteration
    c_plus: np.ndarray | None
    c_minus: np.ndarray | None
    M: float | None
    n_plus: int | None


def step(phi: np.ndarray, img: np.ndarray | None, *, term: str = "region", order: str = "table1",
         reinit: bool = True, dt: float = 15.0, sigma: float = 1.0, ts: int = 7,
         g: np.ndarray | None = None) -> StepResult:
    """One iteration of Table I (steps 2-4), update eq. (18).

    term: 'region' (eq. 17, needs img) or 'edge' (eq. 14, needs g).
    order: 'table1' (update, binarise, smooth) or 'listing' (update, smooth, binarise).
    """
    phi = _f64(phi)
    h, w = phi.shape
    t = 0 if term == "region" else 1
    o = 0 if order == "table1" else 1
    if t == 0:
        img3 = _image3(img)
        nb = img3.shape[2]
        gg = None
    else:
        img3 = None
        nb = 1
        gg = _f64(g)
    K = template2d(sigma, ts)
    phi_out = np.empty((h, w))
    u = np.empty((h, w))
    psi = np.empty((h, w)) if o == 1 else None
    b = np.empty((h, w), np.int8)
    stats = np.zeros(10)
    _load().lseo_step(_dp(img3), h, w, nb, _dp(gg), t, o, int(bool(reinit)), float(dt), _dp(K), ts,
                      _dp(phi), _dp(phi_out), _dp(u), _dp(psi),
                      b.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), _dp(stats))
    if t == 0:
        return StepResult(phi_out, u, psi, b, stats[:nb].copy(), stats[4:4 + nb].copy(),
                          float(stats[8]), int(stats[9]))
    return StepResult(phi_out, u, psi, b, None, None, None, None)


@dataclass
class RunResult:
    phi: np.ndarray
    b: np.ndarray
    iters_done: int
    flips: np.ndarray

    @property
    def mask(self) -> np.ndarray:
        return (self.b > 0).astype(np.uint8)


def run(img: np.ndarray | None, mask: np.ndarray, *, term: str = "region", order: str = "table1",
        reinit_every: int = 1, dt: float = 15.0, sigma: float = 1.0, ts: int = 7, iters: int = 100,
        stop_unchanged: bool = False, g: np.ndarray | None = None, sigma1: float = 1.0,
        ts1: int = 9, edge_scale: float = 255.0) -> RunResult:
    """Whole evolution, Table I steps 1-6.  For term='edge' the edge map is
    computed from img (eq. 14) unless g is given."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    h, w = mask.shape
    t = 0 if term == "region" else 1
    o = 0 if order == "table1" else 1
    if t == 0:
        img3 = _image3(img)
        nb = img3.shape[2]
        gg = None
    else:
        img3 = None
        nb = 1
        gg = _f64(g) if g is not None else edge_map(img, sigma1, ts1, edge_scale)
    K = template2d(sigma, ts)
    phi = np.empty((h, w))
    b = np.empty((h, w), np.int8)
    done = ctypes.c_int(0)
    flips = np.zeros(max(iters, 1), np.int64)
    _load().lseo_run(_dp(img3), h, w, nb, _dp(gg), t, o, int(reinit_every), float(dt), _dp(K), ts,
                     mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(iters),
                     int(bool(stop_unchanged)), _dp(phi),
                     b.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), ctypes.byref(done),
                     flips.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return RunResult(phi, b, int(done.value), flips[: int(done.value)].copy())
