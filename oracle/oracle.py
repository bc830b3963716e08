"""ctypes wrapper of the FP64 CPU oracle (msim_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the synthesis library itself.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "msim_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE double, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Traj(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_points", C.c_int32), ("t", C.POINTER(C.c_double)),
                ("p", C.POINTER(C.c_double)), ("center", C.c_double * 3), ("radius", C.c_double),
                ("speed", C.c_double), ("phase0", C.c_double)]


class _Scene(C.Structure):
    _fields_ = [("size", C.c_double * 3), ("beta", C.c_double * 6), ("src", _Traj), ("rcv", _Traj),
                ("n_mics", C.c_int32), ("mic_offset", C.POINTER(C.c_double)),
                ("n_in", C.c_int64), ("n_out", C.c_int64)]


class _Params(C.Structure):
    _fields_ = [("c", C.c_double), ("fs", C.c_double), ("max_order", C.c_int32), ("taps", C.c_int32),
                ("kaiser_beta", C.c_double), ("cutoff", C.c_double), ("n_tiers", C.c_int32),
                ("tier_max_order", C.c_int32 * 4), ("tier_decim", C.c_int32 * 4),
                ("delay_model", C.c_int32), ("tier_mode", C.c_int32), ("tier_tol", C.c_double),
                ("tier_rmax", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.orc_count_images.restype = C.c_int64
        L.orc_count_images.argtypes = [C.c_int32]
        L.orc_images.restype = C.c_int64
        L.orc_images.argtypes = [dp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp]
        L.orc_image_pos.restype = None
        L.orc_image_pos.argtypes = [dp, C.POINTER(C.c_int32), dp, dp]
        L.orc_i0.restype = C.c_double
        L.orc_i0.argtypes = [C.c_double]
        L.orc_kernel.restype = C.c_double
        L.orc_kernel.argtypes = [C.c_double, C.c_int32, C.c_double, C.c_double]
        L.orc_catmull_rom.restype = C.c_double
        L.orc_catmull_rom.argtypes = [dp, C.c_double]
        L.orc_traj_pos.restype = None
        L.orc_traj_pos.argtypes = [C.POINTER(_Traj), C.c_double, dp]
        L.orc_tau.restype = C.c_double
        L.orc_tau.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.POINTER(C.c_int32), C.c_int, C.c_double]
        for name in ("orc_forward",):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), dp, C.c_int64, C.POINTER(C.c_int64), dp]
        L.orc_adjoint_x.restype = C.c_int
        L.orc_adjoint_x.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), dp, dp]
        L.orc_grad_beta.restype = C.c_int
        L.orc_grad_beta.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), dp, dp, dp]
        L.orc_image_decim.restype = C.c_int32
        L.orc_image_decim.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.POINTER(C.c_int32)]
        L.orc_delays.restype = C.c_int
        L.orc_delays.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.c_int, C.c_int64,
                                 C.POINTER(C.c_int64), dp]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""

    def __init__(self):
        self.bufs = []

    def d(self, a) -> np.ndarray:
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        self.bufs.append(a)
        return a


def _traj(tr, keep: _Keep) -> _Traj:
    t = keep.d(tr.t)
    p = keep.d(tr.p).reshape(-1)
    s = _Traj()
    s.kind = int(tr.kind)
    s.n_points = int(t.shape[0])
    s.t = _dptr(t)
    s.p = _dptr(p)
    s.center = (C.c_double * 3)(*[float(v) for v in tr.center])
    s.radius = float(tr.radius)
    s.speed = float(tr.speed)
    s.phase0 = float(tr.phase0)
    return s


def _scene(sc, keep: _Keep) -> _Scene:
    s = _Scene()
    s.size = (C.c_double * 3)(*[float(v) for v in sc.size])
    s.beta = (C.c_double * 6)(*[float(v) for v in sc.beta])
    s.src = _traj(sc.src, keep)
    s.rcv = _traj(sc.rcv, keep)
    mo = keep.d(sc.mic_offset).reshape(-1)
    s.n_mics = int(sc.mic_offset.shape[0])
    s.mic_offset = _dptr(mo)
    s.n_in = int(sc.x.shape[0])
    s.n_out = int(sc.n_out)
    return s


def _params(par, max_order: int) -> _Params:
    p = _Params()
    p.c = float(par.c)
    p.fs = float(par.fs)
    p.max_order = int(max_order)
    p.taps = int(par.taps)
    p.kaiser_beta = float(par.kaiser_beta)
    p.cutoff = float(par.cutoff)
    tiers = list(par.tiers)
    p.n_tiers = len(tiers)
    mo = [0] * 4
    de = [1] * 4
    for k, (o, d) in enumerate(tiers):
        mo[k] = int(o)
        de[k] = int(d)
    p.tier_max_order = (C.c_int32 * 4)(*mo)
    p.tier_decim = (C.c_int32 * 4)(*de)
    p.delay_model = int(par.delay_model)
    p.tier_mode = int(getattr(par, "tier_mode", 0))
    p.tier_tol = float(getattr(par, "tier_tol", 1e-3))
    p.tier_rmax = int(getattr(par, "tier_rmax", 1024))
    return p


# ---------------------------------------------------------------- public API

def count_images(K: int) -> int:
    return int(lib().orc_count_images(K))


def images(beta, K: int):
    """(m[n,3], hits[n,6], beta_i[n]) of every image with |m|_1 <= K."""
    n = count_images(K)
    m = np.zeros((n, 3), np.int32)
    h = np.zeros((n, 6), np.int32)
    b = np.zeros(n, np.float64)
    bb = np.ascontiguousarray(np.asarray(beta, np.float64))
    lib().orc_images(_dptr(bb), K, m.ctypes.data_as(C.POINTER(C.c_int32)),
                     h.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(b))
    return m, h, b


def image_pos(size, m, q) -> np.ndarray:
    s = np.ascontiguousarray(np.asarray(size, np.float64))
    mm = np.ascontiguousarray(np.asarray(m, np.int32))
    qq = np.ascontiguousarray(np.asarray(q, np.float64))
    out = np.zeros(3)
    lib().orc_image_pos(_dptr(s), mm.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(qq), _dptr(out))
    return out


def i0(x: float) -> float:
    return float(lib().orc_i0(float(x)))


def kernel(u, T: int, kaiser_beta: float = 8.0, cutoff: float = 0.5) -> np.ndarray:
    u = np.atleast_1d(np.asarray(u, np.float64))
    return np.array([lib().orc_kernel(float(v), int(T), float(kaiser_beta), float(cutoff)) for v in u])


def catmull_rom(v4, u: float) -> float:
    a = np.ascontiguousarray(np.asarray(v4, np.float64))
    return float(lib().orc_catmull_rom(_dptr(a), float(u)))


def traj_pos(tr, t: float) -> np.ndarray:
    keep = _Keep()
    s = _traj(tr, keep)
    out = np.zeros(3)
    lib().orc_traj_pos(C.byref(s), float(t), _dptr(out))
    return out


def tau(sc, par, m, mic: int, t: float) -> float:
    keep = _Keep()
    s = _scene(sc, keep)
    p = _params(par, sc.max_order)
    mm = np.ascontiguousarray(np.asarray(m, np.int32))
    return float(lib().orc_tau(C.byref(s), C.byref(p), mm.ctypes.data_as(C.POINTER(C.c_int32)), int(mic), float(t)))


def forward(sc, par, x: Optional[np.ndarray] = None, idx: Optional[Sequence[int]] = None) -> np.ndarray:
    """FP64 output y[mic, n] (all n, or the listed output samples)."""
    keep = _Keep()
    s = _scene(sc, keep)
    p = _params(par, sc.max_order)
    xx = keep.d(sc.x if x is None else x)
    s.n_in = int(xx.shape[0])
    if idx is None:
        y = np.zeros((s.n_mics, sc.n_out))
        lib().orc_forward(C.byref(s), C.byref(p), _dptr(xx), 0, None, _dptr(y))
    else:
        ii = np.ascontiguousarray(np.asarray(idx, np.int64))
        y = np.zeros((s.n_mics, ii.shape[0]))
        lib().orc_forward(C.byref(s), C.byref(p), _dptr(xx), int(ii.shape[0]),
                          ii.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(y))
    return y


def adjoint_x(sc, par, gy: np.ndarray) -> np.ndarray:
    keep = _Keep()
    s = _scene(sc, keep)
    p = _params(par, sc.max_order)
    g = keep.d(gy).reshape(-1)
    gx = np.zeros(sc.x.shape[0])
    lib().orc_adjoint_x(C.byref(s), C.byref(p), _dptr(g), _dptr(gx))
    return gx


def grad_beta(sc, par, gy: np.ndarray, x: Optional[np.ndarray] = None) -> np.ndarray:
    keep = _Keep()
    s = _scene(sc, keep)
    p = _params(par, sc.max_order)
    xx = keep.d(sc.x if x is None else x)
    g = keep.d(gy).reshape(-1)
    gb = np.zeros(6)
    lib().orc_grad_beta(C.byref(s), C.byref(p), _dptr(xx), _dptr(g), _dptr(gb))
    return gb


def image_decim(sc, par, m) -> int:
    """The decimation the oracle's tier-emulating mode uses for image m (0: full rate)."""
    keep = _Keep()
    s = _scene(sc, keep)
    p = _params(par, sc.max_order)
    mm = np.ascontiguousarray(np.asarray(m, np.int32))
    return int(lib().orc_image_decim(C.byref(s), C.byref(p), mm.ctypes.data_as(C.POINTER(C.c_int32))))


def delays(sc, par, mic: int, idx: Sequence[int]) -> np.ndarray:
    """tau[i, k] of every image (oracle enumeration order) at output samples idx."""
    keep = _Keep()
    s = _scene(sc, keep)
    p = _params(par, sc.max_order)
    ii = np.ascontiguousarray(np.asarray(idx, np.int64))
    n = count_images(sc.max_order)
    out = np.zeros((n, ii.shape[0]))
    lib().orc_delays(C.byref(s), C.byref(p), int(mic), int(ii.shape[0]),
                     ii.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(out))
    return out


def loss_and_fd_src(sc, par, target: np.ndarray, knot: int, axis: int, h: float = 1e-6):
    """Central finite difference of L = 0.5 ||y - target||^2 with respect to one
    source knot coordinate, in FP64."""
    def L(scn):
        y = forward(scn, par)
        return 0.5 * float(np.sum((y - target) ** 2))
    sp = sc.copy()
    sm = sc.copy()
    sp.src.p[knot, axis] += h
    sm.src.p[knot, axis] -= h
    return (L(sp) - L(sm)) / (2 * h)
