"""Python binding of the msim library: a Plan over one or more scenes.

Argument marshalling only.  PyTorch supplies device memory and the current HIP
stream; every step of the synthesis runs in libmsim.so.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import MsimError, check


def _d(a, keep: list):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    keep.append(a)
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _traj(tr, keep) -> _lib.Traj:
    s = _lib.Traj()
    s.kind = int(tr.kind)
    s.n_points = int(np.asarray(tr.t).shape[0])
    s.t = _d(tr.t, keep)
    s.p = _d(np.asarray(tr.p).reshape(-1), keep)
    s.center = (C.c_double * 3)(*[float(v) for v in tr.center])
    s.radius = float(tr.radius)
    s.speed = float(tr.speed)
    s.phase0 = float(tr.phase0)
    return s


def _scene(sc, keep) -> _lib.Scene:
    s = _lib.Scene()
    s.size = (C.c_double * 3)(*[float(v) for v in sc.size])
    s.beta = (C.c_double * 6)(*[float(v) for v in sc.beta])
    s.src = _traj(sc.src, keep)
    s.rcv = _traj(sc.rcv, keep)
    s.n_mics = int(np.asarray(sc.mic_offset).shape[0])
    s.mic_offset = _d(np.asarray(sc.mic_offset).reshape(-1), keep)
    s.max_order = int(sc.max_order)
    s.n_in = int(sc.n_in)
    s.n_out = int(sc.n_out)
    return s


def params_struct(par, table_phases: int = 0) -> _lib.Params:
    p = _lib.Params()
    p.c = float(par.c)
    p.fs = float(par.fs)
    p.taps = int(par.taps)
    p.kaiser_beta = float(par.kaiser_beta)
    p.cutoff = float(par.cutoff)
    p.table_phases = int(table_phases)
    tiers = list(par.tiers)
    p.n_tiers = len(tiers)
    mo, de = [0] * 4, [1] * 4
    for k, (o, d) in enumerate(tiers):
        mo[k], de[k] = int(min(o, 2 ** 30)), int(d)
    p.tier_max_order = (C.c_int32 * 4)(*mo)
    p.tier_decim = (C.c_int32 * 4)(*de)
    p.delay_model = int(par.delay_model)
    p.fd_kind = int(getattr(par, "fd_kind", 0))
    p.farrow_order = int(getattr(par, "farrow_order", 9))
    p.knot_slack = float(getattr(par, "knot_slack", 0.0))
    p.tier_mode = int(getattr(par, "tier_mode", 0))
    p.tier_tol = float(getattr(par, "tier_tol", 1e-3))
    p.tier_rmax = int(getattr(par, "tier_rmax", 1024))
    p.adjx_mode = int(getattr(par, "adjx_mode", 0))
    return p


def count_images(max_order: int) -> int:
    n = C.c_int64()
    check(_lib.load().msim_count_images(int(max_order), C.byref(n)))
    return n.value


def suggest_n_out(sc, par) -> int:
    keep: list = []
    s = _scene(sc, keep)
    p = params_struct(par)
    n = C.c_int64()
    check(_lib.load().msim_suggest_n_out(C.byref(s), C.byref(p), C.byref(n)))
    return n.value


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> C.c_void_p:
    st = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(st.cuda_stream)


class Plan:
    """A validated, uploaded synthesis plan for a list of scenes."""

    def __init__(self, scenes: Sequence, par, table_phases: int = 0):
        L = _lib.load()
        self._keep: list = []
        arr = (_lib.Scene * len(scenes))()
        for i, sc in enumerate(scenes):
            arr[i] = _scene(sc, self._keep)
        self.params = params_struct(par, table_phases)
        self._ptr = C.c_void_p()
        check(L.msim_plan_create(arr, len(scenes), C.byref(self.params), C.byref(self._ptr)))
        self.n_scenes = len(scenes)
        n = self.n_scenes
        xo, yo = (C.c_int64 * n)(), (C.c_int64 * n)()
        xt, yt = C.c_int64(), C.c_int64()
        check(L.msim_plan_layout(self._ptr, xo, yo, C.byref(xt), C.byref(yt)))
        self.x_off = np.array(list(xo), np.int64)
        self.y_off = np.array(list(yo), np.int64)
        self.x_total, self.y_total = xt.value, yt.value
        ni = (C.c_int64 * n)()
        taps = C.c_double()
        check(L.msim_plan_stats(self._ptr, ni, C.byref(taps)))
        self.n_images = np.array(list(ni), np.int64)
        self.forward_taps = taps.value
        self.n_in = [int(sc.n_in) for sc in scenes]
        self.n_out = [int(sc.n_out) for sc in scenes]
        self.n_mics = [int(np.asarray(sc.mic_offset).shape[0]) for sc in scenes]
        so, st = (C.c_int64 * n)(), C.c_int64()
        check(L.msim_plan_grad_layout(self._ptr, so, C.byref(st)))
        self.src_off = np.array(list(so), np.int64)
        self.src_total = st.value
        self._ws = {}

    # -------------------------------------------------------------- memory
    def workspace_bytes(self, with_grad: bool = False) -> int:
        b = C.c_size_t()
        check(_lib.load().msim_workspace_size(self._ptr, int(with_grad), C.byref(b)))
        return b.value

    def workspace(self, with_grad: bool = False, device=None) -> torch.Tensor:
        key = bool(with_grad)
        nb = self.workspace_bytes(with_grad)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nb:
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=device or "cuda")
            self._ws[key] = ws
        return ws

    def pack_x(self, xs: Sequence, device="cuda") -> torch.Tensor:
        flat = np.concatenate([np.asarray(x, np.float32).reshape(-1) for x in xs])
        assert flat.shape[0] == self.x_total
        return torch.from_numpy(flat).to(device)

    def unpack_y(self, y: torch.Tensor) -> List[torch.Tensor]:
        return [y[o:o + m * n].view(m, n) for o, m, n in zip(self.y_off, self.n_mics, self.n_out)]

    # ------------------------------------------------------------- compute
    def forward(self, x: torch.Tensor, y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.numel() == self.x_total
        if y is None:
            y = torch.empty(self.y_total, dtype=torch.float32, device=x.device)
        assert y.is_cuda and y.dtype == torch.float32 and y.is_contiguous() and y.numel() == self.y_total
        ws = self.workspace(False, x.device)
        check(_lib.load().msim_forward(self._ptr, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                       C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
        return y

    def forward_noalloc(self, x: torch.Tensor, y: torch.Tensor, stream=None) -> torch.Tensor:
        """The forward with the library's fixed per-GPU scratch instead of a workspace
        (msim_forward_noalloc): nothing is allocated, y is written in place."""
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.numel() == self.x_total
        assert y.is_cuda and y.dtype == torch.float32 and y.is_contiguous() and y.numel() == self.y_total
        check(_lib.load().msim_forward_noalloc(self._ptr, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                               _stream_handle(stream)))
        return y

    def batched_workspace(self, device=None) -> torch.Tensor:
        b = C.c_size_t()
        check(_lib.load().msim_batched_workspace_size(self._ptr, C.byref(b)))
        ws = self._ws.get("batched")
        if ws is None or ws.numel() < b.value:
            ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=device or "cuda")
            self._ws["batched"] = ws
        return ws

    def forward_batched(self, x: torch.Tensor, y: Optional[torch.Tensor] = None, graph: bool = True,
                        stream=None) -> torch.Tensor:
        """All scenes in one persistent launch (captured in a HIP graph when graph=True)."""
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.numel() == self.x_total
        if y is None:
            y = torch.empty(self.y_total, dtype=torch.float32, device=x.device)
        assert y.is_cuda and y.dtype == torch.float32 and y.is_contiguous() and y.numel() == self.y_total
        ws = self.batched_workspace(x.device)
        check(_lib.load().msim_forward_batched(self._ptr, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                               C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream),
                                               int(graph)))
        return y

    def tuning(self) -> dict:
        t = _lib.Tuning()
        check(_lib.load().msim_get_tuning(self._ptr, C.byref(t)))
        return {k: getattr(t, k) for k, _ in _lib.Tuning._fields_}

    def update(self, beta=None, knots=None, stream=None):
        """Replace the walls' coefficients (beta [n_scenes, 6]) and the PWL source knot
        positions (knots [src_total, 3], the gradient layout) in place (msim_plan_update)."""
        b = None if beta is None else np.ascontiguousarray(np.asarray(beta, np.float64).reshape(self.n_scenes, 6))
        k = None if knots is None else np.ascontiguousarray(np.asarray(knots, np.float64).reshape(-1, 3))
        if k is not None and k.shape[0] != self.src_total:
            raise ValueError("knots must hold src_total = %d rows" % self.src_total)
        ptr = lambda a: C.c_void_p(a.ctypes.data) if a is not None else None
        check(_lib.load().msim_plan_update(self._ptr, ptr(b), ptr(k), _stream_handle(stream)))

    def images(self, scene: int) -> np.ndarray:
        """[n_img, 4] int32: (mx, my, mz, decimation R) of the scene's images (plan order)."""
        n = C.c_int64()
        check(_lib.load().msim_get_images(self._ptr, int(scene), None, 0, C.byref(n)))
        out = np.zeros((n.value, 4), np.int32)
        check(_lib.load().msim_get_images(self._ptr, int(scene), C.c_void_p(out.ctypes.data), n.value, C.byref(n)))
        return out

    def fd_error(self) -> dict:
        """Predicted relative errors of the fractional-delay approximations and the budget."""
        e = _lib.FdError()
        check(_lib.load().msim_get_fd_error(self._ptr, C.byref(e)))
        return {k: getattr(e, k) for k, _ in _lib.FdError._fields_}

    def set_tuning(self, threads: int, group_cap: int = 0, outputs_per_lane: int = 0):
        t = _lib.Tuning(threads, group_cap, outputs_per_lane, 0, 0.0, 0)
        check(_lib.load().msim_set_tuning(self._ptr, C.byref(t)))

    def autotune(self, x: torch.Tensor, cache_path: Optional[str] = None, stream=None) -> dict:
        """Chooses the launch shape of the batched forward by timing it (see msim_autotune)."""
        b = C.c_size_t()
        check(_lib.load().msim_autotune_workspace_size(self._ptr, C.byref(b)))
        ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=x.device)
        y = torch.empty(self.y_total, dtype=torch.float32, device=x.device)
        t = _lib.Tuning()
        check(_lib.load().msim_autotune(self._ptr, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                        C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream),
                                        cache_path.encode() if cache_path else None, C.byref(t)))
        del ws
        self._ws.clear()
        return {k: getattr(t, k) for k, _ in _lib.Tuning._fields_}

    def backward(self, x: torch.Tensor, gy: torch.Tensor, want_x: bool = True, want_beta: bool = True,
                 want_src: bool = True, stream=None, batched: bool = False, graph: bool = True, out=None):
        """(dL/dx [x_total] f32, dL/dbeta [n_scenes, 6] f64, dL/dknots [src_total, 3] f64) for
        gy = dL/dy; entries not requested are None.  batched=True runs every scene in one
        persistent launch per kernel (replayed from a HIP graph when graph=True; a graph
        is kept per set of buffers, so a loop passes the same `out`, as from a first call's
        return, to replay it)."""
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.numel() == self.x_total
        assert gy.is_cuda and gy.dtype == torch.float32 and gy.is_contiguous() and gy.numel() == self.y_total
        dev = x.device
        if out is not None:
            gx, gb, gs = out
            if gs is not None and gs.shape[0] != max(self.src_total, 1):
                raise ValueError("out[2] must be the full [max(src_total, 1), 3] buffer")
        else:
            gx = torch.empty(self.x_total, dtype=torch.float32, device=dev) if want_x else None
            gb = torch.empty((self.n_scenes, 6), dtype=torch.float64, device=dev) if want_beta else None
            gs = (torch.zeros((max(self.src_total, 1), 3), dtype=torch.float64, device=dev)
                  if want_src else None)
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        if batched:
            ws = self.batched_workspace(dev)
            check(_lib.load().msim_backward_batched(self._ptr, ptr(x), ptr(gy), ptr(gx), ptr(gb), ptr(gs),
                                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream),
                                                    int(graph)))
        else:
            ws = self.workspace(True, dev)
            check(_lib.load().msim_backward(self._ptr, ptr(x), ptr(gy), ptr(gx), ptr(gb), ptr(gs),
                                            C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
        self.last_backward_buffers = (gx, gb, gs)
        if gs is not None:
            gs = gs[: self.src_total]
        return gx, gb, gs

    def device_status(self, stream=None) -> int:
        f = C.c_int32()
        st = _lib.load().msim_device_status(self._ptr, _stream_handle(stream), C.byref(f))
        if st not in (0, 8):
            check(st)
        return f.value

    def profile_begin(self):
        check(_lib.load().msim_profile_begin(self._ptr))

    def profile_end(self) -> dict:
        pr = _lib.Profile()
        check(_lib.load().msim_profile_end(self._ptr, C.byref(pr)))
        return {k: getattr(pr, k) for k, _ in _lib.Profile._fields_}

    def close(self):
        if getattr(self, "_ptr", None) is not None and self._ptr.value:
            _lib.load().msim_plan_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
