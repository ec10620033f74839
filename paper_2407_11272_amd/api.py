"""Thin torch-facing binding of the C ABI: argument marshalling only.

Each ``wn_*`` function here has the name and meaning of the C entry point in
``include/wn.h``; every step of the computation runs in the HIP library.  PyTorch
provides device memory (tensors, workspaces) and the current HIP stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

_OCC_MODES = {None: L.WN_OCC_NONE, "none": L.WN_OCC_NONE, "threshold": L.WN_OCC_THRESHOLD,
              "sigmoid": L.WN_OCC_SIGMOID}


@dataclass(frozen=True)
class Grid:
    """Voxel grid: ``n[d]`` cells spanning ``[lo[d], hi[d]]`` (centres at idx + 1/2)."""

    lo: tuple = (-0.5, -0.5, -0.5)
    hi: tuple = (0.5, 0.5, 0.5)
    n: tuple = (32, 32, 32)

    @staticmethod
    def cube(res: int, lo: float = -0.5, hi: float = 0.5) -> "Grid":
        return Grid((lo, lo, lo), (hi, hi, hi), (res, res, res))

    @staticmethod
    def of(g) -> "Grid":
        return g if isinstance(g, Grid) else Grid(tuple(g.lo), tuple(g.hi), tuple(g.n))

    @property
    def size(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def to_c(self) -> L.WnGrid:
        g = L.WnGrid()
        for d in range(3):
            g.lo[d] = float(self.lo[d])
            g.hi[d] = float(self.hi[d])
            g.n[d] = int(self.n[d])
        return g


def _stream_handle(device: torch.device | None = None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Workspace:
    """Grow-only device workspace per (device, stream), 256-byte aligned.

    Calls on one stream run in order, so they may share its workspace."""

    _cache: dict = {}

    @classmethod
    def get(cls, nbytes: int, device: torch.device) -> tuple[ctypes.c_void_p, int]:
        key = (device.index, torch.cuda.current_stream(device).cuda_stream)
        buf = cls._cache.get(key)
        if buf is None or buf.numel() < nbytes + 256:
            if buf is not None:   # the old buffer goes: release what the library keeps for it
                torch.cuda.current_stream(device).synchronize()
                old = buf.data_ptr()
                L.check("wn_release_workspace", L.load().wn_release_workspace(ctypes.c_void_p(old + (-old) % 256)))
            cap = max(nbytes + 256, 1 << 20, 0 if buf is None else int(buf.numel() * 1.5))
            buf = torch.zeros(cap, dtype=torch.uint8, device=device)
            cls._cache[key] = buf
        base = buf.data_ptr()
        off = (-base) % 256
        return ctypes.c_void_p(base + off), int(buf.numel() - off)

    @classmethod
    def clear(cls):
        lib = L.load()
        for (dev, _), buf in cls._cache.items():
            torch.cuda.synchronize(dev)
            base = buf.data_ptr()
            L.check("wn_release_workspace", lib.wn_release_workspace(ctypes.c_void_p(base + (-base) % 256)))
        cls._cache.clear()


def _check_mesh(V: torch.Tensor, F: torch.Tensor):
    if not V.is_cuda or not F.is_cuda:
        raise ValueError("V and F must be device tensors (there is no CPU path)")
    if V.dtype != torch.float32 or V.dim() != 2 or V.shape[1] != 3 or not V.is_contiguous():
        raise ValueError("V must be a contiguous float32 [nV, 3] tensor")
    if F.dtype != torch.int32 or F.dim() != 2 or F.shape[1] != 3 or not F.is_contiguous():
        raise ValueError("F must be a contiguous int32 [nF, 3] tensor")


def as_mesh(V: torch.Tensor, F: torch.Tensor, device=None):
    """Cast a mesh to the library's layout (float32 vertices, int32 faces, contiguous)."""
    V, F = torch.as_tensor(V), torch.as_tensor(F)
    device = torch.device(device) if device is not None else (V.device if V.is_cuda else torch.device("cuda"))
    V = V.to(device=device, dtype=torch.float32).contiguous()
    F = F.to(device=device, dtype=torch.int32).contiguous()
    return V, F


# ------------------------------------------------------------ C-ABI mirrors

def wn_workspace_size(op: int, nV: int, nF: int, nQ: int) -> int:
    return int(L.load().wn_workspace_size(op, nV, nF, nQ))


def wn_voxelize(V, F, grid: Grid | None = None, Q: torch.Tensor | None = None, W: torch.Tensor | None = None,
                occupancy: str | None = None, tau: float = 0.5, k: float = 50.0, occ: torch.Tensor | None = None,
                _entry: str = "wn_voxelize"):
    """Winding number at the voxel centres of ``grid`` (or at the rows of ``Q``),
    plus the occupancy map when ``occupancy`` is 'threshold' or 'sigmoid'.
    Returns ``W`` or ``(W, occ)``; outputs may be passed in to avoid allocation."""
    lib = L.load()
    _check_mesh(V, F)
    if (grid is None) == (Q is None):
        raise ValueError("pass exactly one of grid or Q")
    dev = V.device
    if grid is not None:
        grid = Grid.of(grid)
        P, nQ, gptr, qptr = grid.size, 0, ctypes.byref(grid.to_c()), ctypes.c_void_p(0)
        shape = tuple(int(x) for x in grid.n)
    else:
        if Q.dtype != torch.float32 or Q.dim() != 2 or Q.shape[1] != 3 or not Q.is_contiguous() or not Q.is_cuda:
            raise ValueError("Q must be a contiguous float32 [nQ, 3] device tensor")
        P = nQ = Q.shape[0]
        gptr, qptr = None, _ptr(Q)
        shape = (P,)
    mode = _OCC_MODES[occupancy]
    if W is None:
        W = torch.empty(shape, dtype=torch.float32, device=dev)
    if mode != L.WN_OCC_NONE and occ is None:
        occ = torch.empty(shape, dtype=torch.uint8 if mode == L.WN_OCC_THRESHOLD else torch.float32, device=dev)
    need = wn_workspace_size(L.WN_OP_VOXELIZE, V.shape[0], F.shape[0], P)
    ws, wsb = Workspace.get(need, dev)
    st = getattr(lib, _entry)(_ptr(V), V.shape[0], _ptr(F), F.shape[0], gptr, qptr, nQ, _ptr(W), mode, tau, k,
                              _ptr(occ if mode != L.WN_OCC_NONE else None), ws, wsb, _stream_handle(dev))
    L.check(_entry, st)
    return W if mode == L.WN_OCC_NONE else (W, occ)


def wn_build_strips(F, nV: int | None = None):
    """Triangle-strip record stream of host faces F ([nF, 3]) as an int32 numpy array
    [n_records, 2] of (vertex id, face id or -1).  Depends only on F."""
    import numpy as np
    lib = L.load()
    Fh = np.ascontiguousarray(torch.as_tensor(F).cpu().numpy(), dtype=np.int32).reshape(-1, 3)
    nV = int(Fh.max()) + 1 if nV is None and len(Fh) else int(nV or 0)
    n = ctypes.c_int64(0)
    out = np.empty((3 * len(Fh), 2), dtype=np.int32)   # at most 3 records per face: one call
    L.check("wn_build_strips", lib.wn_build_strips(Fh.ctypes.data, len(Fh), nV, out.ctypes.data, len(out),
                                                   ctypes.byref(n)))
    return out[:n.value].copy()


def wn_build_face_pairs(F, nV: int | None = None):
    """Pairs of host faces F ([nF, 3]) that share an edge, for the adjoint's two-faces-per-
    lane kernel: an int32 numpy array [n, 2] of (f, g or -1), every face once.  Depends
    only on F."""
    import numpy as np
    lib = L.load()
    Fh = np.ascontiguousarray(torch.as_tensor(F).cpu().numpy(), dtype=np.int32).reshape(-1, 3)
    nV = int(Fh.max()) + 1 if nV is None and len(Fh) else int(nV or 0)
    n = ctypes.c_int64(0)
    out = np.empty((max(1, len(Fh)), 2), dtype=np.int32)   # at most one entry per face: one call
    L.check("wn_build_face_pairs", lib.wn_build_face_pairs(Fh.ctypes.data, len(Fh), nV, out.ctypes.data, len(out),
                                                           ctypes.byref(n)))
    return out[:n.value].copy()


def _check_pairs(pairs, F):
    if pairs is None:
        return None
    if pairs.dtype != torch.int32 or pairs.dim() != 2 or pairs.shape[1] != 2 or not pairs.is_cuda \
            or not pairs.is_contiguous():
        raise ValueError("pairs must be a contiguous int32 [n, 2] device tensor (wn_build_face_pairs)")
    return pairs


def wn_voxelize_strips(V, F, strips: torch.Tensor, grid: Grid | None = None, Q: torch.Tensor | None = None,
                       W: torch.Tensor | None = None, occupancy: str | None = None, tau: float = 0.5,
                       k: float = 50.0, occ: torch.Tensor | None = None):
    """wn_voxelize with a device strip stream from :func:`wn_build_strips`."""
    lib = L.load()
    _check_mesh(V, F)
    if strips.dtype != torch.int32 or strips.dim() != 2 or strips.shape[1] != 2 or not strips.is_cuda \
            or not strips.is_contiguous():
        raise ValueError("strips must be a contiguous int32 [n, 2] device tensor")
    if (grid is None) == (Q is None):
        raise ValueError("pass exactly one of grid or Q")
    dev = V.device
    if grid is not None:
        grid = Grid.of(grid)
        P, nQ, gptr, qptr = grid.size, 0, ctypes.byref(grid.to_c()), ctypes.c_void_p(0)
        shape = tuple(int(x) for x in grid.n)
    else:
        P = nQ = Q.shape[0]
        gptr, qptr = None, _ptr(Q)
        shape = (P,)
    mode = _OCC_MODES[occupancy]
    if W is None:
        W = torch.empty(shape, dtype=torch.float32, device=dev)
    if mode != L.WN_OCC_NONE and occ is None:
        occ = torch.empty(shape, dtype=torch.uint8 if mode == L.WN_OCC_THRESHOLD else torch.float32, device=dev)
    need = wn_workspace_size(L.WN_OP_VOXELIZE, V.shape[0], max(F.shape[0], (strips.shape[0] + 2) // 3), P)
    ws, wsb = Workspace.get(need, dev)
    st = lib.wn_voxelize_strips(_ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(strips), strips.shape[0], gptr,
                                qptr, nQ, _ptr(W), mode, tau, k, _ptr(occ if mode != L.WN_OCC_NONE else None), ws,
                                wsb, _stream_handle(dev))
    L.check("wn_voxelize_strips", st)
    return W if mode == L.WN_OCC_NONE else (W, occ)


def wn_voxelize_naive(V, F, grid: Grid | None = None, Q: torch.Tensor | None = None, **kw):
    """The naive flux sum of Eq. 4 (centroid samples); arguments as :func:`wn_voxelize`."""
    return wn_voxelize(V, F, grid=grid, Q=Q, _entry="wn_voxelize_naive", **kw)


class SlicedBackward:
    """The adjoint of one (mesh, grid or point list) computed over consecutive point
    ranges in separate calls (``wn_backward_range``): :meth:`begin`, then :meth:`points`
    for ranges of whole 256-point tiles in increasing order that together cover every
    point once, then :meth:`end`.  The result has the same bits as :func:`wn_backward`
    with the same ``pairs`` and ``vertex_sums``.  ``vertex_sums`` (with pairs): the two
    faces of a pair share their running sums at their common vertices, which is faster
    and gives dL/dV only (``end`` then refuses dL/dT).  The object owns its workspace,
    which holds the splits' running sums between calls; all calls go to the current
    stream of V's device."""

    def __init__(self, V, F, grid: Grid | None = None, Q: torch.Tensor | None = None,
                 pairs: torch.Tensor | None = None, vertex_sums: bool = False):
        _check_mesh(V, F)
        self.pairs = _check_pairs(pairs, F)
        self._np = 0 if pairs is None else int(pairs.shape[0])
        self._mode = L.WN_BWD_VERTEX_SUMS if vertex_sums else 0
        if (grid is None) == (Q is None):
            raise ValueError("pass exactly one of grid or Q")
        self.lib = L.load()
        self.V, self.F, self.dev = V, F, V.device
        if grid is not None:
            self.grid = Grid.of(grid)
            self._gc = self.grid.to_c()
            self.P, self._nQ, self._qptr = self.grid.size, 0, ctypes.c_void_p(0)
        else:
            self.grid, self._gc = None, None
            self.P = self._nQ = Q.shape[0]
            self._Q = Q
            self._qptr = _ptr(Q)
        self.tile = L.WN_BWD_TILE
        self.splits = int(self.lib.wn_backward_splits(F.shape[0], self.P))
        if self.splits < 1:
            raise ValueError("sizes out of range for the adjoint")
        need = wn_workspace_size(L.WN_OP_BACKWARD, V.shape[0], F.shape[0], self.P)
        if need == 0:
            raise ValueError("sizes out of range for the adjoint")
        self._buf = torch.empty(need + 256, dtype=torch.uint8, device=self.dev)
        base = self._buf.data_ptr()
        self._ws, self._wsb = ctypes.c_void_p(base + (-base) % 256), need
        self._next = 0

    @property
    def workspace_bytes(self) -> int:
        return self._wsb

    def _call(self, dLdW, p0, n, flags, dLdV=None, dLdT=None):
        g = ctypes.byref(self._gc) if self._gc is not None else None
        st = self.lib.wn_backward_range(_ptr(self.V), self.V.shape[0], _ptr(self.F), self.F.shape[0],
                                        _ptr(self.pairs), self._np, g, self._qptr, self._nQ, _ptr(dLdW), int(p0),
                                        int(n), flags | self._mode, _ptr(dLdV), _ptr(dLdT), self._ws, self._wsb,
                                        _stream_handle(self.dev))
        L.check("wn_backward_range", st)

    def begin(self):
        self._next = 0
        self._call(None, 0, 0, L.WN_BWD_BEGIN)

    def points(self, p0: int, n: int, dLdW: torch.Tensor):
        """Add points [p0, p0 + n): the next range after the previous one (p0 and n whole
        tiles, or the range reaching the last point); dLdW is indexed by the global point
        number."""
        if dLdW.dtype != torch.float32 or not dLdW.is_contiguous() or dLdW.numel() != self.P or not dLdW.is_cuda:
            raise ValueError("dLdW must be a contiguous float32 device tensor with one entry per point")
        if int(p0) != self._next:
            raise ValueError(f"ranges must be consecutive: expected p0 = {self._next}, got {p0}")
        self._call(dLdW, p0, n, 0)
        self._next = int(p0) + int(n)

    def device_error(self) -> int:
        """The device error record of this adjoint's workspace (synchronises)."""
        return int(self.lib.wn_get_device_error(self._ws, _stream_handle(self.dev)))

    def end(self, dLdV: torch.Tensor | None = None, dLdT: torch.Tensor | None = None) -> torch.Tensor:
        if self._next != self.P:
            raise ValueError(f"the ranges covered {self._next} of {self.P} points")
        if self._mode and dLdT is not None:
            raise ValueError("dL/dT is not available with vertex_sums")
        if dLdV is None:
            dLdV = torch.empty_like(self.V)
        self._call(None, 0, 0, L.WN_BWD_END, dLdV, dLdT)
        return dLdV


def wn_backward_naive(V, F, dLdW: torch.Tensor, grid: Grid | None = None, Q: torch.Tensor | None = None, **kw):
    """Adjoint of :func:`wn_voxelize_naive`; arguments as :func:`wn_backward`."""
    return wn_backward(V, F, dLdW, grid=grid, Q=Q, _entry="wn_backward_naive", **kw)


def wn_occupancy(W: torch.Tensor, mode: str = "threshold", tau: float = 0.5, k: float = 50.0,
                 occ: torch.Tensor | None = None) -> torch.Tensor:
    m = _OCC_MODES[mode]
    if m == L.WN_OCC_NONE:
        raise ValueError("mode must be 'threshold' or 'sigmoid'")
    if not W.is_contiguous() or W.dtype != torch.float32 or not W.is_cuda:
        raise ValueError("W must be a contiguous float32 device tensor")
    if occ is None:
        occ = torch.empty(W.shape, dtype=torch.uint8 if m == L.WN_OCC_THRESHOLD else torch.float32, device=W.device)
    st = L.load().wn_occupancy(_ptr(W), W.numel(), m, tau, k, _ptr(occ), _stream_handle(W.device))
    L.check("wn_occupancy", st)
    return occ


def wn_occupancy_backward(W: torch.Tensor, g: torch.Tensor, tau: float = 0.5, k: float = 50.0,
                          dLdW: torch.Tensor | None = None) -> torch.Tensor:
    """dL/dW from g = dL/d(occ) of the soft occupancy sigmoid(k (W - tau))."""
    for name, t in (("W", W), ("g", g)):
        if not t.is_contiguous() or t.dtype != torch.float32 or not t.is_cuda:
            raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if g.numel() != W.numel():
        raise ValueError("g must have one entry per entry of W")
    if dLdW is None:
        dLdW = torch.empty_like(W)
    st = L.load().wn_occupancy_backward(_ptr(W), _ptr(g), W.numel(), tau, k, _ptr(dLdW), _stream_handle(W.device))
    L.check("wn_occupancy_backward", st)
    return dLdW


def wn_release_workspace(ws) -> None:
    """Free what the library keeps for a workspace (graphs, pinned staging); the caller
    synchronises the workspace's stream first."""
    L.check("wn_release_workspace", L.load().wn_release_workspace(ws))


def wn_sigmoid_mse(W: torch.Tensor, target: torch.Tensor, tau: float = 0.5, k: float = 50.0,
                   want_loss: bool = True, want_grad: bool = True, loss: torch.Tensor | None = None,
                   dLdW: torch.Tensor | None = None):
    """(loss [1], dL/dW) of L = mean (sigmoid(k (W - tau)) - target)^2."""
    if W.dtype != torch.float32 or target.dtype != torch.float32 or W.numel() != target.numel():
        raise ValueError("W and target must be float32 tensors of equal size")
    if not (W.is_contiguous() and target.is_contiguous() and W.is_cuda and target.is_cuda):
        raise ValueError("W and target must be contiguous device tensors")
    dev = W.device
    if want_loss and loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    if want_grad and dLdW is None:
        dLdW = torch.empty_like(W)
    need = wn_workspace_size(L.WN_OP_LOSS, 0, 0, W.numel())
    ws, wsb = Workspace.get(need, dev)
    st = L.load().wn_sigmoid_mse(_ptr(W), _ptr(target), W.numel(), tau, k, _ptr(loss if want_loss else None),
                                 _ptr(dLdW if want_grad else None), ws, wsb, _stream_handle(dev))
    L.check("wn_sigmoid_mse", st)
    return loss, dLdW


def wn_backward(V, F, dLdW: torch.Tensor, grid: Grid | None = None, Q: torch.Tensor | None = None,
                want_dLdT: bool = False, dLdV: torch.Tensor | None = None, dLdT: torch.Tensor | None = None,
                _entry: str = "wn_backward", pairs: torch.Tensor | None = None, vertex_sums: bool | None = None):
    """dL/dV [nV, 3] (and dL/dT [nF, 3, 3] if requested) for the given dL/dW.  With
    ``pairs`` (a device copy of :func:`wn_build_face_pairs`) two faces per lane, through
    one wn_backward_range call; ``vertex_sums`` (default: when dL/dT is not wanted) lets
    the two faces of a pair share their sums at their common vertices."""
    lib = L.load()
    _check_mesh(V, F)
    if (grid is None) == (Q is None):
        raise ValueError("pass exactly one of grid or Q")
    dev = V.device
    if grid is not None:
        grid = Grid.of(grid)
        P, nQ, gptr, qptr = grid.size, 0, ctypes.byref(grid.to_c()), ctypes.c_void_p(0)
    else:
        P = nQ = Q.shape[0]
        gptr, qptr = None, _ptr(Q)
    dLdW = dLdW.contiguous()
    if dLdW.dtype != torch.float32 or dLdW.numel() != P or not dLdW.is_cuda:
        raise ValueError("dLdW must be a float32 device tensor with one entry per query point")
    if dLdV is None:
        dLdV = torch.empty_like(V)
    if want_dLdT and dLdT is None:
        dLdT = torch.empty((F.shape[0], 3, 3), dtype=torch.float32, device=dev)
    need = wn_workspace_size(L.WN_OP_BACKWARD, V.shape[0], F.shape[0], P)
    ws, wsb = Workspace.get(need, dev)
    if vertex_sums is None:
        vertex_sums = not want_dLdT
    if vertex_sums and want_dLdT:
        raise ValueError("dL/dT is not available with vertex_sums")
    if pairs is not None:   # the whole range in one wn_backward_range call
        pairs = _check_pairs(pairs, F)
        flags = L.WN_BWD_BEGIN | L.WN_BWD_END | (L.WN_BWD_VERTEX_SUMS if vertex_sums else 0)
        st = lib.wn_backward_range(_ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(pairs), pairs.shape[0], gptr, qptr,
                                   nQ, _ptr(dLdW), 0, P, flags, _ptr(dLdV),
                                   _ptr(dLdT if want_dLdT else None), ws, wsb, _stream_handle(dev))
        L.check("wn_backward_range", st)
        return (dLdV, dLdT) if want_dLdT else dLdV
    st = getattr(lib, _entry)(_ptr(V), V.shape[0], _ptr(F), F.shape[0], gptr, qptr, nQ, _ptr(dLdW), _ptr(dLdV),
                              _ptr(dLdT if want_dLdT else None), ws, wsb, _stream_handle(dev))
    L.check(_entry, st)
    return (dLdV, dLdT) if want_dLdT else dLdV


def wn_flip_duplicate(V, F, eps: float = 0.01):
    """Algorithm 2 (flipping duplication) on the device: returns (V2 [2nV, 3], F2 [2nF, 3])."""
    lib = L.load()
    _check_mesh(V, F)
    dev = V.device
    V2 = torch.empty((2 * V.shape[0], 3), dtype=torch.float32, device=dev)
    F2 = torch.empty((2 * F.shape[0], 3), dtype=torch.int32, device=dev)
    need = wn_workspace_size(L.WN_OP_FLIP, V.shape[0], F.shape[0], 0)
    ws, wsb = Workspace.get(need, dev)
    st = lib.wn_flip_duplicate(_ptr(V), V.shape[0], _ptr(F), F.shape[0], eps, _ptr(V2), _ptr(F2), ws, wsb,
                               _stream_handle(dev))
    L.check("wn_flip_duplicate", st)
    return V2, F2


def _check_f32(name, t, n=None):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements")


def wn_adam(x: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, t: int, lr: float = 1e-3,
            betas=(0.9, 0.999), eps: float = 1e-8) -> None:
    """Adam step number ``t`` (>= 1) on x in place, with moments m, v (updated)."""
    n = x.numel()
    for name, a in (("x", x), ("g", g), ("m", m), ("v", v)):
        _check_f32(name, a, n)
    st = L.load().wn_adam(_ptr(x), _ptr(g), _ptr(m), _ptr(v), n, int(t), lr, betas[0], betas[1], eps,
                          _stream_handle(x.device))
    L.check("wn_adam", st)


_INTEGRALS = {"naive": L.WN_INTEGRAL_NAIVE, "gwn": L.WN_INTEGRAL_GWN}


def wn_morph_step(V: torch.Tensor, F: torch.Tensor, target: torch.Tensor, grid: Grid, m: torch.Tensor,
                  v: torch.Tensor, t0: int, iters: int = 1, integral: str = "naive", tau: float = 0.5,
                  k: float = 50.0, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8,
                  loss_history: torch.Tensor | None = None) -> torch.Tensor:
    """``iters`` morphing iterations (forward, sigmoid-MSE loss, adjoint, Adam with step
    numbers t0+1 ...) on V in place; returns the per-iteration losses (device float [iters])."""
    _check_mesh(V, F)
    grid = Grid.of(grid)
    dev = V.device
    _check_f32("target", target, grid.size)
    _check_f32("m", m, V.numel())
    _check_f32("v", v, V.numel())
    if loss_history is None:
        loss_history = torch.empty(max(0, int(iters)), dtype=torch.float32, device=dev)
    else:
        _check_f32("loss_history", loss_history)
        if loss_history.numel() < iters:
            raise ValueError("loss_history holds fewer than iters floats")
    need = wn_workspace_size(L.WN_OP_MORPH, V.shape[0], F.shape[0], grid.size)
    ws, wsb = Workspace.get(need, dev)
    g = grid.to_c()
    st = L.load().wn_morph_step(_ptr(V), V.shape[0], _ptr(F), F.shape[0], ctypes.byref(g), _ptr(target),
                                _INTEGRALS[integral], tau, k, lr, betas[0], betas[1], eps, int(t0), int(iters),
                                _ptr(m), _ptr(v), _ptr(loss_history), ws, wsb, _stream_handle(dev))
    L.check("wn_morph_step", st)
    return loss_history


class Morpher:
    """Device-resident morphing state: vertices (updated in place), Adam moments and
    the step count.  ``run(n)`` enqueues n iterations without synchronising."""

    def __init__(self, V, F, target, grid, integral: str = "naive", tau: float = 0.5, k: float = 50.0,
                 lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8):
        self.V, self.F = as_mesh(V, F)
        self.V = self.V.clone()
        self.grid = Grid.of(grid)
        self.target = torch.as_tensor(target).to(self.V.device, torch.float32).reshape(-1).contiguous()
        self.m = torch.zeros_like(self.V)
        self.v = torch.zeros_like(self.V)
        self.t = 0
        self.opts = dict(integral=integral, tau=tau, k=k, lr=lr, betas=betas, eps=eps)

    def run(self, iters: int) -> torch.Tensor:
        losses = wn_morph_step(self.V, self.F, self.target, self.grid, self.m, self.v, self.t, iters, **self.opts)
        self.t += int(iters)
        return losses


# ------------------------------------------------------- evaluation chain (Section 3)

def _check_points(name, t):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 2 and t.shape[1] == 3):
        raise ValueError(f"{name} must be a contiguous float32 [n, 3] device tensor")


def wn_cubify(occ: torch.Tensor, grid: Grid):
    """Cube surface of an occupancy grid (uint8/bool, grid.size voxels): (V [nV, 3], F [nF, 3]).
    Reads the two counts back (one synchronisation)."""
    grid = Grid.of(grid)
    occ = occ.reshape(-1)
    if occ.dtype == torch.bool:
        occ = occ.view(torch.uint8)
    if not (occ.is_cuda and occ.dtype == torch.uint8 and occ.is_contiguous() and occ.numel() == grid.size):
        raise ValueError("occ must be a contiguous uint8 device tensor with one entry per voxel")
    dev = occ.device
    n = [int(x) for x in grid.n]
    capV = (n[0] + 1) * (n[1] + 1) * (n[2] + 1)
    capF = 12 * grid.size
    V = torch.empty((capV, 3), dtype=torch.float32, device=dev)
    F = torch.empty((capF, 3), dtype=torch.int32, device=dev)
    counts = torch.empty(2, dtype=torch.int64, device=dev)
    g = grid.to_c()
    lib = L.load()
    ws, wsb = Workspace.get(lib.wn_workspace_size_cubify(ctypes.byref(g)), dev)
    st = lib.wn_cubify(_ptr(occ), ctypes.byref(g), _ptr(V), capV, _ptr(F), capF, _ptr(counts), ws, wsb,
                       _stream_handle(dev))
    L.check("wn_cubify", st)
    nV, nF = (int(x) for x in counts.cpu())
    return V[:nV], F[:nF]


def wn_marching_cubes(f: torch.Tensor, grid: Grid, iso: float = 0.5):
    """Marching cubes of a field at the grid's voxel centres (float32, or uint8/bool read
    as 0/1; grid.size values) at level ``iso`` > 0: (V [nV, 3], F [nF, 3]), closed by a
    layer of zeros around the grid.  Reads the two counts back (one synchronisation)."""
    grid = Grid.of(grid)
    f = f.reshape(-1)
    if f.dtype in (torch.bool, torch.uint8):
        f = f.to(torch.float32)
    if not (f.is_cuda and f.dtype == torch.float32 and f.is_contiguous() and f.numel() == grid.size):
        raise ValueError("f must be a contiguous float32 (or uint8/bool) device tensor with one value per voxel")
    dev = f.device
    g = grid.to_c()
    lib = L.load()
    need = lib.wn_workspace_size_marching(ctypes.byref(g))
    if need == 0:
        raise ValueError("grid too large for marching cubes")
    n = [int(x) for x in grid.n]
    capV = 3 * (n[0] + 2) * (n[1] + 2) * (n[2] + 2)
    capF = 5 * (n[0] + 1) * (n[1] + 1) * (n[2] + 1)
    counts = torch.empty(2, dtype=torch.int64, device=dev)
    ws, wsb = Workspace.get(need, dev)
    # first pass: counts only; then outputs of the exact size
    st = lib.wn_marching_cubes(_ptr(f), ctypes.byref(g), float(iso), None, 0, None, 0, _ptr(counts), ws, wsb,
                               _stream_handle(dev))
    L.check("wn_marching_cubes", st)
    nV, nF = (int(x) for x in counts.cpu())
    assert nV <= capV and nF <= capF
    V = torch.empty((nV, 3), dtype=torch.float32, device=dev)
    F = torch.empty((nF, 3), dtype=torch.int32, device=dev)
    st = lib.wn_marching_cubes(_ptr(f), ctypes.byref(g), float(iso), _ptr(V), nV, _ptr(F), nF, _ptr(counts), ws, wsb,
                               _stream_handle(dev))
    L.check("wn_marching_cubes", st)
    return V, F


def wn_laplacian_smooth(V: torch.Tensor, F: torch.Tensor, lam: float = 0.15, iters: int = 10,
                        keep_volume: bool = True) -> torch.Tensor:
    """Umbrella-operator Laplacian smoothing (Jacobi steps), each step followed by a
    scaling about the origin back to the starting enclosed volume unless ``keep_volume``
    is False; returns new vertices."""
    _check_mesh(V, F)
    out = torch.empty_like(V)
    ws, wsb = Workspace.get(wn_workspace_size(L.WN_OP_SMOOTH, V.shape[0], F.shape[0], 0), V.device)
    st = L.load().wn_laplacian_smooth(_ptr(V), V.shape[0], _ptr(F), F.shape[0], lam, int(iters),
                                      1 if keep_volume else 0, _ptr(out), ws, wsb, _stream_handle(V.device))
    L.check("wn_laplacian_smooth", st)
    return out


def wn_sample_surface(V: torch.Tensor, F: torch.Tensor, u: torch.Tensor):
    """Area-uniform surface samples from uniform numbers u (float64 [n, 3]): (P [n, 3], face [n])."""
    _check_mesh(V, F)
    if not (u.is_cuda and u.dtype == torch.float64 and u.is_contiguous() and u.dim() == 2 and u.shape[1] == 3):
        raise ValueError("u must be a contiguous float64 [n, 3] device tensor")
    n = u.shape[0]
    P = torch.empty((n, 3), dtype=torch.float32, device=V.device)
    face = torch.empty(n, dtype=torch.int32, device=V.device)
    ws, wsb = Workspace.get(wn_workspace_size(L.WN_OP_SAMPLE, 0, F.shape[0], n), V.device)
    st = L.load().wn_sample_surface(_ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(u), n, _ptr(P), _ptr(face), ws,
                                    wsb, _stream_handle(V.device))
    L.check("wn_sample_surface", st)
    return P, face


def wn_nn_distance(A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """d[i] = min_j |A_i - B_j|."""
    _check_points("A", A)
    _check_points("B", B)
    d = torch.empty(A.shape[0], dtype=torch.float32, device=A.device)
    ws, wsb = Workspace.get(wn_workspace_size(L.WN_OP_NN, A.shape[0], B.shape[0], 0), A.device)
    st = L.load().wn_nn_distance(_ptr(A), A.shape[0], _ptr(B), B.shape[0], _ptr(d), ws, wsb, _stream_handle(A.device))
    L.check("wn_nn_distance", st)
    return d


def wn_chamfer_hausdorff(A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """Device float64 [2]: (Chamfer distance, Hausdorff distance) between point sets."""
    _check_points("A", A)
    _check_points("B", B)
    out = torch.empty(2, dtype=torch.float64, device=A.device)
    ws, wsb = Workspace.get(wn_workspace_size(L.WN_OP_NN, A.shape[0], B.shape[0], 0), A.device)
    st = L.load().wn_chamfer_hausdorff(_ptr(A), A.shape[0], _ptr(B), B.shape[0], _ptr(out), ws, wsb,
                                       _stream_handle(A.device))
    L.check("wn_chamfer_hausdorff", st)
    return out


def evaluate_occupancy(occ: torch.Tensor, grid: Grid, V_ref: torch.Tensor, F_ref: torch.Tensor,
                       u_rec: torch.Tensor, u_ref: torch.Tensor, lam: float = 0.15, iters: int = 10,
                       mesher: str = "cubes", iso: float = 0.5):
    """The paper's accuracy measure of an occupancy grid: cube surface (``mesher="cubes"``,
    of a uint8 occupancy) or marching cubes (``"marching"``, of any field at ``iso``),
    Laplacian smoothing, surface samples of the result and of the reference mesh
    (uniform numbers u_rec, u_ref), then (Chamfer, Hausdorff) as a device float64 [2]."""
    if mesher == "cubes":
        Vc, Fc = wn_cubify(occ, grid)
    elif mesher == "marching":
        Vc, Fc = wn_marching_cubes(occ, grid, iso)
    else:
        raise ValueError("mesher must be 'cubes' or 'marching'")
    Vs = wn_laplacian_smooth(Vc, Fc, lam, iters)
    Pa, _ = wn_sample_surface(Vs, Fc, u_rec)
    Pb, _ = wn_sample_surface(V_ref, F_ref, u_ref)
    return wn_chamfer_hausdorff(Pa, Pb)


def wn_get_device_error(device=None) -> int:
    """Status of the last call on the current stream's workspace (synchronises)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ws, _ = Workspace.get(0, dev)
    return int(L.load().wn_get_device_error(ws, _stream_handle(dev)))


def wn_version() -> str:
    return L.load().wn_version().decode()


# ------------------------------------------------------------ conveniences

def voxelize(V, F, grid=None, Q=None, occupancy: str | None = None, tau: float = 0.5, k: float = 50.0,
             strips: bool | None = None):
    """Cast (V, F) to the library layout on the GPU and voxelize.  With faces given on
    the host (numpy, or a CPU tensor) the triangle-strip order is built there first and
    :func:`wn_voxelize_strips` runs (about 1.7x faster on large meshes); faces already on
    the device use :func:`wn_voxelize` unless ``strips=True``.  Both agree to rounding."""
    F_host = None if (isinstance(F, torch.Tensor) and F.is_cuda) else np.asarray(F)
    V, F = as_mesh(V, F)
    if Q is not None:
        Q = torch.as_tensor(Q).to(device=V.device, dtype=torch.float32).contiguous()
    use_strips = (F_host is not None) if strips is None else strips
    if use_strips and F.shape[0] > 0:
        if F_host is None:
            F_host = F.cpu().numpy()
        R = torch.as_tensor(wn_build_strips(np.asarray(F_host, np.int32), V.shape[0])).to(V.device)
        return wn_voxelize_strips(V, F, R, grid=grid, Q=Q, occupancy=occupancy, tau=tau, k=k)
    return wn_voxelize(V, F, grid=grid, Q=Q, occupancy=occupancy, tau=tau, k=k)


# ------------------------------------------------------------ batched launch

@dataclass
class MeshJob:
    """One mesh of a batched launch: device mesh, grid, outputs (allocated if None)."""

    V: torch.Tensor
    F: torch.Tensor
    grid: Grid
    occupancy: str | None = None
    tau: float = 0.5
    k: float = 50.0
    W: torch.Tensor | None = None
    occ: torch.Tensor | None = None
    point_begin: int = 0
    point_count: int = 0   # 0: to the end of the grid
    strips: torch.Tensor | None = None   # device strip stream (wn_build_strips) or None

    def prepare(self):
        _check_mesh(self.V, self.F)
        self.grid = Grid.of(self.grid)
        shape = tuple(int(x) for x in self.grid.n)
        if self.W is None:
            self.W = torch.empty(shape, dtype=torch.float32, device=self.V.device)
        mode = _OCC_MODES[self.occupancy]
        if mode != L.WN_OCC_NONE and self.occ is None:
            self.occ = torch.empty(shape, dtype=torch.uint8 if mode == L.WN_OCC_THRESHOLD else torch.float32,
                                   device=self.V.device)
        return self

    def desc(self) -> L.WnMeshDesc:
        d = L.WnMeshDesc()
        d.V = self.V.data_ptr()
        d.nV = self.V.shape[0]
        d.F = self.F.data_ptr()
        d.nF = self.F.shape[0]
        d.grid = self.grid.to_c()
        d.W = self.W.data_ptr()
        mode = _OCC_MODES[self.occupancy]
        d.occ = self.occ.data_ptr() if mode != L.WN_OCC_NONE else None
        d.occ_mode = mode
        d.tau = self.tau
        d.k = self.k
        d.point_begin = int(self.point_begin)
        d.point_count = int(self.point_count)
        if self.strips is not None:
            d.strips = self.strips.data_ptr()
            d.n_strip_records = int(self.strips.shape[0])
        return d


def _descs(jobs):
    arr = (L.WnMeshDesc * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j.prepare().desc()
    return arr


def wn_workspace_size_batched(jobs) -> int:
    arr = _descs(jobs)
    return int(L.load().wn_workspace_size_batched(arr, len(jobs)))


def wn_voxelize_batched(jobs, graph: bool = True, workspace: tuple | None = None):
    """Forward pass for every MeshJob in one persistent launch; fills job.W / job.occ.

    ``workspace`` = (pointer, bytes) of a caller-owned 256-byte-aligned device buffer;
    by default the per-stream workspace is used."""
    if not jobs:
        return jobs
    lib = L.load()
    arr = _descs(jobs)
    dev = jobs[0].V.device
    need = int(lib.wn_workspace_size_batched(arr, len(jobs)))
    if need == 0:
        raise ValueError("invalid mesh job in batch")
    ws, wsb = workspace if workspace is not None else Workspace.get(need, dev)
    flags = 0 if graph else L.WN_BATCH_NO_GRAPH
    st = lib.wn_voxelize_batched(arr, len(jobs), flags, ws, wsb, _stream_handle(dev))
    L.check("wn_voxelize_batched", st)
    return jobs


def wn_autotune(op: str, jobs) -> dict:
    """Time the launch candidates for ``op`` ('voxelize' and 'naive' use jobs[0],
    'batched' all jobs) and record the fastest; returns the report (synchronises)."""
    import json
    lib = L.load()
    code = {"voxelize": L.WN_OP_VOXELIZE, "batched": L.WN_OP_BATCHED, "naive": L.WN_OP_NAIVE}[op]
    arr = _descs(jobs)
    dev = jobs[0].V.device
    if code == L.WN_OP_BATCHED:
        need = int(lib.wn_workspace_size_batched(arr, len(jobs)))
    else:
        j = jobs[0]
        need = wn_workspace_size(L.WN_OP_VOXELIZE, j.V.shape[0], j.F.shape[0], j.grid.size)
    ws, wsb = Workspace.get(need, dev)
    buf = ctypes.create_string_buffer(4096)
    st = lib.wn_autotune(code, arr, len(jobs), ws, wsb, _stream_handle(dev), buf, len(buf))
    L.check("wn_autotune", st)
    return json.loads(buf.value.decode())
