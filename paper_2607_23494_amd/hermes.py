"""Python binding of libhermes: argument marshalling over the C ABI only.

Every computation runs in the library's HIP kernels.  PyTorch supplies device
memory (tensors) and the current HIP stream.  Importing this module loads
libhermes.so and raises ImportError if it has not been built; there is no
fallback path.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import threading
from typing import Iterable, Sequence

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhermes.so")

F32, F64 = 0, 1
PREC = {"fp32": 0, "bf16x3": 1, "fp16x3": 2}
WIN = {"shell": 0, "sphere": 1, "gauss": 2, "sh_shell": 3}
OP_ASSIGN, OP_FFT, OP_XI, OP_FILTER, OP_ZETA, OP_XI_ANISO, OP_TRIPLET, OP_DDD_GAMMA, OP_READOUT = range(9)
ANISO = {"ring": 0, "ring_bin": 1, "gauss_ring": 2, "disk": 3, "cylinder": 4, "cylshell": 5, "gauss_shell": 6}
MAX_BINS = 64


class HermesError(RuntimeError):
    """A libhermes entry point returned an error status."""

    def __init__(self, status: int, msg: str):
        super().__init__(f"libhermes status {status}: {msg}")
        self.status = status


class _Mark(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("exponent", ctypes.c_double),
                ("offset", ctypes.c_double), ("self_term", ctypes.c_double)]


MARK = {"none": 0, "power_law": 1, "inverse_density": 2}


class _AnisoWindow(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("r_perp", ctypes.c_double),
                ("r_par", ctypes.c_double), ("d_perp", ctypes.c_double), ("d_par", ctypes.c_double)]


class _Window(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("ell", ctypes.c_int32), ("m", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("r_lo", ctypes.c_double), ("r_hi", ctypes.c_double)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2607_23494_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sz = ctypes.c_size_t
    lib.hermes_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.hermes_destroy.argtypes = [vp]
    lib.hermes_destroy.restype = None
    lib.hermes_last_error.restype = ctypes.c_char_p
    lib.hermes_workspace_size.argtypes = [vp, i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
    lib.hermes_assign.argtypes = [vp, vp, vp, i64, f64, i32, i32, vp, vp, vp, sz, vp]
    lib.hermes_fft.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
    lib.hermes_xi.argtypes = [vp, vp, i32, i32, f64, vp, i32, vp, i32, i32, vp, vp, vp, sz, vp]
    lib.hermes_xi_static.argtypes = [vp, vp, i32, i32, f64, vp, i32, vp, i32, i32, vp, vp, vp]
    lib.hermes_xi_aniso.argtypes = [vp, vp, i32, i32, f64, ctypes.POINTER(_AnisoWindow), i32, i32, vp, vp, sz, vp]
    lib.hermes_triplet_mc.argtypes = [vp, vp, vp, vp, i32, i32, f64, vp, vp, i64, f64, f64, i32, i32,
                                      ctypes.c_uint64, vp, vp, sz, vp]
    lib.hermes_ddd_gamma.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, sz, vp]
    lib.hermes_filter_bins.argtypes = [vp, vp, i32, i32, f64, ctypes.POINTER(_Window), i32, vp, vp, vp, sz, vp]
    lib.hermes_zeta_l.argtypes = [vp, vp, vp, i32, f64, vp, i32, i32, i32, vp, vp, sz, vp]
    lib.hermes_readout.argtypes = [vp, vp, i32, i32, f64, vp, vp, i64, ctypes.POINTER(_Mark), vp, vp, vp, sz, vp]
    lib.hermes_readout_fields.argtypes = [vp, vp, i32, i32, i32, f64, vp, vp, i64, ctypes.POINTER(_Mark), vp, vp,
                                          vp, sz, vp]
    lib.hermes_mark_ratio.argtypes = [vp, vp, i32, vp, vp]
    lib.hermes_set_basis.argtypes = [vp, i32]
    lib.hermes_get_basis.argtypes = [vp]
    lib.hermes_get_basis.restype = ctypes.c_int
    lib.hermes_profile_enable.argtypes = [vp, i32]
    lib.hermes_profile_reset.argtypes = [vp]
    lib.hermes_profile_read.argtypes = [vp, i32, ctypes.c_char_p, sz, ctypes.POINTER(i64), ctypes.POINTER(f64)]
    for name in ("hermes_create", "hermes_workspace_size", "hermes_assign", "hermes_fft", "hermes_xi", "hermes_xi_static", "hermes_xi_aniso", "hermes_triplet_mc", "hermes_ddd_gamma",
                 "hermes_filter_bins", "hermes_zeta_l", "hermes_readout", "hermes_profile_enable", "hermes_profile_reset",
                 "hermes_profile_read", "hermes_set_basis", "hermes_readout_fields", "hermes_mark_ratio"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()
_ctx_lock = threading.Lock()
_ctx: dict[int, ctypes.c_void_p] = {}


def _check(status: int) -> None:
    if status != 0:
        raise HermesError(status, _lib.hermes_last_error().decode())


def context(device: int) -> ctypes.c_void_p:
    """The library context of a device (created once per process)."""
    with _ctx_lock:
        c = _ctx.get(device)
        if c is None:
            c = ctypes.c_void_p()
            _check(_lib.hermes_create(ctypes.byref(c), device))
            _ctx[device] = c
        return c


BASES = {"b3": 0, "db2": 1}


def set_basis(name: str, device: int = 0) -> None:
    """Scaling function of every later call on the device's context: "b3"
    (the centred cubic B-spline, default) or "db2" (the orthonormal
    Daubechies D4 function)."""
    if name not in BASES:
        raise ValueError(f"unknown basis {name!r}")
    _check(_lib.hermes_set_basis(context(device), BASES[name]))


def get_basis(device: int = 0) -> str:
    code = _lib.hermes_get_basis(context(device))
    return {v: k for k, v in BASES.items()}[code]


@contextlib.contextmanager
def basis(name: str, device: int = 0):
    """Run a block of calls with the given basis, then restore the previous one."""
    prev = get_basis(device)
    set_basis(name, device)
    try:
        yield
    finally:
        set_basis(prev, device)


def _dev(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("libhermes works on device tensors only")
    return t.device.index if t.device.index is not None else torch.cuda.current_device()


def _stream(device: int, stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream):
    """Allocate on the stream the kernels are launched on: the caching
    allocator then never hands a wrapper's workspace or outputs to work on
    another stream while the library's kernels may still use them."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dtype_code(dtype: torch.dtype) -> int:
    if dtype in (torch.float32, torch.complex64):
        return F32
    if dtype in (torch.float64, torch.complex128):
        return F64
    raise ValueError(f"unsupported dtype {dtype}")


def _edges_arr(edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
    if e.ndim != 1 or e.size < 2:
        raise ValueError("edges must be a 1-D array of at least two values")
    return e


def workspace_size(op: int, n_grid: int, dtype=torch.float32, n_batch: int = 1, n_ells: int = 1,
                   device: int = 0) -> int:
    b = ctypes.c_size_t()
    _check(_lib.hermes_workspace_size(context(device), op, n_grid, _dtype_code(dtype), n_batch, n_ells,
                                      ctypes.byref(b)))
    return int(b.value)


def _workspace(nbytes: int, device: int, work: torch.Tensor | None) -> torch.Tensor:
    if work is not None:
        if work.numel() * work.element_size() < nbytes:
            raise ValueError("workspace tensor too small")
        return work
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=f"cuda:{device}")


# ----------------------------------------------------------------------------
# entry points
# ----------------------------------------------------------------------------

def assign(pos: torch.Tensor, weight: torch.Tensor | None, box_L: float, n_grid: int,
           dtype=torch.float32, eps: torch.Tensor | None = None, sum_w: torch.Tensor | None = None,
           work: torch.Tensor | None = None, stream=None):
    """B3 projection of a catalogue: returns (eps [N,N,N], sum_w [1] float64)."""
    dev = _dev(pos)
    if pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_contiguous():
        raise ValueError("pos must be a contiguous float32 [n, 3] device tensor")
    if weight is not None and (weight.dtype != torch.float32 or weight.numel() != pos.shape[0]
                               or not weight.is_contiguous() or _dev(weight) != dev):
        raise ValueError("weight must be a contiguous float32 [n] tensor on the same device")
    wbytes = workspace_size(OP_ASSIGN, n_grid, dtype, int(pos.shape[0]), 1, dev)
    with _on(stream):
        w = _workspace(wbytes, dev, work)
        if eps is None:
            eps = torch.empty((n_grid, n_grid, n_grid), dtype=dtype, device=pos.device)
        if sum_w is None:
            sum_w = torch.empty(1, dtype=torch.float64, device=pos.device)
        _check(_lib.hermes_assign(context(dev), _ptr(pos), _ptr(weight), pos.shape[0], float(box_L), n_grid,
                                  _dtype_code(eps.dtype), _ptr(eps), _ptr(sum_w), _ptr(w), wbytes,
                                  _stream(dev, stream)))
    return eps, sum_w


def fft(eps: torch.Tensor, sum_w: torch.Tensor, want_delta: bool = True, delta_k: torch.Tensor | None = None,
        delta: torch.Tensor | None = None, stream=None):
    """Contrast and forward r2c FFT: returns (delta_k [N,N,N/2+1] complex, delta or None)."""
    dev = _dev(eps)
    n = eps.shape[0]
    cdt = torch.complex64 if eps.dtype == torch.float32 else torch.complex128
    with _on(stream):
        if delta_k is None:
            delta_k = torch.empty((n, n, n // 2 + 1), dtype=cdt, device=eps.device)
        if want_delta and delta is None:
            delta = torch.empty_like(eps)
        _check(_lib.hermes_fft(context(dev), _ptr(eps), _ptr(sum_w), n, _dtype_code(eps.dtype), _ptr(delta_k),
                               _ptr(delta) if want_delta else None, _stream(dev, stream)))
    return delta_k, (delta if want_delta else None)


def xi(delta_k: torch.Tensor, box_L: float, edges, ells: Sequence[int] = (0,), los_axis: int = 2,
       out: torch.Tensor | None = None, work: torch.Tensor | None = None, stream=None, shot: bool = False):
    """2PCF multipoles by Parseval: device float64 [len(ells), n_bins]; with
    shot=True also the shot-noise factors S_lb of the same shape, as a tuple
    (xi, shot)."""
    dev = _dev(delta_k)
    n = delta_k.shape[0]
    e = _edges_arr(edges)
    el = np.ascontiguousarray(np.asarray(list(ells), dtype=np.int32))
    nb = e.size - 1
    dt = _dtype_code(delta_k.dtype)
    wbytes = workspace_size(OP_XI, n, delta_k.dtype, nb, el.size, dev)
    with _on(stream):
        w = _workspace(wbytes, dev, work)
        if out is None:
            out = torch.empty((el.size, nb), dtype=torch.float64, device=delta_k.device)
        sh = torch.empty((el.size, nb), dtype=torch.float64, device=delta_k.device) if shot else None
        _check(_lib.hermes_xi(context(dev), _ptr(delta_k), n, dt, float(box_L), e.ctypes.data_as(ctypes.c_void_p),
                              nb, el.ctypes.data_as(ctypes.c_void_p), el.size, los_axis, _ptr(out),
                              _ptr(sh) if shot else None, _ptr(w), wbytes, _stream(dev, stream)))
    return (out, sh) if shot else out


def make_aniso_windows(specs: Iterable) -> ctypes.Array:
    """specs: tuples (kind, r_perp, r_par[, d_perp[, d_par]]) with kind in ANISO."""
    specs = list(specs)
    arr = (_AnisoWindow * len(specs))()
    for i, s in enumerate(specs):
        vals = [float(v) for v in s[1:]] + [0.0] * (5 - len(s))
        arr[i] = _AnisoWindow(ANISO[s[0]], 0, *vals)
    return arr


def xi_aniso(delta_k: torch.Tensor, box_L: float, windows, los_axis: int = 2, out: torch.Tensor | None = None,
             work: torch.Tensor | None = None, stream=None):
    """Anisotropic 2PCF for axisymmetric windows: device float64 [n_windows].
    windows: tuples (kind, r_perp, r_par[, d_perp[, d_par]]), kind in ANISO."""
    dev = _dev(delta_k)
    n = delta_k.shape[0]
    arr = make_aniso_windows(windows)
    nw = len(arr)
    wbytes = workspace_size(OP_XI_ANISO, n, delta_k.dtype, nw, 0, dev)
    with _on(stream):
        w = _workspace(wbytes, dev, work)
        if out is None:
            out = torch.empty((nw,), dtype=torch.float64, device=delta_k.device)
        _check(_lib.hermes_xi_aniso(context(dev), _ptr(delta_k), n, _dtype_code(delta_k.dtype), float(box_L), arr, nw,
                                    los_axis, _ptr(out), _ptr(w), wbytes, _stream(dev, stream)))
    return out


def mark_ratio(xi_marked: torch.Tensor, xi_plain: torch.Tensor, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """M(r) = (1 + xi_marked) / (1 + xi) per bin: the marked 2PCF normalised
    by the unmarked pair counts.  Device float64 tensors of one shape."""
    dev = _dev(xi_marked)
    if (xi_marked.dtype != torch.float64 or xi_plain.dtype != torch.float64 or xi_marked.shape != xi_plain.shape
            or not xi_marked.is_contiguous() or not xi_plain.is_contiguous()):
        raise ValueError("xi_marked and xi must be contiguous float64 tensors of one shape")
    with _on(stream):
        if out is None:
            out = torch.empty_like(xi_marked)
        _check(_lib.hermes_mark_ratio(_ptr(xi_marked), _ptr(xi_plain), int(xi_marked.numel()), _ptr(out),
                                      _stream(dev, stream)))
    return out


def triplet_mc(f2: torch.Tensor, f3: torch.Tensor, box_L: float, r12: float, r13: float, n_theta: int,
               n_rot: int, seed: int, centres: torch.Tensor | None = None, weights: torch.Tensor | None = None,
               n_box: int = 0, f1: torch.Tensor | None = None, out: torch.Tensor | None = None,
               work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Monte-Carlo triangle sums: device float64 [n_theta, 4] = (sum a, sum a f2,
    sum a f3, sum a f2 f3) over n_rot rotations of every primary vertex: the
    points `centres` (weights as a) or, without centres, n_box uniform box
    points (f1 as a)."""
    dev = _dev(f2)
    n = f2.shape[0]
    for f in (f1, f3):
        if f is not None and (f.shape != f2.shape or f.dtype != f2.dtype or not f.is_contiguous()):
            raise ValueError("f1, f2, f3 must share shape and dtype and be contiguous")
    if centres is not None and (centres.dtype != torch.float32 or centres.dim() != 2 or centres.shape[1] != 3
                                or not centres.is_contiguous()):
        raise ValueError("centres must be a contiguous float32 [n, 3] device tensor")
    if weights is not None and (centres is None or weights.dtype != torch.float32
                                or weights.numel() != centres.shape[0] or not weights.is_contiguous()):
        raise ValueError("weights must be a contiguous float32 [n] tensor beside centres")
    n_c = int(centres.shape[0]) if centres is not None else int(n_box)
    # a workspace of the minimum size runs the direct path; one sized with the
    # centre count also holds the block-local path's bucket lists
    wmin = workspace_size(OP_TRIPLET, n, f2.dtype, n_theta, 0, dev)
    with _on(stream):
        if work is None:
            w = _workspace(workspace_size(OP_TRIPLET, n, f2.dtype, n_theta, n_c if n_c < 2 ** 31 else 0, dev), dev,
                           None)
        else:
            w = _workspace(wmin, dev, work)
        wbytes = w.numel() * w.element_size()
        if out is None:
            out = torch.empty((n_theta, 4), dtype=torch.float64, device=f2.device)
        _check(_lib.hermes_triplet_mc(context(dev), _ptr(f1), _ptr(f2), _ptr(f3), n, _dtype_code(f2.dtype),
                                      float(box_L), _ptr(centres), _ptr(weights), n_c, float(r12), float(r13),
                                      int(n_theta), int(n_rot), int(seed) & ((1 << 64) - 1), _ptr(out), _ptr(w),
                                      wbytes, _stream(dev, stream)))
    return out


def ddd_gamma(eps: torch.Tensor, fields: torch.Tensor, out: torch.Tensor | None = None,
              work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """3PCF monopole through connection coefficients: device float64 [nb, nb],
    out[b1][b2] = box mean of eps(x) f_b1(x) f_b2(x) for the B3 expansions of
    eps [N,N,N] and fields [nb,N,N,N]."""
    dev = _dev(eps)
    n = eps.shape[0]
    if fields.dim() != 4 or tuple(fields.shape[1:]) != tuple(eps.shape) or fields.dtype != eps.dtype \
            or not fields.is_contiguous() or not eps.is_contiguous():
        raise ValueError("fields must be a contiguous [nb, N, N, N] tensor of eps's dtype")
    nb = fields.shape[0]
    wbytes = workspace_size(OP_DDD_GAMMA, n, eps.dtype, nb, 0, dev)
    with _on(stream):
        w = _workspace(wbytes, dev, work)
        if out is None:
            out = torch.empty((nb, nb), dtype=torch.float64, device=eps.device)
        _check(_lib.hermes_ddd_gamma(context(dev), _ptr(eps), _ptr(fields), nb, n, _dtype_code(eps.dtype), _ptr(out),
                                     _ptr(w), wbytes, _stream(dev, stream)))
    return out


def xi_static(delta_k: torch.Tensor, box_L: float, edges, ells: Sequence[int] = (0,), los_axis: int = 2,
              out: torch.Tensor | None = None, shot_out: torch.Tensor | None = None, stream=None,
              shot: bool = False):
    """hermes_xi_static: as xi() with the library's static scratch instead of a
    workspace (the library allocates nothing; pass `out` (and `shot_out`) to
    allocate nothing here either)."""
    dev = _dev(delta_k)
    n = delta_k.shape[0]
    e = _edges_arr(edges)
    el = np.ascontiguousarray(np.asarray(list(ells), dtype=np.int32))
    nb = e.size - 1
    with _on(stream):
        if out is None:
            out = torch.empty((el.size, nb), dtype=torch.float64, device=delta_k.device)
        if shot and shot_out is None:
            shot_out = torch.empty((el.size, nb), dtype=torch.float64, device=delta_k.device)
        _check(_lib.hermes_xi_static(context(dev), _ptr(delta_k), n, _dtype_code(delta_k.dtype), float(box_L),
                                     e.ctypes.data_as(ctypes.c_void_p), nb, el.ctypes.data_as(ctypes.c_void_p),
                                     el.size, los_axis, _ptr(out), _ptr(shot_out) if shot else None,
                                     _stream(dev, stream)))
    return (out, shot_out) if shot else out


def make_windows(specs: Iterable) -> ctypes.Array:
    """specs: tuples (kind, r_lo, r_hi[, ell, m]) with kind in WIN."""
    specs = list(specs)
    arr = (_Window * len(specs))()
    for i, s in enumerate(specs):
        kind, lo, hi = s[0], s[1], s[2]
        ell, m = (s[3], s[4]) if len(s) > 3 else (0, 0)
        arr[i] = _Window(WIN[kind], int(ell), int(m), 0, float(lo), float(hi))
    return arr


def filter_bins(delta_k: torch.Tensor, box_L: float, windows, store_fields: bool = False,
                moments: bool = True, out: torch.Tensor | None = None, work: torch.Tensor | None = None,
                stream=None):
    """Window-filtered fields and counts-in-cells moments.

    Returns (fields [n_win,N,N,N] or None, moments [n_win,3] float64 or None).
    """
    dev = _dev(delta_k)
    n = delta_k.shape[0]
    win = make_windows(windows)
    nw = len(win)
    rdt = torch.float32 if delta_k.dtype == torch.complex64 else torch.float64
    wbytes = workspace_size(OP_FILTER, n, rdt, nw, 1, dev)
    with _on(stream):
        w = _workspace(wbytes, dev, work)
        if store_fields and out is None:
            out = torch.empty((nw, n, n, n), dtype=rdt, device=delta_k.device)
        mom = torch.empty((nw, 3), dtype=torch.float64, device=delta_k.device) if moments else None
        _check(_lib.hermes_filter_bins(context(dev), _ptr(delta_k), n, _dtype_code(rdt), float(box_L), win, nw,
                                       _ptr(out) if store_fields else None, _ptr(mom), _ptr(w), wbytes,
                                       _stream(dev, stream)))
    return (out if store_fields else None), mom


def zeta_l(delta: torch.Tensor, delta_k: torch.Tensor, box_L: float, edges, l_max: int,
           precision: str = "fp32", out: torch.Tensor | None = None, work: torch.Tensor | None = None,
           stream=None) -> torch.Tensor:
    """3PCF multipoles: device float64 [l_max+1, n_bins, n_bins]."""
    dev = _dev(delta)
    n = delta.shape[0]
    e = _edges_arr(edges)
    nb = e.size - 1
    wbytes = workspace_size(OP_ZETA, n, torch.float32, nb, 1, dev)
    with _on(stream):
        w = _workspace(wbytes, dev, work)
        if out is None:
            out = torch.empty((l_max + 1, nb, nb), dtype=torch.float64, device=delta.device)
        _check(_lib.hermes_zeta_l(context(dev), _ptr(delta), _ptr(delta_k), n, float(box_L),
                                  e.ctypes.data_as(ctypes.c_void_p), nb, l_max, PREC[precision], _ptr(out), _ptr(w),
                                  wbytes, _stream(dev, stream)))
    return out


def readout(field: torch.Tensor, box_L: float, pos: torch.Tensor, weight: torch.Tensor | None = None,
            mark: tuple | None = None, want_values: bool = True, moments: bool = False,
            out: torch.Tensor | None = None, stream=None, moments_out: torch.Tensor | None = None,
            work: torch.Tensor | None = None):
    """Values of a coefficient field at arbitrary positions, optionally turned
    into marks and weighted.  mark = (kind, exponent, offset[, self_term]) with
    kind in MARK.  Returns (values [n_pts] or None, moments [3] float64 or None);
    moments_out, a float64 [3] device tensor, receives the moments in place."""
    if moments_out is not None:
        if moments_out.dtype != torch.float64 or moments_out.numel() != 3 or not moments_out.is_contiguous():
            raise ValueError("moments_out must be a contiguous float64 [3] tensor")
        moments = True
    dev = _dev(field)
    n = field.shape[0]
    if pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_contiguous():
        raise ValueError("pos must be a contiguous float32 [n, 3] device tensor")
    if weight is not None and (weight.dtype != torch.float32 or weight.numel() != pos.shape[0]
                               or not weight.is_contiguous()):
        raise ValueError("weight must be a contiguous float32 [n] tensor")
    mk = None
    if mark is not None:
        st = float(mark[3]) if len(mark) > 3 else 0.0
        mk = _Mark(MARK[mark[0]], 0, float(mark[1]), float(mark[2]), st)
    with _on(stream):
        if want_values and out is None:
            out = torch.empty(pos.shape[0], dtype=field.dtype, device=field.device)
        mom = moments_out if moments_out is not None else (
            torch.empty(3, dtype=torch.float64, device=field.device) if moments else None)
        n_pts = int(pos.shape[0])
        nbytes = workspace_size(OP_READOUT, n, field.dtype, n_pts, device=dev) if n_pts <= 2 ** 31 - 1 else 0
        ws = _workspace(nbytes, dev, work) if nbytes > 0 else None
        _check(_lib.hermes_readout(context(dev), _ptr(field), n, _dtype_code(field.dtype), float(box_L), _ptr(pos),
                                   _ptr(weight), n_pts, ctypes.byref(mk) if mk is not None else None,
                                   _ptr(out) if want_values else None, _ptr(mom), _ptr(ws),
                                   ws.numel() * ws.element_size() if ws is not None else 0, _stream(dev, stream)))
    return (out if want_values else None), mom


def readout_fields(fields: torch.Tensor, box_L: float, pos: torch.Tensor, weight: torch.Tensor | None = None,
                   mark: tuple | None = None, want_values: bool = True, moments: bool = False,
                   out: torch.Tensor | None = None, moments_out: torch.Tensor | None = None,
                   work: torch.Tensor | None = None, stream=None):
    """readout() of several fields [k, N, N, N] at the same positions (one
    bucketing).  Returns (values [k, n_pts] or None, moments [k, 3] or None)."""
    dev = _dev(fields)
    if fields.dim() != 4 or not fields.is_contiguous():
        raise ValueError("fields must be a contiguous [k, N, N, N] device tensor")
    k, n = int(fields.shape[0]), int(fields.shape[1])
    if pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_contiguous():
        raise ValueError("pos must be a contiguous float32 [n, 3] device tensor")
    if weight is not None and (weight.dtype != torch.float32 or weight.numel() != pos.shape[0]
                               or not weight.is_contiguous()):
        raise ValueError("weight must be a contiguous float32 [n] tensor")
    if moments_out is not None:
        if moments_out.dtype != torch.float64 or moments_out.numel() != 3 * k or not moments_out.is_contiguous():
            raise ValueError("moments_out must be a contiguous float64 [k, 3] tensor")
        moments = True
    mk = None
    if mark is not None:
        st = float(mark[3]) if len(mark) > 3 else 0.0
        mk = _Mark(MARK[mark[0]], 0, float(mark[1]), float(mark[2]), st)
    n_pts = int(pos.shape[0])
    with _on(stream):
        if want_values and out is None:
            out = torch.empty((k, n_pts), dtype=fields.dtype, device=fields.device)
        mom = moments_out if moments_out is not None else (
            torch.empty((k, 3), dtype=torch.float64, device=fields.device) if moments else None)
        nbytes = workspace_size(OP_READOUT, n, fields.dtype, n_pts, device=dev) if n_pts <= 2 ** 31 - 1 else 0
        ws = _workspace(nbytes, dev, work) if nbytes > 0 else None
        _check(_lib.hermes_readout_fields(context(dev), _ptr(fields), k, n, _dtype_code(fields.dtype), float(box_L),
                                          _ptr(pos), _ptr(weight), n_pts, ctypes.byref(mk) if mk is not None else None,
                                          _ptr(out) if want_values else None, _ptr(mom), _ptr(ws),
                                          ws.numel() * ws.element_size() if ws is not None else 0,
                                          _stream(dev, stream)))
    return (out if want_values else None), mom


# ----------------------------------------------------------------------------
# per-kernel timing
# ----------------------------------------------------------------------------

def profile_enable(on: bool = True, device: int = 0) -> None:
    """Bracket every library kernel launch with HIP events on its stream."""
    _check(_lib.hermes_profile_enable(context(device), 1 if on else 0))


def profile_reset(device: int = 0) -> None:
    _check(_lib.hermes_profile_reset(context(device)))


def profile_read(device: int = 0) -> dict:
    """{kernel class: (launches, total milliseconds)} since the last reset."""
    out = {}
    buf = ctypes.create_string_buffer(128)
    i = 0
    while True:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        st = _lib.hermes_profile_read(context(device), i, buf, 128, ctypes.byref(n), ctypes.byref(ms))
        if st != 0:
            break
        out[buf.value.decode()] = (int(n.value), float(ms.value))
        i += 1
    return out
