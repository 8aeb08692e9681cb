"""ctypes binding of libtotalconv (argument marshalling only).

Every computation runs in the HIP library; this module converts torch tensors
and numpy arrays into the pointers, sizes and stream handle the C ABI expects
(include/totalconv.h), allocates the device workspace with torch, and turns a
non-zero status into an exception.  If the built library is missing it raises;
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtotalconv.so")

TC_OP_WIGNER, TC_OP_FWD, TC_OP_ADJ, TC_OP_FWD_POL, TC_OP_CUBE, TC_OP_MATRIX = 0, 1, 2, 3, 4, 5
TC_POL_SEPARATE, TC_POL_SUM = 0, 1
TC_LMAX_LIMIT = 16384
TC_OK, TC_EINVAL, TC_EHIP, TC_ENOMEM, TC_EUNSUPPORTED = 0, -1, -2, -3, -4   # include/totalconv.h

_lib = None
_lock = threading.Lock()


class TcDetector(ctypes.Structure):
    """struct tc_detector of include/totalconv.h."""
    _fields_ = [("lmax", ctypes.c_int), ("mbmax", ctypes.c_int), ("nring", ctypes.c_int),
                ("beta", ctypes.c_void_p), ("cosbeta", ctypes.c_void_p), ("blm", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("Cbar", ctypes.c_void_p), ("blm_bar", ctypes.c_void_p)]


class TotalConvError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


def lib():
    """Load libtotalconv.so (built in-tree by paper_1002_1050_amd/build.py)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is not built; run `python -m paper_1002_1050_amd.build` "
                    "(there is no CPU fallback)")
            L = ctypes.CDLL(LIB_PATH)
            I, P, S = ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
            L.tc_last_error.restype = ctypes.c_char_p
            L.tc_last_error.argtypes = []
            L.tc_abi_version.restype = I
            L.tc_abi_version.argtypes = []
            L.totalconv_workspace_bytes.restype = S
            L.totalconv_workspace_bytes.argtypes = [I, I, I, I]
            PP = ctypes.POINTER(P)
            ring_fns = {   # entry points on colatitudes; each has a twin with suffix _x on cosines
                "totalconv_workspace_bytes_rings": (S, [I, I, I, I, P]),
                "wigner_d_rings": (I, [I, I, P, P, I, P, P, P, S, P]),
                "wigner_d_matrix": (I, [I, I, P, P, P, S, P]),
                "totalconv_fwd": (I, [I, I, I, P, P, P, P, P, S, P]),
                "totalconv_adj": (I, [I, I, I, P, P, P, P, P, P, P, S, P]),
                "totalconv_fwd_pol": (I, [I, I, I, P, I, PP, PP, I, PP, P, S, P]),
                "totalconv_adj_pol": (I, [I, I, I, P, I, PP, PP, I, PP, PP, PP, P, S, P]),
            }
            for name, (res, args) in ring_fns.items():
                for n in (name, name + "_x"):
                    getattr(L, n).restype = res
                    getattr(L, n).argtypes = args
            L.tc_rings_from_beta.restype = I
            L.tc_rings_from_beta.argtypes = [I, P, P]
            L.totalconv_fwd_noalloc.restype = I
            L.totalconv_fwd_noalloc.argtypes = [I, I, I, P, P, P, P, P]
            L.tc_set_tile.restype = I
            L.tc_set_tile.argtypes = [I, I]
            L.tc_get_tile.restype = I
            L.tc_get_tile.argtypes = [I, I]
            L.tc_set_tile_ex.restype = I
            L.tc_set_tile_ex.argtypes = [I, I, I, I]
            L.tc_get_tile_ex.restype = I
            L.tc_get_tile_ex.argtypes = [I, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]
            L.tc_plan_create.restype = I
            L.tc_plan_create.argtypes = [ctypes.POINTER(P), I, I, ctypes.POINTER(TcDetector), I, P, P, P]
            L.tc_plan_execute.restype = I
            L.tc_plan_execute.argtypes = [P, P]
            L.tc_plan_destroy.restype = I
            L.tc_plan_destroy.argtypes = [P]
            L.tc_plan_device_bytes.restype = S
            L.tc_plan_device_bytes.argtypes = [P]
            L.tc_plan_tile.restype = I
            L.tc_plan_tile.argtypes = [P]
            L.wigner_d_matrix_workspace_bytes.restype = S
            L.wigner_d_matrix_workspace_bytes.argtypes = [I, I]
            L.totalconv_datacube_workspace_bytes.restype = S
            L.totalconv_datacube_workspace_bytes.argtypes = [I, I, I, I, I]
            L.totalconv_datacube_ring_chunk.restype = I
            L.totalconv_datacube_ring_chunk.argtypes = [I, I, I, I, I]
            L.totalconv_datacube.restype = I
            L.totalconv_datacube.argtypes = [I, I, I, P, I, I, P, P, S, P]
            L.tc_timing_enable.restype = I
            L.tc_timing_enable.argtypes = [I]
            L.tc_timing_read.restype = I
            L.tc_timing_read.argtypes = [I, ctypes.POINTER(ctypes.c_float), I]
            _lib = L
    return _lib


def last_error() -> str:
    return lib().tc_last_error().decode()


def _check(fn: str, rc: int):
    if rc != 0:
        raise TotalConvError(fn, rc, last_error())


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _hptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_device(t, name, dtype):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class _Workspace:
    """Grow-only device workspace per (device, stream)."""

    def __init__(self):
        self._bufs = {}

    def get(self, torch, device, stream, nbytes):
        key = (device.index, stream.value)
        buf = self._bufs.get(key)
        if buf is None or buf.numel() < nbytes:
            self._bufs.pop(key, None)
            buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            self._bufs[key] = buf
        return buf

    def clear(self):
        self._bufs.clear()


workspace_cache = _Workspace()


def rings_from_beta(beta) -> np.ndarray:
    """The ring cosines the library computes on for the colatitudes beta (tc_rings_from_beta)."""
    b = _host(np.atleast_1d(beta), np.float64)
    x = np.empty_like(b)
    _check("tc_rings_from_beta", lib().tc_rings_from_beta(b.size, _hptr(b), _hptr(x)))
    return x


def _fn(name, cos):
    """The C entry point `name` on colatitudes, or its twin `name`_x on ring cosines."""
    return getattr(lib(), name + ("_x" if cos else ""))


def _workspace_bytes(op, lmax, mbmax, rings, cos):
    return int(_fn("totalconv_workspace_bytes_rings", cos)(op, lmax, mbmax, rings.size, _hptr(rings)))


def workspace_bytes(op: int, lmax: int, mbmax: int, beta) -> int:
    """Exact workspace size for these colatitudes; 0 when the arguments are invalid (the entry
    point itself then reports why)."""
    return _workspace_bytes(op, lmax, mbmax, _host(beta, np.float64), False)


def workspace_bytes_x(op: int, lmax: int, mbmax: int, cosbeta) -> int:
    """workspace_bytes for ring cosines."""
    return _workspace_bytes(op, lmax, mbmax, _host(cosbeta, np.float64), True)


def _wigner_d_rings(lmax, mb, msky, rings, cos, device):
    import torch
    device = torch.device(device)
    mb = _host(np.atleast_1d(mb), np.int32)
    ms = _host(np.atleast_1d(msky), np.int32)
    x = _host(np.atleast_1d(rings), np.float64)
    if mb.shape != ms.shape:
        raise ValueError("mb and msky must have the same length")
    out = torch.empty((mb.size, lmax + 1, x.size), dtype=torch.float64, device=device)
    nbytes = lib().totalconv_workspace_bytes(TC_OP_WIGNER, lmax, max(mb.size, 1), max(x.size, 1))
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, nbytes)
    rc = _fn("wigner_d_rings", cos)(lmax, mb.size, _hptr(mb), _hptr(ms), x.size, _hptr(x), _dptr(out),
                                    _dptr(ws), ws.numel(), stream)
    _check("wigner_d_rings" + ("_x" if cos else ""), rc)
    return out


def wigner_d_rings(lmax: int, mb, msky, beta, device="cuda"):
    """d^l_{mb[i],msky[i]}(beta_j) on the GPU, shape (npair, lmax+1, nring) float64."""
    return _wigner_d_rings(lmax, mb, msky, beta, False, device)


def wigner_d_rings_x(lmax: int, mb, msky, cosbeta, device="cuda"):
    """wigner_d_rings on ring cosines."""
    return _wigner_d_rings(lmax, mb, msky, cosbeta, True, device)


def _wigner_d_matrix(l, rings, cos, device, out):
    import torch
    device = torch.device(device)
    x = _host(np.atleast_1d(rings), np.float64)
    shape = (x.size, 2 * l + 1, 2 * l + 1)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=device)
    else:
        _require_device(out, "out", torch.float64)
        if tuple(out.shape) != shape:
            raise ValueError(f"out must have shape {shape}")
        device = out.device
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, int(lib().wigner_d_matrix_workspace_bytes(l, max(x.size, 1))))
    rc = _fn("wigner_d_matrix", cos)(l, x.size, _hptr(x), _dptr(out), _dptr(ws), ws.numel(), stream)
    _check("wigner_d_matrix" + ("_x" if cos else ""), rc)
    return out


def wigner_d_matrix(l: int, beta, device="cuda", out=None):
    """Full matrix d^l_{m m'}(beta_j), -l <= m, m' <= l: float64 (nring, 2l+1, 2l+1) on the GPU."""
    return _wigner_d_matrix(l, beta, False, device, out)


def wigner_d_matrix_x(l: int, cosbeta, device="cuda", out=None):
    """wigner_d_matrix on ring cosines."""
    return _wigner_d_matrix(l, cosbeta, True, device, out)


def _sky_beam(torch, lmax, mbmax, alm, blm, device=None, tag=""):
    """Checks a sky and a beam against lmax / mbmax (complex128, contiguous, on one GPU)."""
    _require_device(alm, "alm" + tag, torch.complex128)
    _require_device(blm, "blm" + tag, torch.complex128)
    if alm.numel() != (lmax + 1) * (lmax + 2) // 2 or blm.numel() != (2 * mbmax + 1) * (lmax + 1):
        raise ValueError(f"alm{tag} / blm{tag} sizes do not match lmax / mbmax")
    device = device or alm.device
    if alm.device != device or blm.device != device:
        raise ValueError(f"alm{tag} and blm{tag} must be on {device}")
    return device


def _totalconv_fwd(lmax, mbmax, rings, cos, alm, blm, out):
    import torch
    device = _sky_beam(torch, lmax, mbmax, alm, blm)
    x = _host(rings, np.float64)
    shape = (2 * mbmax + 1, lmax + 1, x.size)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex128, device=device)
    else:
        _require_device(out, "out", torch.complex128)
        if tuple(out.shape) != shape or out.device != device:
            raise ValueError(f"out must have shape {shape} on {device}")
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, _workspace_bytes(TC_OP_FWD, lmax, mbmax, x, cos))
    rc = _fn("totalconv_fwd", cos)(lmax, mbmax, x.size, _hptr(x), _dptr(alm), _dptr(blm), _dptr(out),
                                   _dptr(ws), ws.numel(), stream)
    _check("totalconv_fwd" + ("_x" if cos else ""), rc)
    return out


def totalconv_fwd(lmax: int, mbmax: int, beta, alm, blm, out=None):
    """C = totalconv(alm, blm) on the colatitudes beta; complex128 (2*mbmax+1, lmax+1, nring)."""
    return _totalconv_fwd(lmax, mbmax, beta, False, alm, blm, out)


def totalconv_fwd_noalloc(lmax: int, mbmax: int, beta, alm, blm, out):
    """totalconv_fwd with its tables in the library's static device array (no workspace, no
    allocation by the library); `out` must be given, complex128 (2*mbmax+1, lmax+1, nring)."""
    import torch
    device = _sky_beam(torch, lmax, mbmax, alm, blm)
    b = _host(beta, np.float64)
    shape = (2 * mbmax + 1, lmax + 1, b.size)
    _require_device(out, "out", torch.complex128)
    if tuple(out.shape) != shape or out.device != device:
        raise ValueError(f"out must have shape {shape} on {device}")
    rc = lib().totalconv_fwd_noalloc(lmax, mbmax, b.size, _hptr(b), _dptr(alm), _dptr(blm), _dptr(out),
                                     _stream_handle(torch, device))
    _check("totalconv_fwd_noalloc", rc)
    return out


def totalconv_fwd_x(lmax: int, mbmax: int, cosbeta, alm, blm, out=None):
    """totalconv_fwd on ring cosines."""
    return _totalconv_fwd(lmax, mbmax, cosbeta, True, alm, blm, out)


def _totalconv_adj(lmax, mbmax, rings, cos, alm, blm, Cbar, want_alm, want_blm):
    import torch
    device = _sky_beam(torch, lmax, mbmax, alm, blm)
    _require_device(Cbar, "Cbar", torch.complex128)
    x = _host(rings, np.float64)
    if Cbar.numel() != (2 * mbmax + 1) * (lmax + 1) * x.size or Cbar.device != device:
        raise ValueError("Cbar must hold (2*mbmax+1, lmax+1, nring) values on the device of alm")
    if not want_alm and not want_blm:
        return None, None
    alm_bar = torch.empty_like(alm) if want_alm else None
    blm_bar = torch.empty_like(blm) if want_blm else None
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, _workspace_bytes(TC_OP_ADJ, lmax, mbmax, x, cos))
    rc = _fn("totalconv_adj", cos)(lmax, mbmax, x.size, _hptr(x), _dptr(alm), _dptr(blm), _dptr(Cbar),
                                   _dptr(alm_bar), _dptr(blm_bar), _dptr(ws), ws.numel(), stream)
    _check("totalconv_adj" + ("_x" if cos else ""), rc)
    return alm_bar, blm_bar


def totalconv_adj(lmax: int, mbmax: int, beta, alm, blm, Cbar, want_alm=True, want_blm=True):
    """(alm_bar, blm_bar) for the cotangent Cbar = dL/dconj(C); either may be None."""
    return _totalconv_adj(lmax, mbmax, beta, False, alm, blm, Cbar, want_alm, want_blm)


def totalconv_adj_x(lmax: int, mbmax: int, cosbeta, alm, blm, Cbar, want_alm=True, want_blm=True):
    """totalconv_adj on ring cosines."""
    return _totalconv_adj(lmax, mbmax, cosbeta, True, alm, blm, Cbar, want_alm, want_blm)


def _ptr_array(ts):
    arr = (ctypes.c_void_p * max(len(ts), 1))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr() if t is not None else None
    return arr


def _pol_inputs(torch, lmax, mbmax, alms, blms):
    alms, blms = list(alms), list(blms)
    if not 1 <= len(alms) <= 3 or len(blms) != len(alms):
        raise ValueError("1 to 3 (alm, blm) pairs are required")
    device = None
    for i, (a, b) in enumerate(zip(alms, blms)):
        device = _sky_beam(torch, lmax, mbmax, a, b, device, f"s[{i}]")
    return alms, blms


def _totalconv_fwd_pol(lmax, mbmax, rings, cos, alms, blms, mode):
    import torch
    alms, blms = _pol_inputs(torch, lmax, mbmax, alms, blms)
    device = alms[0].device
    x = _host(rings, np.float64)
    nout = 1 if mode == TC_POL_SUM else len(alms)
    outs = [torch.empty((2 * mbmax + 1, lmax + 1, x.size), dtype=torch.complex128, device=device)
            for _ in range(nout)]
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, _workspace_bytes(TC_OP_FWD_POL, lmax, mbmax, x, cos))
    rc = _fn("totalconv_fwd_pol", cos)(lmax, mbmax, x.size, _hptr(x), len(alms), _ptr_array(alms),
                                       _ptr_array(blms), mode, _ptr_array(outs), _dptr(ws), ws.numel(), stream)
    _check("totalconv_fwd_pol" + ("_x" if cos else ""), rc)
    return outs


def totalconv_fwd_pol(lmax: int, mbmax: int, beta, alms, blms, mode=TC_POL_SEPARATE):
    """Polarised convolution of 1-3 (alm, blm) pairs sharing one recursion.  Returns a list of
    one C per pair (TC_POL_SEPARATE) or a list holding the summed C (TC_POL_SUM)."""
    return _totalconv_fwd_pol(lmax, mbmax, beta, False, alms, blms, mode)


def totalconv_fwd_pol_x(lmax: int, mbmax: int, cosbeta, alms, blms, mode=TC_POL_SEPARATE):
    """totalconv_fwd_pol on ring cosines."""
    return _totalconv_fwd_pol(lmax, mbmax, cosbeta, True, alms, blms, mode)


def _totalconv_adj_pol(lmax, mbmax, rings, cos, alms, blms, Cbars, mode, want_alm, want_blm):
    import torch
    alms, blms = _pol_inputs(torch, lmax, mbmax, alms, blms)
    Cbars = list(Cbars)
    x = _host(rings, np.float64)
    if len(Cbars) != (1 if mode == TC_POL_SUM else len(alms)):
        raise ValueError("one cotangent per output is required")
    device = alms[0].device
    for i, g in enumerate(Cbars):
        _require_device(g, f"Cbars[{i}]", torch.complex128)
        if g.numel() != (2 * mbmax + 1) * (lmax + 1) * x.size or g.device != device:
            raise ValueError("each Cbar must hold (2*mbmax+1, lmax+1, nring) values on the device of alm")
    abar = [torch.empty_like(a) if want_alm else None for a in alms]
    bbar = [torch.empty_like(b) if want_blm else None for b in blms]
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, _workspace_bytes(TC_OP_ADJ, lmax, mbmax, x, cos))
    rc = _fn("totalconv_adj_pol", cos)(lmax, mbmax, x.size, _hptr(x), len(alms), _ptr_array(alms),
                                       _ptr_array(blms), mode, _ptr_array(Cbars),
                                       _ptr_array(abar) if want_alm else None,
                                       _ptr_array(bbar) if want_blm else None, _dptr(ws), ws.numel(), stream)
    _check("totalconv_adj_pol" + ("_x" if cos else ""), rc)
    return abar, bbar


def totalconv_adj_pol(lmax: int, mbmax: int, beta, alms, blms, Cbars, mode=TC_POL_SEPARATE,
                      want_alm=True, want_blm=True):
    """Gradients ([alm_bar per pair], [blm_bar per pair]) of totalconv_fwd_pol for the cotangents
    Cbars (one per output); entries are None when not requested."""
    return _totalconv_adj_pol(lmax, mbmax, beta, False, alms, blms, Cbars, mode, want_alm, want_blm)


def totalconv_adj_pol_x(lmax: int, mbmax: int, cosbeta, alms, blms, Cbars, mode=TC_POL_SEPARATE,
                        want_alm=True, want_blm=True):
    """totalconv_adj_pol on ring cosines."""
    return _totalconv_adj_pol(lmax, mbmax, cosbeta, True, alms, blms, Cbars, mode, want_alm, want_blm)


def totalconv_datacube(lmax: int, mbmax: int, C, nalpha: int, ngamma: int, out=None):
    """Data cube c(alpha_a, beta_j, gamma_g) of eq. conviqt from the coefficients C
    (complex128 (2*mbmax+1, lmax+1, nring) on the GPU); float64 (nring, nalpha, ngamma)."""
    import torch
    _require_device(C, "C", torch.complex128)
    if C.dim() != 3 or tuple(C.shape[:2]) != (2 * mbmax + 1, lmax + 1):
        raise ValueError("C must have shape (2*mbmax+1, lmax+1, nring)")
    nring = C.shape[2]
    shape = (nring, nalpha, ngamma)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=C.device)
    else:
        _require_device(out, "out", torch.float64)
        if tuple(out.shape) != shape:
            raise ValueError(f"out must have shape {shape}")
    stream = _stream_handle(torch, C.device)
    nbytes = int(lib().totalconv_datacube_workspace_bytes(lmax, mbmax, nring, nalpha, ngamma))
    ws = workspace_cache.get(torch, C.device, stream, nbytes)
    rc = lib().totalconv_datacube(lmax, mbmax, nring, _dptr(C), nalpha, ngamma, _dptr(out), _dptr(ws),
                                  ws.numel(), stream)
    _check("totalconv_datacube", rc)
    return out


def datacube_ring_chunk(lmax: int, mbmax: int, nring: int, nalpha: int, ngamma: int) -> int:
    """Rings the data cube processes per chunk (0 for sizes it refuses)."""
    return int(lib().totalconv_datacube_ring_chunk(lmax, mbmax, nring, nalpha, ngamma))


def set_tile(op: int, R: int):
    """Chains per lane (R) for later calls of `op` in this process; 0 restores the default."""
    _check("tc_set_tile", lib().tc_set_tile(op, R))


def get_tile(op: int, lmax: int) -> int:
    return int(lib().tc_get_tile(op, lmax))


def set_tile_ex(op: int, R: int = 0, TB: int = 0, TR: int = 0):
    """Chains per lane R, l-block TB and adjoint reduction block TR for later calls; 0 = built-in."""
    _check("tc_set_tile_ex", lib().tc_set_tile_ex(op, R, TB, TR))


def get_tile_ex(op: int, lmax: int):
    R, TB, TR = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check("tc_get_tile_ex", lib().tc_get_tile_ex(op, lmax, ctypes.byref(R), ctypes.byref(TB), ctypes.byref(TR)))
    return R.value, TB.value, TR.value


def timing_enable(n: int):
    """Record HIP events around the recursion kernel of the next calls (n pairs per op; 0 = off)."""
    _check("tc_timing_enable", lib().tc_timing_enable(n))


def timing_read(op: int, n: int):
    """Kernel durations (ms) of the last n recorded calls of `op`, oldest first."""
    buf = (ctypes.c_float * max(n, 1))()
    k = lib().tc_timing_read(op, buf, n)
    if k < 0:
        raise TotalConvError("tc_timing_read", k, last_error())
    return [float(buf[i]) for i in range(k)]


class Plan:
    """A batched plan (tc_plan_create): many detectors, one shared sky, one graph launch.

    detectors: list of dicts with keys lmax, mbmax, beta (host colatitudes) or cosbeta (host
    ring cosines), blm (device complex128), and C (forward output) or Cbar / blm_bar (adjoint
    input / output)."""

    def __init__(self, op: int, detectors, lmax_sky: int, alm, alm_bar=None):
        import torch
        if op not in (TC_OP_FWD, TC_OP_ADJ):
            raise ValueError("plans support TC_OP_FWD and TC_OP_ADJ")
        _require_device(alm, "alm", torch.complex128)
        if alm.numel() != (lmax_sky + 1) * (lmax_sky + 2) // 2:
            raise ValueError("alm size does not match lmax_sky")
        if alm_bar is not None:
            _require_device(alm_bar, "alm_bar", torch.complex128)
            if alm_bar.shape != alm.shape or alm_bar.device != alm.device:
                raise ValueError("alm_bar must have the shape and device of alm")
        self._keep = []
        arr = (TcDetector * len(detectors))()
        for i, d in enumerate(detectors):
            L, M = d["lmax"], d["mbmax"]
            if (d.get("beta") is None) == (d.get("cosbeta") is None):
                raise ValueError(f"detector {i}: give exactly one of beta and cosbeta")
            x = _host(d["beta"] if d.get("beta") is not None else d["cosbeta"], np.float64)
            self._keep.append(x)
            shape = (2 * M + 1, L + 1, x.size)
            need = [("blm", (2 * M + 1) * (L + 1))]
            if op == TC_OP_FWD:
                need.append(("C", int(np.prod(shape))))
            else:
                need.append(("Cbar", int(np.prod(shape))))
                if d.get("blm_bar") is not None:
                    need.append(("blm_bar", (2 * M + 1) * (L + 1)))
            for key, n in need:
                if not 0 <= M <= L <= lmax_sky:
                    break          # the library reports the range error
                t = d.get(key)
                if t is None:
                    raise ValueError(f"detector {i}: {key} is required")
                _require_device(t, f"detector {i} {key}", torch.complex128)
                if t.numel() != n or t.device != alm.device:
                    raise ValueError(f"detector {i}: {key} must hold {n} values on the device of alm")
            arr[i].lmax = L
            arr[i].mbmax = M
            arr[i].nring = x.size
            arr[i].beta = _hptr(x).value if d.get("beta") is not None else None
            arr[i].cosbeta = _hptr(x).value if d.get("beta") is None else None
            arr[i].blm = d["blm"].data_ptr()
            arr[i].C = d["C"].data_ptr() if d.get("C") is not None else None
            arr[i].Cbar = d["Cbar"].data_ptr() if d.get("Cbar") is not None else None
            arr[i].blm_bar = d["blm_bar"].data_ptr() if d.get("blm_bar") is not None else None
        self._dets = detectors
        self._alm, self._alm_bar = alm, alm_bar
        self.device = alm.device
        handle = ctypes.c_void_p()
        stream = _stream_handle(torch, self.device)
        rc = lib().tc_plan_create(ctypes.byref(handle), op, len(detectors), arr, lmax_sky,
                                  _dptr(alm), _dptr(alm_bar), stream)
        _check("tc_plan_create", rc)
        self._h = handle

    @property
    def tile(self) -> int:
        return int(lib().tc_plan_tile(self._h))

    @property
    def device_bytes(self) -> int:
        return int(lib().tc_plan_device_bytes(self._h))

    def execute(self):
        import torch
        _check("tc_plan_execute", lib().tc_plan_execute(self._h, _stream_handle(torch, self.device)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
