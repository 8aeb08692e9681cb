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
                ("cosbeta", ctypes.c_void_p), ("blm", ctypes.c_void_p), ("C", ctypes.c_void_p),
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
            L.totalconv_workspace_bytes_rings.restype = S
            L.totalconv_workspace_bytes_rings.argtypes = [I, I, I, I, P]
            L.wigner_d_rings.restype = I
            L.wigner_d_rings.argtypes = [I, I, P, P, I, P, P, P, S, P]
            L.totalconv_fwd.restype = I
            L.totalconv_fwd.argtypes = [I, I, I, P, P, P, P, P, S, P]
            L.totalconv_adj.restype = I
            L.totalconv_adj.argtypes = [I, I, I, P, P, P, P, P, P, P, S, P]
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
            PP = ctypes.POINTER(P)
            L.totalconv_fwd_pol.restype = I
            L.totalconv_fwd_pol.argtypes = [I, I, I, P, I, PP, PP, I, PP, P, S, P]
            L.totalconv_adj_pol.restype = I
            L.totalconv_adj_pol.argtypes = [I, I, I, P, I, PP, PP, I, PP, PP, PP, P, S, P]
            L.wigner_d_matrix_workspace_bytes.restype = S
            L.wigner_d_matrix_workspace_bytes.argtypes = [I, I]
            L.wigner_d_matrix.restype = I
            L.wigner_d_matrix.argtypes = [I, I, P, P, P, S, P]
            L.totalconv_datacube_workspace_bytes.restype = S
            L.totalconv_datacube_workspace_bytes.argtypes = [I, I, I, I, I]
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


def workspace_bytes(op: int, lmax: int, mbmax: int, cosbeta) -> int:
    """Exact workspace size for this ring set; 0 when the arguments are invalid (the entry
    point itself then reports why)."""
    x = _host(cosbeta, np.float64)
    return int(lib().totalconv_workspace_bytes_rings(op, lmax, mbmax, x.size, _hptr(x)))


def wigner_d_rings(lmax: int, mb, msky, cosbeta, device="cuda"):
    """d^l_{mb[i],msky[i]}(beta_j) on the GPU, shape (npair, lmax+1, nring) float64."""
    import torch
    device = torch.device(device)
    mb = _host(np.atleast_1d(mb), np.int32)
    ms = _host(np.atleast_1d(msky), np.int32)
    x = _host(np.atleast_1d(cosbeta), np.float64)
    if mb.shape != ms.shape:
        raise ValueError("mb and msky must have the same length")
    out = torch.empty((mb.size, lmax + 1, x.size), dtype=torch.float64, device=device)
    nbytes = lib().totalconv_workspace_bytes(TC_OP_WIGNER, lmax, max(mb.size, 1), max(x.size, 1))
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, nbytes)
    rc = lib().wigner_d_rings(lmax, mb.size, _hptr(mb), _hptr(ms), x.size, _hptr(x), _dptr(out),
                              _dptr(ws), ws.numel(), stream)
    _check("wigner_d_rings", rc)
    return out


def wigner_d_matrix(l: int, cosbeta, device="cuda", out=None):
    """Full matrix d^l_{m m'}(beta_j), -l <= m, m' <= l: float64 (nring, 2l+1, 2l+1) on the GPU."""
    import torch
    device = torch.device(device)
    x = _host(np.atleast_1d(cosbeta), np.float64)
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
    rc = lib().wigner_d_matrix(l, x.size, _hptr(x), _dptr(out), _dptr(ws), ws.numel(), stream)
    _check("wigner_d_matrix", rc)
    return out


def totalconv_fwd(lmax: int, mbmax: int, cosbeta, alm, blm, out=None):
    """C = totalconv(alm, blm) on the rings cosbeta; complex128 (2*mbmax+1, lmax+1, nring)."""
    import torch
    _require_device(alm, "alm", torch.complex128)
    _require_device(blm, "blm", torch.complex128)
    device = alm.device
    x = _host(cosbeta, np.float64)
    if alm.numel() != (lmax + 1) * (lmax + 2) // 2 or blm.numel() != (2 * mbmax + 1) * (lmax + 1):
        raise ValueError("alm / blm sizes do not match lmax / mbmax")
    shape = (2 * mbmax + 1, lmax + 1, x.size)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex128, device=device)
    else:
        _require_device(out, "out", torch.complex128)
        if tuple(out.shape) != shape:
            raise ValueError(f"out must have shape {shape}")
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, workspace_bytes(TC_OP_FWD, lmax, mbmax, x))
    rc = lib().totalconv_fwd(lmax, mbmax, x.size, _hptr(x), _dptr(alm), _dptr(blm), _dptr(out),
                             _dptr(ws), ws.numel(), stream)
    _check("totalconv_fwd", rc)
    return out


def totalconv_adj(lmax: int, mbmax: int, cosbeta, alm, blm, Cbar, want_alm=True, want_blm=True):
    """(alm_bar, blm_bar) for the cotangent Cbar = dL/dconj(C); either may be None."""
    import torch
    for t, n in ((alm, "alm"), (blm, "blm"), (Cbar, "Cbar")):
        _require_device(t, n, torch.complex128)
    device = alm.device
    x = _host(cosbeta, np.float64)
    if Cbar.numel() != (2 * mbmax + 1) * (lmax + 1) * x.size:
        raise ValueError("Cbar size does not match (2*mbmax+1, lmax+1, nring)")
    alm_bar = torch.empty_like(alm) if want_alm else None
    blm_bar = torch.empty_like(blm) if want_blm else None
    if not want_alm and not want_blm:
        return None, None
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, workspace_bytes(TC_OP_ADJ, lmax, mbmax, x))
    rc = lib().totalconv_adj(lmax, mbmax, x.size, _hptr(x), _dptr(alm), _dptr(blm), _dptr(Cbar),
                             _dptr(alm_bar), _dptr(blm_bar), _dptr(ws), ws.numel(), stream)
    _check("totalconv_adj", rc)
    return alm_bar, blm_bar


def _ptr_array(ts):
    arr = (ctypes.c_void_p * max(len(ts), 1))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr() if t is not None else None
    return arr


def _pol_inputs(torch, lmax, mbmax, alms, blms):
    alms, blms = list(alms), list(blms)
    if not 1 <= len(alms) <= 3 or len(blms) != len(alms):
        raise ValueError("1 to 3 (alm, blm) pairs are required")
    for i, (a, b) in enumerate(zip(alms, blms)):
        _require_device(a, f"alms[{i}]", torch.complex128)
        _require_device(b, f"blms[{i}]", torch.complex128)
        if a.numel() != (lmax + 1) * (lmax + 2) // 2 or b.numel() != (2 * mbmax + 1) * (lmax + 1):
            raise ValueError(f"pair {i}: alm / blm sizes do not match lmax / mbmax")
    return alms, blms


def totalconv_fwd_pol(lmax: int, mbmax: int, cosbeta, alms, blms, mode=TC_POL_SEPARATE):
    """Polarised convolution of 1-3 (alm, blm) pairs sharing one recursion.  Returns a list of
    one C per pair (TC_POL_SEPARATE) or a list holding the summed C (TC_POL_SUM)."""
    import torch
    alms, blms = _pol_inputs(torch, lmax, mbmax, alms, blms)
    device = alms[0].device
    x = _host(cosbeta, np.float64)
    nout = 1 if mode == TC_POL_SUM else len(alms)
    outs = [torch.empty((2 * mbmax + 1, lmax + 1, x.size), dtype=torch.complex128, device=device)
            for _ in range(nout)]
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, workspace_bytes(TC_OP_FWD_POL, lmax, mbmax, x))
    rc = lib().totalconv_fwd_pol(lmax, mbmax, x.size, _hptr(x), len(alms), _ptr_array(alms), _ptr_array(blms),
                                 mode, _ptr_array(outs), _dptr(ws), ws.numel(), stream)
    _check("totalconv_fwd_pol", rc)
    return outs


def totalconv_adj_pol(lmax: int, mbmax: int, cosbeta, alms, blms, Cbars, mode=TC_POL_SEPARATE,
                      want_alm=True, want_blm=True):
    """Gradients ([alm_bar per pair], [blm_bar per pair]) of totalconv_fwd_pol for the cotangents
    Cbars (one per output); entries are None when not requested."""
    import torch
    alms, blms = _pol_inputs(torch, lmax, mbmax, alms, blms)
    Cbars = list(Cbars)
    x = _host(cosbeta, np.float64)
    if len(Cbars) != (1 if mode == TC_POL_SUM else len(alms)):
        raise ValueError("one cotangent per output is required")
    for i, g in enumerate(Cbars):
        _require_device(g, f"Cbars[{i}]", torch.complex128)
        if g.numel() != (2 * mbmax + 1) * (lmax + 1) * x.size:
            raise ValueError("Cbar size does not match (2*mbmax+1, lmax+1, nring)")
    device = alms[0].device
    abar = [torch.empty_like(a) if want_alm else None for a in alms]
    bbar = [torch.empty_like(b) if want_blm else None for b in blms]
    stream = _stream_handle(torch, device)
    ws = workspace_cache.get(torch, device, stream, workspace_bytes(TC_OP_ADJ, lmax, mbmax, x))
    rc = lib().totalconv_adj_pol(lmax, mbmax, x.size, _hptr(x), len(alms), _ptr_array(alms), _ptr_array(blms),
                                 mode, _ptr_array(Cbars), _ptr_array(abar) if want_alm else None,
                                 _ptr_array(bbar) if want_blm else None, _dptr(ws), ws.numel(), stream)
    _check("totalconv_adj_pol", rc)
    return abar, bbar


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

    detectors: list of dicts with keys lmax, mbmax, cosbeta (host array), blm (device
    complex128), and C (forward output) or Cbar / blm_bar (adjoint input / output)."""

    def __init__(self, op: int, detectors, lmax_sky: int, alm, alm_bar=None):
        import torch
        self._keep = []
        arr = (TcDetector * len(detectors))()
        for i, d in enumerate(detectors):
            x = _host(d["cosbeta"], np.float64)
            self._keep.append(x)
            arr[i].lmax = d["lmax"]
            arr[i].mbmax = d["mbmax"]
            arr[i].nring = x.size
            arr[i].cosbeta = _hptr(x).value
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
