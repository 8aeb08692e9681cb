"""The C-ABI library loads, exports every symbol include/*.h declares, and rejects
invalid arguments on the host before touching a GPU (no compute calls here)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    names.discard("defined")
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_1002_1050_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.fail("libtotalconv.so is not built (run python -m paper_1002_1050_amd.build)")
    return _binding.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert {"wigner_d_rings", "totalconv_fwd", "totalconv_adj", "totalconv_workspace_bytes"} <= set(names)
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"


def test_abi_version(L):
    assert L.tc_abi_version() == 2


def test_workspace_query(L):
    from paper_1002_1050_amd import _binding as B
    assert L.totalconv_workspace_bytes(B.TC_OP_FWD, 64, 4, 129) > 0
    assert L.totalconv_workspace_bytes(B.TC_OP_FWD, 64, 65, 129) == 0     # mbmax > lmax
    assert L.totalconv_workspace_bytes(B.TC_OP_FWD, -1, 0, 129) == 0
    assert L.totalconv_workspace_bytes(B.TC_OP_FWD, 16385, 0, 1) == 0
    assert L.totalconv_workspace_bytes(B.TC_OP_ADJ, 64, 4, 0) == 0
    assert L.totalconv_workspace_bytes(7, 64, 4, 10) == 0
    # the adjoint's partial sums dominate: two complex arrays per ring tile over the triangle
    from paper_1002_1050_amd import synthetic as S
    x = S.ring_cosines(8192)
    exact = B.workspace_bytes_x(B.TC_OP_ADJ, 4096, 14, x)
    upper = L.totalconv_workspace_bytes(B.TC_OP_ADJ, 4096, 14, 8192)
    assert 0 < exact <= upper
    assert exact >= 2 * 16 * 29 * 4097 * 4098 // 2


def _call_fwd(L, lmax, mbmax, x, ws_bytes=1 << 30, ws=0x100000):
    x = np.ascontiguousarray(x, np.float64)
    fake = ctypes.c_void_p(0x200000)       # never dereferenced: every call below fails on the host
    return L.totalconv_fwd_x(lmax, mbmax, x.size, x.ctypes.data_as(ctypes.c_void_p), fake, fake, fake,
                             ctypes.c_void_p(ws), ws_bytes, None)


def test_invalid_arguments_rejected_on_host(L):
    from paper_1002_1050_amd import _binding as B
    x = np.linspace(-1, 1, 11)
    assert _call_fwd(L, -1, 0, x) == -1 and "lmax" in B.last_error()
    assert _call_fwd(L, 10, 11, x) == -1 and "mbmax" in B.last_error()
    assert _call_fwd(L, 16385, 0, x) == -1
    bad = x.copy()
    bad[3] = 1.5
    assert _call_fwd(L, 10, 2, bad) == -1 and "cosbeta[3]" in B.last_error()
    bad[3] = np.nan
    assert _call_fwd(L, 10, 2, bad) == -1
    assert _call_fwd(L, 10, 2, x, ws_bytes=16) == -3 and "workspace" in B.last_error()
    assert _call_fwd(L, 10, 2, x, ws=0x100010) == -1 and "aligned" in B.last_error()
    fake = ctypes.c_void_p(0x200000)
    assert L.totalconv_fwd_x(10, 2, 0, None, fake, fake, fake, fake, 1 << 30, None) == -1
    assert L.totalconv_fwd(10, 2, 0, None, fake, fake, fake, fake, 1 << 30, None) == -1
    # wigner_d_rings: |msky| > lmax
    mb = np.array([0], np.int32)
    ms = np.array([11], np.int32)
    rc = L.wigner_d_rings_x(10, 1, mb.ctypes.data_as(ctypes.c_void_p), ms.ctypes.data_as(ctypes.c_void_p),
                            x.size, x.ctypes.data_as(ctypes.c_void_p), fake, fake, 1 << 30, None)
    assert rc == -1 and "msky" in B.last_error()
    # misaligned complex array
    rc = L.totalconv_fwd_x(10, 2, x.size, x.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(0x200008), fake,
                           fake, ctypes.c_void_p(0x100000), 1 << 30, None)
    assert rc == -1 and "aligned" in B.last_error()


def test_adjoint_nothing_requested_is_a_no_op(L):
    x = np.linspace(-1, 1, 5)
    fake = ctypes.c_void_p(0x200000)
    rc = L.totalconv_adj_x(4, 1, x.size, x.ctypes.data_as(ctypes.c_void_p), fake, fake, fake, None, None,
                           None, 0, None)
    assert rc == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1002_1050_amd import _binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        B.lib()


def test_timing_arguments_checked_on_host(L):
    buf = (ctypes.c_float * 4)()
    assert L.tc_timing_enable(-1) == -1
    assert L.tc_timing_enable(65537) == -1
    assert L.tc_timing_read(6, buf, 4) == -1
    assert L.tc_timing_read(-1, buf, 4) == -1
    assert L.tc_timing_read(1, None, 4) == -1
    assert L.tc_timing_read(1, buf, 4) == 0          # timing off: nothing recorded
    assert L.tc_timing_enable(0) == 0


def test_polarised_arguments_checked_on_host(L):
    from paper_1002_1050_amd import _binding as B
    x = np.linspace(-1, 1, 11)
    xp = x.ctypes.data_as(ctypes.c_void_p)
    fake = [0x200000, 0x300000, 0x400000]
    arr = (ctypes.c_void_p * 3)(*fake)
    ws = ctypes.c_void_p(0x100000)
    for npair, mode in ((0, 0), (4, 0), (2, 2), (2, -1)):
        assert L.totalconv_fwd_pol_x(10, 2, x.size, xp, npair, arr, arr, mode, arr, ws, 1 << 30, None) == -1
        assert L.totalconv_adj_pol_x(10, 2, x.size, xp, npair, arr, arr, mode, arr, arr, arr, ws, 1 << 30,
                                   None) == -1
    holed = (ctypes.c_void_p * 3)(fake[0], None, fake[2])
    assert L.totalconv_fwd_pol_x(10, 2, x.size, xp, 3, arr, holed, 0, arr, ws, 1 << 30, None) == -1
    assert "pair 1" in B.last_error()
    assert L.totalconv_fwd_pol_x(10, 2, x.size, xp, 3, arr, arr, 0, holed, ws, 1 << 30, None) == -1
    assert "output 1" in B.last_error()
    assert L.totalconv_fwd_pol_x(10, 2, x.size, xp, 2, None, arr, 0, arr, ws, 1 << 30, None) == -1
    # summed mode needs one cotangent only; nothing requested is a no-op
    one = (ctypes.c_void_p * 1)(fake[0])
    assert L.totalconv_adj_pol_x(10, 2, x.size, xp, 3, arr, arr, 1, one, None, None, ws, 1 << 30, None) == 0


def test_datacube_arguments_checked_on_host(L):
    from paper_1002_1050_amd import _binding as B
    fake = ctypes.c_void_p(0x200000)
    ws = ctypes.c_void_p(0x100000)
    ok = dict(lmax=10, mbmax=2, nring=4, nalpha=5, ngamma=32)
    assert L.totalconv_datacube_workspace_bytes(*ok.values()) > 0
    bad = [dict(ok, ngamma=24), dict(ok, ngamma=16), dict(ok, ngamma=32768), dict(ok, nalpha=0),
           dict(ok, nalpha=900), dict(ok, mbmax=11), dict(ok, lmax=8193, ngamma=16384), dict(ok, nring=0)]
    for b in bad:
        assert L.totalconv_datacube_workspace_bytes(*b.values()) == 0, b
        rc = L.totalconv_datacube(b["lmax"], b["mbmax"], b["nring"], fake, b["nalpha"], b["ngamma"], fake, ws,
                                  1 << 40, None)
        assert rc == -1, b
    assert L.totalconv_datacube(10, 2, 4, fake, 5, 32, fake, ws, 16, None) == -3
    assert L.totalconv_datacube(10, 2, 4, ctypes.c_void_p(0x200008), 5, 32, fake, ws, 1 << 40, None) == -1
    assert "aligned" in B.last_error()


def test_matrix_arguments_checked_on_host(L):
    from paper_1002_1050_amd import _binding as B
    x = np.array([0.3, 0.1])
    xp = x.ctypes.data_as(ctypes.c_void_p)
    fake = ctypes.c_void_p(0x200000)
    ws = ctypes.c_void_p(0x100000)
    assert L.wigner_d_matrix_workspace_bytes(10, 2) > 0
    assert L.wigner_d_matrix_workspace_bytes(-1, 2) == 0 and L.wigner_d_matrix_workspace_bytes(10, 0) == 0
    assert L.wigner_d_matrix_x(-1, 2, xp, fake, ws, 1 << 30, None) == -1
    assert L.wigner_d_matrix_x(16385, 2, xp, fake, ws, 1 << 30, None) == -1
    assert L.wigner_d_matrix_x(10, 2, xp, None, ws, 1 << 30, None) == -1
    assert L.wigner_d_matrix_x(10, 2, xp, ctypes.c_void_p(0x200004), ws, 1 << 30, None) == -1
    assert L.wigner_d_matrix_x(10, 2, xp, fake, ws, 16, None) == -3
    bad = np.array([0.3, 1.5])
    assert L.wigner_d_matrix_x(10, 2, bad.ctypes.data_as(ctypes.c_void_p), fake, ws, 1 << 30, None) == -1
    assert "cosbeta" in B.last_error()
    assert L.tc_set_tile(5, 3) == -1 and L.tc_set_tile(5, 2) == 0 and L.tc_get_tile(5, 10) == 2
    assert L.tc_set_tile(5, 0) == 0 and L.tc_get_tile(5, 10) == 1 and L.tc_get_tile(5, 2000) == 1


def test_cube_chunk_setting(L):
    full = L.totalconv_datacube_workspace_bytes(20, 3, 17, 7, 64)
    assert L.tc_set_tile(4, 3) == 0 and L.tc_get_tile(4, 0) == 3
    assert L.totalconv_datacube_workspace_bytes(20, 3, 17, 7, 64) < full
    assert L.tc_set_tile_ex(4, 3, 32, 0) == -1
    assert L.tc_set_tile(4, 0) == 0 and L.totalconv_datacube_workspace_bytes(20, 3, 17, 7, 64) == full


def test_binding_constants_match_the_header():
    """Every TC_* integer constant that the Python binding names has the header's value."""
    from paper_1002_1050_amd import _binding as B
    text = open(os.path.join(ROOT, "include", "totalconv.h")).read()
    defines = {m.group(1): int(m.group(2)) for m in
               re.finditer(r"#define\s+(TC_[A-Z_0-9]+)\s+\(?(-?\d+)\)?", text)}
    named = [n for n in dir(B) if n.startswith("TC_") and isinstance(getattr(B, n), int)]
    assert {"TC_ENOMEM", "TC_OP_ADJ", "TC_LMAX_LIMIT"} <= set(named)
    for n in named:
        assert n in defines, f"{n} is not defined in include/totalconv.h"
        assert getattr(B, n) == defines[n], n


def _call_fwd_beta(L, lmax, mbmax, beta, ws_bytes=1 << 30, ws=0x100000):
    beta = np.ascontiguousarray(beta, np.float64)
    fake = ctypes.c_void_p(0x200000)       # never dereferenced: every call below fails on the host
    return L.totalconv_fwd(lmax, mbmax, beta.size, beta.ctypes.data_as(ctypes.c_void_p), fake, fake, fake,
                           ctypes.c_void_p(ws), ws_bytes, None)


def test_colatitudes_rejected_on_host(L):
    """The entry points on colatitudes accept beta in [0, pi] (the poles included) and reject
    anything else before any GPU work; the ring-cosine twins keep their own check."""
    from paper_1002_1050_amd import _binding as B
    beta = np.linspace(0.0, np.pi, 9)
    for bad_value in (-1e-300, np.nextafter(np.pi, 4.0), np.nan, np.inf, 4.0):
        bad = beta.copy()
        bad[5] = bad_value
        assert _call_fwd_beta(L, 10, 2, bad) == -1 and "beta[5]" in B.last_error()
        out = np.full(bad.size, 7.0)
        assert L.tc_rings_from_beta(bad.size, bad.ctypes.data_as(ctypes.c_void_p),
                                    out.ctypes.data_as(ctypes.c_void_p)) == -1
        assert np.all(out == 7.0), "nothing is written on failure"
    assert _call_fwd_beta(L, 10, 2, beta, ws_bytes=16) == -3     # valid rings: the workspace check follows
    fake = ctypes.c_void_p(0x200000)
    mb = np.array([0], np.int32)
    rc = L.wigner_d_rings(10, 1, mb.ctypes.data_as(ctypes.c_void_p), mb.ctypes.data_as(ctypes.c_void_p),
                          2, np.array([0.1, -0.2]).ctypes.data_as(ctypes.c_void_p), fake, fake, 1 << 30, None)
    assert rc == -1 and "beta[1]" in B.last_error()
    assert L.tc_rings_from_beta(0, beta.ctypes.data_as(ctypes.c_void_p), beta.ctypes.data_as(ctypes.c_void_p)) == -1
    assert L.tc_rings_from_beta(2, None, beta.ctypes.data_as(ctypes.c_void_p)) == -1
    assert L.tc_rings_from_beta(2, beta.ctypes.data_as(ctypes.c_void_p), None) == -1
    # workspace size on colatitudes: as on the rings they give
    from paper_1002_1050_amd import synthetic as S
    b = S.ring_colatitudes(2048)
    assert B.workspace_bytes(B.TC_OP_ADJ, 1024, 9, b) == B.workspace_bytes_x(B.TC_OP_ADJ, 1024, 9, B.rings_from_beta(b))
    assert B.workspace_bytes(B.TC_OP_ADJ, 1024, 9, -b) == 0
