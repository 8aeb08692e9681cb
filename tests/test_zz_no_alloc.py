"""totalconv_fwd_noalloc (the forward for callers that cannot allocate device memory: its tables
in the library's static device array) against totalconv_fwd (caller workspace), through the C
ABI: equal bit for bit (the same kernels on the same tables), on two calls in a row, the second
with a smaller input, so that what the first call left in the array cannot leak into the second;
and a request whose tables exceed the array is refused on the host."""
import sys

import numpy as np
import pytest

from paper_1002_1050_amd import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1002_1050_amd import _binding
    _binding.lib()
    return _binding


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_noalloc_forward_equals_workspace_forward(B):
    for (L, M, nring, seed) in [(600, 9, 1200, 1), (90, 3, 151, 2)]:      # the second call is smaller
        beta = S.ring_colatitudes(nring)
        alm = dev(S.sky_alm(L, seed) + 0.0j)
        blm = dev(S.random_beam(L, M, seed + 10))
        say(f"totalconv_fwd_noalloc L={L} M={M} nring={nring}")
        out = torch.full((2 * M + 1, L + 1, nring), complex("nan"), dtype=torch.complex128, device="cuda")
        B.totalconv_fwd_noalloc(L, M, beta, alm, blm, out)
        ref = B.totalconv_fwd(L, M, beta, alm, blm)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), "no-allocation forward differs from the workspace forward"


def test_noalloc_forward_refuses_tables_beyond_its_array(B):
    L, M, nring = 16384, 64, 65536           # column tables alone about 50 MB
    alm = torch.zeros(1, dtype=torch.complex128, device="cuda")
    lib = B.lib()
    beta = S.ring_colatitudes(nring)
    rc = lib.totalconv_fwd_noalloc(L, M, nring, B._hptr(beta), B._dptr(alm), B._dptr(alm), B._dptr(alm), None)
    assert rc == B.TC_ENOMEM and "static device array" in B.last_error()
