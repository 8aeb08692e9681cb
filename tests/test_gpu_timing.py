"""Kernel timing events of the C ABI (tc_timing_enable / tc_timing_read)."""
import numpy as np
import pytest

from paper_1002_1050_amd import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_kernel_timing_records_each_call():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1002_1050_amd import _binding as B
    L, M = 200, 4
    x = S.ring_cosines(400)
    alm = torch.from_numpy(S.sky_alm(L, 3)).cuda()
    blm = torch.from_numpy(S.random_beam(L, M, 4)).cuda()
    G = torch.from_numpy(S.random_cbar(L, M, x.size, 5)).cuda()
    print(f"[gpu] timing events, lmax {L}", flush=True)
    B.timing_enable(3)
    try:
        C0 = B.totalconv_fwd_x(L, M, x, alm, blm)
        for _ in range(3):
            C = B.totalconv_fwd_x(L, M, x, alm, blm)
        B.totalconv_adj_x(L, M, x, alm, blm, G)
        torch.cuda.synchronize()
        f = B.timing_read(B.TC_OP_FWD, 8)
        a = B.timing_read(B.TC_OP_ADJ, 8)
        assert len(f) == 3 and len(a) == 1           # capacity 3: the last three forward calls
        assert all(0 < v < 1e4 for v in f + a)
        assert len(B.timing_read(B.TC_OP_FWD, 1)) == 1
        assert B.timing_read(B.TC_OP_WIGNER, 8) == []
        assert torch.equal(C, C0)                     # recording does not change results
    finally:
        B.timing_enable(0)
    assert B.timing_read(B.TC_OP_FWD, 8) == []
