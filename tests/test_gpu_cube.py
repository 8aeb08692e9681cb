"""Data cube (Sec. 4.1, eq. conviqt) on the GPU against the oracle's term-by-term double
sum, through the C ABI.  Gate: per ring, max |dc| / max |c_oracle| <= 1e-12 for the cube
stage alone (seeded random C on both sides), 1e-11 end to end (forward + cube)."""
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


def random_C(L, M, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((2 * M + 1, L + 1, n)) + 1j * rng.standard_normal((2 * M + 1, L + 1, n))


def ring_gate(got, ref):
    num = np.abs(got - ref).reshape(got.shape[0], -1).max(axis=1)
    den = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1)
    return float((num / den).max())


# (lmax, mbmax, nring, nalpha, ngamma): every final radix (2, 4, 8, none), the Nyquist fold
# ngamma = 2 lmax, the smallest grids and the largest FFT (ngamma 16384, 8192-point half length)
CASES = [(1, 0, 3, 1, 2), (2, 1, 5, 3, 4), (8, 2, 17, 5, 16), (20, 3, 9, 7, 64), (31, 4, 6, 9, 64),
         (64, 5, 4, 11, 128), (100, 6, 3, 13, 512), (128, 2, 2, 5, 256), (300, 4, 2, 9, 1024),
         (1000, 3, 2, 7, 2048), (10, 2, 2, 3, 16384), (40, 14, 20, 29, 128), (5, 5, 33, 40, 16)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "L%d_M%d_n%d_a%d_g%d" % c)
def test_cube_stage_against_oracle(B, orc, case):
    L, M, n, Na, Ng = case
    C = random_C(L, M, n, 1000 + L)
    say(f"datacube L={L} M={M} nring={n} nalpha={Na} ngamma={Ng}")
    got = B.totalconv_datacube(L, M, torch.from_numpy(C).cuda(), Na, Ng).cpu().numpy()
    ref = orc.datacube(L, M, C, Na, Ng)
    g = ring_gate(got, ref)
    say(f"  ring gate {g:.2e}")
    assert g <= 1e-12


def test_cube_full_lmax4096_rows_sampled(B, orc):
    """The lmax 4096 / mbmax 14 row shape of the benchmark (nalpha 29, ngamma 8192, 4096-point
    half-length FFT) on 48 rings, sampled points against the oracle."""
    L, M, n, Na, Ng = 4096, 14, 48, 29, 8192
    C = random_C(L, M, n, 4096)
    say("datacube lmax 4096 rows")
    got = B.totalconv_datacube(L, M, torch.from_numpy(C).cuda(), Na, Ng).cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(9))
    j = rng.integers(0, n, 120)
    a = rng.integers(0, Na, 120)
    g = rng.integers(0, Ng, 120)
    g[:4] = [0, Ng // 2, 1, Ng - 1]
    ref = orc.datacube(L, M, C, Na, Ng, points=(j, a, g))
    scale = np.abs(got).max()
    err = np.abs(got[j, a, g] - ref).max() / scale
    say(f"  sampled error / max|c| {err:.2e}")
    assert err <= 1e-12


def test_cube_end_to_end_from_the_forward(B, orc):
    L, M, n, Na, Ng = 90, 4, 64, 9, 256
    x = S.ring_cosines(n)
    alm = S.sky_alm(L, 21)
    blm = S.beam_blm(L, M, 30.0, 0.2)
    say("forward + datacube end to end")
    Cg = B.totalconv_fwd_x(L, M, x, torch.from_numpy(alm).cuda(), torch.from_numpy(blm).cuda())
    got = B.totalconv_datacube(L, M, Cg, Na, Ng).cpu().numpy()
    ref = orc.datacube(L, M, orc.totalconv_fwd(L, M, x, alm, blm), Na, Ng)
    gate = ring_gate(got, ref)
    say(f"  ring gate {gate:.2e}")
    assert gate <= 1e-11


def test_cube_rejects_bad_grids(B):
    C = torch.zeros((5, 11, 4), dtype=torch.complex128, device="cuda")
    for Na, Ng in ((3, 12), (3, 16), (0, 32), (3, 32768)):
        with pytest.raises(B.TotalConvError):
            B.totalconv_datacube(10, 2, C, Na, Ng)      # ngamma not a power of two >= 2 lmax, ...
    with pytest.raises(B.TotalConvError, match="nalpha"):
        B.totalconv_datacube(10, 2, C, 900, 32)        # nalpha * (2 mbmax + 1) > 4096


def test_cube_ring_chunks_give_the_same_cube(B):
    """Rings processed in chunks (here 3 at a time, 6 chunks through the two alpha-sum buffers,
    the FFTs of each chunk on the library's second stream) give the one-chunk cube bit for bit,
    call after call (one timing record per call)."""
    L, M, n, Na, Ng = 20, 3, 17, 7, 64
    C = torch.from_numpy(random_C(L, M, n, 77)).cuda()
    assert B.datacube_ring_chunk(L, M, n, Na, Ng) == n            # one chunk by default
    whole = B.totalconv_datacube(L, M, C, Na, Ng).clone()
    B.set_tile(B.TC_OP_CUBE, 3)
    try:
        assert B.datacube_ring_chunk(L, M, n, Na, Ng) == 3
        B.timing_enable(16)
        for _ in range(3):
            out = torch.full((n, Na, Ng), float("nan"), dtype=torch.float64, device="cuda")
            chunked = B.totalconv_datacube(L, M, C, Na, Ng, out=out)
            torch.cuda.synchronize()
            assert torch.equal(whole, chunked)
        assert len(B.timing_read(B.TC_OP_CUBE, 16)) == 3
    finally:
        B.timing_enable(0)
        B.set_tile(B.TC_OP_CUBE, 0)


def test_cube_full_size_from_the_forward_sampled(B, orc):
    """The benchmark's cube launch at full size: the forward's C at lmax 4096, mbmax 14 on all
    8192 rings (eight ring chunks), nalpha 29, ngamma 8192.  Sampled points, on rings on both
    sides of the chunk boundaries, against the oracle's double sum over the same C rows; gate
    per ring relative to that ring's max |c|."""
    w = S.WORKLOADS["lmax4096"]
    L, M, x = w.lmax, w.mbmax, w.xring()
    Na, Ng = 2 * M + 1, 2 * L
    C = B.totalconv_fwd_x(L, M, x, torch.from_numpy(w.alm()).cuda(), torch.from_numpy(w.blm()).cuda())
    say(f"datacube full size L={L} M={M} nring={x.size} nalpha={Na} ngamma={Ng}")
    cube = B.totalconv_datacube(L, M, C, Na, Ng)
    torch.cuda.synchronize()
    chunk = B.datacube_ring_chunk(L, M, x.size, Na, Ng)
    assert 16 <= chunk < x.size
    nchunk = -(-x.size // chunk)
    rings = np.unique(np.clip(np.array([0, chunk - 1, chunk, 3 * chunk + 5, x.size // 2, x.size - 1]), 0, x.size - 1))
    say(f"  {nchunk} ring chunks; sampled rings {rings.tolist()}")
    sel = torch.from_numpy(rings).cuda()
    Cs = C.index_select(2, sel).cpu().numpy()
    rows = cube.index_select(0, sel)
    scale = rows.abs().reshape(rings.size, -1).max(dim=1).values.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(8192))
    k = np.repeat(np.arange(rings.size), 40)
    a = rng.integers(0, Na, k.size)
    g = rng.integers(0, Ng, k.size)
    g[:4] = [0, Ng // 2, 1, Ng - 1]
    got = rows.cpu().numpy()[k, a, g]
    del C, cube, rows
    torch.cuda.empty_cache()
    ref = orc.datacube(L, M, Cs, Na, Ng, points=(k, a, g))
    err = float((np.abs(got - ref) / scale[k]).max())
    say(f"  {k.size} points: max |dc| / max|c| of the ring {err:.2e}")
    assert nchunk > 1 and err <= 1e-12
