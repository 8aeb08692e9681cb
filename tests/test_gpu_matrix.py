"""Full reduced Wigner matrix at one l (Sec. 3.1) on the GPU against the oracle's
d^l_{m m'} (the l-recursion in long double, pinned to Wigner's explicit sum and the
Jacobi form), through the C ABI.  Gate: absolute error (|d| <= 1), 1e-12 up to l = 300,
1e-10 up to l = 4096, 3e-10 at l = 8192 (the d gate of wigner_d_rings); plus the
orthogonality d d^T = 1 of every matrix as a property at any size."""
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
    yield _binding
    _binding.set_tile(_binding.TC_OP_MATRIX, 0)


# poles, the equator, rings a hair away from the poles, and ordinary rings
RINGS = np.array([1.0, -1.0, 0.0, 1 - 2.0 ** -40, -(1 - 2.0 ** -40), 0.37, -0.81, 0.9999, 2.0 ** -30])


def all_pairs(l):
    m = np.repeat(np.arange(-l, l + 1), 2 * l + 1)
    mp = np.tile(np.arange(-l, l + 1), 2 * l + 1)
    return m, mp


@pytest.mark.parametrize("l", [0, 1, 2, 7, 40, 300])
def test_matrix_small_l_every_element(B, orc, l):
    say(f"wigner_d_matrix l={l} nring={RINGS.size}")
    got = B.wigner_d_matrix_x(l, RINGS).cpu().numpy()
    m, mp = all_pairs(l)
    ref = orc.wigner_d(l, m, mp, RINGS)[:, l, :]                   # [pair][ring]
    ref = ref.T.reshape(RINGS.size, 2 * l + 1, 2 * l + 1)
    err = np.abs(got - ref).max()
    say(f"  max abs err {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("l,gate", [(4096, 1e-10), (8192, 3e-10)])
def test_matrix_large_l_sampled_and_orthogonal(B, orc, l, gate):
    x = RINGS[[2, 3, 5, 6, 7]]
    say(f"wigner_d_matrix l={l} nring={x.size}")
    got = B.wigner_d_matrix_x(l, x)
    rng = np.random.Generator(np.random.PCG64(l))
    m = np.concatenate([rng.integers(-l, l + 1, 400), np.full(40, l), np.full(40, 0), np.arange(-20, 20)])
    mp = np.concatenate([rng.integers(-l, l + 1, 400), rng.integers(-l, l + 1, 40), rng.integers(-l, l + 1, 40),
                         np.arange(-20, 20)[::-1]])
    ref = orc.wigner_d(l, m, mp, x)[:, l, :]
    g = got.cpu().numpy()[:, m + l, mp + l].T
    err = np.abs(g - ref).max()
    say(f"  sampled max abs err {err:.2e}")
    assert err <= gate
    for j in range(x.size):                                      # d(beta) is orthogonal
        dj = got[j]
        e = (dj @ dj.T - torch.eye(2 * l + 1, dtype=torch.float64, device=dj.device)).abs().max().item()
        say(f"  ring {j}: max |d d^T - 1| {e:.2e}")
        assert e <= 10 * gate


def test_matrix_tiles_agree(B):
    """The built-in two-wave workgroups (128-step flushes, a partial last row tile at l 1500) and
    the one-wave R 1 and R 2 builds write the same matrix bit for bit, poles included."""
    l = 1500
    x = np.concatenate([RINGS[2:7], [1.0, -1.0]])
    B.set_tile(B.TC_OP_MATRIX, 0)
    c = B.wigner_d_matrix_x(l, x)
    B.set_tile(B.TC_OP_MATRIX, 1)
    a = B.wigner_d_matrix_x(l, x)
    B.set_tile(B.TC_OP_MATRIX, 2)
    b = B.wigner_d_matrix_x(l, x)
    B.set_tile(B.TC_OP_MATRIX, 0)
    assert torch.equal(a, b) and torch.equal(a, c)


def test_matrix_benchmark_launch_sampled(B, orc):
    """The benchmark's launch: the full matrix at l = 4096 on its 16 rings (every ring, both
    sides, all row tiles), sampled elements of every ring against the oracle."""
    l, nring = 4096, 16
    x = S.ring_cosines(2 * nring + 1)[1:nring + 1]
    say(f"wigner_d_matrix l={l} nring={nring} (benchmark rings)")
    got = B.wigner_d_matrix_x(l, x)
    rng = np.random.Generator(np.random.PCG64(16 * l))
    m = np.concatenate([rng.integers(-l, l + 1, 300), [l, -l, 0, l, -l], np.arange(l - 70, l + 1)])
    mp = np.concatenate([rng.integers(-l, l + 1, 300), [l, -l, 0, -l, l], rng.integers(-l, l + 1, 71)])
    ref = orc.wigner_d(l, m, mp, x)[:, l, :]
    g = got.cpu().numpy()[:, m + l, mp + l].T
    err = np.abs(g - ref).max()
    say(f"  {m.size} elements x {nring} rings: max abs err {err:.2e}")
    assert err <= 1e-10
