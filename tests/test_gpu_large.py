"""The large batched case at full size: four detectors at lmax 8192, mbmax 16 on the
16384-ring grid, sky C_l = 1/(l(l+1)+1) exp(-l^2/8192^2), seeded elliptical Gaussian beams.

The rings are processed in chunks of 4096 (2048 mirror pairs, (j, 16383 - j)); C of one chunk
is 17.7 GB per detector.  Each test runs a batched plan (one persistent launch over the four
detectors) on one full chunk:
* forward, on the polar and on the equatorial chunk: sampled columns, covering every mb and
  every msky decile, against the oracle over all 4096 rings (per-column gate 1e-11, widened by the epsilon skip's own bound
  for columns that are cold on every ring of the chunk), and the plain call bitwise equal to
  the plan on detector 0;
* adjoint, on the equatorial and on the polar chunk, with a seeded Gaussian cotangent: sampled
  rows of the summed sky gradient against the oracle (every mb and ring of those msky rows,
  1e-11; on the polar chunk rows whose chains start deep below 2^-900 and fold during the walk),
  and the dot-product identities <G, C> = <sky_bar, a> (all detectors) and
  <G_d, C_d> = <b_d, beam_bar_d> (each detector; a property that holds at any size) for the beam
  gradients.
"""
import sys

import numpy as np
import pytest

from paper_1002_1050_amd import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W = S.WORKLOADS["large4"]
L, M, NRING = W.lmax, W.mbmax, W.nring
HALF = 2048                     # mirror pairs per chunk
GATE = 1e-11


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def chunk_rings(c):
    """Indices of chunk c: rings j with min(j, N-1-j) in [c HALF, (c+1) HALF), ascending, so
    that position p and 4095 - p hold a mirror pair."""
    j = np.arange(NRING)
    k = np.minimum(j, NRING - 1 - j)
    return np.nonzero((k >= c * HALF) & (k < (c + 1) * HALF))[0]


def need_memory(nbytes):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes:
        pytest.skip(f"needs {nbytes / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1002_1050_amd import _binding
    _binding.lib()
    return _binding


@pytest.fixture(scope="module")
def inputs(B):
    say(f"large4 inputs: sky lmax {L}, {len(W.detectors)} beams mbmax {M}")
    alm = W.alm()
    blms = [d.blm() for d in W.detectors]
    return alm, blms


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


SKIP = 2.0 ** -100              # level below which the method drops a term's d (Sec. 4.2.1)


def weight_sums(alm, blm, mb, ms):
    """sum_l |conj(b_{l,mb}) s_{l,msky}| over l >= max(|mb|, msky), per column."""
    out = np.empty(mb.size)
    for c in range(mb.size):
        m = int(ms[c])
        l0 = max(abs(int(mb[c])), m)
        start = S.alm_index(L, m, m)
        s = alm[start + (l0 - m):start + (L + 1 - m)]
        out[c] = float(np.sum(np.abs(blm[mb[c] + M, l0:]) * np.abs(s)))
    return out


def skip_aware_gate(got, ref, wsum, tag):
    """Per column: max_j |dC| <= 1e-11 max_j |C| + 2^-100 sum_l |w_l|.  The second term is the
    most the epsilon skip can drop (every dropped term has |d| < 2^-100); it is below the first
    for columns that are hot somewhere on the chunk and can exceed it only for columns that
    are cold on every ring of the chunk.  A column with no weight (zero beam row) must be
    exactly zero.  Returns the largest relative error over the columns whose skip bound is
    under a tenth of the relative gate, and their count."""
    err = np.abs(got - ref).max(axis=1)
    big = np.abs(ref).max(axis=1)
    skip = SKIP * wsum
    strict = (big > 0) & (skip <= 0.1 * GATE * big)
    for c in range(ref.shape[0]):
        say(f"    {tag} col {c}: max|C| {big[c]:.3e}  max|dC| {err[c]:.3e}  skip bound {skip[c]:.3e}"
            f"  {'strict' if strict[c] else 'skip-bounded'}")
    assert np.all(err <= GATE * big + skip), "column outside the gate"
    return (float((err[strict] / big[strict]).max()) if np.any(strict) else 0.0), int(strict.sum())


def sampled_columns(d, seed=8192):
    """Ten columns for detector d: one msky per decile of [0, L]; mb from the detector's share
    of [-M, M] (the mb with ((mb + M) // 2) % 4 == d: both parities, the beams being zero for
    odd mb), so the four detectors cover every mb."""
    rng = np.random.Generator(np.random.PCG64(seed + d))
    edges = np.linspace(0, L + 1, 11).astype(int)
    ms = np.array([rng.integers(edges[k], edges[k + 1]) for k in range(10)], np.int32)
    mbs = np.array([m for m in range(-M, M + 1) if ((m + M) // 2) % 4 == d])
    mb = np.array([mbs[k % mbs.size] for k in range(10)], np.int32)
    return mb, ms


# forward chunks: the polar one (chains start far below 2^-900 for most msky) and the one next to
# the equator (every column hot, the mirror pairs closest to pi/2)
FWD_CHUNKS = {"polar": 0, "equatorial": NRING // (2 * HALF) - 1}


@pytest.mark.parametrize("chunk", ["polar", "equatorial"])
def test_large4_batched_forward_chunk(B, orc, inputs, chunk):
    alm, blms = inputs
    rings = chunk_rings(FWD_CHUNKS[chunk])
    x = S.ring_cosines(NRING)[rings]
    shape = (2 * M + 1, L + 1, x.size)
    need_memory(5 * 16 * int(np.prod(shape)) + 2 * 10**9)
    a_d = dev(alm)
    dets = [{"lmax": L, "mbmax": M, "cosbeta": x, "blm": dev(b),
             "C": torch.empty(shape, dtype=torch.complex128, device="cuda")} for b in blms]
    say(f"large4 forward plan: {len(dets)} detectors, lmax {L}, mbmax {M}, {chunk} chunk of {x.size} rings")
    plan = B.Plan(B.TC_OP_FWD, dets, L, a_d)
    plan.execute()
    torch.cuda.synchronize()
    plan.close()
    worst = 0.0
    for d, det in enumerate(dets):
        mb, ms = sampled_columns(d)
        idx = torch.from_numpy(((mb + M) * (L + 1) + ms).astype(np.int64)).to("cuda")
        got = det["C"].reshape(-1, x.size).index_select(0, idx).cpu().numpy()
        if d == 0:
            say("  plain call, detector 0")
            plain = B.totalconv_fwd_x(L, M, x, a_d, det["blm"])
            same = torch.equal(plain.reshape(-1, x.size).index_select(0, idx).cpu(), torch.from_numpy(got))
            del plain
            assert same, "plain call differs from the batched plan"
        det["C"] = None
        torch.cuda.empty_cache()
        ref = orc.totalconv_fwd(L, M, x, alm, blms[d], cols=(mb, ms))
        say(f"  detector {d}: mb {mb.tolist()}, msky {ms.tolist()}")
        g, nhot = skip_aware_gate(got, ref, weight_sums(alm, blms[d], mb, ms), f"det {d}")
        say(f"  detector {d}: relative error {g:.3e} over {nhot} strictly gated columns")
        worst = max(worst, g)
    assert worst <= GATE


# msky rows of the summed sky gradient checked on each chunk: on the polar chunk, rows that turn
# hot within it, so that their chains start far below 2^-900, pass many rescales and fold (loading
# their cotangents) during the walk
ADJ_CHUNKS = {"equatorial": (NRING // (2 * HALF) - 1, [4096, 7000, 8000]),
              "polar": (0, [0, 700, 1500])}


@pytest.mark.parametrize("chunk", ["equatorial", "polar"])
def test_large4_batched_adjoint_chunk(B, orc, inputs, chunk):
    alm, blms = inputs
    c, msel = ADJ_CHUNKS[chunk]
    rings = chunk_rings(c)
    x = S.ring_cosines(NRING)[rings]
    shape = (2 * M + 1, L + 1, x.size)
    nC = 16 * int(np.prod(shape))
    P = (L + 1) * (L + 2) // 2
    plan_uv = 4 * 2 * 16 * (2 * M + 1) * P          # per-detector U and V of one ring tile
    need_memory(4 * nC + plan_uv + 2 * 10**9)
    a_d = dev(alm)
    dets = [{"lmax": L, "mbmax": M, "cosbeta": x, "blm": dev(b),
             "C": torch.empty(shape, dtype=torch.complex128, device="cuda")} for b in blms]
    say(f"large4 forward for the dot products: {chunk} chunk of {x.size} rings")
    plan = B.Plan(B.TC_OP_FWD, dets, L, a_d)
    plan.execute()
    torch.cuda.synchronize()
    plan.close()
    lhs = []
    for d, det in enumerate(dets):
        g = torch.Generator(device="cuda")
        g.manual_seed(7000 + d)
        det["Cbar"] = torch.randn(shape, dtype=torch.complex128, device="cuda", generator=g)
        lhs.append(torch.vdot(det["Cbar"].flatten(), det["C"].flatten()).item())
        det["C"] = None
        torch.cuda.empty_cache()
        det["blm_bar"] = torch.empty((2 * M + 1, L + 1), dtype=torch.complex128, device="cuda")
    alm_bar = torch.empty_like(a_d)
    say("large4 adjoint plan")
    plan = B.Plan(B.TC_OP_ADJ, dets, L, a_d, alm_bar)
    plan.execute()
    torch.cuda.synchronize()
    plan.close()
    # dot-product identities
    tot = sum(lhs)
    rhs_a = torch.vdot(alm_bar, a_d).item()
    say(f"  <G,C> = {tot:.9e}  <sky_bar,a> = {rhs_a:.9e}")
    assert abs(tot - rhs_a) <= GATE * abs(tot)
    for d, det in enumerate(dets):
        rhs_b = torch.sum(torch.conj(det["blm"]) * det["blm_bar"]).item()
        say(f"  detector {d}: <G,C> = {lhs[d]:.9e}  <b,beam_bar> = {rhs_b:.9e}")
        assert abs(lhs[d] - rhs_b) <= GATE * abs(lhs[d])
    # sampled rows of the summed sky gradient: every mb and ring of msky in msel
    nb = 2 * M + 1
    cols_mb = np.repeat(np.arange(-M, M + 1), len(msel)).astype(np.int32)
    cols_ms = np.tile(np.array(msel), nb).astype(np.int32)
    idx = torch.from_numpy(((cols_mb + M) * (L + 1) + cols_ms).astype(np.int64)).to("cuda")
    ref = {m: np.zeros(L + 1 - m, np.complex128) for m in msel}
    for d, det in enumerate(dets):
        Gs = det["Cbar"].reshape(-1, x.size).index_select(0, idx).cpu().numpy()
        det["Cbar"] = None
        torch.cuda.empty_cache()
        say(f"  oracle column sums, detector {d}")
        u = orc.column_sums(L, M, x, Gs, (cols_mb, cols_ms))
        u = (u[..., 0].astype(np.float64) + 1j * u[..., 1].astype(np.float64)).reshape(nb, len(msel), L + 1)
        for k, m in enumerate(msel):
            ref[m] += (blms[d][:, m:] * u[:, k, m:]).sum(axis=0)
    ga = alm_bar.cpu().numpy()
    worst = 0.0
    for m in msel:
        start = S.alm_index(L, m, m)
        got = ga[start:start + L + 1 - m]
        e = float(np.linalg.norm(got - ref[m]) / np.linalg.norm(ref[m]))
        say(f"  sky-gradient row msky={m}: rel {e:.3e}")
        worst = max(worst, e)
    assert worst <= GATE
