"""Host logic of bench.py that runs without a GPU: the one-GPU contract, the traffic lookup and
the algorithmic flop count per term."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1002_1050_amd import synthetic as S  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_traffic_only_for_the_measured_source_and_tile(monkeypatch):
    import hashlib
    src = os.path.join(ROOT, "paper_1002_1050_amd", "csrc", "tc_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if sha not in bench.MEASURED_TRAFFIC["kernel_source_sha256"]:   # counters of an older source: null
        for kernel, tiles in bench.MEASURED_TRAFFIC["lmax4096"].items():
            for key in tiles:
                assert bench.hbm_traffic(kernel, "lmax4096", tuple(int(v) for v in key.split(","))) is None
        monkeypatch.setitem(bench.MEASURED_TRAFFIC, "kernel_source_sha256", [sha])
    table = bench.MEASURED_TRAFFIC["lmax4096"]
    for kernel, tiles in table.items():
        for key, nbytes in tiles.items():
            tile = tuple(int(v) for v in key.split(","))
            got = bench.hbm_traffic(kernel, "lmax4096", tile)
            assert got == nbytes and nbytes > 1.5e10
    assert bench.hbm_traffic("k_adj", "lmax4096", (2, 32, 4)) is None      # tile not measured
    assert bench.hbm_traffic("k_adj", "lmax8192", (8, 64, 4)) is None      # workload not measured
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "kernel_source_sha256", ["0" * 64])
    assert bench.hbm_traffic("k_adj", "lmax4096", (8, 64, 4)) is None      # other source


def test_forward_flops_per_term_weights_the_two_forms():
    w = S.WORKLOADS["lmax4096"]
    sym = w.blm()                                  # elliptical Gaussian: rows equal up to a sign
    assert bench.forward_flops_per_term(w, sym, True) == pytest.approx(bench.FLOPS_PER_TERM_PAIRED_ROWS)
    assert bench.forward_flops_per_term(w, sym, False) == bench.FLOPS_PER_TERM_UNPAIRED
    gen = S.random_beam(w.lmax, w.mbmax, 5)        # only the mb = 0 row is symmetric
    f = bench.forward_flops_per_term(w, gen, True)
    L, M = w.lmax, w.mbmax
    ms = np.arange(L + 1)
    n = {mb: float(np.sum(L - np.maximum(abs(mb), ms) + 1)) for mb in range(-M, M + 1)}
    want = (n[0] * 4.5 + (sum(n.values()) - n[0]) * 6.5) / sum(n.values())
    assert f == pytest.approx(want)
