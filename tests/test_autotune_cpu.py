"""Host logic of the autotuner (no GPU): a candidate tile that does not fit in device memory is
skipped, any other failure propagates, and the fastest remaining tile wins."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1002_1050_amd import _binding as B  # noqa: E402
from paper_1002_1050_amd import autotune  # noqa: E402


@pytest.fixture
def fake(monkeypatch, tmp_path):
    """Replace the GPU parts: tile setting records the tile, timing returns a fixed time per R."""
    monkeypatch.setenv("TC_TUNE_CACHE", str(tmp_path / "tiles.json"))
    monkeypatch.setattr(autotune, "_gpu_name", lambda: "cpu-test")
    monkeypatch.setattr(autotune, "_release", lambda: None)
    state = {"t": (0, 0, 0)}
    monkeypatch.setattr(B, "set_tile_ex", lambda op, R, TB, TR: state.update(t=(R, TB, TR)))
    monkeypatch.setattr(B, "get_tile_ex", lambda op, lmax: (8, 64, 4))
    ms = {2: 3.0, 4: 2.0, 8: 1.0}                  # R 8 fastest, then R 4

    def fake_time(fn, reps=2):
        fn()
        return ms[state["t"][0]] + (0.5 if state["t"][1] == 32 else 0.0)

    monkeypatch.setattr(autotune, "_time", fake_time)
    return state


def test_tile_out_of_memory_is_skipped(monkeypatch, fake):
    def adj(*a, **k):
        if fake["t"][0] == 8:                      # the fastest tile does not fit
            raise torch.cuda.OutOfMemoryError("out of memory")
        return None, None

    monkeypatch.setattr(B, "totalconv_adj_x", adj)
    best = autotune.tune_plain(B.TC_OP_ADJ, 100, 4, np.zeros(8), None, None, None, reps=1, use_cache=False)
    assert best == (4, 64, 4)


def test_library_enomem_is_skipped_and_other_errors_propagate(monkeypatch, fake):
    def fwd_enomem(*a, **k):
        if fake["t"][0] == 8:
            raise B.TotalConvError("totalconv_fwd", B.TC_ENOMEM, "workspace")
        return None

    monkeypatch.setattr(B, "totalconv_fwd_x", fwd_enomem)
    assert autotune.tune_plain(B.TC_OP_FWD, 100, 4, np.zeros(8), None, None, reps=1,
                               use_cache=False) == (4, 64, 4)

    def fwd_invalid(*a, **k):
        raise B.TotalConvError("totalconv_fwd", B.TC_EINVAL, "bad argument")

    monkeypatch.setattr(B, "totalconv_fwd_x", fwd_invalid)
    with pytest.raises(B.TotalConvError):
        autotune.tune_plain(B.TC_OP_FWD, 100, 4, np.zeros(8), None, None, reps=1, use_cache=False)


def test_no_tile_fits(monkeypatch, fake):
    def adj(*a, **k):
        raise torch.cuda.OutOfMemoryError("out of memory")

    monkeypatch.setattr(B, "totalconv_adj_x", adj)
    with pytest.raises(MemoryError):
        autotune.tune_plain(B.TC_OP_ADJ, 100, 4, np.zeros(8), None, None, None, reps=1, use_cache=False)
    assert fake["t"] == (0, 0, 0)                  # the built-in tile is restored
