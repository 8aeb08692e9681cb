"""Tile autotuner: picks (R, TB, TR) for plain calls and batched plans.

R is the chain block (chains per lane; a workgroup covers 256 R ring slots of a
column), TB the l block (values of l per LDS coefficient block), TR the
adjoint's reduction block (steps per wave reduction).

Each candidate runs the real launch (after one untimed warm-up) and is timed with
HIP events on the stream it runs on; the fastest wins.  Results are cached in a
JSON file (``$TC_TUNE_CACHE``, else ``~/.cache/paper_1002_1050_amd/tiles.json``)
keyed by the operation, sizes and GPU name, so a later process reuses them.
"""
from __future__ import annotations

import json
import os

from . import _binding as B

CANDIDATES = {
    B.TC_OP_FWD: [(r, tb, 4) for tb in (32, 64) for r in (2, 4, 8)],
    B.TC_OP_ADJ: [(r, tb, 4) for tb in (32, 64) for r in (2, 4, 8)],
    B.TC_OP_FWD_POL: [(r, tb, 4) for tb in (32, 64) for r in (2, 4)],
}


def _key(t):
    return "R%d_TB%d_TR%d" % t


def _cache_path():
    return os.environ.get("TC_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1002_1050_amd", "tiles.json")


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _out_of_memory(e):
    """A device allocation that failed: torch's out-of-memory error or the library's TC_ENOMEM."""
    import torch
    return isinstance(e, torch.cuda.OutOfMemoryError) or (
        isinstance(e, B.TotalConvError) and e.code == B.TC_ENOMEM)


def _release():
    import torch
    B.workspace_cache.clear()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _time(fn, reps=2):
    import torch
    fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _gpu_name():
    import torch
    return torch.cuda.get_device_name(0).replace(" ", "_")


def tune_plain(op, lmax, mbmax, cosbeta, alm, blm, Cbar=None, reps=2, use_cache=True):
    """Best (R, TB, TR) for a plain totalconv_fwd / totalconv_adj / totalconv_fwd_pol call of this
    shape (for the polarised forward, alm and blm are the lists of pairs)."""
    npair = len(alm) if op == B.TC_OP_FWD_POL else 1
    key = f"plain:{op}:{lmax}:{mbmax}:{len(cosbeta)}:{npair}:{_gpu_name()}"
    cache = _load() if use_cache else {}
    if key in cache:
        return tuple(cache[key]["tile"])
    times = {}
    default = B.get_tile_ex(op, lmax)
    try:
        for t in CANDIDATES[op]:
            B.set_tile_ex(op, *t)
            try:
                if op == B.TC_OP_FWD:
                    times[t] = _time(lambda: B.totalconv_fwd_x(lmax, mbmax, cosbeta, alm, blm), reps)
                elif op == B.TC_OP_FWD_POL:   # alm, blm: lists of pairs; separate outputs
                    times[t] = _time(lambda: B.totalconv_fwd_pol_x(lmax, mbmax, cosbeta, alm, blm), reps)
                else:
                    B.workspace_cache.clear()
                    times[t] = _time(lambda: B.totalconv_adj_x(lmax, mbmax, cosbeta, alm, blm, Cbar), reps)
            except Exception as e:   # noqa: BLE001 - only a tile that does not fit in memory is skipped
                if not _out_of_memory(e):
                    raise
                _release()
    finally:
        B.set_tile_ex(op, 0, 0, 0)
    if not times:
        raise MemoryError(f"no tile of op {op} fits in device memory at lmax {lmax}, mbmax {mbmax}")
    best = min(times, key=times.get)
    cache = _load()
    cache[key] = {"tile": list(best), "ms": {_key(k): v for k, v in times.items()}, "default": list(default)}
    _store(cache)
    return best


def tune_plan(op, make_plan, reps=2, use_cache=True, key_extra=""):
    """Best (R, TB, TR) for a batched plan; make_plan() builds the plan for the current tile."""
    key = f"plan:{op}:{key_extra}:{_gpu_name()}"
    cache = _load() if use_cache else {}
    if key in cache:
        return tuple(cache[key]["tile"]), cache[key]["ms"]
    times = {}
    try:
        for t in CANDIDATES[op]:
            B.set_tile_ex(op, *t)
            try:
                plan = make_plan()
            except Exception as e:   # noqa: BLE001 - only a plan that does not fit is skipped
                if not _out_of_memory(e):
                    raise
                _release()
                continue
            times[t] = _time(plan.execute, reps)
            plan.close()
    finally:
        B.set_tile_ex(op, 0, 0, 0)
    if not times:
        raise MemoryError(f"no tile of plan op {op} fits in device memory")
    best = min(times, key=times.get)
    cache = _load()
    cache[key] = {"tile": list(best), "ms": {_key(k): v for k, v in times.items()}}
    _store(cache)
    return best, cache[key]["ms"]
