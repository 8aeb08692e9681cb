#!/usr/bin/env python3
"""Throughput of the total convolution on one MI355X: forward + adjoint.

One step = totalconv_fwd (C from sky and beam) + totalconv_adj (sky and beam
gradients from a fixed cotangent), both through the C ABI on torch's current
stream, on the lmax 4096 / mbmax 14 / 8192-ring workload (synthetic seeded sky
and beam, inputs resident in HBM before timing).  `value` counts the
(l, mb, msky, beta) terms of both passes per second.

Prints one JSON line.  Also reports, for the dominant kernel, its algorithmic
FP64 rate against the vector-FP64 peak (HIP events around each launch on the
stream it runs on) and its HBM bytes per launch (rocprofv3 counters recorded
for this kernel source and tile), the CPU oracle timed on a bounded sample of
the same workload, and side legs: the sixteen-detector batched plan against
sixteen plain calls (forward and adjoint), the polarised forward, the data cube
and the fixed-l Wigner matrix.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CU x 128 FP64 flop/clk x 2.4 GHz
# Algorithmic FP64 flops per (l, mb, msky, beta) term with the mirror-ring pairing:
# one recursion step (5 flops: sub, 3 mul, fma as written in the paper) serves two
# terms, and each term adds a complex weight times a real d (4 flops).
FLOPS_PER_TERM_PAIRED = 6.5
FLOPS_PER_TERM_UNPAIRED = 9.0
# forward on a column whose beam rows mb and -mb differ by a sign: one complex weight per
# step serves both rings of a mirror pair (5 recursion + 4 accumulation flops per 2 terms)
FLOPS_PER_TERM_PAIRED_ROWS = 4.5


def forward_flops_per_term(w, blm, paired):
    """Algorithmic flops per term of the forward: 4.5 on the columns whose beam rows mb and -mb
    are equal up to a sign for every l >= |mb| (the library then sums even and odd l apart),
    6.5 on the others (9 without mirror pairs), weighted by the terms of each column."""
    if not paired:
        return FLOPS_PER_TERM_UNPAIRED
    L, M = w.lmax, w.mbmax
    ms = np.arange(L + 1)
    tot = fast = 0
    for mb in range(-M, M + 1):
        n = float(np.sum(L - np.maximum(abs(mb), ms) + 1))
        p, m = blm[mb + M, abs(mb):], blm[-mb + M, abs(mb):]
        tot += n
        if np.array_equal(m, p) or np.array_equal(m, -p):
            fast += n
    return (fast * FLOPS_PER_TERM_PAIRED_ROWS + (tot - fast) * FLOPS_PER_TERM_PAIRED) / tot


# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes over
# this bench (the kernels' dispatches at lmax 4096), each counter scaled by what it
# reads for a device-to-device copy of known size in the same run, per kernel and tile
# (R, TB, TR).  Valid only for the kernel source they were taken on (SHA-256 of
# tc_kernels.hip) and the tile the bench runs; otherwise null.
def _bytes(fetch_kib, write_kib, copy_fetch_kib, copy_write_kib=2097152.0):
    """FETCH_SIZE KiB x 1024 x (2 GiB / copy's FETCH_SIZE bytes) + the same for WRITE_SIZE."""
    return int(fetch_kib * 1024 * (2147483648 / (copy_fetch_kib * 1024))
               + write_kib * 1024 * (2147483648 / (copy_write_kib * 1024)))


MEASURED_TRAFFIC = {
    # FETCH_SIZE and WRITE_SIZE of the kernels as built from this source, each scaled by the
    # counts of a 2 GiB device-to-device copy in the same run
    "kernel_source_sha256": ["accdb2a8b4aad6c420f4213ccefc993ad46b38da8747be5129beade2de1ad0ee"],
    "lmax4096": {
        # the forward: its two launches, k_fwd_rows and k_fwd, together
        "k_fwd": {"8,64,4": _bytes(1449012.8 + 3725.5, 16475947.9 + 0.0, 1048611.6),
                  "4,64,4": _bytes(973078.5 + 3726.5, 16633820.6 + 0.0, 1048611.6)},
        "k_adj": {"8,64,4": _bytes(11091143.9, 17801268.9, 1048611.6)},
    },
}


def hbm_traffic(kernel, workload, tile):
    import hashlib
    src = os.path.join(ROOT, "paper_1002_1050_amd", "csrc", "tc_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha not in MEASURED_TRAFFIC["kernel_source_sha256"]:
        return None
    return MEASURED_TRAFFIC.get(workload, {}).get(kernel, {}).get(",".join(str(int(v)) for v in tile))


def parse():
    p = argparse.ArgumentParser(description=__doc__)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="lmax4096")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="wall-clock budget of the oracle sample (0 disables)")
    p.add_argument("--fwd-only", action="store_true", help="time the forward alone")
    p.add_argument("--batched-reps", type=int, default=3,
                   help="interleaved repetitions of the sixteen-detector batched-vs-plain comparison (0 skips)")
    p.add_argument("--pol-reps", type=int, default=2,
                   help="timed repetitions of the polarised forward (three pairs, separate and summed; 0 skips)")
    p.add_argument("--cube-reps", type=int, default=2,
                   help="timed repetitions of the data-cube stage on the forward's output (0 skips)")
    p.add_argument("--matrix-reps", type=int, default=2,
                   help="timed repetitions of the full-matrix generator at l = lmax on 16 rings (0 skips)")
    p.add_argument("--config-reps", type=int, default=5,
                   help="timed repetitions of the lmax 64 / 1024 / 2048 workloads (0 skips)")
    p.add_argument("--large-reps", type=int, default=3,
                   help="timed repetitions of one 4096-ring chunk of the four lmax 8192 detectors (0 skips)")
    p.add_argument("--no-tune", action="store_true", help="use the built-in tiles instead of the autotuner")
    p.add_argument("--tile-fwd", default="", help="forward tile 'R,TB' (skips its autotuning)")
    p.add_argument("--tile-adj", default="", help="adjoint tile 'R,TB[,TR]' (skips its autotuning)")
    p.add_argument("--copy-calibration-gib", type=float, default=0.0,
                   help="first run one device-to-device copy of this many GiB (a reference kernel of known "
                        "traffic for hardware byte counters)")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, x, alm, blm, G_cols_fn, seconds):
    """Oracle forward + adjoint column sums on a seeded sample of whole columns."""
    import oracle
    rng = np.random.Generator(np.random.PCG64(2024))
    nb = 2 * w.mbmax + 1
    order = rng.permutation(nb * (w.lmax + 1))
    done_terms = 0
    ncols = 0
    elapsed = 0.0          # oracle time only (the cotangent copies are excluded)
    batch = 16
    for i in range(0, order.size, batch):
        sel = order[i:i + batch]
        mb = (sel // (w.lmax + 1) - w.mbmax).astype(np.int32)
        ms = (sel % (w.lmax + 1)).astype(np.int32)
        G = G_cols_fn(sel)
        ts = time.perf_counter()
        oracle.totalconv_fwd(w.lmax, w.mbmax, x, alm, blm, cols=(mb, ms))
        oracle.column_sums(w.lmax, w.mbmax, x, G, (mb, ms))
        te = time.perf_counter()
        elapsed += te - ts
        done_terms += 2 * int(np.sum(w.lmax + 1 - np.maximum(np.abs(mb), ms))) * w.nring
        ncols += sel.size
        if elapsed >= seconds:
            break
    rate = done_terms / elapsed
    return {
        "value": rate,
        "unit": "terms/s",
        "cores": int(oracle.max_threads()),
        "kind": "oracle",
        # the whole workload (forward + adjoint over every column) at the sampled rate
        "full_workload_extrapolated_s": round(2 * w.terms() / rate, 1),
        "sample": f"{ncols} seeded random (mb, msky) columns x all {w.nring} rings of the {w.name} "
                  f"workload, forward + adjoint column sums, x87 long double, {elapsed:.1f} s; "
                  f"{host_cpu()}",
    }


def host_cpu():
    """The host's CPU model and the cores this process may run on."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {len(os.sched_getaffinity(0))} cores in the process affinity set"


def truncate_sky(S, alm, lmax_sky, lmax):
    out = np.zeros(S.alm_size(lmax), np.complex128)
    for m in range(lmax + 1):
        out[S.alm_index(lmax, m, m):S.alm_index(lmax, lmax, m) + 1] = \
            alm[S.alm_index(lmax_sky, m, m):S.alm_index(lmax_sky, lmax, m) + 1]
    return out


def batched_compare(reps, tune):
    """Sixteen detectors (lmax 512..4096 x mbmax 4..14, 2 lmax rings each, one sky at lmax 4096):
    sixteen plain totalconv_fwd calls on one stream (each with its own tile) against one
    tc_plan_execute of the graph-captured plan.  Interleaved repetitions."""
    import torch
    from paper_1002_1050_amd import _binding as B
    from paper_1002_1050_amd import autotune
    from paper_1002_1050_amd import synthetic as S
    w = S.WORKLOADS["batched16"]
    dev = torch.device("cuda:0")
    alm_h = S.sky_alm(w.lmax, w.sky_seed)
    alm = torch.from_numpy(alm_h).to(dev)
    dets, plain = [], []
    for d in w.detectors:
        beta = d.colatitudes()
        x = B.rings_from_beta(beta)       # the library's rings, for the autotuner's cosine calls
        blm = torch.from_numpy(d.blm()).to(dev)
        C = torch.empty((2 * d.mbmax + 1, d.lmax + 1, d.nring), dtype=torch.complex128, device=dev)
        a_d = torch.from_numpy(truncate_sky(S, alm_h, w.lmax, d.lmax)).to(dev)
        t = autotune.tune_plain(B.TC_OP_FWD, d.lmax, d.mbmax, x, a_d, blm, reps=1) if tune else (0, 0, 0)
        dets.append({"lmax": d.lmax, "mbmax": d.mbmax, "beta": beta, "blm": blm, "C": C})
        plain.append((d, beta, x, a_d, blm, C, t))
        log(f"  detector lmax={d.lmax} mbmax={d.mbmax} nring={d.nring} plain tile (R, TB, TR)={t}")

    def run_plain():
        for d, beta, x, a_d, blm, C, t in plain:
            B.set_tile_ex(B.TC_OP_FWD, *t)
            B.totalconv_fwd(d.lmax, d.mbmax, beta, a_d, blm, out=C)
        B.set_tile_ex(B.TC_OP_FWD, 0, 0, 0)

    tp_ = (0, 0, 0)
    if tune:
        tp_, tms = autotune.tune_plan(B.TC_OP_FWD, lambda: B.Plan(B.TC_OP_FWD, dets, w.lmax, alm), reps=1,
                                      key_extra="batched16")
        log(f"  plan tile (R, TB, TR)={tp_} (trial ms {tms})")
    B.set_tile_ex(B.TC_OP_FWD, *tp_)
    plan = B.Plan(B.TC_OP_FWD, dets, w.lmax, alm)
    B.set_tile_ex(B.TC_OP_FWD, 0, 0, 0)
    s = torch.cuda.current_stream(dev)
    run_plain()
    plan.execute()
    torch.cuda.synchronize()
    tp, tb = [], []
    for i in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(s)
        run_plain()
        e[1].record(s)
        torch.cuda.synchronize()
        e[2].record(s)
        plan.execute()
        e[3].record(s)
        torch.cuda.synchronize()
        tp.append(e[0].elapsed_time(e[1]))
        tb.append(e[2].elapsed_time(e[3]))
        log(f"  rep {i + 1}/{reps}: plain {tp[-1]:.1f} ms, batched {tb[-1]:.1f} ms")
    ratios = [a / b for a, b in zip(tp, tb)]
    terms = w.terms()
    res = {
        "workload": "sixteen detectors, lmax {512,1024,2048,4096} x mbmax {4,6,9,14}, 2 lmax rings each, "
                    "one sky at lmax 4096, forward",
        "terms": terms,
        "plain_ms_median": float(np.median(tp)),
        "batched_ms_median": float(np.median(tb)),
        "plain_terms_per_s": terms / (np.median(tp) * 1e-3),
        "batched_terms_per_s": terms / (np.median(tb) * 1e-3),
        "speedup_median": float(np.median(ratios)),
        "speedup_min": float(np.min(ratios)),
        "speedup_max": float(np.max(ratios)),
        "plan_tile": list(tp_) if tune else "built-in",
        "plan_R": plan.tile,
        "reps": reps,
    }
    plan.close()
    torch.cuda.empty_cache()
    try:
        res["adjoint"] = batched_adjoint_compare(w, dets, plain, alm, reps, tune)
    except Exception as e:   # noqa: BLE001 - reported in the JSON line; the forward leg stands
        log(f"batched adjoint comparison failed: {type(e).__name__}: {e}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        res["adjoint"] = {"error": f"{type(e).__name__}: {e}"}
    return res


def batched_adjoint_compare(w, dets, plain, alm, reps, tune):
    """The adjoint of the same sixteen detectors, each forward output C as its cotangent: sixteen
    plain totalconv_adj calls (each with its own tile), each detector's sky gradient added into
    the full one, against one tc_plan_execute of the adjoint plan at its built-in tile (the plan
    sums the sky gradients in its graph).  Interleaved repetitions."""
    import torch
    from paper_1002_1050_amd import _binding as B
    from paper_1002_1050_amd import autotune
    from paper_1002_1050_amd import synthetic as S
    dev = alm.device
    adets = [{"lmax": d["lmax"], "mbmax": d["mbmax"], "beta": d["beta"], "blm": d["blm"],
              "Cbar": d["C"], "blm_bar": torch.empty_like(d["blm"])} for d in dets]
    alm_bar = torch.empty_like(alm)
    plain_bar = torch.zeros_like(alm)
    legs = []
    for d, beta, x, a_d, blm, C, _ in plain:
        # full-layout positions of the detector's truncated sky (m-major, l inner)
        ix = np.concatenate([np.arange(S.alm_index(w.lmax, m, m), S.alm_index(w.lmax, d.lmax, m) + 1)
                             for m in range(d.lmax + 1)])
        t = autotune.tune_plain(B.TC_OP_ADJ, d.lmax, d.mbmax, x, a_d, blm, C, reps=1) if tune else (0, 0, 0)
        legs.append((d, beta, a_d, blm, C, t, torch.from_numpy(ix).to(dev)))
        log(f"  adjoint detector lmax={d.lmax} mbmax={d.mbmax} plain tile (R, TB, TR)={t}")

    def run_plain():
        plain_bar.zero_()
        for d, beta, a_d, blm, C, t, ix in legs:
            B.set_tile_ex(B.TC_OP_ADJ, *t)
            ab, _ = B.totalconv_adj(d.lmax, d.mbmax, beta, a_d, blm, C)
            plain_bar.index_add_(0, ix, ab)
        B.set_tile_ex(B.TC_OP_ADJ, 0, 0, 0)

    # the plan is autotuned like the forward's: its partial sums (one U and one V row per column,
    # about 25 GB for these sixteen detectors) do not depend on the tile
    tp_ = (0, 0, 0)
    tms = {}
    if tune:
        tp_, tms = autotune.tune_plan(B.TC_OP_ADJ, lambda: B.Plan(B.TC_OP_ADJ, adets, w.lmax, alm, alm_bar), reps=1,
                                      key_extra="batched16")
        log(f"  adjoint plan tile (R, TB, TR)={tp_} (trial ms {tms})")
    B.set_tile_ex(B.TC_OP_ADJ, *tp_)
    plan = B.Plan(B.TC_OP_ADJ, adets, w.lmax, alm, alm_bar)
    B.set_tile_ex(B.TC_OP_ADJ, 0, 0, 0)
    s = torch.cuda.current_stream(dev)
    run_plain()
    plan.execute()
    torch.cuda.synchronize()
    tp, tb = [], []
    for i in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(s)
        run_plain()
        e[1].record(s)
        torch.cuda.synchronize()
        e[2].record(s)
        plan.execute()
        e[3].record(s)
        torch.cuda.synchronize()
        tp.append(e[0].elapsed_time(e[1]))
        tb.append(e[2].elapsed_time(e[3]))
        log(f"  adjoint rep {i + 1}/{reps}: plain {tp[-1]:.1f} ms, batched {tb[-1]:.1f} ms")
    ratios = [a / b for a, b in zip(tp, tb)]
    terms = w.terms()
    res = {
        "workload": "the same sixteen detectors, adjoint (sky gradient summed over detectors, beam "
                    "gradient per detector), each forward output as its cotangent",
        "plain_ms_median": float(np.median(tp)),
        "batched_ms_median": float(np.median(tb)),
        "plain_terms_per_s": terms / (np.median(tp) * 1e-3),
        "batched_terms_per_s": terms / (np.median(tb) * 1e-3),
        "speedup_median": float(np.median(ratios)),
        "speedup_min": float(np.min(ratios)),
        "speedup_max": float(np.max(ratios)),
        "plan_tile": list(tp_) if tune else "built-in",
        "plan_R": plan.tile,
        "reps": reps,
    }
    plan.close()
    return res


def config_timing(name, reps, tune):
    """One plain workload (small, medium, adjoint): forward and adjoint through the entry points on
    colatitudes, timed with the library's HIP events around each recursion kernel (median of reps
    after one warm-up; the adjoint's kernel time is its launches over the ring tiles) and as whole
    calls; cotangent a seeded Gaussian drawn on the device."""
    import torch
    from paper_1002_1050_amd import _binding as B
    from paper_1002_1050_amd import synthetic as S
    w = S.WORKLOADS[name]
    dev = torch.device("cuda:0")
    beta = w.colatitudes()
    x = B.rings_from_beta(beta)
    alm = torch.from_numpy(w.alm()).to(dev)
    blm_h = w.blm()
    blm = torch.from_numpy(blm_h).to(dev)
    C = torch.empty((2 * w.mbmax + 1, w.lmax + 1, w.nring), dtype=torch.complex128, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(w.lmax)
    G = torch.randn(C.shape, dtype=torch.complex128, device=dev, generator=gen)
    tf = ta = (0, 0, 0)
    if tune:
        from paper_1002_1050_amd import autotune
        tf = autotune.tune_plain(B.TC_OP_FWD, w.lmax, w.mbmax, x, alm, blm, reps=1)
        ta = autotune.tune_plain(B.TC_OP_ADJ, w.lmax, w.mbmax, x, alm, blm, G, reps=1)
    B.set_tile_ex(B.TC_OP_FWD, *tf)
    B.set_tile_ex(B.TC_OP_ADJ, *ta)
    s = torch.cuda.current_stream(dev)
    B.totalconv_fwd(w.lmax, w.mbmax, beta, alm, blm, out=C)
    B.totalconv_adj(w.lmax, w.mbmax, beta, alm, blm, G)
    torch.cuda.synchronize()
    B.timing_enable(reps)
    fwd, adj = [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(s)
        B.totalconv_fwd(w.lmax, w.mbmax, beta, alm, blm, out=C)
        e[1].record(s)
        B.totalconv_adj(w.lmax, w.mbmax, beta, alm, blm, G)
        e[2].record(s)
        torch.cuda.synchronize()
        fwd.append(e[0].elapsed_time(e[1]))
        adj.append(e[1].elapsed_time(e[2]))
    kf = float(np.median(B.timing_read(B.TC_OP_FWD, reps)))
    ka = float(np.median(B.timing_read(B.TC_OP_ADJ, reps)))
    B.timing_enable(0)
    B.set_tile_ex(B.TC_OP_FWD, 0, 0, 0)
    B.set_tile_ex(B.TC_OP_ADJ, 0, 0, 0)
    terms = w.terms()
    fpt_f = forward_flops_per_term(w, blm_h, True)
    fpt_a = FLOPS_PER_TERM_PAIRED
    cf, ca = float(np.median(fwd)), float(np.median(adj))
    res = {"workload": f"lmax={w.lmax}, mbmax={w.mbmax}, {w.nring} rings, forward + adjoint", "terms_per_pass": terms,
           "tiles_R_TB_TR": {"forward": list(tf), "adjoint": list(ta)},
           "forward_call_ms": round(cf, 4), "adjoint_call_ms": round(ca, 4),
           "forward_kernel_ms": round(kf, 4), "adjoint_kernel_ms": round(ka, 4),
           "terms_per_s": 2 * terms / ((cf + ca) * 1e-3),
           "forward_frac": round(fpt_f * terms / (kf * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4),
           "adjoint_frac": round(fpt_a * terms / (ka * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4),
           "reps": reps}
    log(f"  {name}: forward {cf:.3f} ms (kernel {kf:.3f}), adjoint {ca:.3f} ms (kernel {ka:.3f}), "
        f"{res['terms_per_s']:.3e} terms/s, frac {res['forward_frac']} / {res['adjoint_frac']}")
    del C, G
    torch.cuda.empty_cache()
    return res


def large_chunk_timing(reps, chunk=1):
    """The four lmax 8192 detectors (mbmax 16, 16384 rings) on one chunk of 4096 rings (2048 mirror
    pairs; the chunk next to the polar one by default): the batched forward plan and the batched
    adjoint plan (sky gradient summed over the detectors, every beam gradient), each forward
    output as its own cotangent; whole plan executions timed with events on the stream, median
    of reps after one warm-up."""
    import torch
    from paper_1002_1050_amd import _binding as B
    from paper_1002_1050_amd import synthetic as S
    w = S.WORKLOADS["large4"]
    L, M, N, half = w.lmax, w.mbmax, w.nring, 2048
    dev = torch.device("cuda:0")
    j = np.arange(N)
    k = np.minimum(j, N - 1 - j)
    rings = np.nonzero((k >= chunk * half) & (k < (chunk + 1) * half))[0]
    beta = w.colatitudes()[rings]
    alm = torch.from_numpy(w.alm()).to(dev)
    shape = (2 * M + 1, L + 1, beta.size)
    dets = [{"lmax": L, "mbmax": M, "beta": beta, "blm": torch.from_numpy(d.blm()).to(dev),
             "C": torch.empty(shape, dtype=torch.complex128, device=dev)} for d in w.detectors]
    terms = len(dets) * S.count_terms(L, M, beta.size)
    s = torch.cuda.current_stream(dev)

    def timed(plan):
        plan.execute()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            plan.execute()
            e1.record(s)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return out

    fplan = B.Plan(B.TC_OP_FWD, dets, L, alm)
    tf = timed(fplan)
    fplan.close()
    for d in dets:
        d["Cbar"] = d.pop("C")
        d["blm_bar"] = torch.empty_like(d["blm"])
    alm_bar = torch.empty_like(alm)
    aplan = B.Plan(B.TC_OP_ADJ, dets, L, alm, alm_bar)
    ta = timed(aplan)
    aplan.close()
    del dets
    torch.cuda.empty_cache()
    f, a = float(np.median(tf)), float(np.median(ta))
    log(f"  large4 chunk {chunk}: forward plan {f:.1f} ms, adjoint plan {a:.1f} ms ({tf} / {ta})")
    return {"workload": f"four detectors lmax={L}, mbmax={M}, ring chunk {chunk} of 4 ({beta.size} of {N} rings), "
                        "batched forward and adjoint plans", "terms_per_pass": terms,
            "forward_ms_median": f, "adjoint_ms_median": a, "forward_ms": tf, "adjoint_ms": ta,
            "terms_per_s": 2 * terms / ((f + a) * 1e-3),
            "forward_frac": round(FLOPS_PER_TERM_PAIRED_ROWS * terms / (f * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4),
            "adjoint_frac": round(FLOPS_PER_TERM_PAIRED * terms / (a * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4),
            "frac_note": "4.5 (forward) and 6.5 (adjoint) flops per term of each detector, as if each walked its "
                         "own recursion; the four detectors share rings and lmax, so the forward plan walks "
                         "each column once for all four, and its fraction can exceed 1",
            "reps": reps}


def datacube_timing(w, C, reps):
    """Data cube of eq. conviqt from the forward's C: nalpha = 2 mbmax + 1, ngamma = 2 lmax.
    Algorithmic bytes: C read once, the cube written once."""
    import torch
    from paper_1002_1050_amd import _binding as B
    na, ng = 2 * w.mbmax + 1, 2 * w.lmax
    cube = torch.empty((w.nring, na, ng), dtype=torch.float64, device=C.device)
    B.totalconv_datacube(w.lmax, w.mbmax, C, na, ng, out=cube)   # warm-up
    torch.cuda.synchronize()
    B.timing_enable(64)
    t0 = time.perf_counter()
    for _ in range(reps):
        B.totalconv_datacube(w.lmax, w.mbmax, C, na, ng, out=cube)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    calls = B.timing_read(B.TC_OP_CUBE, reps)   # one record per call, around all of its kernels
    B.timing_enable(0)
    kms = float(np.mean(calls))
    nbytes = C.numel() * 16 + cube.numel() * 8
    chunk = B.datacube_ring_chunk(w.lmax, w.mbmax, w.nring, na, ng)
    nchunk = -(-w.nring // chunk)
    del cube
    torch.cuda.empty_cache()
    log(f"  data cube: kernels {kms:.2f} ms ({nchunk} ring chunks of {chunk}), {nbytes / (kms * 1e-3) / 1e9:.0f} GB/s")
    return {"workload": f"data cube, nalpha={na}, ngamma={ng}, {w.nring} rings, lmax={w.lmax}, mbmax={w.mbmax}",
            "kernel_ms": round(kms, 3), "call_ms": round(wall * 1e3, 3), "algorithmic_bytes": nbytes,
            "hbm_gb_per_s": nbytes / (kms * 1e-3) / 1e9, "ring_chunks": nchunk, "rings_per_chunk": chunk}


def matrix_timing(w, reps, nring=16):
    """Full matrix d^l_{m m'}, -l <= m, m' <= l, at l = lmax on nring seeded rings.
    The output is written once: 8 bytes per element, the kernel's algorithmic HBM traffic."""
    import torch
    from paper_1002_1050_amd import _binding as B
    from paper_1002_1050_amd import synthetic as S
    l = w.lmax
    beta = S.ring_colatitudes(2 * nring + 1)[1:nring + 1]
    out = torch.empty((nring, 2 * l + 1, 2 * l + 1), dtype=torch.float64, device="cuda:0")
    B.wigner_d_matrix(l, beta, out=out)   # warm-up
    torch.cuda.synchronize()
    B.timing_enable(reps)
    t0 = time.perf_counter()
    for _ in range(reps):
        B.wigner_d_matrix(l, beta, out=out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    kms = float(np.mean(B.timing_read(B.TC_OP_MATRIX, reps)))
    B.timing_enable(0)
    n = out.numel()
    del out
    torch.cuda.empty_cache()
    log(f"  full matrix l={l}: kernel {kms:.2f} ms, {n / (kms * 1e-3):.3e} elements/s, {8 * n / (kms * 1e-3) / 1e9:.0f} GB/s")
    return {"workload": f"full Wigner matrix at l={l}, {nring} rings", "elements": n, "kernel_ms": round(kms, 3),
            "call_ms": round(wall * 1e3, 3), "elements_per_s": n / (kms * 1e-3),
            "hbm_gb_per_s": 8 * n / (kms * 1e-3) / 1e9}


def polarised_compare(w, beta, alm, blm, reps, tune):
    """Polarised forward on the same workload: temperature, gradient and curl pairs (three
    seeded skies, three beams) sharing one recursion, as three outputs and as their sum.
    Terms count each pair's (l, mb, msky, beta) terms."""
    import torch
    from paper_1002_1050_amd import _binding as B
    from paper_1002_1050_amd import synthetic as S
    dev = alm.device
    alms = [alm] + [torch.from_numpy(S.sky_alm(w.lmax, w.sky_seed + 1 + p)).to(dev) for p in range(2)]
    blms = [blm] + [torch.from_numpy(S.random_beam(w.lmax, w.mbmax, 77 + p)).to(dev) for p in range(2)]
    tile = B.get_tile_ex(B.TC_OP_FWD_POL, w.lmax)
    if tune:
        from paper_1002_1050_amd import autotune
        tile = autotune.tune_plain(B.TC_OP_FWD_POL, w.lmax, w.mbmax, B.rings_from_beta(beta), alms, blms, reps=1)
    B.set_tile_ex(B.TC_OP_FWD_POL, *tile)
    terms = 3 * w.terms()
    res = {"workload": f"polarised forward and adjoint, three (sky, beam) pairs, lmax={w.lmax}, "
                       f"mbmax={w.mbmax}, {w.nring} rings", "terms": terms, "tile_R_TB": list(tile[:2])}
    for name, mode in (("separate", B.TC_POL_SEPARATE), ("summed", B.TC_POL_SUM)):
        outs = B.totalconv_fwd_pol(w.lmax, w.mbmax, beta, alms, blms, mode)   # warm-up
        del outs
        torch.cuda.synchronize()
        B.timing_enable(reps)
        t0 = time.perf_counter()
        for _ in range(reps):
            outs = B.totalconv_fwd_pol(w.lmax, w.mbmax, beta, alms, blms, mode)
            del outs
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        kms = float(np.mean(B.timing_read(B.TC_OP_FWD_POL, reps)))
        B.timing_enable(0)
        res[name] = {"kernel_ms": round(kms, 3), "call_ms": round(wall * 1e3, 3),
                     "terms_per_s": terms / (kms * 1e-3)}
        log(f"  polarised {name}: kernel {kms:.1f} ms, {terms / (kms * 1e-3):.3e} terms/s")
        torch.cuda.empty_cache()
    B.set_tile_ex(B.TC_OP_FWD_POL, 0, 0, 0)
    # the adjoint (totalconv_adj_pol, sky and beam gradients of every pair), the forward's outputs
    # as cotangents: one per output (separate) or the first for the summed output; whole calls
    # timed with events on the stream
    outs = B.totalconv_fwd_pol(w.lmax, w.mbmax, beta, alms, blms, B.TC_POL_SEPARATE)
    res["adjoint"] = {}
    s = torch.cuda.current_stream(dev)
    for name, mode, cbars in (("separate", B.TC_POL_SEPARATE, outs), ("summed", B.TC_POL_SUM, outs[:1])):
        g = B.totalconv_adj_pol(w.lmax, w.mbmax, beta, alms, blms, cbars, mode)   # warm-up
        del g
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            g = B.totalconv_adj_pol(w.lmax, w.mbmax, beta, alms, blms, cbars, mode)
            del g
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res["adjoint"][name] = {"call_ms": round(ms, 3), "terms_per_s": terms / (ms * 1e-3)}
        log(f"  polarised adjoint {name}: call {ms:.1f} ms, {terms / (ms * 1e-3):.3e} terms/s")
    del outs
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    from paper_1002_1050_amd import _binding as B
    from paper_1002_1050_amd import synthetic as S

    if args.copy_calibration_gib > 0:
        n = int(args.copy_calibration_gib * (1 << 30)) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 8} bytes read and written")
        del src, dst
    w = S.WORKLOADS[args.workload]
    if w.detectors:
        raise SystemExit("batched workloads are timed by bench_batched")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    beta = w.colatitudes()
    x = B.rings_from_beta(beta)           # the library's rings, for the autotuner's cosine calls
    alm_h, blm_h = w.alm(), w.blm()
    alm = torch.from_numpy(alm_h).to(dev)
    blm = torch.from_numpy(blm_h).to(dev)
    terms = w.terms()
    log(f"workload {w.name}: lmax={w.lmax} mbmax={w.mbmax} nring={w.nring} terms/pass={terms:.4e}")

    # untimed set-up: C, the target C_T from a second sky, cotangent G = C - C_T
    C = torch.empty((2 * w.mbmax + 1, w.lmax + 1, w.nring), dtype=torch.complex128, device=dev)
    B.totalconv_fwd(w.lmax, w.mbmax, beta, alm, blm, out=C)
    T = B.totalconv_fwd(w.lmax, w.mbmax, beta, torch.from_numpy(S.sky_alm(w.lmax, w.target_seed or 1050)).to(dev), blm)
    G = C - T
    del T
    torch.cuda.synchronize()
    log("set-up done")

    def given(spec):
        v = [int(u) for u in spec.split(",")]
        return (v[0], v[1], v[2] if len(v) > 2 else 4)

    tf = given(args.tile_fwd) if args.tile_fwd else None
    ta = given(args.tile_adj) if args.tile_adj else None
    if not args.no_tune and (tf is None or ta is None):
        from paper_1002_1050_amd import autotune
        if tf is None:
            tf = autotune.tune_plain(B.TC_OP_FWD, w.lmax, w.mbmax, x, alm, blm, reps=1)
        if ta is None:
            ta = autotune.tune_plain(B.TC_OP_ADJ, w.lmax, w.mbmax, x, alm, blm, G, reps=1)
        log(f"autotuned tiles (R, TB, TR): forward {tf}, adjoint {ta}")
        torch.cuda.empty_cache()
    tf = tf or B.get_tile_ex(B.TC_OP_FWD, w.lmax)
    ta = ta or B.get_tile_ex(B.TC_OP_ADJ, w.lmax)
    B.set_tile_ex(B.TC_OP_FWD, *tf)
    B.set_tile_ex(B.TC_OP_ADJ, *ta)
    tiles = {"forward": list(tf), "adjoint": list(ta)}

    def step():
        B.totalconv_fwd(w.lmax, w.mbmax, beta, alm, blm, out=C)
        if not args.fwd_only:
            B.totalconv_adj(w.lmax, w.mbmax, beta, alm, blm, G)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    stream = torch.cuda.current_stream(dev)
    ev = []
    B.timing_enable(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        B.totalconv_fwd(w.lmax, w.mbmax, beta, alm, blm, out=C)
        e[1].record(stream)
        if not args.fwd_only:
            B.totalconv_adj(w.lmax, w.mbmax, beta, alm, blm, G)
        e[2].record(stream)
        ev.append(e)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    adj_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev])) if not args.fwd_only else 0.0
    # HIP events recorded by the library on this stream directly around each recursion kernel
    k_fwd = B.timing_read(B.TC_OP_FWD, args.steps)
    k_adj = B.timing_read(B.TC_OP_ADJ, args.steps) if not args.fwd_only else []
    B.timing_enable(0)
    kfwd_ms = float(np.mean(k_fwd))
    kadj_ms = float(np.mean(k_adj)) if k_adj else 0.0
    log(f"timed {args.steps} steps in {elapsed:.3f} s; forward {fwd_ms:.2f} ms, adjoint {adj_ms:.2f} ms; "
        f"kernels: k_fwd {kfwd_ms:.2f} ms, k_adj {kadj_ms:.2f} ms")

    passes = 1 if args.fwd_only else 2
    ms_per_step = elapsed / args.steps * 1e3
    value = passes * terms / (elapsed / args.steps)
    paired = bool(np.all(x[::-1][: w.nring // 2] == -x[: w.nring // 2]))
    fpt_adj = FLOPS_PER_TERM_PAIRED if paired else FLOPS_PER_TERM_UNPAIRED
    fpt_fwd = forward_flops_per_term(w, blm_h, paired)
    dom_name, dom_ms = ("k_adj", kadj_ms) if kadj_ms > kfwd_ms else ("k_fwd", kfwd_ms)
    fpt = fpt_adj if dom_name == "k_adj" else fpt_fwd
    fpt_other = fpt_fwd if dom_name == "k_adj" else fpt_adj
    achieved = fpt * terms / (dom_ms * 1e-3) / 1e12
    roofline = {
        "bound": "alu",
        "kernel": dom_name,
        "achieved": round(achieved, 3),
        "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
        "traffic": hbm_traffic(dom_name, w.name, ta if dom_name == "k_adj" else tf),
        "flops_per_term": fpt,
        "terms_per_launch": terms,
        "launch_ms": round(dom_ms, 3),
        "launch_ms_per_step": [round(v, 3) for v in (k_adj if dom_name == "k_adj" else k_fwd)],
        "other_kernel": {"name": "k_fwd" if dom_name == "k_adj" else "k_adj",
                         "launch_ms": round(kfwd_ms if dom_name == "k_adj" else kadj_ms, 3),
                         "flops_per_term": round(fpt_other, 4),
                         "frac": round(fpt_other * terms / ((kfwd_ms if dom_name == "k_adj" else kadj_ms) or float("inf"))
                                       / 1e9 / FP64_VECTOR_PEAK_TFLOPS, 4)},
    }
    result = {
        "metric": "(l,mb,msky,beta) convolution terms/s, forward + adjoint",
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"total convolution {'forward' if args.fwd_only else 'forward + adjoint'}, "
                        f"lmax={w.lmax}, mbmax={w.mbmax}, msky 0..{w.lmax}, {w.nring} equispaced rings",
            "lmax": w.lmax, "mbmax": w.mbmax, "nring": w.nring,
            "terms_per_pass": terms, "passes_per_step": passes,
        },
        "forward_ms": round(fwd_ms, 3),
        "adjoint_ms": round(adj_ms, 3),
        "forward_terms_per_s": terms / (fwd_ms * 1e-3),
        "adjoint_terms_per_s": (terms / (adj_ms * 1e-3)) if adj_ms else None,
        "roofline": roofline,
        "tiles_R_TB_TR": tiles,
    }
    def side_leg(name, fn, *a):
        """A side measurement that raises (say, short of device memory on a shared board) is
        recorded as an error; the step's own line above is already complete."""
        try:
            return fn(*a)
        except Exception as e:   # noqa: BLE001 - reported in the JSON line, never swallowed silently
            log(f"{name} failed: {type(e).__name__}: {e}")
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            return {"error": f"{type(e).__name__}: {e}"}

    if args.cube_reps > 0:
        log("data cube")
        result["datacube"] = side_leg("data cube", datacube_timing, w, C, args.cube_reps)
    if args.matrix_reps > 0:
        log("full matrix")
        result["matrix"] = side_leg("full matrix", matrix_timing, w, args.matrix_reps)
    if args.cpu_seconds > 0:
        nring = w.nring
        Gc = G.reshape(-1, nring)

        def g_cols(sel):
            idx = torch.from_numpy(np.asarray(sel, np.int64)).to(dev)
            return Gc.index_select(0, idx).cpu().numpy()

        log(f"cpu baseline: oracle on a sample, about {args.cpu_seconds:.0f} s")
        import oracle
        result["cpu_baseline"] = cpu_baseline(w, oracle.ring_grid_x(beta), alm_h, blm_h, g_cols, args.cpu_seconds)
        del Gc
    B.set_tile_ex(B.TC_OP_FWD, 0, 0, 0)
    B.set_tile_ex(B.TC_OP_ADJ, 0, 0, 0)
    if args.pol_reps > 0:
        del C
        torch.cuda.empty_cache()
        log("polarised forward")
        result["polarised"] = side_leg("polarised forward", polarised_compare, w, beta, alm, blm, args.pol_reps,
                                       not args.no_tune)
        C = None
    if args.batched_reps > 0:
        del C, G
        torch.cuda.empty_cache()
        log("batched sixteen-detector comparison")
        result["batched"] = side_leg("batched comparison", batched_compare, args.batched_reps, not args.no_tune)
    C = G = None
    torch.cuda.empty_cache()
    if args.config_reps > 0:
        log("the other workloads")
        result["configs"] = {n: side_leg(f"workload {n}", config_timing, n, args.config_reps, not args.no_tune)
                             for n in ("small", "medium", "adjoint")}
    if args.large_reps > 0:
        log("four lmax 8192 detectors, one ring chunk")
        result["large4_chunk"] = side_leg("large chunk", large_chunk_timing, args.large_reps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
