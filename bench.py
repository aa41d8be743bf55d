"""Benchmark of the early-abandoning pruned DTW hot path on one MI355X.

One step = the nearest-neighbour subsequence search of the noisy
multi-sinusoid workload (2,000,000-point series, query of length 256 cut from
an independent realisation plus N(0, 0.1) noise) at every window of the
workload, r in {0, 13, 26, 52} (0, 5, 10, 20 % of 256): z-normalised window
statistics, pruned and early-abandoned DTW of every candidate, shared
best-so-far.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line (rank 0): candidates/s over the step, effective and
nominal cells/s, pruned fraction, the VALU roofline of the dominant kernel
(5 float32 operations per evaluated cell against the 157.3 TFLOP/s vector
peak) and the FP64 CPU oracle timed on a bounded sample on this host; beside
the timed steps, the same searches with the lower-bound cascade
(`lb_cascade`) and as one batched call (`batched`).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NN-search candidates/s + effective DTW GCUPS (1 MI355X); fwd+bwd pairs/s"
PEAK_HBM = 8.0e12  # bytes/s, MI355X HBM3E
PEAK_FP32_VALU = 157.3e12        # FLOP/s, MI355X vector FP32 (256 CUs x 2.4 GHz x 256)
OPS_PER_CELL = 5                 # sub, mul, add, two 2-input mins
BORDER_MIN_WINDOW = 24           # windows served by the bordered band kernel
M = 256
N_SERIES = 2_000_000


# The sources each measured kernel is compiled from (by name prefix): a
# counter figure taken on other sources no longer describes the kernel.
KERNEL_SOURCES = {
    "nn_band_kernel": ("band.h", "common.h"),
    "ed_search_kernel": ("ed.hip", "band.h", "common.h"),
    "wide_kernel": ("wide.h", "band.h", "common.h"),
    "wf_fwd_kernel": ("wf.hip", "wf.h", "common.h"),
    "wf_grad_kernel": ("wf.hip", "wf.h", "common.h"),
}


def kernel_source_hash(kernel: str):
    files = next((v for k, v in KERNEL_SOURCES.items() if kernel.startswith(k)), None)
    if files is None:
        return None
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2010_05371_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (scaled FETCH_SIZE + WRITE_SIZE), if they were taken on the
    kernel's current source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get("kernels", {}).get(kernel)
    if not isinstance(e, dict) or e.get("source_hash") != kernel_source_hash(kernel):
        return None
    return e.get("bytes")


def cpu_baseline(q32, x32, windows, budget_s: float):
    """The FP64 oracle (brute force, every window) on a bounded sample of offsets."""
    import numpy as np

    import gen
    import oracle
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    threads = oracle.default_threads()
    # calibrate on a small sample, then size the sample to the budget
    probe = 64 * threads
    t0 = time.perf_counter()
    for w in windows:
        oracle.nn_dists(q, x, w, np.arange(probe), nthreads=threads)
    dt = time.perf_counter() - t0
    n = int(max(probe, min(x.size - q.size + 1, probe * budget_s / max(dt, 1e-6))))
    offs = np.linspace(0, x.size - q.size, n).astype(np.int64)
    t0 = time.perf_counter()
    for w in windows:
        oracle.nn_dists(q, x, w, offs, nthreads=threads)
    dt = time.perf_counter() - t0
    # the same oracle on one thread, on a sample a tenth as large
    n1 = max(probe // 4, n // (10 * threads))
    offs1 = np.linspace(0, x.size - q.size, n1).astype(np.int64)
    t0 = time.perf_counter()
    for w in windows:
        oracle.nn_dists(q, x, w, offs1, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n * len(windows) / dt, "unit": "candidates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} evenly spaced offsets of the 2,000,000-point series, each at windows "
                      f"{list(windows)}, brute-force FP64 full-matrix DTW with two-pass "
                      f"z-normalisation ({dt:.1f} s on {threads} threads)",
            "one_core_value": n1 * len(windows) / dt1,
            "one_core_sample": f"{n1} evenly spaced offsets at each window ({dt1:.1f} s)",
            "cpu_model": _cpu_model()}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_eap_scan(q32, x32, windows, budget_s: float, gpu_per_window):
    """The paper's method on the CPU: the nearest-neighbour scan with the
    EAPrunedDTW model (Algorithm 3) bounded by a shared best-so-far, over a
    contiguous prefix of the offsets at each window, multi-threaded; its
    evaluated cells per candidate beside the GPU's."""
    import numpy as np

    import gen
    import oracle
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    threads = oracle.default_threads()
    K = x.size - q.size + 1
    probe = 256 * threads
    t0 = time.perf_counter()
    for w in windows:
        oracle.eap_scan(q, x, w, np.arange(probe), nthreads=threads)
    dt = time.perf_counter() - t0
    n = int(max(probe, min(K, probe * budget_s / max(dt, 1e-6))))
    per_window = {}
    t_all = 0.0
    for w in windows:
        t0 = time.perf_counter()
        k, d, cells = oracle.eap_scan(q, x, w, np.arange(n), nthreads=threads)
        dtw = time.perf_counter() - t0
        t_all += dtw
        g = gpu_per_window[str(w)]
        per_window[str(w)] = {"candidates_per_s": n / dtw, "best_offset_in_prefix": k,
                              "cells_per_candidate": cells / n,
                              "gpu_cells_per_candidate": g["cells_evaluated"] / K}
    return {"value": n * len(windows) / t_all, "unit": "candidates/s", "cores": threads,
            "kind": "oracle EAPrunedDTW model scan",
            "sample": f"the first {n} offsets of the 2,000,000-point series at each window "
                      f"{list(windows)} ({t_all:.1f} s on {threads} threads)",
            "per_window": per_window}


def lb_cascade(eap, q, x, windows, K, steps, plain_rec):
    """The same searches with the lower-bound cascade in front of the DTW
    (reported beside the plain search, outside its timed steps): wall time per
    window, the cascade's counters, and the answer check against the plain
    search."""
    import time as _t

    import torch

    out = {}
    tot_ms = 0.0
    for w in windows:
        eap.nn_search_lb(q, x, w)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        for _ in range(steps):
            (k, d), st = eap.nn_search_lb(q, x, w, stats=True)
        torch.cuda.synchronize()
        ms = (_t.perf_counter() - t0) * 1e3 / steps
        tot_ms += ms
        kp, dp = plain_rec[w][-1][0], plain_rec[w][-1][1]
        out[str(w)] = {"offset": k, "dist": d, "same_as_plain": (k, d) == (kp, dp), "wall_ms": round(ms, 4),
                       "gpu_ms": round(st["kernel_ms"], 4), "bounds_ms": round(st["lb_ms"], 4),
                       "dtw_ms": round(st["main_kernel_ms"], 4),
                       "pruned_kim": st["pruned_kim"], "pruned_keogh_eq": st["pruned_keogh_eq"],
                       "pruned_recheck": st["pruned_recheck"], "dtw_candidates": st["dtw_candidates"],
                       "cells_evaluated": st["cells_evaluated"]}
    return {"candidates_per_s": K * len(windows) / (tot_ms / 1e3), "ms_per_step": round(tot_ms, 4),
            "per_window": out}


def batched(eap, q, x, windows, K, steps, plain_rec):
    """The same four searches as one batched call (reported beside the plain
    search, outside its timed steps): the band-window launches run side by
    side on concurrent streams, and the CUs one launch's late waves leave idle
    take the others' waves."""
    import time as _t

    import torch

    qs = [(q, w) for w in windows]
    res = eap.nn_search_batch(qs, x)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    for _ in range(steps):
        res = eap.nn_search_batch(qs, x)
    torch.cuda.synchronize()
    ms = (_t.perf_counter() - t0) * 1e3 / steps
    same = all(tuple(r) == (plain_rec[w][-1][0], plain_rec[w][-1][1]) for r, w in zip(res, windows))
    return {"candidates_per_s": K * len(windows) / (ms / 1e3), "ms_per_step": round(ms, 4),
            "same_as_plain": same, "streams": eap.get_option("batch_branches")}


def _events_ms(pairs):
    return float(sum(a.elapsed_time(b) for a, b in pairs) / max(len(pairs), 1))


def c5_section(eap, steps, cpu_budget):
    """Differentiation workload: 4,096 pairs of z-normalised random walks of
    length 256 (the second a warped noisy copy), window 26.  Forward with the
    path record, backward to both series' gradients, and the distance-only
    forward, called through the C ABI on torch's current stream with inputs
    resident on the GPU.  Per-launch times come from HIP events around each
    call (the recorded forward and the distance-only forward are one kernel
    launch each); the autograd.Function wall time is reported beside them."""
    import ctypes

    import torch

    import gen
    S32, T32, w = gen.c5()
    dev = torch.device("cuda:0")
    S = torch.from_numpy(S32).to(dev)
    T = torch.from_numpy(T32).to(dev)
    P, L = S.shape
    ctx = eap.context(0)
    ctx.bind_stream()
    lib, h, p = ctx._lib, ctx.handle, eap._ptr
    rec = torch.empty(int(lib.eapdtw_dtw_ckpt_bytes(P, L, w)), device=dev, dtype=torch.uint8)
    out = torch.empty(P, device=dev)
    gout = torch.ones(P, device=dev)
    gS, gT = torch.empty_like(S), torch.empty_like(T)
    cls_rec = eap.dtw_kernel_class(P, L, w, True)
    cls_fwd = eap.dtw_kernel_class(P, L, w, False)

    def fwd_rec():
        ctx.check(lib.eapdtw_dtw_fwd(h, p(S), p(T), P, L, w, p(out), ctypes.c_void_p(rec.data_ptr())))

    def bwd():
        ctx.check(lib.eapdtw_dtw_bwd(h, p(S), p(T), P, L, w, ctypes.c_void_p(rec.data_ptr()),
                                     p(gout), p(gS), p(gT)))

    def fwd_only():
        ctx.check(lib.eapdtw_dtw_fwd(h, p(S), p(T), P, L, w, p(out), None))

    def wall_ms(fns):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for fn in fns:
                fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    def launch_ms(fn):
        """Average GPU time of one call in a burst of back-to-back calls (the
        host queues ahead of the GPU, so the events bracket the launch
        itself)."""
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        evs[0].record()
        for k in range(steps):
            fn()
            evs[k + 1].record()
        torch.cuda.synchronize()
        return _events_ms(list(zip(evs[:-1], evs[1:])))

    def step_launch_ms():
        """GPU time of the recorded forward and of the backward as they run
        in the forward + backward loop (events between the alternating calls;
        a gap where the GPU waits for the host counts in the launch after it)."""
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
        torch.cuda.synchronize()
        evs[0].record()
        for k in range(steps):
            fwd_rec()
            evs[2 * k + 1].record()
            bwd()
            evs[2 * k + 2].record()
        torch.cuda.synchronize()
        return (_events_ms([(evs[2 * k], evs[2 * k + 1]) for k in range(steps)]),
                _events_ms([(evs[2 * k + 1], evs[2 * k + 2]) for k in range(steps)]))

    for _ in range(3):
        fwd_rec()
        bwd()
        fwd_only()
    fb_ms = wall_ms((fwd_rec, bwd))
    f_ms = wall_ms((fwd_only,))
    fwd_rec_step_ms, bwd_step_ms = step_launch_ms()
    fwd_rec_ms = launch_ms(fwd_rec)
    bwd_ms = launch_ms(bwd)
    fwd_ms = launch_ms(fwd_only)
    # the same two calls captured once as a HIP graph and replayed: one host
    # launch per step keeps the GPU fed back to back (the C-ABI loop above is
    # bound by the host's per-call work, and the GPU idles between calls)
    gS_eager, gT_eager = gS.clone(), gT.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx.bind_stream()
        for _ in range(3):
            fwd_rec()
            bwd()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ctx.bind_stream()
        fwd_rec()
        bwd()
    ctx.bind_stream()
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    graph_same = bool(torch.equal(gS, gS_eager) and torch.equal(gT, gT_eager))
    del graph
    # the same through autograd.Function (Python wall time per step)
    Sg, Tg = S.clone().requires_grad_(True), T.clone().requires_grad_(True)
    for _ in range(2):
        eap.DTWFunction.apply(Sg, Tg, w).sum().backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        Sg.grad = None
        Tg.grad = None
        eap.DTWFunction.apply(Sg, Tg, w).sum().backward()
    torch.cuda.synchronize()
    ag_ms = (time.perf_counter() - t0) * 1e3 / steps
    same = bool(torch.equal(Sg.grad, gS) and torch.equal(Tg.grad, gT))
    # the same pairs one call each (the first 256, distance-only forward)
    n1 = min(P, 256)
    o1 = torch.empty(1, device=dev)

    def per_pair():
        for i in range(n1):
            ctx.check(lib.eapdtw_dtw_fwd(h, p(S[i]), p(T[i]), 1, L, w, p(o1), None))

    per_pair()
    pp_ms = wall_ms((per_pair,)) if steps >= 1 else float("nan")
    cells = P * _band_cells(L, L, w)
    k_rec = f"wf_fwd_kernel<{cls_rec['lanes']}, {cls_rec['slots']}, {2 if cls_rec['codes_in_lds'] else 1}>"
    k_fwd = f"wf_fwd_kernel<{cls_fwd['lanes']}, {cls_fwd['slots']}, 0>"
    res = {
        "workload": "dtw fwd+bwd: 4,096 warped random-walk pairs, length 256, window 26",
        "pairs": P, "len": L, "window": w, "steps": steps,
        "fwd_bwd_pairs_per_s": P / (fb_ms / 1e3), "fwd_bwd_ms": round(fb_ms, 4),
        "fwd_pairs_per_s": P / (f_ms / 1e3), "fwd_ms": round(f_ms, 4),
        "per_pair_calls_fwd_pairs_per_s": n1 / (pp_ms / 1e3),
        "graph_fwd_bwd_pairs_per_s": P / (graph_ms / 1e3), "graph_fwd_bwd_ms": round(graph_ms, 4),
        "graph_grads_equal_eager": graph_same,
        "autograd_fwd_bwd_pairs_per_s": P / (ag_ms / 1e3), "autograd_fwd_bwd_ms": round(ag_ms, 4),
        "autograd_grads_equal_c_abi": same,
        # per-launch GPU times: in the forward + backward loop, and in bursts
        # of back-to-back calls of one kind
        "recorded_fwd_launch_ms": round(fwd_rec_step_ms, 4), "bwd_launch_ms": round(bwd_step_ms, 4),
        "recorded_fwd_burst_launch_ms": round(fwd_rec_ms, 4), "bwd_burst_launch_ms": round(bwd_ms, 4),
        "fwd_launch_ms": round(fwd_ms, 4),
        "band_cells": cells,
        "roofline_fwd_bwd": _valu_roofline(k_rec, cells, fwd_rec_step_ms),
        "roofline_fwd": _valu_roofline(k_fwd, cells, fwd_ms),
    }
    if cpu_budget > 0:
        res["cpu_baseline"] = _c5_cpu(S32, T32, w, cpu_budget)
    return res


def _band_cells(ls, lt, r):
    """In-band cells of an ls x lt matrix under window r (Section 2.1)."""
    n = 0
    for i in range(ls):
        lo, hi = max(0, i - r), min(lt - 1, i + r)
        n += max(0, hi - lo + 1)
    return n


def _valu_roofline(kernel, cells, ms):
    achieved = OPS_PER_CELL * cells / (ms / 1e3)
    traffic = load_traffic(kernel)
    return {"bound": "alu", "kernel": kernel, "achieved": achieved / 1e12,
            "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
            "traffic": traffic, "ops_per_cell": OPS_PER_CELL, "cells_per_launch": cells,
            "launch_ms": round(ms, 5),
            "hbm_gbs": traffic / (ms / 1e3) / 1e9 if traffic else None}


def _c5_cpu(S32, T32, w, budget_s):
    """The FP64 oracle's DTW with its path gradient on a sample of the pairs."""
    import gen
    import oracle
    t0 = time.perf_counter()
    n = 0
    while n < S32.shape[0] and time.perf_counter() - t0 < budget_s:
        oracle.dtw_grad(gen.as_oracle(S32[n]), gen.as_oracle(T32[n]), w)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {n} pairs, FP64 full-matrix DTW with the optimal path's "
                      f"gradient, one thread ({dt:.1f} s)"}


def c1_section(eap, steps):
    """Small search: a 128-point random-walk query against an independent
    20,000-point random walk, window 13 (per call: candidates/s, effective and
    nominal GCUPS, the pruned-or-abandoned fraction, the main kernel's VALU
    fraction)."""
    import numpy as np
    import torch

    import gen
    q32, x32, w = gen.c1()
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    K = x.numel() - q.numel() + 1
    for _ in range(3):
        eap.nn_search(q, x, w)
    torch.cuda.synchronize()
    walls, sts = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        (k, d), st = eap.nn_search(q, x, w, stats=True)
        walls.append((time.perf_counter() - t0) * 1e3)
        sts.append(st)
    wall = float(np.median(walls))
    main_ms = float(np.median([s_["main_kernel_ms"] for s_ in sts]))
    st = sts[-1]
    r = _valu_roofline(f"nn_band_kernel<{w}, 4, false, false>", st["cells_evaluated"], main_ms)
    return {"workload": "nn_search random walk n=20,000, m=128, window 13", "candidates": K,
            "steps": steps, "candidates_per_s": K / (wall / 1e3), "call_ms": round(wall, 4),
            "main_kernel_ms": round(main_ms, 4), "best": [int(k), float(d)],
            "effective_gcups": st["cells_evaluated"] / (wall / 1e3) / 1e9,
            "nominal_gcups": st["cells_nominal"] / (wall / 1e3) / 1e9,
            "pruned_fraction": 1.0 - st["cells_evaluated"] / st["cells_nominal"], "roofline": r}


C3_KERNEL = "wide_kernel<64, 1, false>"  # the tiled kernel: 64-row tiles, pairwise, whole window


ERP_OPS_PER_CELL = 7  # |a-b|, |b-g| (subtractions), three additions, a 3-way minimum (2)


def erp_section(eap, steps):
    """ERP (edit distance with real penalty) of a batch of pairs: 262,144 pairs
    of a z-normalised random walk of length 256 and a warped noisy copy (4,096
    distinct pairs, repeated), gap value 0, no bound, windows 13 / 26 / 52;
    one pair per lane, so the batch is sized to give every SIMD two waves."""
    import numpy as np
    import torch

    import gen
    X, Y = gen.erp_pairs()
    x, y = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    P, L = X.shape
    per = {}
    for w in (13, 26, 52):
        eap.erp_pairs(x, y, w, 0.0, stats=True)
        ms = []
        for _ in range(steps):
            _, st = eap.erp_pairs(x, y, w, 0.0, stats=True)
            ms.append(st["main_kernel_ms"])
        m = sum(ms) / len(ms)
        cells = st["cells_evaluated"]
        achieved = ERP_OPS_PER_CELL * cells / (m / 1e3)
        per[str(w)] = {"kernel_ms": round(m, 4), "pairs_per_s": P / (m / 1e3), "cells": cells,
                       "cells_per_s": cells / (m / 1e3),
                       "roofline": {"bound": "alu", "kernel": f"erp_pairs_kernel<{w}>",
                                    "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                                    "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                                    "traffic": None, "ops_per_cell": ERP_OPS_PER_CELL}}
    return {"workload": "ERP of 262,144 pairs of length 256 (random walk vs warped copy), g = 0",
            "pairs": P, "len": L, "steps": steps, "per_window": per}


def c3_section(eap, steps):
    """All pairs (Section 2.3 pruning, bound = squared Euclidean distance per
    pair): 2,000 z-normalised random walks of length 512, full window; the
    unordered pairs (DTW is symmetric, so they give the ordered 2M)."""
    import torch

    import gen
    X32, w = gen.c3()
    X = torch.from_numpy(X32).cuda()
    N = X.shape[0]
    eap.pairwise(X, w)
    torch.cuda.synchronize()
    sts = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = eap.pairwise(X, w, stats=True)
        sts.append(st)
    wall = (time.perf_counter() - t0) * 1e3 / steps
    st = sts[-1]
    main_ms = sum(s["main_kernel_ms"] for s in sts) / len(sts)
    npairs = N * (N - 1) // 2
    r = _valu_roofline(C3_KERNEL, st["cells_evaluated"], main_ms)
    r["cells_computed_per_launch"] = st["cells_computed"]
    return {"workload": "all pairs: 2,000 random walks of length 512, full window, ub = ED",
            "pairs": npairs, "steps": steps, "pairs_per_s": npairs / (wall / 1e3),
            "call_ms": round(wall, 4), "main_kernel_ms": round(main_ms, 4),
            "cells_nominal": st["cells_nominal"], "cells_evaluated": st["cells_evaluated"],
            "pruned_fraction": 1.0 - st["cells_evaluated"] / st["cells_nominal"],
            "roofline": r}


def c4_section(eap, steps, variants=True):
    """Batched uneven search: 64 random-walk queries (lengths 64-1024, windows
    5-20 %) against a 10,000,000-point random walk, as one batched call and as
    64 single-query calls."""
    import torch

    import gen
    queries, windows, series = gen.c4()
    x = torch.from_numpy(series).cuda()
    qs = [(torch.from_numpy(q).cuda(), w) for q, w in zip(queries, windows)]
    cands = sum(x.numel() - q.numel() + 1 for q, _ in qs)
    eap.nn_search_batch(qs, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res, st = eap.nn_search_batch(qs, x, stats=True)
    b_ms = (time.perf_counter() - t0) * 1e3 / steps
    single = [eap.nn_search(q, x, w) for q, w in qs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev = 0
    for _ in range(steps):
        single = []
        for q, w in qs:
            r1, s1 = eap.nn_search(q, x, w, stats=True)
            single.append(r1)
            ev += s1["cells_evaluated"]
    s_ms = (time.perf_counter() - t0) * 1e3 / steps
    same = all(a == b for a, b in zip(res, single))
    if not variants:
        return _c4_line(qs, cands, steps, b_ms, s_ms, same, st, ev, None)
    # the batched call without the graph (every launch issued by the host)
    eap.set_option("graph", 0)
    try:
        eap.nn_search_batch(qs, x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res_ng = eap.nn_search_batch(qs, x)
        ng_ms = (time.perf_counter() - t0) * 1e3 / steps
    finally:
        eap.set_option("graph", 1)
    # with the autotuner's choices per (length, window) bucket (the tuning
    # runs once, outside the timed calls)
    t0 = time.perf_counter()
    eap.set_option("autotune", 1)
    try:
        eap.nn_search_batch(qs, x)
        tune_s = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res_at = eap.nn_search_batch(qs, x)
        at_ms = (time.perf_counter() - t0) * 1e3 / steps
    finally:
        eap.set_option("autotune", 0)
    return _c4_line(qs, cands, steps, b_ms, s_ms, same, st, ev,
                    {"batched_no_graph_ms": round(ng_ms, 3), "no_graph_same_answers": res_ng == res,
                     "batched_autotuned_ms": round(at_ms, 3), "autotune_seconds": round(tune_s, 2),
                     "autotuned_same_answers": res_at == res})


def _c4_line(qs, cands, steps, b_ms, s_ms, same, st, ev, extra):
    line = {"workload": "batched uneven search: 64 queries (m 64-1024, r 5-20%) vs 10,000,000 points",
            "queries": len(qs), "candidates": cands, "steps": steps,
            "batched_candidates_per_s": cands / (b_ms / 1e3), "batched_ms": round(b_ms, 3),
            "single_calls_candidates_per_s": cands / (s_ms / 1e3), "single_calls_ms": round(s_ms, 3),
            "speedup_batched_vs_single": s_ms / b_ms, "same_answers": same,
            "batched_cells_evaluated": st["cells_evaluated"],
            "batched_cells_nominal": st["cells_nominal"],
            "single_cells_evaluated": ev // steps,
            "batched_effective_gcups": st["cells_evaluated"] / (b_ms / 1e3) / 1e9}
    if extra:
        line.update(extra)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of CPU oracle work for cpu_baseline (0 = skip)")
    ap.add_argument("--n", type=int, default=N_SERIES)
    ap.add_argument("--lb-steps", type=int, default=5,
                    help="repetitions of the lower-bound cascade searches reported beside "
                         "the plain ones (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="repetitions of the four searches as one batched call reported "
                         "beside the plain ones (0 = skip)")
    ap.add_argument("--batch-streams", type=int, default=0,
                    help="streams of the batched call's band launches (0 = the library's "
                         "default)")
    ap.add_argument("--c5-steps", type=int, default=50,
                    help="steps of the differentiation workload (4,096 pairs fwd and fwd+bwd; "
                         "0 = skip)")
    ap.add_argument("--erp-steps", type=int, default=5,
                    help="repetitions per window of the ERP pairs workload (0 = skip)")
    ap.add_argument("--c1-steps", type=int, default=10,
                    help="calls of the small search workload (0 = skip)")
    ap.add_argument("--c4-variants", type=int, default=1,
                    help="1 = also time the batched call without its graph and with the "
                         "autotuner's choices (0 = skip)")
    ap.add_argument("--c3-steps", type=int, default=3,
                    help="repetitions of the all-pairs workload (0 = skip)")
    ap.add_argument("--c4-steps", type=int, default=2,
                    help="repetitions of the batched uneven search and of its 64 single calls "
                         "(0 = skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-mebibyte buffer once (a plain copy of known size "
                         "that calibrates HBM byte counters in a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2010_05371_amd as eap

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    q32, x32, windows = gen.c2(n=args.n, m=M)
    q = torch.from_numpy(q32).to(dev)
    x = torch.from_numpy(x32).to(dev)
    K = x32.size - q32.size + 1
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe * (1 << 18), device=dev, dtype=torch.float32)
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst

    def step(record):
        for w in windows:
            (k, d), st = eap.nn_search(q, x, w, stats=True)
            if record is not None:
                record.setdefault(w, []).append((k, d, st))

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    rec = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    cand_per_step = K * len(windows)

    per_window = {}
    tot_eval = tot_nom = 0
    dom = None
    for w in windows:
        rs = rec[w]
        st = rs[-1][2]
        main_ms = float(np.mean([r[2]["main_kernel_ms"] for r in rs]))
        call_ms = float(np.mean([r[2]["kernel_ms"] for r in rs]))
        ev, nom, comp = st["cells_evaluated"], st["cells_nominal"], st["cells_computed"]
        tot_eval += ev
        tot_nom += nom
        per_window[str(w)] = {
            "offset": rs[-1][0], "dist": rs[-1][1], "call_ms": round(call_ms, 4),
            "main_kernel_ms": round(main_ms, 4), "candidates_per_s": K / (call_ms / 1e3),
            "cells_nominal": nom, "cells_evaluated": ev, "cells_computed": comp,
            "pruned_fraction": 1.0 - ev / nom, "abandoned": st["abandoned"],
            "effective_gcups_kernel": ev / (main_ms / 1e3) / 1e9,
        }
        if dom is None or main_ms > per_window[str(dom)]["main_kernel_ms"]:
            dom = w
    dw = per_window[str(dom)]
    achieved = OPS_PER_CELL * dw["cells_evaluated"] / (dw["main_kernel_ms"] / 1e3)
    kname = f"nn_band_kernel<{dom}, 4, false, {'true' if dom >= BORDER_MIN_WINDOW else 'false'}>"
    traffic = load_traffic(kname)
    line = {
        "metric": METRIC,
        "value": cand_per_step / (ms_per_step / 1e3),
        "unit": "candidates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "nn_search noisy multi-sinusoid n=2,000,000 m=256 windows {0,13,26,52}",
                   "n": int(x32.size), "m": M, "windows": list(windows),
                   "candidates_per_window": K},
        "effective_gcups": tot_eval / (ms_per_step / 1e3) / 1e9,
        "nominal_gcups": tot_nom / (ms_per_step / 1e3) / 1e9,
        "pruned_fraction": 1.0 - tot_eval / tot_nom,
        "per_window": per_window,
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU, "traffic": traffic,
                     "ops_per_cell": OPS_PER_CELL,
                     "cells_computed_per_launch": dw["cells_computed"],
                     "cells_per_launch": dw["cells_evaluated"],
                     "launch_ms": dw["main_kernel_ms"],
                     # HBM bandwidth of the same launch (measured bytes / event time)
                     # against the 8 TB/s peak: the path is not bandwidth-bound
                     "hbm_gbs": (traffic / (dw["main_kernel_ms"] / 1e3) / 1e9) if traffic else None,
                     "hbm_frac": (traffic / (dw["main_kernel_ms"] / 1e3) / PEAK_HBM) if traffic else None},
    }
    if args.lb_steps > 0:
        line["lb_cascade"] = lb_cascade(eap, q, x, windows, K, args.lb_steps, rec)
    if args.batch_steps > 0:
        if args.batch_streams > 0:
            eap.set_option("batch_branches", args.batch_streams)
        line["batched"] = batched(eap, q, x, windows, K, args.batch_steps, rec)
    if args.c1_steps > 0:
        line["c1_search"] = c1_section(eap, args.c1_steps)
    if args.c5_steps > 0:
        line["c5_fwd_bwd"] = c5_section(eap, args.c5_steps, min(args.cpu_budget, 5.0))
    if args.c3_steps > 0:
        line["c3_pairwise"] = c3_section(eap, args.c3_steps)
    if args.erp_steps > 0:
        line["erp_pairs"] = erp_section(eap, args.erp_steps)
    if args.c4_steps > 0:
        line["c4_batched"] = c4_section(eap, args.c4_steps, args.c4_variants != 0)
    if args.cpu_budget > 0:
        line["cpu_baseline"] = cpu_baseline(q32, x32, windows, args.cpu_budget)
        line["cpu_eap_scan"] = cpu_eap_scan(q32, x32, windows, min(args.cpu_budget, 8.0),
                                            per_window)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
