"""Autotuner of the FP64 contraction block shapes.

The pipelined GEMM has six block configurations (tn_options.gemm_config, numbered
1..6: 16x512 k8, 16x256 k16, 32x128 k32, 32x128 k16, 64x64 k32, 64x64 k16). GEMM ops
fall in three classes by their runtime row count (<= 16, <= 32, more). For each class
in turn, every candidate is run on the given networks with the classes already tuned
held at their choice, and the candidate with the least device time spent in GEMM ops
(summed over the networks, from tn_profile_last) is kept. All candidates compute the
same products; only the blocking differs.
"""
from __future__ import annotations

import time

CANDIDATES = {0: [1, 2, 3, 4, 5, 6], 1: [3, 4, 5, 6], 2: [3, 4, 5, 6]}
NAMES = {0: "built-in", 1: "16x512 k8", 2: "16x256 k16", 3: "32x128 k32", 4: "32x128 k16", 5: "64x64 k32",
         6: "64x64 k16"}


def autotune(T, handles, slices, chis, envs, stream=None, reps: int = 1):
    """Returns (config [3 ints], report dict). T is the tnapprox binding."""
    cfg = [0, 0, 0]
    report = {}
    t0 = time.perf_counter()
    for cls in range(3):
        times = {}
        for cand in [0] + CANDIDATES[cls]:
            trial = list(cfg)
            trial[cls] = cand
            best = None
            for _ in range(reps):
                T.tn_contract_approx_batch(handles, slices, chis, envs, stream=stream, gemm_config=trial)
                t = sum(T.tn_profile_last(h)["gemm"] for h in handles)
                best = t if best is None else min(best, t)
            times[cand] = best
        cfg[cls] = min(times, key=lambda c: (times[c], c))
        report[f"rows<={16 if cls == 0 else 32}" if cls < 2 else "rows>32"] = {
            NAMES[c]: round(v, 4) for c, v in times.items()}
    report["chosen"] = [NAMES[c] for c in cfg]
    report["seconds"] = round(time.perf_counter() - t0, 2)
    return cfg, report
