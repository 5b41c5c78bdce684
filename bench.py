#!/usr/bin/env python3
"""Throughput of the density-matrix approximate contraction on one MI355X.

Workload (one step): the 64x64 open 2D Ising lattice (J=1, h=0) at the 8 inverse
temperatures linspace(0.30, 0.60, 8), each at max_rank chi in {32, 64} and
env_size in {1, 2}: 32 networks, contracted in ONE persistent launch (one
workgroup per network). Inputs are uploaded once before timing (tn_create).

Prints one JSON line: networks/s over the timed steps (plain FP64 method), the
roofline of the interpreter kernel (algorithmic GEMM flops per launch over its
HIP-event duration), the per-site error of every result against the stored oracle
values, the same workload once in each other form (split BF16x3 / FP16x3
contractions; learned warm start of the eigensolve with an MLP trained on the GPU
beforehand) with its networks/s and worst error, and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "networks/s + MFMA util at |dlnZ|/N<=1e-8: mixed+batched+learned vs plain FP64"
PEAK_FP64_TFLOPS = 78.6          # MI355X FP64 (matrix and vector)
HBM_PEAK_GBS = 8000.0
GROUPS = [(32, 1), (32, 2), (64, 1), (64, 2)]
CUS = 256
# HBM bytes per launch of interp_kernel on this workload: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0
# (factors from a 256 MiB copy), from profiles/interp_kernel_w2_64x64_fp64_hbm.txt. Set to
# None whenever the kernel changes until the counters are taken again.
TRAFFIC_BYTES = 6.953e9
SPLIT_TAU_REL = 1e-10   # keep cutoff of the split-precision forms (relative to the largest eigenvalue)


def workload():
    from paper_2406_09769_amd import inputs
    nets, chis, envs = [], [], []
    for chi, env in GROUPS:
        for beta in inputs.w2_betas():
            nets.append(inputs.ising_2d(64, 64, beta))
            chis.append(chi)
            envs.append(env)
    return nets, chis, envs


def golden_errors(results, chis, envs):
    path = os.path.join(ROOT, "tests", "golden", "w2_oracle.json")
    if not os.path.exists(path):
        return None
    from paper_2406_09769_amd import inputs
    gold = json.load(open(path))["rows"]
    betas = inputs.w2_betas() * len(GROUPS)
    errs = []
    for r, chi, env, b in zip(results, chis, envs, betas):
        g = next(x for x in gold if x["chi"] == chi and x["env"] == env and abs(x["beta"] - b) < 1e-12)
        errs.append(abs(r.log_abs - g["log_abs"]) / 4096 if r.sign == g["sign"] else float("inf"))
    return errs


def train_model(T):
    """The warm-start MLP trained on rows the method harvests from small lattices."""
    from paper_2406_09769_amd import inputs
    ds = T.Dataset(400_000)
    for (L, b, chi) in ((16, 0.35, 16), (16, 0.44, 16), (16, 0.5, 16), (20, 0.44, 24)):
        net = inputs.ising_2d(L, L, b)
        T.tn_harvest(T.create_network(net), net.slices, chi, 1, ds)
    m = T.Model(seed=7)
    m.train(ds, steps=3000, batch=128, lr=3e-3, seed=11)
    return m


def cpu_baseline(sample: int):
    """The oracle, untuned, on `sample` networks of the same workload (host cores)."""
    import numpy as np  # noqa: F401
    from paper_2406_09769_amd import inputs
    from oracle import dm
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:
        threads = os.cpu_count()
    picks = []
    betas = inputs.w2_betas()
    for i in range(sample):
        chi, env = GROUPS[i % len(GROUPS)]
        picks.append((chi, env, betas[(3 * i + 3) % len(betas)]))
    t0 = time.perf_counter()
    for chi, env, b in picks:
        dm.contract_approx(inputs.ising_2d(64, 64, b), chi, env)
    dt = time.perf_counter() - t0
    return {"value": len(picks) / dt, "unit": "networks/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(picks)} of the 32 networks, one per (chi, env) in turn at betas "
                      f"{sorted(set(round(p[2], 4) for p in picks))}; {dt:.1f} s on the host"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=8, help="networks timed in the CPU oracle (0 = skip)")
    ap.add_argument("--no-forms", action="store_true", help="skip the runs of the other forms")
    ap.add_argument("--no-tune", action="store_true", help="skip the GEMM block autotuner (built-in shapes)")
    ap.add_argument("--cubic", type=int, default=0, metavar="CHI",
                    help="only contract the 8x8x8 3D lattice (beta 0.2217, plane slices) once at max_rank CHI "
                         "and print its time (the chip-wide op path) and exit")
    ap.add_argument("--cubic-precision", choices=["fp64", "bf16x3", "fp16x3"], default="fp64",
                    help="contraction arithmetic of the --cubic run")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a buffer of MIB MiB once on the GPU (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.cubic > 0:
        import torch
        from paper_2406_09769_amd import inputs, tnapprox as T
        net = inputs.ising_3d(8, 8, 8, 0.2217)
        h = T.create_network(net)
        prec = {"fp64": T.TN_FP64, "bf16x3": T.TN_SPLIT_BF16X3, "fp16x3": T.TN_SPLIT_FP16X3}[args.cubic_precision]
        stats = T.tn_plan_stats(h, net.slices, args.cubic, 1)
        T.tn_contract_approx(h, net.slices, args.cubic, 1, precision=prec)   # plan, workspace, graph capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = T.tn_contract_approx(h, net.slices, args.cubic, 1, precision=prec)
        dt = time.perf_counter() - t0
        print(json.dumps({"workload": "ising3d_8x8x8_open_J1_h0 beta 0.2217 plane slices", "chi": args.cubic,
                          "precision": args.cubic_precision,
                          "seconds": round(dt, 4), "kernel_s": round(r.seconds, 4), "log_abs": r.log_abs,
                          "sign": r.sign, "gemm_flops": r.flops, "plan": stats}), flush=True)
        return
    if args.copy_probe > 0:
        import torch
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the workload's networks "
              "are independent and would be split across GPUs, which this build does not do.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_09769_amd import tnapprox as T
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream

    nets, chis, envs = workload()
    handles = [T.create_network(n) for n in nets]
    slices = [n.slices for n in nets]
    print(f"[bench] {len(nets)} networks uploaded; warmup {args.warmup}, timed steps {args.steps}",
          file=sys.stderr, flush=True)
    gemm_config, tune_report = [0, 0, 0], None
    if not args.no_tune:
        from paper_2406_09769_amd.autotune import autotune
        gemm_config, tune_report = autotune(T, handles, slices, chis, envs, stream=stream)
        print(f"[bench] autotuned GEMM blocks: {json.dumps(tune_report)}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        T.tn_contract_approx_batch(handles, slices, chis, envs, stream=stream, gemm_config=gemm_config)
        print(f"[bench] warmup step {i} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kernel_s = []
    rs = None
    for i in range(args.steps):
        rs = T.tn_contract_approx_batch(handles, slices, chis, envs, stream=stream, gemm_config=gemm_config)
        kernel_s.append(rs[0].seconds)
        print(f"[bench] step {i}: {rs[0].seconds * 1e3:.1f} ms in the kernel", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = len(nets) / (ms_per_step / 1e3)

    prof = {}
    for name, i in (("beta0.44_chi64_env1", 8 * 2 + 3), ("beta0.44_chi32_env1", 3)):
        prof[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in T.tn_profile_last(handles[i]).items()
                      if not k.startswith("learned")}
    print(f"[bench] per-op device seconds of one network: {json.dumps(prof)}", file=sys.stderr, flush=True)
    flops = sum(r.flops for r in rs)
    eig_flops = sum(r.eig_flops for r in rs)
    ksec = sum(kernel_s) / len(kernel_s)
    achieved = flops / ksec / 1e12
    errs = golden_errors(rs, chis, envs)

    forms = {}
    # the split forms drop eigenvalues below 1e-10 of the largest: the split products do not
    # resolve them, and keeping their noise directions only raises the kept ranks (the worst
    # error against the oracle is the same as with 1e-15); the last form is plain FP64 with the
    # keep cutoff at 1e-12, the method's own speed / accuracy knob
    form_list = [] if args.no_forms else [
        ("split_bf16x3", lambda: dict(precision=T.TN_SPLIT_BF16X3, tau_rel=SPLIT_TAU_REL)),
        ("split_fp16x3", lambda: dict(precision=T.TN_SPLIT_FP16X3, tau_rel=SPLIT_TAU_REL)),
        ("learned_warm_start", lambda: dict(eig=T.TN_EIG_LEARNED, model=train_model(T))),
        ("fp64_tau_rel_1e-12", lambda: dict(tau_rel=1e-12))]
    for name, make_kw in form_list:
        kw = make_kw()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rf = T.tn_contract_approx_batch(handles, slices, chis, envs, stream=stream, **kw)
        torch.cuda.synchronize()
        dtf = time.perf_counter() - t1
        ef = golden_errors(rf, chis, envs)
        forms[name] = {"networks_per_s": round(len(nets) / dtf, 4), "kernel_ms": round(rf[0].seconds * 1e3, 3),
                       "max_dlnZ_per_site_vs_oracle": (max(ef) if ef else None),
                       "within_1e-8": (sum(e <= 1e-8 for e in ef) if ef else None)}
        if name.startswith("learned"):
            forms[name]["warm_starts_accepted"] = sum(r.n_learned for r in rf)
            forms[name]["eigensolves"] = sum(r.n_eig for r in rf)
        print(f"[bench] form {name}: {json.dumps(forms[name])}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "networks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "form": "plain FP64 (exact eigensolve), 32 networks in one persistent launch",
        "config": {"workload": "ising2d_64x64_open_J1_h0 x 8 betas linspace(0.30,0.60,8) x chi{32,64} x env{1,2}",
                   "networks": len(nets), "lattice": "64x64", "chi": [32, 64], "env_size": [1, 2]},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 5), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 7), "traffic": TRAFFIC_BYTES,
                     "workgroups": len(nets), "frac_of_cus_in_use": round(achieved / (PEAK_FP64_TFLOPS * len(nets) / CUS), 6),
                     "kernel": "interp_kernel", "kernel_ms": round(ksec * 1e3, 3),
                     "gemm_flops_per_launch": flops, "eig_flops_per_launch": eig_flops},
        "accuracy": {"max_dlnZ_per_site_vs_oracle": (max(errs) if errs else None),
                     "within_1e-8": (sum(e <= 1e-8 for e in errs) if errs else None)},
        "forms": forms,
        "gemm_blocks": {"config": gemm_config, "autotune": tune_report},
    }
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
