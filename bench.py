#!/usr/bin/env python3
"""Throughput of the density-matrix approximate contraction on one MI355X.

Workload (one step): the 64x64 open 2D Ising lattice (J=1, h=0) at the 8 inverse
temperatures linspace(0.30, 0.60, 8), each at max_rank chi in {32, 64} and
env_size in {1, 2}: 32 networks, contracted in ONE persistent launch (one
workgroup per network, replayed from a captured HIP graph). Inputs are uploaded
once before timing (tn_create).

Prints one JSON line: networks/s over the timed steps (plain FP64 method), the
roofline of the interpreter kernel (algorithmic GEMM flops per launch over its
HIP-event duration), the per-site error of every result against the stored oracle
values, and the same workload in each other form, every form timed as the median
of several launches: split BF16x3 / FP16x3 contractions of environments and density
matrices, the learned warm start of the eigensolve (an MLP trained on the GPU
beforehand on density matrices of the 6x6, 64x64 and 3D lattice workloads), and
their combination, the mixed + batched + learned form. Each form reports how many
of its results lie within 1e-8 per site of the oracle and its networks/s counting
only those, next to plain FP64 at the same keep cutoff. The CPU oracle is timed on
a bounded sample of the same workload.
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
PEAK_16BIT_TFLOPS = 2500.0      # MI355X dense BF16 / FP16 matrix cores
# HBM bytes per launch of interp_kernel on this workload: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0
# (factors from a 256 MiB copy), from profiles/interp_kernel_w2_64x64_fp64_hbm.txt. None
# whenever the kernel has changed since the counters were taken.
TRAFFIC_BYTES = 3.687e9
SPLIT_TAU_REL = 1e-10   # keep cutoff of the split-precision forms (relative to the largest eigenvalue)
BOUND = 1e-8            # accuracy the forms are counted at (per site, against the oracle)


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sample: int):
    """The oracle, untuned, on `sample` networks of the same workload (all host threads the
    BLAS uses), and on one network with one thread."""
    from paper_2406_09769_amd import inputs
    from oracle import dm
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count()
    betas = inputs.w2_betas()
    full = [(chi, env, b) for chi, env in GROUPS for b in betas]      # the step's 32 networks
    sample = min(sample, len(full))
    picks = [full[(i * len(full)) // sample] for i in range(sample)]   # spread over the step
    t0 = time.perf_counter()
    for chi, env, b in picks:
        dm.contract_approx(inputs.ising_2d(64, 64, b), chi, env)
    dt = time.perf_counter() - t0
    out = {"value": len(picks) / dt, "unit": "networks/s", "cores": int(threads), "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": (f"all 32 networks of the step" if len(picks) == len(full) else
                      f"{len(picks)} of the 32 networks (chi, env, beta): "
                      f"{[(c, e, round(b, 4)) for c, e, b in picks]}") + f"; {dt:.1f} s on the host"}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            dm.contract_approx(inputs.ising_2d(64, 64, betas[0]), 32, 2)
            d1 = time.perf_counter() - t1
        out["one_thread"] = {"value": 1.0 / d1, "unit": "networks/s",
                             "sample": f"1 network (beta {betas[0]:g}, chi 32, env 2), {d1:.1f} s"}
    return out


def time_form(T, handles, slices, chis, envs, reps, **kw):
    """Median wall time of `reps` launches of the batch (after one untimed launch)."""
    import statistics
    import torch
    T.tn_contract_approx_batch(handles, slices, chis, envs, **kw)
    walls, kern, rs = [], [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs = T.tn_contract_approx_batch(handles, slices, chis, envs, **kw)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t)
        kern.append(rs[0].seconds)
    return statistics.median(walls), statistics.median(kern), rs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=32, help="networks timed in the CPU oracle (0 = skip)")
    ap.add_argument("--no-forms", action="store_true", help="skip the runs of the other forms")
    ap.add_argument("--form-reps", type=int, default=5, help="timed launches per form (median)")
    ap.add_argument("--no-tune", action="store_true", help="skip the GEMM block autotuner (built-in shapes)")
    ap.add_argument("--cubic", type=int, default=0, metavar="CHI",
                    help="only contract the 8x8x8 3D lattice (beta 0.2217, plane slices) once at max_rank CHI "
                         "and print its time (the chip-wide op path) and exit")
    ap.add_argument("--cubic-precision", choices=["fp64", "bf16x3", "fp16x3", "bf16x3_all"], default="fp64",
                    help="contraction arithmetic of the --cubic run")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a buffer of MIB MiB once on the GPU (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.cubic > 0:
        import torch
        from paper_2406_09769_amd import inputs, tnapprox as T
        net = inputs.ising_3d(8, 8, 8, 0.2217)
        h = T.create_network(net)
        prec = {"fp64": T.TN_FP64, "bf16x3": T.TN_SPLIT_BF16X3, "fp16x3": T.TN_SPLIT_FP16X3,
                "bf16x3_all": T.TN_SPLIT_BF16X3_ALL}[args.cubic_precision]
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
    # Every form runs the same 32 networks in one launch and is timed as the median of
    # --form-reps launches. The split forms drop eigenvalues below 1e-10 of the largest: their
    # 16-bit products resolve nothing below that (the FP32 sums inside each 16-bit matrix
    # instruction leave about 6e-8 of ||L||), and plain FP64 at the same cutoff is timed beside
    # them, so that the arithmetic is compared at equal method settings.
    from paper_2406_09769_amd.learned import train_warm_start_model
    model = None if args.no_forms else train_warm_start_model(T)
    form_list = [] if args.no_forms else [
        ("fp64", dict()),
        ("fp64_tau_rel_1e-10", dict(tau_rel=SPLIT_TAU_REL)),
        ("split_bf16x3", dict(precision=T.TN_SPLIT_BF16X3, tau_rel=SPLIT_TAU_REL)),
        ("split_fp16x3", dict(precision=T.TN_SPLIT_FP16X3, tau_rel=SPLIT_TAU_REL)),
        ("split_bf16x3_all", dict(precision=T.TN_SPLIT_BF16X3_ALL, tau_rel=SPLIT_TAU_REL)),
        ("learned_warm_start", dict(eig=T.TN_EIG_LEARNED, model=model)),
        ("mixed_batched_learned", dict(precision=T.TN_SPLIT_BF16X3, tau_rel=SPLIT_TAU_REL, eig=T.TN_EIG_LEARNED,
                                       model=model)),
    ]
    for name, kw in form_list:
        wall, kern, rf = time_form(T, handles, slices, chis, envs, args.form_reps, stream=stream, **kw)
        ef = golden_errors(rf, chis, envs)
        within = sum(e <= BOUND for e in ef) if ef else None
        fl = sum(r.flops for r in rf)
        sfl = sum(r.split_flops for r in rf)
        forms[name] = {"networks_per_s": round(len(nets) / wall, 4), "median_wall_ms": round(wall * 1e3, 3),
                       "kernel_ms": round(kern * 1e3, 3),
                       "max_dlnZ_per_site_vs_oracle": (max(ef) if ef else None),
                       "within_1e-8": within,
                       "networks_per_s_within_1e-8": (round(within / wall, 4) if ef else None),
                       "gemm_flops": fl,
                       "fp64_mfma_frac": round((fl - sfl) / kern / 1e12 / PEAK_FP64_TFLOPS, 8)}
        if sfl:
            # each split contraction issues six 16-bit products per FP64 one
            forms[name]["split_flops"] = sfl
            forms[name]["issued_16bit_mfma_flops"] = 6 * sfl
            forms[name]["mfma_16bit_frac"] = round(6 * sfl / kern / 1e12 / PEAK_16BIT_TFLOPS, 9)
        if kw.get("eig") == T.TN_EIG_LEARNED:
            forms[name]["warm_starts_accepted"] = sum(r.n_learned for r in rf)
            forms[name]["eigensolves"] = sum(r.n_eig for r in rf)
        print(f"[bench] form {name}: {json.dumps(forms[name])}", file=sys.stderr, flush=True)
    metric_summary = None
    if "mixed_batched_learned" in forms:
        mx, fp = forms["mixed_batched_learned"], forms["fp64"]
        metric_summary = {
            "mixed_batched_learned_networks_per_s_within_1e-8": mx["networks_per_s_within_1e-8"],
            "plain_fp64_networks_per_s_within_1e-8": fp["networks_per_s_within_1e-8"],
            "ratio": round(mx["networks_per_s_within_1e-8"] / fp["networks_per_s_within_1e-8"], 4),
            "mixed_mfma_16bit_frac": mx.get("mfma_16bit_frac"),
            "plain_fp64_mfma_frac": fp["fp64_mfma_frac"]}

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
        "metric_summary": metric_summary,
        "gemm_blocks": {"config": gemm_config, "autotune": tune_report},
    }
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
