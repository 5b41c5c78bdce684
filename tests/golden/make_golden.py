"""Write oracle values for the full-size workloads into tests/golden/*.json.

Calls only oracle/ (and the seeded input generators). Usage:
    python tests/golden/make_golden.py w2   # 64x64 2D Ising, 8 betas x chi {32,64} x env {1,2}
    python tests/golden/make_golden.py w4   # 64 signed-J random 3-regular graphs, beta 1, chi 64
    python tests/golden/make_golden.py w5   # 32 random 3-SAT #CSP formulas, n 150, m 450, chi 32
    python tests/golden/make_golden.py w4spread  # how far FP64 fixes each W4 result (see spread())
    python tests/golden/make_golden.py w5small   # 8 random 3-SAT formulas, n 50, m 150, chi 32
    python tests/golden/make_golden.py w5smallspread  # how far FP64 fixes each of those results
    python tests/golden/make_golden.py w4eignoise      # add the eigensolver backward-error row to w4_spread
    python tests/golden/make_golden.py w5smalleignoise # ... and to w5_small_spread
    python tests/golden/make_golden.py w3   # 8x8x8 3D Ising at the 3 betas, chi 16, plane slices
    python tests/golden/make_golden.py w3chi32 0.2217   # the same lattice at chi 32, one beta
    python tests/golden/make_golden.py w3spread 0.25 [--hows=evr,perturbed_0,perturbed13_0]
                                            # how far FP64 fixes the W3 result at these betas
"""
import json
import math
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2406_09769_amd import inputs  # noqa: E402
from oracle import dm  # noqa: E402


def w2(out_path):
    rows = []
    for chi in (32, 64):
        for env in (1, 2):
            for beta in inputs.w2_betas():
                net = inputs.ising_2d(64, 64, beta)
                t = time.time()
                st = dm.Stats()
                v, s = dm.contract_approx(net, chi, env, stats=st)
                rows.append({"beta": beta, "chi": chi, "env": env, "log_abs": v, "sign": s,
                             "n_eig": st.n_eig, "seconds": time.time() - t})
                print(json.dumps(rows[-1]), flush=True)
    json.dump({"workload": "ising2d 64x64 open, J=1, h=0",
               "generator": "paper_2406_09769_amd.inputs.ising_2d(64, 64, beta)",
               "oracle": "oracle.dm.contract_approx(net, chi, env) with default cutoffs",
               "rows": rows}, open(out_path, "w"), indent=1)


def _w3_one(beta):
    net = inputs.ising_3d(8, 8, 8, beta)
    t = time.time()
    st = dm.Stats()
    v, s = dm.contract_approx(net, 16, 1, stats=st)
    row = {"beta": beta, "chi": 16, "env": 1, "log_abs": v, "sign": s, "n_eig": st.n_eig,
           "seconds": time.time() - t}
    print(json.dumps(row), flush=True)
    return row


def w3_chi32(out_path, beta):
    """The 8x8x8 lattice at chi 32 for one beta. Every right environment holds up to
    (32 * 2^9)^2 doubles (2.1 GB): only every 8th is kept and the rest recomputed (a memory
    schedule, bit-identical to keeping them all). Rows for other betas in out_path stay."""
    net = inputs.ising_3d(8, 8, 8, beta)
    t = time.time()
    st = dm.Stats()
    v, s = dm.contract_approx(net, 32, 1, stats=st, env_checkpoint=8)
    row = {"beta": beta, "chi": 32, "env": 1, "log_abs": v, "sign": s, "n_eig": st.n_eig,
           "seconds": time.time() - t}
    print(json.dumps(row), flush=True)
    old = json.load(open(out_path))["rows"] if os.path.exists(out_path) else []
    rows = sorted([r for r in old if r["beta"] != beta] + [row], key=lambda r: r["beta"])
    json.dump({"workload": "ising3d 8x8x8 open, J=1, h=0, one z-plane per slice, chi 32",
               "generator": "paper_2406_09769_amd.inputs.ising_3d(8, 8, 8, beta)",
               "oracle": "oracle.dm.contract_approx(net, 32, 1, env_checkpoint=8) with default cutoffs",
               "rows": rows}, open(out_path, "w"), indent=1)


def w3(out_path):
    rows = [_w3_one(b) for b in inputs.w3_betas()]    # one at a time: each peaks near 20 GB
    json.dump({"workload": "ising3d 8x8x8 open, J=1, h=0, one z-plane per slice",
               "generator": "paper_2406_09769_amd.inputs.ising_3d(8, 8, 8, beta)",
               "oracle": "oracle.dm.contract_approx(net, 16, 1) with default cutoffs",
               "rows": rows}, open(out_path, "w"), indent=1)


def _w3_spread_one(args):
    """One alternative FP64 evaluation of a W3 lattice: LAPACK's MRRR driver ("evr"), or the
    default solver on inputs scaled by (1 + a z), z standard normal with the given seed,
    a = 1e-15 ("perturbed_<seed>") or a = 1e-13 ("perturbed13_<seed>", the relative rounding
    bound of an FP64 sum of about 10^3 terms, the depth of this lattice's contractions), or
    the default solver with every pairwise contraction result scaled by (1 + 1e-15 z)
    ("gemmnoise_<seed>"), or the default solver on L + eps ||L|| S, S symmetric Gaussian of
    unit spectral norm ("eignoise_<seed>")."""
    import copy
    import numpy as np
    import scipy.linalg as sl
    beta, how = args
    net = inputs.ising_3d(8, 8, 8, beta)
    if how == "evr":
        dm.EIGH = lambda L: sl.eigh(L, driver="evr")
    elif how.startswith("eignoise_"):
        # every density matrix handed to the default solver with a symmetric perturbation of
        # spectral norm eps * ||L||: the backward error any FP64 symmetric eigensolver is
        # allowed (an absolute-accuracy solver may show all of it)
        rng = np.random.default_rng(int(how.rsplit("_", 1)[1]))

        def eigh_noisy(L):
            Z = rng.standard_normal(L.shape)
            S = 0.5 * (Z + Z.T)
            S /= np.linalg.norm(S, 2)
            return np.linalg.eigh(L + np.finfo(float).eps * np.linalg.norm(L, 2) * S)
        dm.EIGH = eigh_noisy
    elif how.startswith("gemmnoise_"):
        # every pairwise contraction result scaled by (1 + 1e-15 z): the size of the rounding
        # differences another FP64 summation order leaves in each contraction
        rng = np.random.default_rng(int(how.rsplit("_", 1)[1]))
        td = np.tensordot
        dm.np.tensordot = lambda a, b, axes=2: (lambda r: r * (1.0 + 1e-15 * rng.standard_normal(r.shape)))(
            td(a, b, axes=axes))
    else:
        amp = 1e-13 if how.startswith("perturbed13_") else 1e-15
        rng = np.random.default_rng(int(how.rsplit("_", 1)[1]))
        net = copy.deepcopy(net)
        net.tensors = [t * (1.0 + amp * rng.standard_normal(t.shape)) for t in net.tensors]
    v = dm.contract_approx(net, 16, 1)[0]
    print(json.dumps({"beta": beta, "how": how, "log_abs": v}), flush=True)
    return beta, how, v


def w3spread(out_path, betas, hows):
    """Deviation per site of each alternative evaluation from the stored oracle value; rows
    already in out_path are kept and extended."""
    gold = {r["beta"]: r for r in json.load(open(os.path.join(HERE, "w3_oracle.json")))["rows"]}
    old = {r["beta"]: r for r in json.load(open(out_path))["rows"]} if os.path.exists(out_path) else {}
    jobs = [(b, h) for b in betas for h in hows]
    if len(jobs) == 1:
        res = [_w3_spread_one(jobs[0])]
    else:
        with Pool(2) as pool:
            res = pool.map(_w3_spread_one, jobs)
    for b in betas:
        row = {k: v for k, v in old.get(b, {"beta": b}).items() if k != "spread"}
        row.update({h: abs(v - gold[b]["log_abs"]) / 512 for bb, h, v in res if bb == b})
        old[b] = {"beta": b, "spread": max(v for k, v in row.items() if k != "beta"),
                  **{k: v for k, v in row.items() if k != "beta"}}
    json.dump({"workload": "8x8x8 lattice of w3_oracle.json, chi 16",
               "what": "largest |dlnZ|/N between the stored oracle value and the oracle under an "
                       "alternative LAPACK eigensolver (evr), relative input noise of 1e-15 "
                       "(perturbed_s) or 1e-13 (perturbed13_s, the rounding bound of an FP64 sum "
                       "of about 10^3 terms), 1e-15 relative noise on every pairwise "
                       "contraction result (gemmnoise_s, another summation order's rounding), or "
                       "a symmetric perturbation of norm eps ||L|| of every density matrix "
                       "(eignoise_s, the backward error an FP64 eigensolver may have)",
               "rows": [old[b] for b in sorted(old)]}, open(out_path, "w"), indent=1)


def _spread_one(i, kind="w4"):
    """Oracle result of instance i (W4 graphs, or the small #CSP formulas for kind "w5small")
    under three other equally valid FP64 evaluations: LAPACK's MRRR driver (evr) in place of
    the default divide-and-conquer one, and the default solver on the network with every
    tensor entry scaled by (1 + 1e-15 z), z standard normal (two seeds). Returns the largest
    |dlnZ|/N from the stored value."""
    import copy
    import numpy as np
    import scipy.linalg as sl
    if kind == "w4":
        gold = json.load(open(os.path.join(HERE, "w4_oracle.json")))["rows"][i]
        net, chi = inputs.rrg_batch(i + 1)[i], 64
    else:
        gold = json.load(open(os.path.join(HERE, "w5_small_oracle.json")))["rows"][i]
        net, chi = inputs.csp_batch(i + 1, n_vars=50)[i], 32
    assert net.name == gold["name"]
    vals = {}
    dm.EIGH = lambda L: sl.eigh(L, driver="evr")
    try:
        vals["evr"] = dm.contract_approx(net, chi, 1)[0]
    finally:
        dm.EIGH = np.linalg.eigh
    for seed in (0, 1):
        rng = np.random.default_rng(seed)
        net2 = copy.deepcopy(net)
        net2.tensors = [t * (1.0 + 1e-15 * rng.standard_normal(t.shape)) for t in net.tensors]
        vals[f"perturbed_{seed}"] = dm.contract_approx(net2, chi, 1)[0]
    dev = {k: abs(v - gold["log_abs"]) / net.n_sites for k, v in vals.items()}
    row = {"index": i, "name": net.name, "spread": max(dev.values()), **dev}
    print(json.dumps(row), flush=True)
    return row


def _eignoise_one(args):
    """Instance i of a batch workload under the default solver on L + eps ||L|| S for every
    density matrix (S symmetric Gaussian of unit spectral norm, seed 0): the backward error
    any FP64 symmetric eigensolver is allowed. Returns (i, |dlnZ|/N from the stored value)."""
    import numpy as np
    kind, i = args
    if kind == "w4":
        gold = json.load(open(os.path.join(HERE, "w4_oracle.json")))["rows"][i]
        net, chi = inputs.rrg_batch(i + 1)[i], 64
    else:
        gold = json.load(open(os.path.join(HERE, "w5_small_oracle.json")))["rows"][i]
        net, chi = inputs.csp_batch(i + 1, n_vars=50)[i], 32
    assert net.name == gold["name"]
    rng = np.random.default_rng(0)

    def eigh_noisy(L):
        Z = rng.standard_normal(L.shape)
        S = 0.5 * (Z + Z.T)
        S /= np.linalg.norm(S, 2)
        return np.linalg.eigh(L + np.finfo(float).eps * np.linalg.norm(L, 2) * S)
    dm.EIGH = eigh_noisy
    try:
        v = dm.contract_approx(net, chi, 1)[0]
    finally:
        dm.EIGH = np.linalg.eigh
    d = abs(v - gold["log_abs"]) / net.n_sites
    print(json.dumps({"kind": kind, "index": i, "eignoise_0": d}), flush=True)
    return i, d


WORKERS = int(os.environ.get("GOLDEN_WORKERS", "4"))


def add_eignoise(kind, path, count, workers=None):
    workers = workers or WORKERS
    """Adds the eignoise_0 deviation to every row of a stored spread file and raises each
    row's spread to it where it is larger."""
    with Pool(workers) as pool:
        res = dict(pool.map(_eignoise_one, [(kind, i) for i in range(count)]))
    d = json.load(open(path))
    for r in d["rows"]:
        r["eignoise_0"] = res[r["index"]]
        r["spread"] = max(r["spread"], r["eignoise_0"])
    d["what"] += ("; eignoise_0: each density matrix given a symmetric perturbation of norm "
                  "eps ||L|| before its eigensolve, the backward error any FP64 eigensolver may have")
    json.dump(d, open(path, "w"), indent=1)


def _spread_w5small(i):
    return _spread_one(i, "w5small")


def spread_w5small(out_path, workers=None):
    with Pool(workers or WORKERS) as pool:
        rows = sorted(pool.map(_spread_w5small, range(8)), key=lambda r: r["index"])
    json.dump({"workload": "the 8 formulas of w5_small_oracle.json",
               "what": "largest |dlnZ|/N between the stored oracle value and the oracle under an "
                       "alternative LAPACK eigensolver (evr) or 1e-15 relative input noise (2 seeds)",
               "rows": rows}, open(out_path, "w"), indent=1)


def spread(out_path, workers=None):
    with Pool(workers or WORKERS) as pool:
        rows = sorted(pool.map(_spread_one, range(64)), key=lambda r: r["index"])
    json.dump({"workload": "the 64 graphs of w4_oracle.json",
               "what": "largest |dlnZ|/N between the stored oracle value and the oracle under an "
                       "alternative LAPACK eigensolver (evr) or 1e-15 relative input noise (2 seeds)",
               "rows": rows}, open(out_path, "w"), indent=1)


def _one(args):
    kind, i, chi = args
    if kind == "w4":
        net = inputs.rrg_batch(i + 1)[i]
    elif kind == "w5":
        net = inputs.csp_batch(i + 1)[i]
    else:
        net = inputs.csp_batch(i + 1, n_vars=50)[i]
    t = time.time()
    st = dm.Stats()
    v, s = dm.contract_approx(net, chi, 1, stats=st)
    row = {"index": i, "name": net.name, "n_sites": net.n_sites, "n_tensors": len(net.tensors),
           "chi": chi, "env": 1, "log_abs": v, "sign": s, "n_eig": st.n_eig, "seconds": time.time() - t}
    print(json.dumps(row), flush=True)
    return row


def batch(kind, count, chi, out_path, workers=None):
    with Pool(workers or WORKERS) as pool:
        rows = sorted(pool.map(_one, [(kind, i, chi) for i in range(count)]), key=lambda r: r["index"])
    desc = {"w4": ("64 signed-J random 3-regular graphs, n_i = 2*U{50..150}, J ~ N(0,1), beta 1, "
                   "seed 4000+i, greedy path", "paper_2406_09769_amd.inputs.rrg_batch(64)"),
            "w5": ("32 random 3-SAT #CSP formulas, n 150, m 450, seed 5000+i, greedy path",
                   "paper_2406_09769_amd.inputs.csp_batch(32)"),
            "w5small": ("8 random 3-SAT #CSP formulas, n 50, m 150, seed 5000+i, greedy path",
                        "paper_2406_09769_amd.inputs.csp_batch(8, n_vars=50)")}[kind]
    json.dump({"workload": desc[0], "generator": desc[1],
               "oracle": f"oracle.dm.contract_approx(net, {chi}, 1) with default cutoffs",
               "rows": rows}, open(out_path, "w"), indent=1)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "w2"
    if which == "w2":
        w2(os.path.join(HERE, "w2_oracle.json"))
    elif which == "w4":
        batch("w4", 64, 64, os.path.join(HERE, "w4_oracle.json"))
    elif which == "w5":
        batch("w5", 32, 32, os.path.join(HERE, "w5_oracle.json"))
    elif which == "w4spread":
        spread(os.path.join(HERE, "w4_spread.json"))
    elif which == "w3":
        w3(os.path.join(HERE, "w3_oracle.json"))
    elif which == "w3chi32":
        w3_chi32(os.path.join(HERE, "w3_chi32_oracle.json"), float(sys.argv[2]))
    elif which == "w3spread":
        args = [a for a in sys.argv[2:] if not a.startswith("--hows=")]
        hows = [a[7:].split(",") for a in sys.argv[2:] if a.startswith("--hows=")]
        w3spread(os.path.join(HERE, "w3_spread.json"), [float(x) for x in args],
                 hows[0] if hows else ["evr", "perturbed_0"])
    elif which == "w5small":
        batch("w5small", 8, 32, os.path.join(HERE, "w5_small_oracle.json"))
    elif which == "w5smallspread":
        spread_w5small(os.path.join(HERE, "w5_small_spread.json"))
    elif which == "w4eignoise":
        add_eignoise("w4", os.path.join(HERE, "w4_spread.json"), 64)
    elif which == "w5smalleignoise":
        add_eignoise("w5small", os.path.join(HERE, "w5_small_spread.json"), 8)
