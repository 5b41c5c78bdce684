"""Write oracle values for the full-size workloads into tests/golden/*.json.

Calls only oracle/ (and the seeded input generators). Usage:
    python tests/golden/make_golden.py w2        # 64x64 2D Ising, 8 betas x chi {32,64} x env {1,2}
"""
import json
import math
import os
import sys
import time

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


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "w2"
    if which == "w2":
        w2(os.path.join(HERE, "w2_oracle.json"))
