"""Full-size uneven batches in one launch against stored oracle values (plain FP64).

* 64 random 3-regular graphs with Gaussian couplings (n = 2*U{50..150}, beta 1,
  chi 64, single-vertex slices on the greedy path), one workgroup per graph;
* 32 random 3-SAT model counts (n 150, m 450, chi 32) as #CSP networks.

Expected values: tests/golden/w4_oracle.json and w5_oracle.json, written by
tests/golden/make_golden.py from oracle.dm alone. Bound: |dlnZ|/N <= 1e-10 with N
the number of spins or variables.
"""
import json
import os

import numpy as np
import pytest

from paper_2406_09769_amd import inputs

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
BOUND = 1e-10


@pytest.fixture(scope="module")
def T():
    from paper_2406_09769_amd import tnapprox
    return tnapprox


def _check_batch(T, nets, gold, chi, label):
    hs = [T.create_network(n) for n in nets]
    rs = T.tn_contract_approx_batch(hs, [n.slices for n in nets], chi, 1)
    errs = []
    for net, g, r in zip(nets, gold, rs):
        assert net.name == g["name"]
        assert r.sign == g["sign"], (net.name, r.sign, g["sign"])
        errs.append(abs(r.log_abs - g["log_abs"]) / net.n_sites)
    print(f"{label}: {len(nets)} networks in {rs[0].seconds:.3f} s of kernel time, "
          f"{sum(r.n_eig for r in rs)} eigensolves, max |dlnZ|/N {max(errs):.2e}", flush=True)
    assert max(errs) <= BOUND
    assert [r.n_eig for r in rs] == [g["n_eig"] for g in gold]


def test_rrg_batch_of_64_matches_oracle():
    from paper_2406_09769_amd import tnapprox as T
    gold = json.load(open(os.path.join(GOLD, "w4_oracle.json")))["rows"]
    _check_batch(T, inputs.rrg_batch(64), gold, 64, "random 3-regular, chi 64")


def test_csp_batch_of_32_matches_oracle():
    from paper_2406_09769_amd import tnapprox as T
    gold = json.load(open(os.path.join(GOLD, "w5_oracle.json")))["rows"]
    _check_batch(T, inputs.csp_batch(32), gold, 32, "3-SAT #CSP, chi 32")
