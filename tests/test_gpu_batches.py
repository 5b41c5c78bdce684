"""Uneven batches in one launch against stored oracle values (plain FP64).

* 64 random 3-regular graphs with Gaussian couplings (n = 2*U{50..150}, beta 1,
  chi 64, single-vertex slices on the greedy path), one workgroup per graph, bound
  1e-10 per site. The rank rule never cuts where the spectrum does not separate by
  10%, so every kept subspace is fixed by FP64 arithmetic: under other valid FP64
  evaluations (another LAPACK eigensolver, 1e-15 relative input noise, an eps ||L||
  perturbation of every density matrix) the oracle moves by at most 2.5e-12 per site
  (tests/golden/w4_spread.json).
* Random 3-SAT model counts as #CSP networks: 8 formulas of 50 variables (m 150, chi
  32) and the full 32 formulas of 150 variables (m 450). Their 0/1 tensors put
  eigenvalues of many density matrices close to the 1e-12 cutoff, where a keep decision
  can flip under the backward error of an FP64 eigensolver: with an eps ||L|| error the
  oracle moves by up to 1.2e-10 per variable (w5_small_spread.json), with an n eps ||L||
  error one decision of the formula of seed 5004 flips and moves it by 5.9e-9, the
  deviation the GPU shows there. Stated bound for #CSP: 1e-8 per variable. The
  150-variable batch takes minutes on the device, so it runs as one batch in 16 parts
  (each network's op list cut into consecutive pieces, one launch per piece, the same
  results bit for bit) that report their progress.

Expected values: tests/golden/*.json, written by tests/golden/make_golden.py from
oracle/ alone. N is the number of spins or variables.
"""
import json
import os

import pytest

from paper_2406_09769_amd import inputs

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
BOUND = 1e-10
CSP_BOUND = 1e-8


@pytest.fixture(scope="module")
def T():
    from paper_2406_09769_amd import tnapprox
    return tnapprox


def _run(T, nets, chi):
    hs = [T.create_network(n) for n in nets]
    return T.tn_contract_approx_batch(hs, [n.slices for n in nets], chi, 1)


def test_rrg_batch_of_64_matches_oracle(T):
    gold = json.load(open(os.path.join(GOLD, "w4_oracle.json")))["rows"]
    nets = inputs.rrg_batch(64)
    print("random 3-regular batch: 64 graphs, chi 64, one launch", flush=True)
    hs = [T.create_network(n) for n in nets]
    n_qr = sum(T.tn_plan_stats(h, n.slices, 64, 1)["qr_svd"] for h, n in zip(hs, nets))
    rs = T.tn_contract_approx_batch(hs, [n.slices for n in nets], 64, 1)
    worst = 0.0
    for net, g, r in zip(nets, gold, rs):
        assert net.name == g["name"]
        assert r.sign == g["sign"], net.name
        err = abs(r.log_abs - g["log_abs"]) / net.n_sites
        assert err <= BOUND, (net.name, err)
        worst = max(worst, err)
    print(f"kernel {rs[0].seconds:.2f} s, {sum(r.n_eig for r in rs)} eigensolves ({n_qr} by the QR-SVD branch); "
          f"worst |dlnZ|/N {worst:.2e}", flush=True)
    assert n_qr > 0


def _csp_check(nets, gold, rs, bound_of):
    worst = 0.0
    for net, g, r in zip(nets, gold, rs):
        assert net.name == g["name"]
        assert r.sign == g["sign"], net.name
        assert r.n_eig == g["n_eig"]
        err = abs(r.log_abs - g["log_abs"]) / net.n_sites
        b = bound_of(net.name)
        print(f"  {net.name}: |dlnZ|/N {err:.2e} (bound {b:.1e})", flush=True)
        assert err <= b, (net.name, err, b)
        worst = max(worst, err / b)
    return worst


def test_csp_batch_matches_oracle(T):
    gold = json.load(open(os.path.join(GOLD, "w5_small_oracle.json")))["rows"]
    nets = inputs.csp_batch(8, n_vars=50)
    print("3-SAT #CSP batch: 8 formulas, n 50, m 150, chi 32, one launch", flush=True)
    rs = _run(T, nets, 32)
    worst = _csp_check(nets, gold, rs, lambda name: CSP_BOUND)
    print(f"kernel {rs[0].seconds:.2f} s, {sum(r.n_eig for r in rs)} eigensolves, worst error / bound "
          f"{worst:.2f}", flush=True)


# The 150-variable batches run for minutes; their progress lines only reach a terminal
# with pytest -s, and a run that prints nothing for minutes is taken for hung. They run
# when TN_LONG_GPU_TESTS=1 (with -s).
LONG = pytest.mark.skipif(os.environ.get("TN_LONG_GPU_TESTS") != "1",
                          reason="minutes of GPU time with no output under capture; set TN_LONG_GPU_TESTS=1 and use -s")


def _progress(done, total):
    print(f"  part {done}/{total} done", flush=True)


@pytest.fixture(scope="module")
def w5_full(T):
    gold = json.load(open(os.path.join(GOLD, "w5_oracle.json")))["rows"]
    nets = inputs.csp_batch(32)
    hs = [T.create_network(n) for n in nets]
    # plan each formula here (several seconds of host work each, kept on the handle for the
    # batch) so that the run reports progress while it plans
    for i, (h, n) in enumerate(zip(hs, nets)):
        st = T.tn_plan_stats(h, n.slices, 32, 1)
        print(f"  planned formula {i + 1}/32: {st['ops']} ops", flush=True)
    return gold, nets, hs




@LONG
def test_csp_full_size_batch_exact(T, w5_full):
    gold, nets, hs = w5_full
    print("3-SAT #CSP: 32 formulas, n 150, m 450, chi 32, one batch in 16 parts, exact eigensolve", flush=True)
    rs = T.tn_contract_approx_batch(hs, [n.slices for n in nets], 32, 1, chunks=16, progress=_progress)
    worst = _csp_check(nets, gold, rs, lambda name: CSP_BOUND)
    print(f"kernel {rs[0].seconds:.2f} s, {sum(r.n_eig for r in rs)} eigensolves, worst error / bound "
          f"{worst:.2f}", flush=True)


@LONG
def test_csp_full_size_batch_learned_vs_exact(T, w5_full):
    """The learned warm start on the 150-variable formulas (MLP trained on density matrices
    of the lattice workloads, exact solve as fallback when a residual exceeds 1e-6): the same
    bound as the exact solve; warm starts accepted and the eigensolve time of both are
    printed (the QR-SVD branch's small matrices take no warm start)."""
    from paper_2406_09769_amd.learned import train_warm_start_model
    gold, nets, hs = w5_full
    m = train_warm_start_model(T, report=lambda s: print("  " + s, flush=True))
    print("3-SAT #CSP: 32 formulas, n 150, chi 32, one batch in 16 parts, learned warm start", flush=True)
    rs = T.tn_contract_approx_batch(hs, [n.slices for n in nets], 32, 1, eig=T.TN_EIG_LEARNED, model=m,
                                    chunks=16, progress=_progress)
    worst = _csp_check(nets, gold, rs, lambda name: CSP_BOUND)
    n_qr = sum(T.tn_plan_stats(h, n.slices, 32, 1)["qr_svd"] for h, n in zip(hs, nets))
    print(f"kernel {rs[0].seconds:.2f} s, {sum(r.n_learned for r in rs)} of {sum(r.n_eig for r in rs)} eigensolves "
          f"by the warm start ({n_qr} by the QR-SVD branch), worst error / bound {worst:.2f}", flush=True)
