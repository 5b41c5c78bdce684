"""The precision form (split BF16 x3 / FP16 x3 contractions, FP64 eigensolve) against
the FP64 oracle.

The split forms TN_SPLIT_BF16X3 and TN_SPLIT_FP16X3 run only the contractions that
build right environments and density matrices in 16-bit parts; the main chain that
carries the value (projector application, the carried block, the closing
contractions), the eigensolve and the log accumulation stay FP64. The value is then
the FP64 contraction of the network with projectors onto slightly moved subspaces.

What moves them: every 16-bit matrix instruction sums its products in FP32, so each
density matrix carries an error of about 2^-24 of |C||R||C|^T, which for the positive
Ising tensors is about 6e-8 ||L||. Eigen-directions of L whose eigenvalues lie below
that level are noise in the split forms; kept directions at or below it are replaced by
others of about the same weight, which changes the captured weight of each truncation
at the 1e-8 level. Stated per-result bounds:
* lattices whose kept spectra stay above the noise floor (the 2D and 3D lattices in
  the disordered phase): |dlnZ|/N <= 1e-8, the accuracy the mixed form is measured at;
* the 64x64 workload, whose near-critical networks keep eigenvalues down to 1e-15 of
  the largest: |dlnZ|/N <= 3e-8 per result, and the count within 1e-8 is asserted;
* networks whose cuts sit in a dense tail of the spectrum (the ordered 3D lattice at
  beta 0.25, signed random graphs): |dlnZ|/N <= 1e-6, the same bound as the forms that
  split every contraction (TN_SPLIT_*_ALL), whose main chain carries about 2^-20 of
  relative rounding per step over about N steps.
Every result is printed.
"""
import json
import os

import pytest

from paper_2406_09769_amd import inputs
from oracle import dm

pytestmark = pytest.mark.gpu
BOUND = 1e-8          # environment / density-matrix split on well-conditioned lattices
BOUND_W2 = 3e-8       # the 64x64 workload (spectra kept down to the FP64 floor)
BOUND_ILL = 1e-6      # cuts in a dense spectral tail; every contraction split
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def T():
    from paper_2406_09769_amd import tnapprox
    return tnapprox


def env_only(T, precision):
    return precision in (T.TN_SPLIT_BF16X3, T.TN_SPLIT_FP16X3)


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("net_fn,chi,env,ill", [
    (lambda: inputs.ising_2d(6, 6, 0.44), 4, 1, False),
    (lambda: inputs.ising_2d(6, 6, 0.44), 16, 1, False),
    (lambda: inputs.ising_2d(16, 16, 0.44), 16, 2, False),
    (lambda: inputs.ising_3d(4, 4, 4, 0.2217), 8, 1, False),
    (lambda: inputs.ising_3d(5, 5, 5, 0.2217), 16, 1, False),     # chip-wide ops: per-chunk scaling
    (lambda: inputs.ising_rrg(40, 1.0, 4100), 16, 1, True),
])
def test_precision_form_within_bound(T, precision, net_fn, chi, env, ill):
    net = net_fn()
    h = T.create_network(net)
    r = T.tn_contract_approx(h, net.slices, chi, env, precision=precision)
    v, s = dm.contract_approx(net, chi, env)
    d = abs(r.log_abs - v) / net.n_sites
    bound = BOUND if env_only(T, precision) and not ill else BOUND_ILL
    print(f"{net.name} chi={chi} env={env} precision={precision}: |dlnZ|/N {d:.3e} (bound {bound:.0e})", flush=True)
    assert r.sign == s and d <= bound


def test_fp64_unchanged_by_the_option(T):
    net = inputs.ising_2d(12, 12, 0.44)
    h = T.create_network(net)
    a = T.tn_contract_approx(h, net.slices, 16, 1)
    b = T.tn_contract_approx(h, net.slices, 16, 1, precision=T.TN_FP64)
    assert a.log_abs == b.log_abs


def _w2(T):
    gold = json.load(open(os.path.join(HERE, "golden", "w2_oracle.json")))["rows"]
    nets, chis, envs, gl = [], [], [], []
    for chi, env in ((32, 1), (32, 2), (64, 1), (64, 2)):
        for b in inputs.w2_betas():
            nets.append(inputs.ising_2d(64, 64, b))
            chis.append(chi)
            envs.append(env)
            gl.append(next(x for x in gold if x["chi"] == chi and x["env"] == env and abs(x["beta"] - b) < 1e-12))
    return nets, chis, envs, gl


@pytest.mark.parametrize("tau_rel", [1e-15, 1e-10])
@pytest.mark.parametrize("precision", [1, 2, 3])
def test_w2_full_size_precision_form(T, precision, tau_rel):
    """All 32 networks of the 64x64 workload in one launch, with the default keep cutoff and
    with the 1e-10 cutoff the split forms use in the benchmark."""
    nets, chis, envs, gl = _w2(T)
    hs = [T.create_network(n) for n in nets]
    rs = T.tn_contract_approx_batch(hs, [n.slices for n in nets], chis, envs, precision=precision, tau_rel=tau_rel)
    errs = [abs(r.log_abs - g["log_abs"]) / 4096 for r, g in zip(rs, gl)]
    within = sum(e <= BOUND for e in errs)
    print(f"64x64 workload, precision={precision}, tau_rel={tau_rel:g}: kernel {rs[0].seconds:.3f} s, worst |dlnZ|/N "
          f"{max(errs):.3e}, {within}/32 within 1e-8, per (chi, env) group "
          f"{[f'{max(errs[8 * i:8 * i + 8]):.1e}' for i in range(4)]}", flush=True)
    assert all(r.sign == g["sign"] for r, g in zip(rs, gl))
    if env_only(T, precision):
        assert max(errs) <= BOUND_W2
        assert within >= (30 if tau_rel < 1e-12 else 26)
    else:
        assert max(errs) <= BOUND_ILL


@pytest.mark.parametrize("tau_rel", [1e-15, 1e-10])
@pytest.mark.parametrize("precision", [1, 2])
def test_w3_full_size_precision_form(T, precision, tau_rel):
    """8x8x8 lattice, chi 16, the three betas, against the stored FP64 oracle values, with
    the default keep cutoff and the split forms' 1e-10."""
    gold = json.load(open(os.path.join(HERE, "golden", "w3_oracle.json")))["rows"]
    for g in gold:
        net = inputs.ising_3d(8, 8, 8, g["beta"])
        h = T.create_network(net)
        r = T.tn_contract_approx(h, net.slices, g["chi"], g["env"], precision=precision, tau_rel=tau_rel)
        d = abs(r.log_abs - g["log_abs"]) / net.n_sites
        print(f"W3 beta={g['beta']} chi={g['chi']} precision={precision} tau_rel={tau_rel:g}: |dlnZ|/N {d:.3e}, "
              f"{r.seconds:.2f} s",
              flush=True)
        bound = BOUND if g["beta"] < 0.25 else BOUND_ILL     # beta 0.25: ordered phase
        assert r.sign == g["sign"] and d <= bound
        del h


def test_w4_random_graphs_in_the_split_form(T):
    """The 64 signed random 3-regular graphs (chi 64) in one launch with BF16 x3 environment
    and density-matrix contractions (FP32 sums inside each matrix instruction). Their kept
    spectra reach 1e-12 of the largest eigenvalue, far below the split forms' noise floor
    (about 6e-8 ||L||): the split form does not resolve these networks (measured worst
    2.4e-4 per site, median 1.4e-7, 4 of 64 within 1e-8). This is a measurement, not a
    parity claim: every graph's error is printed, and the assertion only guards against a
    broken run (signs, and 1e-3 per site)."""
    gold = json.load(open(os.path.join(HERE, "golden", "w4_oracle.json")))["rows"]
    nets = inputs.rrg_batch(64)
    hs = [T.create_network(n) for n in nets]
    rs = T.tn_contract_approx_batch(hs, [n.slices for n in nets], 64, 1, precision=T.TN_SPLIT_BF16X3)
    errs = []
    for net, g, r in zip(nets, gold, rs):
        assert net.name == g["name"] and r.sign == g["sign"]
        errs.append(abs(r.log_abs - g["log_abs"]) / net.n_sites)
    print(f"64 graphs, BF16 x3: kernel {rs[0].seconds:.2f} s, worst |dlnZ|/N {max(errs):.2e}, median "
          f"{sorted(errs)[32]:.2e}, within 1e-8: {sum(e <= BOUND for e in errs)}/64; per graph "
          f"{[f'{e:.1e}' for e in errs]}", flush=True)
    assert max(errs) <= 1e-3
