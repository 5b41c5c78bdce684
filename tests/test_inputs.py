"""Pins of the input generators (the site tensors of the paper's section 8.1 and
the #CSP networks) against brute-force enumeration, independent of the method."""
import math

import numpy as np
import pytest

from paper_2406_09769_amd import inputs
from oracle import exact


@pytest.mark.parametrize("beta_j", [0.7, -1.3, 0.0, 2.5])
def test_bond_pair_gives_boltzmann(beta_j):
    q, r = inputs.ising_bond_pair(beta_j)
    want = np.array([[math.exp(beta_j), math.exp(-beta_j)], [math.exp(-beta_j), math.exp(beta_j)]])
    assert np.allclose(q @ r.T, want, rtol=1e-14, atol=1e-14)
    if beta_j >= 0:  # the paper's symmetric W
        c, s = math.sqrt(math.cosh(beta_j)), math.sqrt(math.sinh(beta_j))
        w = np.array([[c + s, c - s], [c - s, c + s]]) / math.sqrt(2)
        assert np.allclose(q, w) and np.allclose(r, w)


def test_ising_2d_site_tensors_match_brute_force():
    net = inputs.ising_2d(4, 4, 0.44)
    bf = exact.brute_force_ising(16, net.meta["bonds"], net.meta["couplings"], 0.44)
    assert abs(math.log(exact.einsum_network(net)) - bf) < 1e-12
    assert abs(bf - exact.tm_2d(4, 4, 0.44)) < 1e-12


def test_ising_3d_site_tensors_match_brute_force():
    net = inputs.ising_3d(2, 2, 3, 0.2217)
    bf = exact.brute_force_ising(12, net.meta["bonds"], net.meta["couplings"], 0.2217)
    assert abs(math.log(exact.einsum_network(net)) - bf) < 1e-12
    assert abs(bf - exact.tm_3d(2, 2, 3, 0.2217)) < 1e-12
    assert [len(s) for s in net.slices] == [6, 6]


def test_signed_rrg_matches_brute_force():
    net = inputs.ising_rrg(14, 1.0, seed=7)
    assert any(j < 0 for j in net.meta["couplings"])
    bf = exact.brute_force_ising(14, net.meta["bonds"], net.meta["couplings"], 1.0)
    assert abs(math.log(exact.einsum_network(net)) - bf) < 1e-11
    assert all(t.shape == (2, 2, 2) for t in net.tensors)


def test_rrg_is_simple_and_regular():
    net = inputs.ising_rrg(100, 1.0, seed=4000)
    bonds = net.meta["bonds"]
    deg = np.zeros(100, int)
    for u, v in bonds:
        assert u != v
        deg[u] += 1
        deg[v] += 1
    assert np.all(deg == 3)
    assert len({tuple(sorted(b)) for b in bonds}) == len(bonds)
    order = [s[0] for s in net.slices]
    assert order[0] == 0 and sorted(order) == list(range(100))


def test_rrg_batch_sizes():
    sizes = [len(n.tensors) for n in inputs.rrg_batch(8)]
    assert all(100 <= s <= 300 and s % 2 == 0 for s in sizes)


def test_csp_counts_match_brute_force():
    rng = np.random.default_rng(3)
    clauses = inputs.random_3sat(8, 11, rng)
    net = inputs.csp_network(8, clauses)
    count = exact.brute_force_count(8, clauses)
    assert len(net.edges) <= 52
    assert abs(exact.einsum_network(net) - count) < 1e-9
    assert net.n_sites == 8


def test_csp_copy_chains_and_degenerate_degrees():
    # variable 0 in 5 clauses (chain of 3 COPY3), variable 5 in none (scalar 2), variable 6 once
    clauses = [[(0, False), (1, True), (2, False)], [(0, True), (3, False), (4, False)],
               [(0, False), (1, False), (6, True)], [(0, False), (2, True), (3, True)],
               [(0, True), (4, True), (1, False)]]
    net = inputs.csp_network(7, clauses)
    count = exact.brute_force_count(7, clauses)
    assert abs(exact.einsum_network(net) - count) < 1e-9
    assert len(net.meta["var_vertices"][0]) == 3
    assert net.tensors[net.meta["var_vertices"][5][0]].ndim == 0


def test_w2_betas():
    b = inputs.w2_betas()
    assert len(b) == 8 and b[0] == 0.3 and abs(b[-1] - 0.6) < 1e-15
