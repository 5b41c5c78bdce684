"""The oracle's exact routes and the density-matrix oracle against exact values computed
independently of this repository (tests/golden/exact_values.json).

The values are those of the Ising network of section 8.1 on the open lattices of the
section 8.3 experiments, and Onsager's free energy of the square lattice. Because the
method is exact once the kept rank reaches the full bond dimension (every density
matrix then keeps its whole support), the density-matrix oracle at full rank with the
cutoffs off must reproduce each lattice value to rounding; the transfer-matrix and
brute-force routes must reproduce them at any rank.
"""
import json
import math
import os

import pytest

from oracle import dm, exact
from paper_2406_09769_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_values.json")))
TOL = GOLD["tolerance_abs"]


def _ising2d(ly, lx):
    return [r for r in GOLD["ising2d"] if (r["ly"], r["lx"]) == (ly, lx)]


def test_brute_force_matches_the_exact_small_lattices():
    for r in _ising2d(4, 4):                            # 5x5 (25 spins) is past brute force
        net = inputs.ising_2d(r["ly"], r["lx"], r["beta"])
        bf = exact.brute_force_ising(net.n_sites, net.meta["bonds"], net.meta["couplings"], r["beta"])
        assert abs(bf - r["log_z"]) <= TOL
    (r3,) = [r for r in GOLD["ising3d"] if (r["lz"], r["ly"], r["lx"]) == (3, 2, 2)]
    net = inputs.ising_3d(3, 2, 2, r3["beta"])
    bf = exact.brute_force_ising(net.n_sites, net.meta["bonds"], net.meta["couplings"], r3["beta"])
    assert abs(bf - r3["log_z"]) <= TOL


def test_transfer_matrices_match_the_exact_values():
    for r in GOLD["ising2d"]:
        assert abs(exact.tm_2d(r["ly"], r["lx"], r["beta"]) - r["log_z"]) <= TOL, r
    for r in GOLD["ising3d"]:
        assert abs(exact.tm_3d(r["lz"], r["ly"], r["lx"], r["beta"]) - r["log_z"]) <= TOL, r


def test_onsager_free_energy_matches_the_exact_values():
    for r in GOLD["onsager_f"]:
        assert abs(exact.onsager_f(r["beta"]) - r["f"]) <= 1e-13
        assert abs(exact.onsager_f_double(r["beta"]) - r["f"]) <= 1e-12


@pytest.mark.parametrize("env", [1, 2])
def test_density_matrix_oracle_reproduces_6x6_and_small_3d(env):
    (r,) = _ising2d(6, 6)
    v, s = dm.contract_approx(inputs.ising_2d(6, 6, r["beta"]), 16, env, tau_rel=0, tau_deg=0)
    assert s == 1 and abs(v - r["log_z"]) <= TOL
    (r3,) = [r for r in GOLD["ising3d"] if (r["lz"], r["ly"], r["lx"]) == (3, 2, 2)]
    v, s = dm.contract_approx(inputs.ising_3d(3, 2, 2, r3["beta"]), 16, env, tau_rel=0, tau_deg=0)
    assert s == 1 and abs(v - r3["log_z"]) <= TOL


@pytest.mark.slow
def test_density_matrix_oracle_reproduces_the_12_wide_strips_at_full_rank():
    """Width 12: the full bond dimension is 2^6 = 64, so rank 64 is exact at every beta."""
    for r in _ising2d(64, 12):
        net = inputs.ising_2d(64, 12, r["beta"])
        v, s = dm.contract_approx(net, 64, 1, tau_rel=0, tau_deg=0)
        assert s == 1 and abs(v - r["log_z"]) / net.n_sites <= 1e-13, r
        v, s = dm.contract_approx(net, 64, 1)            # default cutoffs drop weight below 1e-12 of w1
        assert s == 1 and abs(v - r["log_z"]) / net.n_sites <= 1e-10, r


@pytest.mark.slow
def test_density_matrix_oracle_reproduces_the_4x4_slabs_at_full_rank():
    """A 4x4 plane has 16 leaves, full bond 2^8 = 256 (one beta: about 30 s)."""
    for r in GOLD["ising3d"]:
        if (r["lz"], r["ly"], r["lx"]) == (4, 4, 4) and r["beta"] == 0.2217:
            v, s = dm.contract_approx(inputs.ising_3d(4, 4, 4, r["beta"]), 256, 1, tau_rel=0, tau_deg=0)
            assert s == 1 and abs(v - r["log_z"]) / 64 <= 1e-13, r
