"""C-ABI tests that need no GPU: the library loads, exports every declared entry
point, validates its inputs, and its host planner reproduces the oracle's
structural plan (leaf order and embedding) exactly."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2406_09769_amd import inputs
from oracle import dm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def T():
    from paper_2406_09769_amd import tnapprox
    return tnapprox


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(tn_\w+)\s*\(", text, re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported(T):
    names = declared_symbols()
    assert {"tn_create", "tn_contract_approx", "tn_contract_approx_batch", "tn_destroy"} <= set(names)
    lib = ctypes.CDLL(T.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def _plans_equal(T, net, env):
    st = dm.Stats()
    dm.contract_approx(net, 2, env, stats=st)
    pj = T.tn_plan_json(net.tensors, net.edges, net.slices, env)
    assert len(pj["partitions"]) == len(st.plans)
    for (leaf_edges, placement), pp in zip(st.plans, pj["partitions"]):
        assert list(leaf_edges) == pp["leaves"]
        assert [list(x) for x in placement] == [list(x) for x in pp["placement"]]


@pytest.mark.parametrize("env", [1, 2, 3])
def test_plan_2d_matches_oracle(T, env):
    _plans_equal(T, inputs.ising_2d(6, 7, 0.44), env)


def test_plan_3d_matches_oracle(T):
    _plans_equal(T, inputs.ising_3d(3, 3, 4, 0.25), 1)
    _plans_equal(T, inputs.ising_3d(4, 2, 3, 0.25), 2)


@pytest.mark.parametrize("seed,env", [(3, 1), (4, 2), (5, 6)])
def test_plan_rrg_matches_oracle(T, seed, env):
    _plans_equal(T, inputs.ising_rrg(60, 1.0, seed=seed), env)


@pytest.mark.parametrize("seed,env", [(1, 1), (2, 3)])
def test_plan_csp_matches_oracle(T, seed, env):
    rng = np.random.default_rng(seed)
    _plans_equal(T, inputs.csp_network(40, inputs.random_3sat(40, 110, rng)), env)


def test_plan_full_size_2d_matches_oracle_structure(T):
    net = inputs.ising_2d(64, 64, 0.44)
    pj = T.tn_plan_json(net.tensors, net.edges, net.slices, 2)
    assert len(pj["partitions"]) == 32
    for p in pj["partitions"][:-1]:
        assert len(p["leaves"]) == 64


def test_plan_rejects_malformed_networks(T):
    good = inputs.ising_2d(3, 3, 0.44)
    with pytest.raises(T.TnError) as e:
        T.tn_plan_json(good.tensors, good.edges[:-1], good.slices, 1)   # dangling modes
    assert e.value.status == T.TN_EINVAL
    bad = list(good.edges)
    t0, m0, t1, m1 = bad[0]
    bad[0] = (t0, m0, t0, m1)
    with pytest.raises(T.TnError):
        T.tn_plan_json(good.tensors, bad, good.slices, 1)                # self-loop
    with pytest.raises(T.TnError):
        T.tn_plan_json(good.tensors, good.edges, good.slices[:-1], 1)    # path misses tensors
    with pytest.raises(T.TnError):
        T.tn_plan_json(good.tensors, good.edges, [good.slices[0] + [0]] + good.slices[1:], 1)
    with pytest.raises(T.TnError):
        T.tn_plan_json(good.tensors, good.edges, good.slices, 0)         # env_size < 1


def test_create_validates_before_touching_a_device(T):
    net = inputs.ising_2d(3, 3, 0.44)
    tensors = [t.copy() for t in net.tensors]
    tensors[4][0, 0, 0, 0] = math.nan
    with pytest.raises(T.TnError) as e:
        T.tn_create(tensors, net.edges)
    assert e.value.status == T.TN_ENUMERIC
    edges = list(net.edges)
    t0, m0, t1, m1 = edges[0]
    edges[0] = (t0, m0, t1, (m1 + 1) % net.tensors[t1].ndim)
    with pytest.raises(T.TnError) as e:
        T.tn_create(net.tensors, edges)
    assert e.value.status == T.TN_EINVAL


def test_error_strings(T):
    for s in range(6):
        assert T.LIB.tn_error_string(s)


def _twin_block(order):
    """Two order-`order` tensors joined by `order` bond-2 edges, absorbed one at a time: the
    right environment of the first cut spans 2^(2 (order - 2)) elements even at rank 1."""
    shapes = [(2,) * order, (2,) * order]
    edges = [(0, m, 1, m) for m in range(order)]
    return shapes, edges, [[0], [1]]


def test_plan_refuses_intermediates_of_2_to_the_31_elements(T):
    shapes, edges, slices = _twin_block(17)            # largest environment 2^30: planned
    T.tn_plan_json(shapes, edges, slices, 1)
    shapes, edges, slices = _twin_block(18)            # 2^32: refused before any table is built
    with pytest.raises(T.TnError) as e:
        T.tn_plan_json(shapes, edges, slices, 1)
    assert e.value.status == T.TN_EUNSUPPORTED
    assert "2^31" in str(e.value)
