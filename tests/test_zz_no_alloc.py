"""The allocation-free entry point against tn_contract_approx.

Both run the same kernels on the same op list, so the results must be bit-identical;
two calls in a row (the second on a smaller network) also check that what the shared
device scratch keeps from the last call changes nothing.
"""
import pytest

from paper_2406_09769_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2406_09769_amd import tnapprox
    return tnapprox


def test_noalloc_matches_the_allocating_entry_point_on_two_calls(T):
    cases = [(inputs.ising_2d(16, 16, 0.44), 16, 2), (inputs.ising_2d(6, 6, 0.44), 4, 1)]
    for net, chi, env in cases:     # the second call is smaller than the first
        print(f"noalloc: {net.name} chi={chi} env={env}", flush=True)
        h = T.create_network(net)
        a = T.tn_contract_approx_noalloc(h, net.slices, chi, env)
        h2 = T.create_network(net)
        b = T.tn_contract_approx(h2, net.slices, chi, env)
        assert a.sign == b.sign and a.log_abs == b.log_abs, (a, b)
        assert a.flops == b.flops and a.n_eig == b.n_eig


def test_noalloc_learned_and_split_options(T):
    net = inputs.ising_2d(12, 12, 0.5)
    h = T.create_network(net)
    h2 = T.create_network(net)
    for prec in (T.TN_SPLIT_BF16X3, T.TN_FP64):
        a = T.tn_contract_approx_noalloc(h, net.slices, 8, 1, precision=prec)
        b = T.tn_contract_approx(h2, net.slices, 8, 1, precision=prec)
        assert a.log_abs == b.log_abs and a.sign == b.sign


def test_noalloc_refuses_chip_wide_networks(T):
    net = inputs.ising_3d(5, 5, 5, 0.2217)
    h = T.create_network(net)
    assert T.tn_plan_stats(h, net.slices, 16, 1)["grid_ops"] > 0
    with pytest.raises(T.TnError) as e:
        T.tn_contract_approx_noalloc(h, net.slices, 16, 1)
    assert e.value.status == T.TN_EUNSUPPORTED
