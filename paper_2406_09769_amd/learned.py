"""Training recipe of the learned warm start: every step runs in the library.

The MLP is trained on rows the method itself harvests (tn_harvest) from density matrices
of the lattice workloads: the 6x6 lattice at rank 4 and 16, two 64x64 lattices at
inverse temperatures outside the timed set, and a 4x4x4 cubic lattice (the 3D workload's
single-workgroup size). Training is tn_model_train (Adam on the device).
"""
from __future__ import annotations

from . import inputs


def harvest_networks():
    return [(inputs.ising_2d(6, 6, 0.44), 4), (inputs.ising_2d(6, 6, 0.44), 16),
            (inputs.ising_2d(64, 64, 0.40), 32), (inputs.ising_2d(64, 64, 0.50), 32),
            (inputs.ising_3d(4, 4, 4, 0.2217), 16)]


def train_warm_start_model(T, steps: int = 3000, seed: int = 7, report=None):
    """A model of the binding T (tnapprox) trained on the harvested rows; returns it.
    Training runs in launches of 500 Adam steps (the optimiser state carries over);
    report(text), if given, is called after the harvest and after each launch."""
    ds = T.Dataset(600_000)
    for net, chi in harvest_networks():
        T.tn_harvest(T.create_network(net), net.slices, chi, 1, ds)
    if report:
        report(f"harvested {ds.size()} rows")
    m = T.Model(seed=seed)
    done = 0
    while done < steps:
        k = min(500, steps - done)
        loss = m.train(ds, steps=k, batch=128, lr=3e-3, seed=11 + done)
        done += k
        if report:
            report(f"trained {done} steps, last batch loss {loss:.3e}")
    return m
