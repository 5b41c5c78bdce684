"""Seeded synthetic input networks for the density-matrix contraction path.

This module builds closed tensor networks and their contraction paths. It is the
only code that both the GPU path and the CPU oracle consume: it holds none of the
density-matrix method's arithmetic, only the construction of the inputs.

Networks (all FP64, row-major):

* classical Ising model on open 2D and 3D lattices and on random 3-regular graphs
  with signed couplings. Each site tensor is a COPY tensor with one bond matrix on
  every leg (paper section 8.1, the Ising tensor construction), so that contracting
  two site tensors over a bond gives the Boltzmann weight exp(beta J s_i s_j).
  Spin +1 maps to index 0.
* #CSP counting networks for random 3-SAT: COPY tensors for the variables and a
  0/1 clause tensor that is zero on the single falsifying assignment (the #CSP
  application named in the paper's introduction). Variable value False maps to
  index 0.

A contraction path is a list of slices (lists of vertex ids); consecutive slices
are fused into partitions by the method's env_size argument.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Network:
    """A closed tensor network plus the contraction path it is meant to follow.

    tensors[t] is a float64 ndarray; edges[e] = (t0, m0, t1, m1) joins mode m0 of
    tensor t0 with mode m1 of tensor t1. Every mode appears in exactly one edge.
    slices is the ordered path; n_sites is the number of spins or variables, the
    N of the per-site error |dlnZ|/N.
    """

    tensors: list
    edges: list
    slices: list
    n_sites: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    def check(self) -> None:
        seen = {}
        for e, (t0, m0, t1, m1) in enumerate(self.edges):
            if t0 == t1:
                raise ValueError(f"edge {e} is a self-loop")
            for t, m in ((t0, m0), (t1, m1)):
                if (t, m) in seen:
                    raise ValueError(f"mode {m} of tensor {t} used twice")
                seen[(t, m)] = e
            if self.tensors[t0].shape[m0] != self.tensors[t1].shape[m1]:
                raise ValueError(f"edge {e} joins modes of different size")
        for t, a in enumerate(self.tensors):
            for m in range(a.ndim):
                if (t, m) not in seen:
                    raise ValueError(f"mode {m} of tensor {t} is dangling")
        flat = [v for s in self.slices for v in s]
        if sorted(flat) != list(range(len(self.tensors))):
            raise ValueError("slices do not partition the vertices")


# ---------------------------------------------------------------- bond matrices

def ising_bond_pair(beta_j: float):
    """Real factors (Q, R) with Q @ R.T = [[e^{bJ}, e^{-bJ}], [e^{-bJ}, e^{bJ}]].

    For bJ >= 0 both factors equal the paper's symmetric square-root matrix W
    (section 8.1). For bJ < 0 that W is complex, so the sinh factor's sign moves
    onto R: with H = [[1,1],[1,-1]], Q = H diag(sqrt cosh, sqrt|sinh|) H / sqrt2 and
    R = H diag(sqrt cosh, sgn(J) sqrt|sinh|) H / sqrt2. Q goes on the lower-id
    endpoint of the bond, R on the higher-id endpoint.
    """
    c = math.sqrt(math.cosh(beta_j))
    s = math.sqrt(abs(math.sinh(beta_j)))
    sg = 1.0 if beta_j >= 0 else -1.0
    h = np.array([[1.0, 1.0], [1.0, -1.0]])
    q = h @ np.diag([c, s]) @ h / math.sqrt(2.0)
    r = h @ np.diag([c, sg * s]) @ h / math.sqrt(2.0)
    return q, r


def _copy_with_factors(factors):
    """t[j_1..j_d] = sum_i prod_e F_e[i, j_e]: a COPY tensor with F_e on each leg."""
    d = len(factors)
    if d == 0:
        return np.array(2.0)
    t = np.zeros((2,) * d)
    for i in range(2):
        outer = np.array(1.0)
        for f in factors:
            outer = np.multiply.outer(outer, f[i])
        t += outer
    return t


def ising_network(n_vertices: int, bonds, couplings, beta: float):
    """Site tensors and edges of an Ising model on an arbitrary graph.

    bonds is a list of (u, v) vertex pairs, couplings the J of each bond. Modes of
    each tensor follow the order in which its bonds appear in the list.
    """
    legs = [[] for _ in range(n_vertices)]  # per vertex: list of (edge id, factor)
    for e, ((u, v), j) in enumerate(zip(bonds, couplings)):
        if u == v:
            raise ValueError("self-loop bond")
        q, r = ising_bond_pair(beta * j)
        lo, hi = (u, v) if u < v else (v, u)
        legs[lo].append((e, q))
        legs[hi].append((e, r))
    tensors = [_copy_with_factors([f for _, f in lg]) for lg in legs]
    ends = {}
    for v, lg in enumerate(legs):
        for m, (e, _) in enumerate(lg):
            ends.setdefault(e, []).append((v, m))
    edges = []
    for e in range(len(bonds)):
        (t0, m0), (t1, m1) = ends[e]
        edges.append((t0, m0, t1, m1))
    return tensors, edges


# ---------------------------------------------------------------- lattices

def ising_2d(ly: int, lx: int, beta: float, j: float = 1.0) -> Network:
    """Open ly x lx square lattice; vertex id y*lx + x; slices are the rows."""
    vid = lambda y, x: y * lx + x
    bonds = []
    for y in range(ly):
        for x in range(lx):
            if x + 1 < lx:
                bonds.append((vid(y, x), vid(y, x + 1)))
            if y + 1 < ly:
                bonds.append((vid(y, x), vid(y + 1, x)))
    tensors, edges = ising_network(ly * lx, bonds, [j] * len(bonds), beta)
    slices = [[vid(y, x) for x in range(lx)] for y in range(ly)]
    net = Network(tensors, edges, slices, ly * lx, f"ising2d_{ly}x{lx}_b{beta:g}",
                  {"kind": "ising2d", "ly": ly, "lx": lx, "beta": beta, "j": j,
                   "bonds": bonds, "couplings": [j] * len(bonds)})
    net.check()
    return net


def ising_3d(lz: int, ly: int, lx: int, beta: float, j: float = 1.0) -> Network:
    """Open lz x ly x lx cubic lattice; slices are z-planes listed row-major in (y, x)."""
    vid = lambda z, y, x: (z * ly + y) * lx + x
    bonds = []
    for z in range(lz):
        for y in range(ly):
            for x in range(lx):
                if x + 1 < lx:
                    bonds.append((vid(z, y, x), vid(z, y, x + 1)))
                if y + 1 < ly:
                    bonds.append((vid(z, y, x), vid(z, y + 1, x)))
                if z + 1 < lz:
                    bonds.append((vid(z, y, x), vid(z + 1, y, x)))
    n = lz * ly * lx
    tensors, edges = ising_network(n, bonds, [j] * len(bonds), beta)
    slices = [[vid(z, y, x) for y in range(ly) for x in range(lx)] for z in range(lz)]
    net = Network(tensors, edges, slices, n, f"ising3d_{lz}x{ly}x{lx}_b{beta:g}",
                  {"kind": "ising3d", "dims": (lz, ly, lx), "beta": beta, "j": j,
                   "bonds": bonds, "couplings": [j] * len(bonds)})
    net.check()
    return net


# ---------------------------------------------------------------- greedy path

def greedy_path(n_vertices: int, adjacency) -> list:
    """Linear vertex order by minimum boundary growth; each slice is one vertex.

    Start at vertex 0. Then repeatedly take the unabsorbed vertex minimising
    (edges to unabsorbed vertices) - (edges into the absorbed set); ties go to the
    most edges into the absorbed set, then to the smallest id. adjacency[v] lists
    the neighbour of every edge of v (with repetition for parallel edges).
    """
    if n_vertices == 0:
        return []
    absorbed = np.zeros(n_vertices, dtype=bool)
    into = np.zeros(n_vertices, dtype=np.int64)  # edges into the absorbed set
    deg = np.array([len(a) for a in adjacency], dtype=np.int64)
    order = []
    v = 0
    while True:
        order.append(v)
        absorbed[v] = True
        for u in adjacency[v]:
            into[u] += 1
        if len(order) == n_vertices:
            break
        score = (deg - into) - into
        cand = np.flatnonzero(~absorbed)
        # lexicographic: min score, max into, min id
        best = min(cand, key=lambda u: (score[u], -into[u], u))
        v = int(best)
    return [[v] for v in order]


def _adjacency_from_edges(n_vertices, edges):
    adj = [[] for _ in range(n_vertices)]
    for (t0, _, t1, _) in edges:
        adj[t0].append(t1)
        adj[t1].append(t0)
    return adj


# ---------------------------------------------------------------- random 3-regular

def random_regular_bonds(n: int, degree: int, rng: np.random.Generator):
    """Simple random regular graph by the pairing model, rejecting loops and multi-edges."""
    if (n * degree) % 2:
        raise ValueError("n * degree must be even")
    for _ in range(10000):
        stubs = np.repeat(np.arange(n), degree)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        key = np.sort(pairs, axis=1)
        if len(np.unique(key[:, 0] * n + key[:, 1])) != len(key):
            continue
        return [(int(a), int(b)) for a, b in key]
    raise RuntimeError("pairing model failed to produce a simple graph")


def ising_rrg(n: int, beta: float, seed: int, degree: int = 3) -> Network:
    """Signed-coupling Ising model on a random regular graph, J_ij ~ N(0, 1), greedy path."""
    rng = np.random.default_rng(seed)
    bonds = random_regular_bonds(n, degree, rng)
    js = rng.standard_normal(len(bonds)).tolist()
    tensors, edges = ising_network(n, bonds, js, beta)
    slices = greedy_path(n, _adjacency_from_edges(n, edges))
    net = Network(tensors, edges, slices, n, f"rrg{degree}_n{n}_s{seed}",
                  {"kind": "rrg", "n": n, "beta": beta, "seed": seed,
                   "bonds": bonds, "couplings": js})
    net.check()
    return net


def rrg_batch(count: int = 64, beta: float = 1.0, base_seed: int = 4000):
    """Uneven batch: instance i has n_i = 2 * U{50..150} vertices, seeded with base_seed + i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        n = 2 * int(rng.integers(50, 151))
        out.append(ising_rrg(n, beta, base_seed + i))
    return out


# ---------------------------------------------------------------- #CSP (3-SAT)

def random_3sat(n_vars: int, n_clauses: int, rng: np.random.Generator):
    """Clauses as lists of (variable, negated); three distinct variables per clause."""
    clauses = []
    for _ in range(n_clauses):
        vs = rng.choice(n_vars, size=3, replace=False)
        neg = rng.integers(0, 2, size=3)
        clauses.append([(int(v), bool(g)) for v, g in zip(vs, neg)])
    return clauses


def csp_network(n_vars: int, clauses) -> Network:
    """#SAT counting network: clause tensors plus COPY tensors for the variables.

    A clause tensor has one 2-valued leg per literal and is 0 only on the assignment
    that makes every literal false. A variable that occurs d times is a COPY tensor
    of order d; for d > 3 it is a chain of d-2 order-3 COPY tensors. d = 2 is an
    identity matrix, d = 1 the vector [1, 1], d = 0 the scalar 2.
    Vertices: clauses first (ids 0..m-1), then variable tensors.
    """
    tensors = []
    for cl in clauses:
        t = np.ones((2, 2, 2))
        bad = tuple(1 if neg else 0 for (_, neg) in cl)
        t[bad] = 0.0
        tensors.append(t)
    # occurrences of each variable: (clause vertex, mode)
    occ = [[] for _ in range(n_vars)]
    for c, cl in enumerate(clauses):
        for m, (v, _) in enumerate(cl):
            occ[v].append((c, m))
    edges = []
    var_vertices = []
    for v in range(n_vars):
        d = len(occ[v])
        mine = []
        if d == 0:
            tensors.append(np.array(2.0))
            mine.append(len(tensors) - 1)
        elif d == 1:
            tensors.append(np.ones(2))
            mine.append(len(tensors) - 1)
            edges.append((occ[v][0][0], occ[v][0][1], mine[0], 0))
        elif d == 2:
            tensors.append(np.eye(2))
            mine.append(len(tensors) - 1)
            edges.append((occ[v][0][0], occ[v][0][1], mine[0], 0))
            edges.append((occ[v][1][0], occ[v][1][1], mine[0], 1))
        else:
            copy3 = np.zeros((2, 2, 2))
            copy3[0, 0, 0] = copy3[1, 1, 1] = 1.0
            ids = []
            for _ in range(d - 2):
                tensors.append(copy3.copy())
                ids.append(len(tensors) - 1)
            mine = ids
            # chain: link i joins mode 2 of ids[i] with mode 0 of ids[i+1]
            for i in range(len(ids) - 1):
                edges.append((ids[i], 2, ids[i + 1], 0))
            # occurrences: first two on ids[0] modes 0,1; then mode 1 of ids[1..]; last on mode 2 of ids[-1]
            slots = [(ids[0], 0), (ids[0], 1)] + [(ids[i], 1) for i in range(1, len(ids))] + [(ids[-1], 2)]
            for (c, m), (t, mm) in zip(occ[v], slots):
                edges.append((c, m, t, mm))
        var_vertices.append(mine)
    n = len(tensors)
    slices = greedy_path(n, _adjacency_from_edges(n, edges))
    net = Network(tensors, edges, slices, n_vars, f"csp_n{n_vars}_m{len(clauses)}",
                  {"kind": "csp", "n_vars": n_vars, "clauses": clauses,
                   "var_vertices": var_vertices})
    net.check()
    return net


def random_3sat_network(n_vars: int, ratio: float, seed: int) -> Network:
    rng = np.random.default_rng(seed)
    m = int(round(ratio * n_vars))
    net = csp_network(n_vars, random_3sat(n_vars, m, rng))
    net.name = f"3sat_n{n_vars}_m{m}_s{seed}"
    net.meta["seed"] = seed
    return net


def csp_batch(count: int = 32, n_vars: int = 150, ratio: float = 3.0, base_seed: int = 5000):
    return [random_3sat_network(n_vars, ratio, base_seed + i) for i in range(count)]


# ---------------------------------------------------------------- named workloads

def w2_betas():
    """The eight inverse temperatures of the 64x64 2D workload: linspace(0.30, 0.60, 8)."""
    return [float(b) for b in np.linspace(0.30, 0.60, 8)]


def w3_betas():
    return [0.20, 0.2217, 0.25]
