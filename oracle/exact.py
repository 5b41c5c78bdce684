"""Exact references that pin the oracle (TEST INFRASTRUCTURE ONLY).

None of these uses the density-matrix method. They compute the same partition
functions by independent routes:

* brute force over all spin (or variable) assignments, straight from the Ising
  partition function of section 8.1 and from the #CSP definition (a count of
  satisfying assignments);
* the row transfer matrix of an open 2D lattice and the plane transfer matrix
  of an open 3D slab, applied one bond at a time on the 2^(width) state vector;
* Onsager's closed-form free energy per site of the infinite square lattice;
* exact contraction of a small network with numpy.einsum (for the generator).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


# ---------------------------------------------------------------- brute force

def brute_force_ising(n: int, bonds, couplings, beta: float) -> float:
    """ln Z = ln sum_s exp(beta * sum_(ij) J_ij s_i s_j), s in {-1, +1}^n (n <= 24)."""
    if n > 24:
        raise ValueError("too many spins for brute force")
    total_max = None
    chunks = []
    step = 1 << min(n, 20)
    for start in range(0, 1 << n, step):
        idx = np.arange(start, min(start + step, 1 << n), dtype=np.int64)
        spins = 1 - 2 * ((idx[:, None] >> np.arange(n)[None, :]) & 1)  # bit 0 -> +1
        energy = np.zeros(len(idx))
        for (u, v), j in zip(bonds, couplings):
            energy += j * spins[:, u] * spins[:, v]
        x = beta * energy
        m = x.max()
        chunks.append((m, np.log(np.sum(np.exp(x - m)))))
        total_max = m if total_max is None else max(total_max, m)
    return float(total_max + np.log(sum(np.exp(m - total_max + l) for m, l in chunks)))


def brute_force_count(n_vars: int, clauses) -> int:
    """Number of assignments satisfying every clause (n_vars <= 24)."""
    if n_vars > 24:
        raise ValueError("too many variables for brute force")
    idx = np.arange(1 << n_vars, dtype=np.int64)
    ok = np.ones(len(idx), dtype=bool)
    for cl in clauses:
        sat = np.zeros(len(idx), dtype=bool)
        for v, neg in cl:
            bit = (idx >> v) & 1          # 1 = True
            sat |= (bit == 0) if neg else (bit == 1)
        ok &= sat
    return int(ok.sum())


# ---------------------------------------------------------------- transfer matrices

def _apply_pair(psi, width, a, b, w):
    """Multiply psi by the Boltzmann weight w(s_a, s_b) of one bond (diagonal)."""
    shape = [2] * width
    p = psi.reshape(shape)
    # weight tensor broadcast over axes a, b
    wt = np.ones([2 if i in (a, b) else 1 for i in range(width)])
    idx = [slice(None) if i in (a, b) else 0 for i in range(width)]
    wt[tuple(idx)] = w if a < b else w.T
    return (p * wt).reshape(-1)


def _apply_vertical(psi, width, a, bmat):
    """psi[..., s_a, ...] <- sum_s' B[s_a, s'] psi[..., s', ...] (a bond to the next row)."""
    p = psi.reshape([2] * width)
    p = np.moveaxis(np.tensordot(bmat, p, axes=([1], [a])), 0, a)
    return p.reshape(-1)


def boltzmann(beta_j):
    return np.array([[math.exp(beta_j), math.exp(-beta_j)],
                     [math.exp(-beta_j), math.exp(beta_j)]])


def tm_2d(ly: int, lx: int, beta: float, j: float = 1.0) -> float:
    """ln Z of the open ly x lx Ising lattice by the row transfer matrix (lx <= 20)."""
    b = boltzmann(beta * j)
    psi = np.ones(1 << lx)
    log = 0.0
    for y in range(ly):
        for x in range(lx - 1):
            psi = _apply_pair(psi, lx, x, x + 1, b)
        if y + 1 < ly:
            for x in range(lx):
                psi = _apply_vertical(psi, lx, x, b)
        m = np.max(np.abs(psi))
        psi /= m
        log += math.log(m)
    return log + math.log(np.sum(psi))


def tm_3d(lz: int, ly: int, lx: int, beta: float, j: float = 1.0) -> float:
    """ln Z of the open lz x ly x lx Ising lattice by the plane transfer matrix (ly*lx <= 20)."""
    b = boltzmann(beta * j)
    w = ly * lx
    site = lambda y, x: y * lx + x
    psi = np.ones(1 << w)
    log = 0.0
    for z in range(lz):
        for y in range(ly):
            for x in range(lx):
                if x + 1 < lx:
                    psi = _apply_pair(psi, w, site(y, x), site(y, x + 1), b)
                if y + 1 < ly:
                    psi = _apply_pair(psi, w, site(y, x), site(y + 1, x), b)
        if z + 1 < lz:
            for s in range(w):
                psi = _apply_vertical(psi, w, s, b)
        m = np.max(np.abs(psi))
        psi /= m
        log += math.log(m)
    return log + math.log(np.sum(psi))


# ---------------------------------------------------------------- Onsager

def onsager_f(beta: float, j: float = 1.0) -> float:
    """Free energy per site -beta*F/N = lim lnZ/N of the square-lattice Ising model.

    f(K) = ln(2 cosh 2K) + (1/2pi) int_0^pi ln[(1 + sqrt(1 - k^2 sin^2 t)) / 2] dt,
    k = 2 sinh 2K / cosh^2 2K, K = beta*J (Onsager's solution).
    """
    k_ = beta * j
    kap = 2.0 * math.sinh(2 * k_) / math.cosh(2 * k_) ** 2
    g = lambda t: math.log((1.0 + math.sqrt(max(0.0, 1.0 - kap * kap * math.sin(t) ** 2))) / 2.0)
    val, _ = integrate.quad(g, 0.0, math.pi, limit=400, epsabs=1e-15, epsrel=1e-15)
    return math.log(2.0 * math.cosh(2 * k_)) + val / (2.0 * math.pi)


def onsager_f_double(beta: float, j: float = 1.0) -> float:
    """The same free energy from the double-integral form:
    f = ln 2 + (1/2pi^2) int int ln[cosh^2 2K - sinh 2K (cos a + cos b)] da db."""
    k_ = beta * j
    c2, s2 = math.cosh(2 * k_) ** 2, math.sinh(2 * k_)
    inner = lambda a: integrate.quad(lambda b: math.log(c2 - s2 * (math.cos(a) + math.cos(b))),
                                     0.0, math.pi, limit=200, epsabs=1e-14, epsrel=1e-14)[0]
    val, _ = integrate.quad(inner, 0.0, math.pi, limit=200, epsabs=1e-13, epsrel=1e-13)
    return math.log(2.0) + val / (2.0 * math.pi ** 2)


# ---------------------------------------------------------------- full einsum

def einsum_network(net) -> float:
    """Exact value of a small closed network by one numpy.einsum call (returns Z)."""
    letters = {}
    alphabet = [chr(c) for c in range(ord('a'), ord('z') + 1)] + \
               [chr(c) for c in range(ord('A'), ord('Z') + 1)]
    if len(net.edges) > len(alphabet):
        raise ValueError("network too large for einsum")
    subs = []
    for t, a in enumerate(net.tensors):
        s = [None] * a.ndim
        subs.append(s)
    for e, (t0, m0, t1, m1) in enumerate(net.edges):
        subs[t0][m0] = alphabet[e]
        subs[t1][m1] = alphabet[e]
    expr = ",".join("".join(s) for s in subs) + "->"
    path = np.einsum_path(expr, *net.tensors, optimize=("greedy", 1 << 24))[0]
    return float(np.einsum(expr, *net.tensors, optimize=path))
