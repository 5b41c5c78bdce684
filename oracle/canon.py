"""Canonicalisation twin of the density-matrix oracle (TEST INFRASTRUCTURE ONLY).

The paper states that the density-matrix algorithm and truncation of the explicit
(untruncated) tree by canonicalisation give the same output (section 3.2, the
apply-then-truncate MPO-MPS algorithm, and the cost lemma of Appendix F that runs
both on the same update order). This module computes the approximate contraction
that way, to pin the density-matrix oracle at chi below the full bond dimension:

1. with the same leaf order and embedding as the oracle, each position's group is
   contracted into one site tensor of the untruncated MPS; an edge that passes over
   a position is carried through it by an identity;
2. the MPS is brought to right-canonical form by QR from the right end
   (Definition canonical_form, Algorithm canonize);
3. a left-to-right sweep takes the SVD of each site, keeps singular vectors with
   the same rank rule applied to the squared singular values, and pushes the
   remainder into the next site.

It shares the structural plan with oracle.dm but none of its numerical steps.
"""
from __future__ import annotations

import math

import numpy as np

from .dm import T, contract, absorb_all, absorb_in_order, closing_order, plan_partition, partitions_of

CLUSTER_FLOOR = 0.1        # separation rule above CLUSTER_FLOOR * tau_rel * w1, as in dm.keep

LN2 = math.log(2.0)


def _keep_from_spectrum(w, chi, tau_rel, tau_deg):
    """Kept rank for eigenvalues w (descending) under the oracle's rank rule."""
    dim = len(w)
    w1 = w[0] if dim else 0.0
    k = min(chi, dim)
    while k >= 1 and w[k - 1] <= tau_rel * w1:
        k -= 1
    while 1 <= k < dim and w[k] > CLUSTER_FLOOR * tau_rel * w1 and w[k - 1] - w[k] <= tau_deg * w[k - 1]:
        k -= 1
    return k if k > 0 else min(chi, dim)


def _scale_pow2(data):
    m = float(np.max(np.abs(data))) if data.size else 0.0
    if m == 0.0:
        return data, 0
    _, e = math.frexp(m)
    return np.ldexp(data, -e), e


def _canon_sweep(plan, j, chi, tau_rel, tau_deg):
    n = len(plan.leaves)
    gpos = {}
    for gi, g in enumerate(plan.groups):
        for i in g:
            gpos[i] = gi + 1
    span = {}  # internal label -> (p, q) positions of its two ends
    for i, u in enumerate(plan.units):
        for l in u.t.labels:
            span.setdefault(l, []).append(gpos[i])
    span = {l: (min(ps), max(ps)) for l, ps in span.items() if len(ps) == 2}

    # untruncated site tensors with per-cut copies of every crossing edge
    sites = []
    for k in range(1, n + 1):
        s = absorb_all(None, [plan.units[i].t for i in plan.groups[k - 1]])
        labs = []
        for l in s.labels:
            if l in span:
                p, q = span[l]
                if p == q:
                    raise AssertionError("internal edge left open in a group")
                labs.append((l, p) if k == p else (l, q - 1))
            else:
                labs.append(l)
        s = T(s.data, tuple(labs))
        for l, (p, q) in span.items():
            if p < k < q:
                d = None
                for i in plan.groups[p - 1]:
                    if l in plan.units[i].t.labels:
                        d = plan.units[i].t.dim(l)
                s = contract(s, T(np.eye(d), ((l, k - 1), (l, k))))
        sites.append(s)

    def left_labels(k):
        return [lab for lab in sites[k - 1].labels if isinstance(lab, tuple) and len(lab) == 2
                and lab[0] in span and lab[1] == k - 1]

    def right_labels(k):
        return [lab for lab in sites[k - 1].labels if isinstance(lab, tuple) and len(lab) == 2
                and lab[0] in span and lab[1] == k]

    # merge positions 1 and 2 (the first tree vertex)
    first = contract(sites[0], sites[1])
    sites = [None, first] + sites[2:]
    bond = {}  # cut -> label of the single canonical bond

    # right-canonical form by QR from the right
    for k in range(n, 2, -1):
        s = sites[k - 1]
        left = [l for l in s.labels if (isinstance(l, tuple) and len(l) == 2 and l[0] in span
                                         and l[1] == k - 1) or l == bond.get(k - 1)]
        rest = [l for l in s.labels if l not in left]
        s = s.transpose_to(tuple(left) + tuple(rest))
        dl = int(np.prod([s.dim(l) for l in left]))
        m = s.data.reshape(dl, -1)
        q, r = np.linalg.qr(m.T)           # m = r^T q^T
        c = ('rc', j, k - 1)
        sites[k - 1] = T(q.T.reshape((q.shape[1],) + s.data.shape[len(left):]), (c,) + tuple(rest))
        rt = T(r.T.reshape([s.dim(l) for l in left] + [q.shape[1]]), tuple(left) + (c,))
        sites[k - 2] = contract(sites[k - 2], rt)
        bond[k - 1] = c

    # left sweep with truncated SVDs
    acc = 0.0
    out = []
    cur = sites[1]
    rows = [plan.leaves[0], plan.leaves[1]]
    for k in range(2, n):
        c = bond[k]
        cur = cur.transpose_to(tuple(rows) + (c,))
        data, e = _scale_pow2(cur.data)
        acc += e * LN2
        nr = int(np.prod(data.shape[:-1]))
        m = data.reshape(nr, -1)
        u, sv, vt = np.linalg.svd(m, full_matrices=False)
        w = np.zeros(nr)
        w[:len(sv)] = sv ** 2
        kk = _keep_from_spectrum(w, chi, tau_rel, tau_deg)
        kk_avail = min(kk, u.shape[1])
        uk = u[:, :kk_avail]
        if kk > kk_avail:  # rank-deficient fallback: pad with an orthonormal complement
            full, _ = np.linalg.qr(np.concatenate([uk, np.eye(nr)], axis=1))
            uk = full[:, :kk]
        b = ('b', j, k - 1)
        ut = T(uk.reshape(list(data.shape[:-1]) + [kk]), tuple(rows) + (b,))
        out.append((ut, 1 if k == 2 else k))
        carry = T(uk.T @ m, (b, c))
        cur = contract(carry, sites[k])
        rows = [b, plan.leaves[k]]
    cur = cur.transpose_to(tuple(rows))
    data, e = _scale_pow2(cur.data)
    acc += e * LN2
    out.append((T(data, tuple(rows)), n))
    return out, acc


def contract_canon(net, chi: int, env_size: int, tau_rel=1e-12, tau_deg=0.1):
    """ln|Z|, sign(Z) by canonicalisation-based truncation on the oracle's plan."""
    path_index = {}
    for s in net.slices:
        for v in s:
            path_index[v] = len(path_index)
    acc = 0.0
    sgn = 1
    absorbed = set()
    mps, leaves = [], []
    for j, part in enumerate(partitions_of(net.slices, env_size)):
        plan = plan_partition(net, j, part, absorbed, path_index, mps, leaves)
        n = len(plan.leaves)
        if n == 0:
            z = float(absorb_in_order(closing_order(plan.units)).data)
            if z == 0.0:
                return -math.inf, 0
            acc += math.log(abs(z))
            sgn *= 1 if z > 0 else -1
            mps, leaves = [], []
        elif n <= 2:
            root = absorb_in_order(closing_order(plan.units)).transpose_to(plan.leaves)
            data, e = _scale_pow2(root.data)
            acc += e * LN2
            mps, leaves = [(T(data, root.labels), 1)], list(plan.leaf_edges)
        else:
            mps, extra = _canon_sweep(plan, j, chi, tau_rel, tau_deg)
            acc += extra
            leaves = list(plan.leaf_edges)
        absorbed |= set(part)
    return acc, sgn
