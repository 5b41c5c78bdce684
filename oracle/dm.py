"""Density-matrix approximate contraction: plain, slow FP64 reference (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py). Written from the paper, not
shared with the GPU path.

What is computed (paper sections 4.2, 6.2, 6.3 and Appendix C):

* The closed network is contracted along a maximally unbalanced partition path
  (Algorithm partitioned_contract restricted to a linear path): partition P_j is
  the union of env_size consecutive slices, and the absorbed set grows by one
  partition at a time.
* After each absorption, the union of the current boundary MPS and the partition's
  tensors is approximated by a new MPS (the MPS tree of Definition "MPS tree",
  root at the last leaf) with Algorithm density_matrix_alg: a post-order sweep over
  the tree where, at each non-root vertex, the density matrix (Definition
  "density matrix") is formed from cached environments (Eq. dm_cache), its leading
  eigenvectors are kept and merged into the parent vertex.
* The value is returned as ln|Z| and the sign of Z; intermediate blocks are
  rescaled by exact powers of two whose exponents are summed in FP64.

Readings of the paper that this file fixes (the paper leaves them open):

* leaf order: surviving old leaves keep their old position; the new leaves of a
  partition tensor follow its anchor (the lowest old position among the leaves it
  contracts, else propagated from its lowest-path-index anchored neighbour in the
  partition, else appended), then path indices, then the edge id;
* embedding: a partition tensor sits at the position of its first new leaf; one
  without new leaves sits at the first position whose key is not below its own
  (direct) anchor if it contracts old leaves, else at the position of its
  lowest-path-index neighbour in the partition placed in an earlier pass (passes
  repeat until stable), else at the last position; an old
  MPS tensor sits at the new position of its own leaf (else likewise by its old
  position); a leaf whose owning tensor sits elsewhere is carried to its position
  by an identity matrix (the identity insertion of section 6.2);
* keep() (the paper's leading_eigenvectors says nothing about ties or numerical
  zeros): top eigenpairs, at most chi, dropping eigenvalues <= tau_rel * w1
  (tau_rel = 1e-12) and never cutting where the spectrum does not separate:
  while w_k - w_{k+1} <= tau_deg * w_k (tau_deg = 0.1) and w_{k+1} exceeds
  CLUSTER_FLOOR * tau_rel * w1 (CLUSTER_FLOOR = 0.1), the cut moves up by one.
  Why: any backward-stable FP64 eigensolver returns the spectrum of L + E with
  ||E|| up to a small multiple of eps ||L||. A cut at relative gap g turns the kept
  subspace by about eps w1 / (g w_k) and moves the result by about eps / g, so
  tau_deg = 0.1 keeps every cut's sensitivity near 1e-15; and an eigenvalue kept
  at 1e-15 w1 is indistinguishable from E, its eigenvector a random direction of
  the near-null space, which later partitions can amplify (on #CSP networks such a
  direction moved lnZ by 1e-7 per variable), so tau_rel = 1e-12 keeps only
  eigenvalues the FP64 solve resolves. The rule is blind to zero padding;
* the first tree vertex holds positions 1 and 2 (the first non-leaf node of the
  MPS tree joins the first two leaves).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LN2 = math.log(2.0)
TAU_REL = 1e-12
TAU_DEG = 0.1
CLUSTER_FLOOR = 0.1        # the separation rule applies to w_{k+1} > CLUSTER_FLOOR * tau_rel * w1

# The symmetric eigensolver keep() calls. Any backward-stable one gives an equally
# valid result; swapping it (e.g. for LAPACK's relatively robust representation
# driver) measures how far the method's result is fixed by FP64 arithmetic on a
# given network.
EIGH = np.linalg.eigh


# ---------------------------------------------------------------- labelled tensors

@dataclass
class T:
    """A dense tensor whose modes carry hashable labels (edge names)."""

    data: np.ndarray
    labels: tuple

    def __post_init__(self):
        assert self.data.ndim == len(self.labels), (self.data.shape, self.labels)
        assert len(set(self.labels)) == len(self.labels), self.labels

    def size(self):
        return int(np.prod(self.data.shape, dtype=np.int64)) if self.data.ndim else 1

    def dim(self, lab):
        return self.data.shape[self.labels.index(lab)]

    def transpose_to(self, labels):
        perm = [self.labels.index(l) for l in labels]
        return T(np.transpose(self.data, perm), tuple(labels))


def contract(a: T, b: T) -> T:
    """Sum over every label the two tensors share (pairwise contraction, section 2.2)."""
    shared = [l for l in a.labels if l in b.labels]
    ia = [a.labels.index(l) for l in shared]
    ib = [b.labels.index(l) for l in shared]
    out = np.tensordot(a.data, b.data, axes=(ia, ib))
    labels = tuple(l for l in a.labels if l not in shared) + tuple(l for l in b.labels if l not in shared)
    return T(out, labels)


def _result_log_size(a: T, b: T) -> float:
    s = 0.0
    for l in a.labels:
        if l not in b.labels:
            s += math.log(a.dim(l))
    for l in b.labels:
        if l not in a.labels:
            s += math.log(b.dim(l))
    return s


def absorb_in_order(units):
    """Contract tensors one at a time into a running intermediate, in the given order."""
    cur = units[0]
    for u in units[1:]:
        cur = contract(cur, u)
    return cur


def closing_order(units):
    """The partition's tensors sorted for a sweep along the old leaf positions.

    Used when everything of a partition step is contracted at once (at most two
    new leaves): a sweep in position order keeps the intermediate as small as the
    boundary, whereas a greedy order can leave a whole row of bonds open.
    """
    return [u.t for u in sorted(units, key=lambda u: u.sweep)]


def absorb_all(start, units):
    """Contract a list of tensors one at a time into a running intermediate.

    The next tensor is the one giving the smallest intermediate (ties: list order).
    The paper leaves the contraction order inside a density matrix free (it uses a
    path optimiser); any order gives the same value up to rounding.
    """
    rest = list(units)
    cur = start
    if cur is None:
        cur = rest.pop(0)
    while rest:
        best = min(range(len(rest)), key=lambda i: (_result_log_size(cur, rest[i]), i))
        cur = contract(cur, rest.pop(best))
    return cur


def rescale(t: T):
    """Multiply by 2^-e with e the frexp exponent of max|t|; returns (tensor, e)."""
    m = float(np.max(np.abs(t.data))) if t.data.size else 0.0
    if m == 0.0 or not math.isfinite(m):
        return t, 0
    _, e = math.frexp(m)
    return T(np.ldexp(t.data, -e), t.labels), e


# ---------------------------------------------------------------- keep rule

def keep(L: np.ndarray, chi: int, tau_rel=TAU_REL, tau_deg=TAU_DEG):
    """Leading eigenvectors of a symmetric PSD density matrix (leading_eigenvectors).

    Returns (U, w, k, fallback) with U = the k leading eigenvectors, w all
    eigenvalues in descending order. k starts at min(chi, dim), drops eigenvalues
    <= tau_rel*w1 (below what an FP64 solve resolves), then steps down while the
    spectrum does not separate at the cut (w_{k+1} > CLUSTER_FLOOR*tau_rel*w1 and
    w_k - w_{k+1} <= tau_deg*w_k). Zero rows and columns added to L only add
    eigenvalues below both floors, so they never change k. If nothing survives,
    min(chi, dim) vectors are kept and fallback is True.
    """
    w, v = EIGH(L)
    w = w[::-1].copy()
    v = v[:, ::-1].copy()
    dim = len(w)
    w1 = w[0] if dim else 0.0
    k = min(chi, dim)
    while k >= 1 and w[k - 1] <= tau_rel * w1:
        k -= 1
    while 1 <= k < dim and w[k] > CLUSTER_FLOOR * tau_rel * w1 and w[k - 1] - w[k] <= tau_deg * w[k - 1]:
        k -= 1
    fallback = False
    if k == 0:
        k = min(chi, dim)
        fallback = True
    return v[:, :k], w, k, fallback


def keep_qr_svd(C: np.ndarray, R: np.ndarray, chi: int, tau_rel=TAU_REL, tau_deg=TAU_DEG):
    """The QR-SVD branch of Algorithm density_matrix_alg for a vertex whose open size
    (rows of C) exceeds its crossing size (columns of C): instead of forming the
    density matrix L = C R C^T, orthogonalise C = Q Rc, take the leading eigenvectors
    of the small matrix Rc R Rc^T under keep(), and map them back through Q. L and
    Rc R Rc^T share their nonzero spectrum (L = Q (Rc R Rc^T) Q^T), so the kept rank and
    subspace are those of keep(L). Returns (U, w, k, fallback) like keep(), with w the
    spectrum of the small matrix."""
    Q, Rc = np.linalg.qr(C)                # reduced: Q has min(rows, cols) columns
    M = Rc @ R @ Rc.T
    M = 0.5 * (M + M.T)
    Uh, w, k, fb = keep(M, chi, tau_rel, tau_deg)
    return Q @ Uh, w, k, fb


# ---------------------------------------------------------------- structural plan

@dataclass
class Unit:
    """One tensor of the union network of a partition step."""

    t: T
    kind: str          # 'mps', 'site' or 'id'
    ref: int           # mps: old own-leaf position (1-based); site: vertex id; id: position
    order: int = 0     # tie-break order (mps first, then sites in path order, then ids)
    sweep: tuple = ()  # order of the closing sweep: (old position or anchor, kind, path index)


@dataclass
class PartitionPlan:
    leaves: list       # new leaf labels in order (position 1..n)
    leaf_edges: list   # same, as original edge ids
    groups: list       # groups[k-1] = list of unit indices at position k
    units: list        # the union network after identity insertion
    placement: list    # per unit: (kind, ref, position)


def partitions_of(slices, env_size):
    return [sum(slices[i:i + env_size], []) for i in range(0, len(slices), env_size)]


def plan_partition(net, j, part, absorbed, path_index, mps_units, old_leaves):
    """Leaf order, embedding and identity insertion for one absorption.

    mps_units: list of (T, own_position); old_leaves: list of original edge ids in
    order. Returns a PartitionPlan. Pure graph logic: no tensor data is touched
    except to copy references.
    """
    pset = set(part)
    edges = net.edges
    endpoints = lambda e: (edges[e][0], edges[e][2])

    def far_end(e):
        a, b = endpoints(e)
        return b if a in absorbed else a

    # old leaves: contracted (far end in P) or surviving
    contracted = {}  # position -> edge
    surviving = []   # (position, edge)
    for p, e in enumerate(old_leaves, start=1):
        if far_end(e) in pset:
            contracted[p] = e
        else:
            surviving.append((p, e))

    # anchors of partition tensors (path order)
    order_p = sorted(part, key=lambda v: path_index[v])
    anchor = {}
    for t in order_p:
        cand = [p for p, e in contracted.items() if far_end(e) == t]
        anchor[t] = min(cand) if cand else None
    direct = dict(anchor)
    inc = net.meta.setdefault('_incidence', None)
    if inc is None:
        inc = [[] for _ in net.tensors]
        for e, (t0, m0, t1, m1) in enumerate(edges):
            inc[t0].append((e, m0, t1))
            inc[t1].append((e, m1, t0))
        net.meta['_incidence'] = inc
    nbrs = {t: [o for (_, _, o) in inc[t] if o in pset] for t in part}
    for t in order_p:
        if anchor[t] is None:
            got = [u for u in nbrs[t] if anchor[u] is not None]
            if got:
                u = min(got, key=lambda u: path_index[u])
                anchor[t] = anchor[u]
    INF = math.inf
    for t in order_p:
        if anchor[t] is None:
            anchor[t] = INF

    # new leaves and their sort keys
    keyed = []
    for p, e in surviving:
        keyed.append(((p, 0, 0, 0, 0), e))
    done = absorbed | pset
    for t in order_p:
        for (e, _, other) in inc[t]:
            if other not in done:
                keyed.append(((anchor[t], 1, path_index[t], path_index[other], e), e))
    keyed.sort(key=lambda ke: ke[0])
    keys = [k for k, _ in keyed]
    leaf_edges = [e for _, e in keyed]
    n = len(leaf_edges)
    pos_of_edge = {e: i + 1 for i, e in enumerate(leaf_edges)}

    def first_pos_at_or_after(a):
        for i, k in enumerate(keys):
            if k[0] >= a:
                return i + 1
        return n

    # union network units
    units = []
    for (t, own) in mps_units:
        units.append(Unit(t, 'mps', own, 0, (own, 0, 0)))
    for t in order_p:
        a = net.tensors[t]
        labs = [None] * a.ndim
        for (e, m, _) in inc[t]:
            labs[m] = ('e', e)
        units.append(Unit(T(a, tuple(labs)), 'site', t, 1 + path_index[t],
                          (anchor[t], 1, path_index[t])))

    if n == 0:
        return PartitionPlan([], [], [], units, [(u.kind, u.ref, 0) for u in units])

    # embedding
    pos = [None] * len(units)
    site_unit = {}
    for i, u in enumerate(units):
        if u.kind == 'mps':
            own_edge = old_leaves[u.ref - 1]
            if own_edge in pos_of_edge:
                pos[i] = pos_of_edge[own_edge]
            else:
                pos[i] = first_pos_at_or_after(u.ref)
        else:
            site_unit[u.ref] = i
            mine = [pos_of_edge[lab[1]] for lab in u.t.labels
                    if lab[0] == 'e' and lab[1] in pos_of_edge]
            if mine:
                pos[i] = min(mine)
            elif direct[u.ref] is not None:
                pos[i] = first_pos_at_or_after(direct[u.ref])
    # leafless tensors without contracted leaves follow their lowest-path-index
    # neighbour in the partition that was placed before the current pass; passes
    # repeat until nothing changes
    while True:
        prev = list(pos)
        for t in order_p:
            i = site_unit[t]
            if prev[i] is None:
                placed = [u for u in nbrs[t] if prev[site_unit[u]] is not None]
                if placed:
                    pos[i] = prev[site_unit[min(placed, key=lambda u: path_index[u])]]
        if pos == prev:
            break
    pos = [n if p is None else p for p in pos]

    # identity insertion: each position's leaf must live in its own group
    big = 1 << 40
    for k in range(1, n + 1):
        lab = ('e', leaf_edges[k - 1])
        owner = next(i for i, u in enumerate(units) if lab in u.t.labels)
        if pos[owner] != k:
            s = ('s', j, k)
            ut = units[owner].t
            units[owner].t = T(ut.data, tuple(s if l == lab else l for l in ut.labels))
            d = ut.dim(lab)
            units.append(Unit(T(np.eye(d), (s, lab)), 'id', k, big + k, (math.inf, 2, k)))
            pos.append(k)

    groups = [[] for _ in range(n)]
    for i, p in enumerate(pos):
        groups[p - 1].append(i)
    for g in groups:
        g.sort(key=lambda i: units[i].order)
    placement = [(u.kind, u.ref, p) for u, p in zip(units, pos)]
    leaves = [('e', e) for e in leaf_edges]
    return PartitionPlan(leaves, leaf_edges, groups, units, placement)


def crossing_labels(plan: PartitionPlan):
    """X_k for every cut k: labels of union edges joining positions <= k and > k."""
    where = {}
    for gi, g in enumerate(plan.groups):
        for i in g:
            for l in plan.units[i].t.labels:
                where.setdefault(l, []).append(gi + 1)
    n = len(plan.groups)
    X = {k: [] for k in range(1, n)}
    for l, ps in where.items():
        if len(ps) == 2:
            for k in range(min(ps), max(ps)):
                X[k].append(l)
    return {k: sorted(v, key=repr) for k, v in X.items()}


# ---------------------------------------------------------------- the algorithm

@dataclass
class Stats:
    n_eig: int = 0
    n_fallback: int = 0
    max_asym: float = 0.0      # max |L - L^T| / max|L| before symmetrisation
    min_ratio: float = 1.0     # min w_min / w_1 over all density matrices
    kept: list = field(default_factory=list)
    dims: list = field(default_factory=list)   # (rows, crossing size) of every vertex's C
    plans: list = field(default_factory=list)
    harvest: list = field(default_factory=list)


def _bra(lab, leaf):
    return lab if lab == leaf else ('bra', lab)


def contract_approx(net, chi: int, env_size: int, tau_rel=TAU_REL, tau_deg=TAU_DEG,
                    gauge_rng=None, stats: Stats | None = None, harvest=False, env_checkpoint=None,
                    qr_svd=False):
    """Approximate ln|Z| and sign(Z) of a closed network (returns (log_abs, sign)).

    gauge_rng: if given, every kept basis U is rotated by a random orthogonal
    matrix (the result must not change: only span(U) matters).
    harvest: keep every (density matrix, kept rank) pair in stats.harvest.
    env_checkpoint: None keeps every right environment of a partition step in
    memory; an integer c keeps only every c-th one (and the lowest stretch) and
    recomputes the others from the nearest kept one above when the forward sweep
    reaches them. A memory schedule only: the same operations on the same operands,
    so the result is bit-identical.
    qr_svd: at every vertex whose open size exceeds its crossing size take the QR-SVD
    branch of the algorithm (keep_qr_svd) instead of forming the density matrix; the
    default forms it everywhere (same kept subspaces, up to rounding).
    """
    if chi < 1 or env_size < 1:
        raise ValueError("chi and env_size must be >= 1")
    stats = stats if stats is not None else Stats()
    path_index = {}
    for s in net.slices:
        for v in s:
            path_index[v] = len(path_index)
    parts = partitions_of(net.slices, env_size)

    acc = 0.0
    sgn = 1
    absorbed = set()
    mps = []        # list of (T, own position)
    leaves = []     # original edge ids, in order
    for j, part in enumerate(parts):
        plan = plan_partition(net, j, part, absorbed, path_index, mps, leaves)
        stats.plans.append((plan.leaf_edges, plan.placement))
        n = len(plan.leaves)
        units = plan.units
        if n == 0:
            z = absorb_in_order(closing_order(units))
            val = float(z.data)
            if val == 0.0:
                return -math.inf, 0
            acc += math.log(abs(val))
            sgn *= 1 if val > 0 else -1
            mps, leaves = [], []
        elif n <= 2:
            root = absorb_in_order(closing_order(units)).transpose_to(plan.leaves)
            root, e = rescale(root)
            acc += e * LN2
            if not np.any(root.data):
                return -math.inf, 0
            mps, leaves = [(root, 1)], list(plan.leaf_edges)
        else:
            mps, extra = _dm_sweep(plan, j, chi, tau_rel, tau_deg, gauge_rng, stats, harvest, env_checkpoint,
                                   qr_svd)
            acc += extra
            leaves = list(plan.leaf_edges)
            if mps is None:
                return -math.inf, 0
        absorbed |= set(part)
    return acc, sgn


def _dm_sweep(plan, j, chi, tau_rel, tau_deg, gauge_rng, stats, harvest, env_checkpoint=None, qr_svd=False):
    """Algorithm density_matrix_alg on the MPS tree of one partition step.

    Right environments R_k (k = n-1 .. 2) are the memoised density matrices
    DM(u, v) of Eq. dm_cache for the subtree to the right of cut k; the forward
    sweep forms L = C R_k C^T at each tree vertex, keeps its leading eigenvectors
    and merges U^T into the parent (the next C).
    """
    n = len(plan.leaves)
    grp = lambda k: [plan.units[i].t for i in plan.groups[k - 1]]
    X = crossing_labels(plan)

    def env(k, r_next):
        """R_k from R_{k+1} (None for k = n-1): the group at k+1 absorbed ket then bra,
        its leaf traced between them."""
        leaf = plan.leaves[k]          # leaf of position k+1
        ket = grp(k + 1)
        bra = [T(t.data, tuple(_bra(l, leaf) for l in t.labels)) for t in ket]
        r = absorb_all(r_next, ket + bra)
        want = tuple(X[k]) + tuple(('bra', l) for l in X[k])
        assert set(r.labels) == set(want), (r.labels, want)
        r, _ = rescale(r.transpose_to(want))
        return r

    # right environments, k = n-1 down to 2; with a checkpoint interval c only R_k with
    # (n-1-k) % c == 0 and the lowest stretch (reached first by the forward sweep) stay
    R = {}
    low = 2 + ((n - 3) % env_checkpoint if env_checkpoint else 0)
    prev = None
    for k in range(n - 1, 1, -1):
        r = env(k, prev)
        if env_checkpoint is None or (n - 1 - k) % env_checkpoint == 0 or k <= low:
            R[k] = r
        prev = r
    prev = None

    def env_at(k):
        if k not in R:                 # recompute the stretch below the next kept R
            top = min(i for i in R if i > k)
            r = R[top]
            for i in range(top - 1, k - 1, -1):
                r = env(i, r)
                R[i] = r
        return R[k]

    acc = 0.0
    c = absorb_all(None, grp(1) + grp(2))
    rows = [plan.leaves[0], plan.leaves[1]]
    c = c.transpose_to(tuple(rows) + tuple(X[2]))
    c, e = rescale(c)
    acc += e * LN2
    out = []
    for k in range(2, n):
        nr = int(np.prod([c.dim(l) for l in rows]))
        cm = c.data.reshape(nr, -1)
        rk = env_at(k)
        if env_checkpoint is not None:
            del R[k]                   # the forward sweep never returns to it
        d = int(np.prod([rk.dim(l) for l in X[k]])) if X[k] else 1
        rm = rk.data.reshape(d, d)
        if qr_svd and nr > d:
            U, w, kk, fb = keep_qr_svd(cm, rm, chi, tau_rel, tau_deg)
            L = None
        else:
            L = cm @ rm @ cm.T
            mx = float(np.max(np.abs(L))) if L.size else 0.0
            if mx > 0:
                stats.max_asym = max(stats.max_asym, float(np.max(np.abs(L - L.T))) / mx)
            L = 0.5 * (L + L.T)
            U, w, kk, fb = keep(L, chi, tau_rel, tau_deg)
        stats.n_eig += 1
        stats.dims.append((nr, d))
        stats.n_fallback += int(fb)
        stats.kept.append(kk)
        if w[0] > 0:
            stats.min_ratio = min(stats.min_ratio, float(w[-1] / w[0]))
        if harvest and L is not None:
            stats.harvest.append((L.copy(), kk, nr, d))
        if gauge_rng is not None:
            q, _ = np.linalg.qr(gauge_rng.standard_normal((kk, kk)))
            U = U @ q
        b = ('b', j, k - 1)
        ut = T(U.reshape([c.dim(l) for l in rows] + [kk]), tuple(rows) + (b,))
        out.append((ut, 1 if k == 2 else k))
        c = contract(ut, c)  # (b, X_k)
        c = absorb_all(c, grp(k + 1))
        rows = [b, plan.leaves[k]]
        tail = tuple(X[k + 1]) if k + 1 < n else ()
        c = c.transpose_to(tuple(rows) + tail)
        c, e = rescale(c)
        acc += e * LN2
    if not np.any(c.data):
        return None, acc
    out.append((c, n))
    return out, acc
