"""ORACLE (test infrastructure only): a plain CPU FP64 barycentric Lagrange treecode.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this.
It takes the steps of the paper's Algorithm 3 (Section 6.3) in the paper's order:

1. build the tree of source clusters and the target batches (Section 6.1);
2. for every source cluster, compute the proxy charges of Eq.
   particle-cluster-approx-rearranged (Section 6.2) with Chebyshev points of the
   second kind and the barycentric Lagrange basis (Eqs. Lagrange_polynomials,
   barycentric_weights);
3. for every target batch, run ComputePotential from the root with the MAC of
   Eq. MAC, evaluating accepted batch-cluster pairs by the approximation and the
   others by the direct sum of Eq. direct-sum_2.

Singularity subtraction (Section 4.3) enters by linearity (the paper states that
the treecode takes it in without giving the details): each cluster carries two charge sets,
f^_k from q_j = f_j w_j and w^_k from q_j = w_j. For Yukawa the approximated pair
sum is sum_k G(|r_i - s_k|) (f^_k - f_i w^_k); for Coulomb it is
sum_k [f^_k - f_i exp(-|r_i - s_k|^2/a^2) w^_k] / |r_i - s_k|. Near pairs use the
subtracted particle sums, skipping distance exactly zero, and the analytic term
(4 pi f_i / k^2, or 2 pi a^2 f_i) is added once per target at the end.

Readings where the paper is silent (each shared, by statement only, with the GPU
implementation):
* root box = the given domain box, else the bounding box of the sources; the
  root is split at the midpoint of that box; every cluster (root included) is
  shrunk to the bounding box of its particles, and a non-root cluster is split at
  the midpoint of its shrunk box;
* dimension d is split iff ext_d >= ext_max * (1/sqrt 2) (the aspect rule) and
  ext_d > 0; the child digit is 4*[x >= mid_x] + 2*[y >= mid_y] + [z >= mid_z]
  over split dimensions; children are the non-empty digits in increasing order
  and keep their particles' relative order; a cluster is a leaf iff it holds at
  most N_L particles (or cannot be split);
* nodes are numbered level by level (parents in order, children in digit order);
* cluster centre = midpoint of the shrunk box, radius = half its diagonal,
  R = distance between centres; the distance part of the MAC is
  (r_B + r_C) < theta * R and the size part is (n+1)^3 < N_S, both strict;
* proxy nodes s_k = c + h cos(pi k / n) with the end nodes set exactly to the box
  faces (s_0 = hi, s_n = lo); a particle that coincides with a node takes the
  Kronecker basis there; a zero-extent dimension puts all mass on node 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SQRT1_2 = 0.70710678118654752440


@dataclass
class Tree:
    perm: np.ndarray          # tree position -> original index
    begin: np.ndarray         # per node, [begin, end) in tree positions
    end: np.ndarray
    lo: np.ndarray            # (n_nodes, 3) shrunk box
    hi: np.ndarray
    level: np.ndarray
    parent: np.ndarray
    children: list = field(default_factory=list)  # per node: list of child ids

    @property
    def n_nodes(self):
        return self.begin.size

    def is_leaf(self, c):
        return len(self.children[c]) == 0

    def leaves(self):
        return [c for c in range(self.n_nodes) if not self.children[c]]

    def count(self, c):
        return int(self.end[c] - self.begin[c])


def build_tree(x, y, z, leaf_size: int, domain=None) -> Tree:
    pts = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64),
                    np.asarray(z, np.float64)], axis=1)
    n = pts.shape[0]
    if domain is not None:
        root_lo = np.array(domain[0], dtype=np.float64)
        root_hi = np.array(domain[1], dtype=np.float64)
    else:
        root_lo = pts.min(axis=0)
        root_hi = pts.max(axis=0)
    # level-ordered construction; each node holds its particles' original indices
    nodes_idx = [np.arange(n, dtype=np.int64)]
    split_lo = [root_lo]
    split_hi = [root_hi]
    parent = [-1]
    level = [0]
    children = [[]]
    begin = [0]
    cur = [0]
    while cur:
        nxt = []
        for c in cur:
            idx = nodes_idx[c]
            if idx.size <= leaf_size:
                continue
            slo, shi = split_lo[c], split_hi[c]
            ext = shi - slo
            lmax = ext.max()
            if not lmax > 0.0:
                continue
            split = (ext >= lmax * SQRT1_2) & (ext > 0.0)
            mid = 0.5 * (slo + shi)
            p = pts[idx]
            digit = np.zeros(idx.size, dtype=np.int64)
            for d, bit in ((0, 4), (1, 2), (2, 1)):
                if split[d]:
                    digit += bit * (p[:, d] >= mid[d])
            groups = [(dg, idx[digit == dg]) for dg in range(8)]
            groups = [(dg, g) for dg, g in groups if g.size]
            if len(groups) < 2:
                continue
            off = begin[c]
            for dg, g in groups:
                cid = len(nodes_idx)
                nodes_idx.append(g)
                q = pts[g]
                split_lo.append(q.min(axis=0))
                split_hi.append(q.max(axis=0))
                parent.append(c)
                level.append(level[c] + 1)
                children.append([])
                begin.append(off)
                off += g.size
                children[c].append(cid)
                nxt.append(cid)
        cur = nxt
    nn = len(nodes_idx)
    lo = np.empty((nn, 3))
    hi = np.empty((nn, 3))
    for c in range(nn):
        q = pts[nodes_idx[c]]
        lo[c] = q.min(axis=0)
        hi[c] = q.max(axis=0)
    begin = np.array(begin, dtype=np.int64)
    end = begin + np.array([g.size for g in nodes_idx], dtype=np.int64)
    perm = np.empty(n, dtype=np.int64)
    for c in range(nn):
        if not children[c]:
            perm[begin[c]:end[c]] = nodes_idx[c]
    return Tree(perm=perm, begin=begin, end=end, lo=lo, hi=hi,
                level=np.array(level, dtype=np.int64), parent=np.array(parent, dtype=np.int64),
                children=children)


def geometry(tree: Tree):
    """centre (n_nodes, 3) and radius (n_nodes,) of every cluster's shrunk box."""
    c = 0.5 * (tree.lo + tree.hi)
    h = 0.5 * (tree.hi - tree.lo)
    r = np.sqrt(h[:, 0] * h[:, 0] + h[:, 1] * h[:, 1] + h[:, 2] * h[:, 2])
    return c, r


# ----------------------------------------------------------------------------------
# Section 6.2: interpolation points, barycentric basis, proxy charges

def cheb2_nodes(lo: float, hi: float, n: int) -> np.ndarray:
    """s_k = c + h cos(pi k / n), k = 0..n, with s_0 = hi and s_n = lo exactly."""
    k = np.arange(n + 1, dtype=np.float64)
    s = 0.5 * (lo + hi) + 0.5 * (hi - lo) * np.cos(np.pi * k / n)
    s[0] = hi
    s[n] = lo
    return s


def barycentric_weights(n: int) -> np.ndarray:
    b = np.array([(-1.0) ** k for k in range(n + 1)])
    b[0] *= 0.5
    b[n] *= 0.5
    return b


def lagrange_basis(t: np.ndarray, s: np.ndarray, b: np.ndarray) -> np.ndarray:
    """L_k(t_j) for all j, k by the barycentric formula; exact node hits give the
    Kronecker basis. Returns (len(t), len(s))."""
    t = np.asarray(t, dtype=np.float64)
    if s[0] == s[-1]:  # zero-extent dimension: all mass on node 0
        L = np.zeros((t.size, s.size))
        L[:, 0] = 1.0
        return L
    diff = t[:, None] - s[None, :]
    hit = diff == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        a = b[None, :] / diff
        L = a / a.sum(axis=1, keepdims=True)
    rows = hit.any(axis=1)
    if np.any(rows):
        L[rows] = hit[rows].astype(np.float64)
    return L


def proxy_charges(px, py, pz, q, lo, hi, n):
    """f^_{k1 k2 k3} = sum_j L_k1(x_j) L_k2(y_j) L_k3(z_j) q_j for q of shape
    (m, N_S) (several charge sets at once). Returns nodes (3, n+1) and charges
    (m, n+1, n+1, n+1)."""
    b = barycentric_weights(n)
    sx, sy, sz = (cheb2_nodes(lo[d], hi[d], n) for d in range(3))
    Lx = lagrange_basis(px, sx, b)
    Ly = lagrange_basis(py, sy, b)
    Lz = lagrange_basis(pz, sz, b)
    q = np.atleast_2d(q)
    fh = np.einsum("ja,jb,jc,mj->mabc", Lx, Ly, Lz, q, optimize=True)
    return np.stack([sx, sy, sz]), fh


# ----------------------------------------------------------------------------------
# Section 6.3: Algorithm 3

FAR, NEAR, OPEN = "far", "near", "open"


def classify(dist_ok: bool, size_ok: bool, leaf: bool) -> str:
    """Outcome of one batch-cluster pair under Eq. MAC (Section 6.2) and the
    ComputePotential step of Algorithm 3 (Section 6.3).

    The approximation is used only when both parts of the MAC hold: the cluster
    is well separated from the batch (distance part) and holds more sources than
    the approximation has proxy charges (size part). A well-separated cluster that
    is too small is summed directly as a whole. A cluster that is not well
    separated is resolved into its children, unless it has none, in which case
    it is summed directly."""
    if dist_ok:
        return FAR if size_ok else NEAR
    return NEAR if leaf else OPEN


def interaction_lists(tree: Tree, theta: float, n: int, ncoef: int | None = None,
                      batch_tree: Tree | None = None):
    """Per target batch: (far clusters, near clusters) of the source tree, in the
    order a depth-first visit from the root that takes children in order meets
    them (Algorithm 3 starts that visit at the root for every batch).

    Batches are the leaves of `batch_tree` (default: the source tree itself, when
    targets are the sources). `ncoef` is the size part of the MAC (a cluster is
    approximated only if ncoef < N_S), (n+1)^3 unless given. Returns (batches,
    far, near) with batches the leaf ids of the batch tree in node order."""
    cen, rad = geometry(tree)
    bt = tree if batch_tree is None else batch_tree
    bcen, brad = geometry(bt)
    if ncoef is None:
        ncoef = (n + 1) ** 3
    batches = bt.leaves()
    far, near = [], []
    for B in batches:
        fl, nl = [], []
        work = [0]  # clusters still to classify; the last one is taken next
        while work:
            C = work.pop()
            d = bcen[B] - cen[C]
            R = np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
            dist_ok = bool((brad[B] + rad[C]) < theta * R)
            size_ok = ncoef < tree.count(C)
            kind = classify(dist_ok, size_ok, tree.is_leaf(C))
            if kind == FAR:
                fl.append(C)
            elif kind == NEAR:
                nl.append(C)
            else:
                work.extend(reversed(tree.children[C]))
        far.append(fl)
        near.append(nl)
    return batches, far, near


def _pair_kernel(kernel, d, d2, kappa, alpha):
    """(K1, K2) per the subtracted forms; K2 is None for plain kernels."""
    if kernel == "yukawa_ss":
        g = np.exp(-kappa * d) / d
        return g, g
    if kernel == "coulomb_ss":
        return 1.0 / d, np.exp(-d2 / (alpha * alpha)) / d
    if kernel == "yukawa":
        return np.exp(-kappa * d) / d, None
    return 1.0 / d, None


def treecode(x, y, z, f, w, kernel: str, kappa, theta: float, degree: int, leaf_size: int,
             alpha: float = 1.0, domain=None, tree: Tree | None = None, return_parts=False,
             targets=None):
    """u (n_orb, N_t) in the caller's target order. f may be (N,) or (n_orb, N);
    kappa a scalar or per-orbital sequence (Yukawa only).

    targets: None (the targets are the sources: batches are the source tree's
    leaves), or (tx, ty, tz, tf) with tf of shape (N_t,) or (n_orb, N_t) (the
    values f_i of the subtracted kernels; may be None for the plain ones). The
    target batches are then the leaves of a tree built on the targets by the same
    rule (Section 6.1), with N_B = N_L and the root box the targets' bounding box.
    Pairs at distance exactly zero are skipped, so targets that coincide with
    sources are well defined."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    f = np.atleast_2d(np.asarray(f, np.float64))
    w = np.asarray(w, np.float64)
    n_orb, N = f.shape
    kap = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (n_orb,))
    ss = kernel in ("yukawa_ss", "coulomb_ss")
    if tree is None:
        tree = build_tree(x, y, z, leaf_size, domain)
    perm = tree.perm
    X, Y, Zs, W = x[perm], y[perm], z[perm], w[perm]
    F = f[:, perm]
    Q = F * W[None, :]
    if targets is None:
        btree = tree
        TX, TY, TZ, TF = X, Y, Zs, F
        n_t = N
    else:
        tx, ty, tz = (np.asarray(a, np.float64) for a in targets[:3])
        n_t = tx.size
        tf = targets[3]
        tf = (np.zeros((n_orb, n_t)) if tf is None
              else np.broadcast_to(np.atleast_2d(np.asarray(tf, np.float64)), (n_orb, n_t)))
        btree = build_tree(tx, ty, tz, leaf_size)
        tp = btree.perm
        TX, TY, TZ, TF = tx[tp], ty[tp], tz[tp], tf[:, tp]
    ncoef = (degree + 1) ** 3
    # proxy charges of every cluster that can ever be approximated
    nodes, fhat, what = {}, {}, {}
    for c in range(tree.n_nodes):
        if tree.count(c) > ncoef:
            b, e = tree.begin[c], tree.end[c]
            qs = np.vstack([Q[:, b:e], W[None, b:e]])
            nd, ch = proxy_charges(X[b:e], Y[b:e], Zs[b:e], qs, tree.lo[c], tree.hi[c], degree)
            nodes[c] = nd
            fhat[c] = ch[:n_orb].reshape(n_orb, -1)
            what[c] = ch[n_orb].reshape(-1)
    # batch-cluster interactions
    batches, far, near = interaction_lists(tree, theta, degree,
                                           batch_tree=None if targets is None else btree)
    U = np.zeros((n_orb, n_t))
    for B, fl, nl in zip(batches, far, near):
        b0, b1 = btree.begin[B], btree.end[B]
        tx_, ty_, tz_ = TX[b0:b1, None], TY[b0:b1, None], TZ[b0:b1, None]
        for o in range(n_orb):
            acc = np.zeros(b1 - b0)
            fi = TF[o, b0:b1]
            for C in fl:
                sx, sy, sz = nodes[C]
                gx, gy, gz = np.meshgrid(sx, sy, sz, indexing="ij")
                dx = tx_ - gx.reshape(1, -1)
                dy = ty_ - gy.reshape(1, -1)
                dz = tz_ - gz.reshape(1, -1)
                d2 = dx * dx + dy * dy + dz * dz
                d = np.sqrt(d2)
                k1, k2 = _pair_kernel(kernel, d, d2, kap[o], alpha)
                acc += k1 @ fhat[C][o]
                if ss:
                    acc -= fi * (k2 @ what[C])
            for C in nl:
                s0, s1 = tree.begin[C], tree.end[C]
                dx = tx_ - X[None, s0:s1]
                dy = ty_ - Y[None, s0:s1]
                dz = tz_ - Zs[None, s0:s1]
                d2 = dx * dx + dy * dy + dz * dz
                d = np.sqrt(d2)
                zero = d == 0.0
                dsafe = np.where(zero, 1.0, d)
                k1, k2 = _pair_kernel(kernel, dsafe, d2, kap[o], alpha)
                k1 = np.where(zero, 0.0, k1)
                acc += k1 @ Q[o, s0:s1]
                if ss:
                    k2 = np.where(zero, 0.0, k2)
                    acc -= fi * (k2 @ W[s0:s1])
            if kernel == "yukawa_ss":
                acc += 4.0 * np.pi * fi / (kap[o] * kap[o])
            elif kernel == "coulomb_ss":
                acc += 2.0 * np.pi * alpha * alpha * fi
            U[o, b0:b1] = acc
    out = np.empty_like(U)
    out[:, btree.perm] = U
    if return_parts:
        return out, dict(tree=tree, batch_tree=btree, batches=batches, far=far, near=near,
                         fhat=fhat, what=what, nodes=nodes)
    return out
