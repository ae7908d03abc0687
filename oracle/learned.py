"""ORACLE (test infrastructure only): the learned degree/MAC selection of the
interaction lists, in plain numpy FP64.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this.

The selection is a project addition on Algorithm 3 (Section 6.3): the
ComputePotential traversal of every target batch from the root, where a pair
that passes the permissive test (r_B + r_C) < theta_max R and holds more than
(4+1)^3 sources is approximated at the lowest degree n in 4..12 with
(n+1)^3 < N_S whose predicted error meets every orbital's budget, else opened
(a leaf, or a pair failing theta_max at a leaf, is summed directly; a pair with
at most 125 sources is summed directly). Per orbital, the network (oracle/mlp.py)
sees the log-features (r_C, R - r_B, kappa, N_S, l1), standardised, with
l1 = |q^|_1 + max_B |f| |w^|_1 from the cluster's degree-4 proxy charges of f w
and of w (Section 6.2), and predicts log10 error minus the pair scale
log10(l1) - kappa (R - r_B) log10(e) - log10(R - r_B). If any orbital's raw
log-feature lies outside the training range [lo, hi], the pair takes the fixed
MAC (theta_fb, degree_fb) of Algorithm 3 instead.

The GPU evaluates the network in FP32; decisions whose margin (distance of a
compared quantity from its threshold, in log units) is below `tie` can
legitimately differ, and `learned_lists` reports them as ties.
"""
from __future__ import annotations

import numpy as np

from oracle import bltc
from oracle.mlp import forward

DEG_MIN, DEG_MAX = 4, 12
LOG10E = np.log10(np.e)


def split_params(flat, sizes=(5, 64, 64, 64, 9)):
    out, off = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append(np.asarray(flat[off:off + a * b], np.float64).reshape(b, a))
        off += a * b
        out.append(np.asarray(flat[off:off + b], np.float64))
        off += b
    return out


def cluster_l1(tree, x, y, z, F, W, C, degree=DEG_MIN):
    """|q^_o|_1 per orbital and |w^|_1 of cluster C's degree-4 proxy charges (the
    sources in tree order are x[perm] ...)."""
    b, e = tree.begin[C], tree.end[C]
    Q = np.vstack([F[:, b:e] * W[None, b:e], W[None, b:e]])
    _, ch = bltc.proxy_charges(x[b:e], y[b:e], z[b:e], Q, tree.lo[C], tree.hi[C], degree)
    return np.array([np.abs(c).sum() for c in ch])


def learned_lists(tree, x, y, z, F, W, kappa, params, norm, log_tol, theta_max, theta_fb,
                  degree_fb, reference=None, tie=2e-4):
    """Per batch (leaf order): far [(C, degree)] and near [C] in traversal order.
    x, y, z, F (n_orb, N), W are in the tree's order. `reference` (optional):
    per batch a dict C -> ("far", degree) or ("near",) of another implementation;
    where it differs from this one at a tie the traversal follows the reference.
    Returns (far, near, ties, mismatches)."""
    P = split_params(params)
    nrm = np.asarray(norm, np.float64)
    shift, scale, lo, hi = nrm[0:5], nrm[5:10], nrm[10:15], nrm[15:20]
    kappa = np.asarray(kappa, np.float64)
    n_orb = F.shape[0]
    cen, rad = bltc.geometry(tree)
    l1_cache = {}
    far_all, near_all, ties, mism = [], [], [], []
    for bi, B in enumerate(tree.leaves()):
        fmax = np.abs(F[:, tree.begin[B]:tree.end[B]]).max(axis=1)
        ref = reference[bi] if reference is not None else None
        far, near = [], []

        def decide(C, cnt, R, rC):
            d = max(R - rad[B], 1e-12)
            if C not in l1_cache:
                l1_cache[C] = cluster_l1(tree, x, y, z, F, W, C)
            l1s = l1_cache[C]
            fallback, margin, degs = False, np.inf, []
            for o in range(n_orb):
                l1 = max(l1s[o] + fmax[o] * l1s[n_orb], 1e-30)
                raw = np.log(np.array([rC, d, kappa[o], cnt, l1]))
                margin = min(margin, np.min(np.abs(raw - lo)), np.min(np.abs(raw - hi)))
                if np.any(raw < lo) or np.any(raw > hi):
                    fallback = True
                    continue
                pred = forward(P, ((raw - shift) * scale)[None])[0][0]
                scl = np.log10(l1) - LOG10E * kappa[o] * d - np.log10(d)
                d_o = -1
                for deg in range(DEG_MIN, DEG_MAX + 1):
                    if (deg + 1) ** 3 >= cnt:
                        break
                    v = pred[deg - DEG_MIN] + scl - log_tol[o]
                    margin = min(margin, abs(v))
                    if v <= 0:
                        d_o = deg
                        break
                degs.append(d_o)
            if fallback:
                nf = degree_fb + 1
                dist = (rad[B] + rC) < theta_fb * R
                if dist and nf ** 3 < cnt:
                    return ("far", degree_fb), margin
                return (("open",) if not dist else ("near",)), margin
            if min(degs) >= 0:
                return ("far", max(degs)), margin
            return ("open",), margin

        def visit(C):
            dv = cen[B] - cen[C]
            R = np.sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2])
            rC = rad[C]
            cnt = tree.count(C)
            leaf = tree.is_leaf(C)
            if not ((rad[B] + rC) < theta_max * R):
                dec = ("near",) if leaf else ("open",)
            elif cnt <= (DEG_MIN + 1) ** 3:
                dec = ("near",)
            else:
                dec, margin = decide(C, cnt, R, rC)
                if dec == ("open",) and leaf:
                    dec = ("near",)
                if ref is not None:
                    other = ref.get(C, ("open",))
                    if other != dec:
                        (ties if margin < tie else mism).append((bi, C, dec, other, margin))
                        if margin < tie:
                            dec = other
            if dec[0] == "far":
                far.append((C, dec[1]))
            elif dec[0] == "near":
                near.append(C)
            else:
                for ch in tree.children[C]:
                    visit(ch)

        visit(0)
        far_all.append(far)
        near_all.append(near)
    return far_all, near_all, ties, mism
