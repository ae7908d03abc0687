"""ORACLE (test infrastructure only): the learned degree/MAC selection of the
interaction lists, and the treecode sum over such lists, in plain numpy FP64.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this.

The selection is a project addition on Algorithm 3 (Section 6.3). Every target
batch B visits the source tree depth first from the root, children in order. A
cluster C that fails the permissive distance test (r_B + r_C) < theta_max R is
resolved into its children (a leaf is summed directly), as Algorithm 3 does. A
cluster that passes it and holds at most (4+1)^3 sources is summed directly (no
degree has fewer charges than sources). Otherwise, per orbital o, the network
(oracle/mlp.py) sees the log-features

    (r_C, d = R - r_B, c_o, N_S, l1_o),
    standardised as (ln(raw + offset) - shift) * scale,

with the decay rate c_o = kappa_o for the Yukawa kernels and 0 for the Coulomb
kernels (the kappa -> 0 limit of exp(-kappa r)/r is 1/r), offset 0.25 on c and 0
on the others (so that c = 0 maps to a finite value), and
l1_o = |q^_o|_1 + g max_B |f_o| |w^|_1 from C's degree-4 proxy charges of f w and
of w (Section 6.2): the size of the charges the pair's far field carries. The
subtracted charges -f_i w^ enter with the ratio g of their kernel to the first
one's: g = 1 for the subtracted Yukawa kernel (both terms carry
exp(-kappa r)/r); for the subtracted Coulomb kernel the Gaussian
exp(-r^2/a^2) at the least distance dm = max(R - r_B - r_C, 0) that a target of
B and a proxy point of C can have, a bound over the pair; g = 0 for the plain
kernels (no subtraction). It predicts, for degrees 4..12, log10 of the pair's largest error
minus the pair scale s_o = log10(l1_o) - c_o d log10(e) - log10(d) (log10 of the
size of the pair's far field). The
pair is approximated at the lowest degree n with (n+1)^3 < N_S whose predicted
error meets the batch's budget for every orbital (the largest such degree over
the orbitals is used), and resolved into its children otherwise (a leaf is
summed directly). If any orbital's log-feature lies outside the training range
[lo, hi], the pair takes the fixed MAC (theta_fb, degree_fb) of Algorithm 3.

Budget of a batch: a batch's error is a sum over its far pairs, so the per-pair
budget shrinks with their number. With tol_o the caller's absolute budget for
orbital o and M_B the number of far pairs of B in the fixed-MAC lists at
(theta_max, degree 4), the pair budget is tol_o / max(M_B, 1): the error of a
target's far field is at most the sum of its pairs' errors (triangle
inequality), whatever their signs.

The GPU evaluates the network in FP32, so a decision whose margin (distance of a
compared log quantity from its threshold) is below `tie` may legitimately come
out the other way there. `learned_lists` reports such decisions; it never takes
another implementation's decision.
"""
from __future__ import annotations

import numpy as np

from oracle import bltc
from oracle.mlp import forward

DEG_MIN, DEG_MAX = 4, 12
LOG10E = np.log10(np.e)
YUKAWA_KERNELS = ("yukawa_ss", "yukawa")
# added to the raw features before the logarithm: only the decay rate, which is
# 0 for the Coulomb kernels
LOG_OFFSET = np.array([0.0, 0.0, 0.25, 0.0, 0.0])


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


def decay(kernel, kappa_o):
    """The network's third raw input: the kernel's decay rate, kappa for the
    Yukawa kernels, 0 for the Coulomb kernels."""
    return kappa_o if kernel in YUKAWA_KERNELS else 0.0


def subtracted_weight(kernel, R, rB, rC, alpha):
    """g: the weight of the subtracted charges in the l1 feature (see above)."""
    if kernel == "yukawa_ss":
        return 1.0
    if kernel == "coulomb_ss":
        dm = max(R - rB - rC, 0.0)
        return float(np.exp(-dm * dm / (alpha * alpha)))
    return 0.0


def pair_scale(l1, d, c):
    """log10 of the size of a pair's far field, l1 exp(-c d) / d, c the decay rate."""
    return np.log10(l1) - LOG10E * c * d - np.log10(d)


def lowest_degree(pred, scale, log_tol, cnt):
    """Lowest degree n in 4..12 with (n+1)^3 < cnt and pred[n-4] + scale <= log_tol,
    or -1; and the smallest distance of a compared value from the threshold."""
    margin = np.inf
    for deg in range(DEG_MIN, DEG_MAX + 1):
        if (deg + 1) ** 3 >= cnt:
            break
        v = pred[deg - DEG_MIN] + scale - log_tol
        margin = min(margin, abs(v))
        if v <= 0:
            return deg, margin
    return -1, margin


def candidate_counts(tree, theta_max):
    """M_B per batch: far pairs of the fixed-MAC lists at (theta_max, degree 4)."""
    _, far, _ = bltc.interaction_lists(tree, theta_max, DEG_MIN)
    return np.array([len(fl) for fl in far], dtype=np.int64)


def learned_lists(tree, x, y, z, F, W, kernel, kappa, params, norm, log_tol, theta_max,
                  theta_fb, degree_fb, alpha=1.0, tie=2e-4):
    """Per batch (leaf order): far [(C, degree)] and near [C] in visiting order,
    and the decisions within `tie` of a threshold as (batch index, C, margin).
    x, y, z, F (n_orb, N), W are in the tree's order; log_tol (n_orb,) is log10 of
    the caller's absolute budget per orbital. Returns (far, near, ties)."""
    P = split_params(params)
    nrm = np.asarray(norm, np.float64)
    shift, scale, lo, hi = nrm[0:5], nrm[5:10], nrm[10:15], nrm[15:20]
    n_orb = F.shape[0]
    kappa = np.broadcast_to(np.asarray(kappa, np.float64), (n_orb,))
    log_tol = np.asarray(log_tol, np.float64)
    cen, rad = bltc.geometry(tree)
    m_b = candidate_counts(tree, theta_max)
    l1_cache = {}
    far_all, near_all, ties = [], [], []
    for bi, B in enumerate(tree.leaves()):
        fmax = np.abs(F[:, tree.begin[B]:tree.end[B]]).max(axis=1)
        budget = log_tol - np.log10(max(int(m_b[bi]), 1))
        far, near = [], []

        def decide(C, cnt, R, rC):
            d = max(R - rad[B], 1e-12)
            if C not in l1_cache:
                l1_cache[C] = cluster_l1(tree, x, y, z, F, W, C)
            l1s = l1_cache[C]
            fallback, margin, degs = False, np.inf, []
            g = subtracted_weight(kernel, R, rad[B], rC, alpha)
            for o in range(n_orb):
                l1 = max(l1s[o] + g * fmax[o] * l1s[n_orb], 1e-30)
                c = decay(kernel, kappa[o])
                raw = np.log(np.array([rC, d, c, cnt, l1]) + LOG_OFFSET)
                margin = min(margin, np.min(np.abs(raw - lo)), np.min(np.abs(raw - hi)))
                if np.any(raw < lo) or np.any(raw > hi):
                    fallback = True
                    continue
                pred = forward(P, ((raw - shift) * scale)[None])[0][0]
                d_o, m_o = lowest_degree(pred, pair_scale(l1, d, c), budget[o], cnt)
                margin = min(margin, m_o)
                degs.append(d_o)
            if fallback:
                dist = (rad[B] + rC) < theta_fb * R
                return bltc.classify(dist, (degree_fb + 1) ** 3 < cnt, False), degree_fb, margin
            if min(degs) >= 0:
                return bltc.FAR, max(degs), margin
            return bltc.OPEN, 0, margin

        work = [0]
        while work:
            C = work.pop()
            dv = cen[B] - cen[C]
            R = np.sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2])
            rC = rad[C]
            cnt = tree.count(C)
            deg = 0
            if not ((rad[B] + rC) < theta_max * R):
                kind = bltc.OPEN
            elif cnt <= (DEG_MIN + 1) ** 3:
                kind = bltc.NEAR
            else:
                kind, deg, margin = decide(C, cnt, R, rC)
                if margin < tie:
                    ties.append((bi, C, margin))
            if kind == bltc.OPEN and tree.is_leaf(C):
                kind = bltc.NEAR
            if kind == bltc.FAR:
                far.append((C, deg))
            elif kind == bltc.NEAR:
                near.append(C)
            else:
                work.extend(reversed(tree.children[C]))
        far_all.append(far)
        near_all.append(near)
    return far_all, near_all, ties


def lists_treecode(tree, x, y, z, F, W, kernel, kappa, far, near, alpha=1.0):
    """The treecode sum over given lists (per batch, far [(C, degree)] and near [C]),
    with proxy charges of each far cluster at its own degree (Eq.
    particle-cluster-approx-rearranged) and the subtracted pair sums and analytic
    term of Section 4.3, as in oracle/bltc.py. x, y, z, F (n_orb, N), W are in
    the tree's order; returns U (n_orb, N) in the tree's order."""
    n_orb, N = F.shape
    kap = np.broadcast_to(np.asarray(kappa, np.float64), (n_orb,))
    ss = kernel in ("yukawa_ss", "coulomb_ss")
    Q = F * W[None, :]
    charges = {}
    U = np.zeros((n_orb, N))
    for B, fl, nl in zip(tree.leaves(), far, near):
        b0, b1 = tree.begin[B], tree.end[B]
        tx, ty, tz = x[b0:b1, None], y[b0:b1, None], z[b0:b1, None]
        for o in range(n_orb):
            acc = np.zeros(b1 - b0)
            fi = F[o, b0:b1]
            for C, deg in fl:
                if (C, deg) not in charges:
                    s0, s1 = tree.begin[C], tree.end[C]
                    charges[(C, deg)] = bltc.proxy_charges(
                        x[s0:s1], y[s0:s1], z[s0:s1], np.vstack([Q[:, s0:s1], W[None, s0:s1]]),
                        tree.lo[C], tree.hi[C], deg)
                (sx, sy, sz), ch = charges[(C, deg)]
                gx, gy, gz = np.meshgrid(sx, sy, sz, indexing="ij")
                dx = tx - gx.reshape(1, -1)
                dy = ty - gy.reshape(1, -1)
                dz = tz - gz.reshape(1, -1)
                d2 = dx * dx + dy * dy + dz * dz
                k1, k2 = bltc._pair_kernel(kernel, np.sqrt(d2), d2, kap[o], alpha)
                acc += k1 @ ch[o].reshape(-1)
                if ss:
                    acc -= fi * (k2 @ ch[n_orb].reshape(-1))
            for C in nl:
                s0, s1 = tree.begin[C], tree.end[C]
                dx = tx - x[None, s0:s1]
                dy = ty - y[None, s0:s1]
                dz = tz - z[None, s0:s1]
                d2 = dx * dx + dy * dy + dz * dz
                d = np.sqrt(d2)
                zero = d == 0.0
                k1, k2 = bltc._pair_kernel(kernel, np.where(zero, 1.0, d), d2, kap[o], alpha)
                acc += np.where(zero, 0.0, k1) @ Q[o, s0:s1]
                if ss:
                    acc -= fi * (np.where(zero, 0.0, k2) @ W[s0:s1])
            if kernel == "yukawa_ss":
                acc += 4.0 * np.pi * fi / (kap[o] * kap[o])
            elif kernel == "coulomb_ss":
                acc += 2.0 * np.pi * alpha * alpha * fi
            U[o, b0:b1] = acc
    return U
