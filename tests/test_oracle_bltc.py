"""Pins of the treecode oracle: interpolation identities, polynomial reproduction
of the proxy charges, the tree rules, MAC validity and coverage, theta = 0
against the direct sum, and the error trends of Section 6.4."""
import numpy as np
import pytest

from oracle import bltc
from oracle.direct import direct_sum
from workloads.configs import uniform_cube
from workloads.rng import SplitMix64


@pytest.mark.parametrize("n", [1, 2, 5, 8, 12])
def test_barycentric_basis_matches_lagrange_products(n):
    # textbook Lagrange form prod_{m != k} (t - s_m)/(s_k - s_m) on the same nodes
    s = bltc.cheb2_nodes(-0.3, 1.7, n)
    b = bltc.barycentric_weights(n)
    t = SplitMix64(n).uniform(50, -0.3, 1.7)
    L = bltc.lagrange_basis(t, s, b)
    ref = np.ones((t.size, n + 1))
    for k in range(n + 1):
        for m in range(n + 1):
            if m != k:
                ref[:, k] *= (t - s[m]) / (s[k] - s[m])
    np.testing.assert_allclose(L, ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(L.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    # nodes hit exactly give the Kronecker basis, including the box faces
    np.testing.assert_array_equal(bltc.lagrange_basis(s, s, b), np.eye(n + 1))


def test_chebyshev_second_kind_nodes():
    s = bltc.cheb2_nodes(-1.0, 1.0, 6)
    np.testing.assert_allclose(s, np.cos(np.pi * np.arange(7) / 6), atol=1e-16)
    s = bltc.cheb2_nodes(2.0, 5.0, 4)
    assert s[0] == 5.0 and s[-1] == 2.0 and np.all(np.diff(s) < 0)


@pytest.mark.parametrize("n", [3, 6, 8])
def test_proxy_charges_reproduce_polynomial_moments(n):
    # interpolation of degree n is exact for monomials x^a y^b z^c, a, b, c <= n:
    # sum_k s^a s^b s^c q^_k = sum_j x_j^a y_j^b z_j^c q_j
    g = SplitMix64(100 + n)
    N = 400
    lo = np.array([0.5, -1.0, 2.0])
    hi = np.array([1.5, 0.25, 2.4])
    px = g.uniform(N, lo[0], hi[0])
    py = g.uniform(N, lo[1], hi[1])
    pz = g.uniform(N, lo[2], hi[2])
    q = g.uniform(N, -1, 1)
    lo_s = np.array([px.min(), py.min(), pz.min()])
    hi_s = np.array([px.max(), py.max(), pz.max()])
    nodes, fh = bltc.proxy_charges(px, py, pz, q, lo_s, hi_s, n)
    fh = fh[0]
    sx, sy, sz = nodes
    c = 0.5 * (lo_s + hi_s)
    for a, bb, cc in [(0, 0, 0), (1, 0, 0), (0, 1, 2), (n, 0, 1), (n, n, n), (2, n - 1, 1)]:
        lhs = np.einsum("abc,a,b,c->", fh, (sx - c[0]) ** a, (sy - c[1]) ** bb, (sz - c[2]) ** cc)
        rhs = np.sum((px - c[0]) ** a * (py - c[1]) ** bb * (pz - c[2]) ** cc * q)
        scale = np.sum(np.abs(q)) * np.max(np.abs(hi_s - lo_s)) ** (a + bb + cc)
        assert abs(lhs - rhs) <= 1e-12 * scale


def _tree_case(n=6000, leaf=200, seed=3, domain=None):
    x, y, z, f, w = uniform_cube(n, seed=seed)
    # make it non-uniform: squeeze half of the points toward a corner
    x = np.where(np.arange(n) % 2 == 0, x, -1.0 + 0.1 * (x + 1.0))
    return x, y, z, f, w, bltc.build_tree(x, y, z, leaf, domain)


def test_tree_rules():
    x, y, z, f, w, t = _tree_case()
    P = np.stack([x, y, z], axis=1)
    n = x.size
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    for c in range(t.n_nodes):
        b, e = t.begin[c], t.end[c]
        pts = P[t.perm[b:e]]
        assert np.array_equal(t.lo[c], pts.min(axis=0)) and np.array_equal(t.hi[c], pts.max(axis=0))
        ch = t.children[c]
        if not ch:
            assert e - b <= 200
            continue
        assert e - b > 200 and 2 <= len(ch) <= 8
        assert t.begin[ch[0]] == b and t.end[ch[-1]] == e
        for a_, b_ in zip(ch[:-1], ch[1:]):
            assert t.end[a_] == t.begin[b_]
        # children lie on one side of every split plane of the parent's box
        slo = t.lo[c] if c else P.min(axis=0)
        shi = t.hi[c] if c else P.max(axis=0)
        ext = shi - slo
        split = ext >= ext.max() * bltc.SQRT1_2
        mid = 0.5 * (slo + shi)
        for k in ch:
            kp = P[t.perm[t.begin[k]:t.end[k]]]
            for d in range(3):
                if split[d]:
                    side = kp[:, d] >= mid[d]
                    assert side.all() or (~side).all()
    # level numbering: parents before children, levels non-decreasing
    assert np.all(np.diff(t.level) >= 0)


def test_aspect_rule_splits_flat_boxes_in_two_or_four():
    g = SplitMix64(9)
    n = 3000
    x = g.uniform(n, 0, 4.0)
    y = g.uniform(n, 0, 1.0)
    z = g.uniform(n, 0, 1.0)
    t = bltc.build_tree(x, y, z, 500)
    assert len(t.children[0]) == 2  # only the long x side is bisected
    x = g.uniform(n, 0, 4.0)
    y = g.uniform(n, 0, 4.0)
    t = bltc.build_tree(x, y, z, 500)
    assert len(t.children[0]) == 4


def test_lists_cover_every_source_once_and_obey_the_mac():
    x, y, z, f, w, t = _tree_case(n=5000, leaf=150)
    theta, deg = 0.6, 4
    batches, far, near = bltc.interaction_lists(t, theta, deg)
    cen, rad = bltc.geometry(t)
    N = x.size
    for B, fl, nl in zip(batches, far, near):
        cover = np.zeros(N, dtype=np.int64)
        for C in fl:
            R = np.linalg.norm(cen[B] - cen[C])
            assert rad[B] + rad[C] < theta * R and (deg + 1) ** 3 < t.count(C)
            cover[t.begin[C]:t.end[C]] += 1
        for C in nl:
            R = np.linalg.norm(cen[B] - cen[C])
            ok = rad[B] + rad[C] < theta * R
            assert (not ok and not t.children[C]) or (ok and (deg + 1) ** 3 >= t.count(C))
            cover[t.begin[C]:t.end[C]] += 1
        assert np.all(cover == 1)


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss", "yukawa", "coulomb"])
def test_theta_zero_is_the_direct_sum(kernel):
    x, y, z, f, w = uniform_cube(2500, seed=21)
    u = bltc.treecode(x, y, z, f, w, kernel, 1.3, 0.0, 5, 300)[0]
    ref, ab = direct_sum(kernel, x, y, z, f, w, kappa=1.3, return_abs=True)
    assert np.max(np.abs(u - ref) / (ab + np.abs(ref))) < 1e-13


def test_error_falls_with_degree_and_meets_1e6_at_degree_8():
    x, y, z, f, w = uniform_cube(6000, seed=1)
    ref = direct_sum("yukawa_ss", x, y, z, f, w, kappa=1.0)
    errs = []
    for n in (2, 4, 6, 8):
        u = bltc.treecode(x, y, z, f, w, "yukawa_ss", 1.0, 0.7, n, 100)[0]
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    assert all(a > b for a, b in zip(errs[:-1], errs[1:])), errs
    assert errs[-1] < 1e-6


def test_error_rises_with_theta():
    x, y, z, f, w = uniform_cube(6000, seed=2)
    ref = direct_sum("coulomb_ss", x, y, z, f, w)
    errs = []
    for th in (0.4, 0.6, 0.8):
        u = bltc.treecode(x, y, z, f, w, "coulomb_ss", 0.0, th, 4, 100)[0]
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    assert errs[0] < errs[1] < errs[2], errs


def test_batched_orbitals_equal_separate_calls():
    x, y, z, f, w = uniform_cube(3000, seed=4)
    g = SplitMix64(44)
    F = np.stack([f, g.uniform(f.size, -1, 1), g.uniform(f.size, 0, 2)])
    kap = [0.7, 1.5, 3.0]
    U = bltc.treecode(x, y, z, F, w, "yukawa_ss", kap, 0.7, 5, 200)
    for o in range(3):
        u = bltc.treecode(x, y, z, F[o], w, "yukawa_ss", kap[o], 0.7, 5, 200)[0]
        np.testing.assert_allclose(U[o], u, rtol=0, atol=1e-14 * np.abs(u).max())


def _independent_geometry(t, x, y, z):
    """Centre and radius of every cluster computed from its points directly
    (midpoint and half-diagonal of their bounding box), not by the oracle."""
    P = np.stack([x, y, z], axis=1)
    cen = np.empty((t.n_nodes, 3))
    rad = np.empty(t.n_nodes)
    for c in range(t.n_nodes):
        q = P[t.perm[t.begin[c]:t.end[c]]]
        lo, hi = q.min(axis=0), q.max(axis=0)
        cen[c] = 0.5 * (lo + hi)
        rad[c] = 0.5 * np.sqrt(np.sum((hi - lo) ** 2))
    return cen, rad


@pytest.mark.parametrize("theta,deg", [(0.6, 4), (0.8, 2), (0.3, 1), (0.7, 6)])
def test_lists_are_maximal_every_opened_ancestor_failed_the_distance_test(theta, deg):
    # Algorithm 3 descends into a cluster only when the distance part of Eq. MAC
    # fails for it: every proper ancestor of a listed cluster must fail it, and a
    # listed non-leaf must have passed it (far, or near because it was too small)
    x, y, z, f, w, t = _tree_case(n=5000, leaf=120)
    cen, rad = _independent_geometry(t, x, y, z)
    K = (deg + 1) ** 3
    batches, far, near = bltc.interaction_lists(t, theta, deg)

    def dist_ok(B, C):
        return rad[B] + rad[C] < theta * np.linalg.norm(cen[B] - cen[C])

    n_far = n_small = 0
    for B, fl, nl in zip(batches, far, near):
        for kind, lst in (("far", fl), ("near", nl)):
            for C in lst:
                A = t.parent[C]
                while A >= 0:
                    assert not dist_ok(B, A), (B, C, A)
                    A = t.parent[A]
                if kind == "far":
                    assert dist_ok(B, C) and K < t.count(C)
                    n_far += 1
                elif t.children[C]:
                    assert dist_ok(B, C) and K >= t.count(C)
                    n_small += 1
                else:
                    assert not dist_ok(B, C) or K >= t.count(C)
    assert n_far > 0
    if deg == 6:  # (n+1)^3 = 343 exceeds N_L: some separated non-leaves are too small
        assert n_small > 0


def test_lists_visit_clusters_depth_first_in_child_order():
    # the far and near entries of a batch, merged in visiting order, follow the
    # tree's depth-first order (a recursive visit from the root, children in order)
    x, y, z, f, w, t = _tree_case(n=4000, leaf=100)
    order = []

    def dfs(c):
        order.append(c)
        for ch in t.children[c]:
            dfs(ch)

    dfs(0)
    rank = {c: i for i, c in enumerate(order)}
    batches, far, near = bltc.interaction_lists(t, 0.7, 3)
    for fl, nl in zip(far, near):
        for lst in (fl, nl):
            assert all(rank[a] < rank[b] for a, b in zip(lst[:-1], lst[1:]))
        # ranges of the listed clusters tile the sources in increasing order
        merged = sorted(fl + nl, key=rank.get)
        assert t.begin[merged[0]] == 0 and t.end[merged[-1]] == x.size
        for a, b in zip(merged[:-1], merged[1:]):
            assert t.end[a] == t.begin[b]


def _targets_case(n_t=700, seed=5):
    g = SplitMix64(seed)
    x, y, z, f, w = uniform_cube(3000, seed=31)
    tx, ty, tz = g.uniform(n_t, -1.2, 1.2), g.uniform(n_t, -1.2, 1.2), g.uniform(n_t, -1.2, 1.2)
    tf = g.uniform(n_t, -1, 1)
    tx[:40], ty[:40], tz[:40] = x[:40], y[:40], z[:40]  # targets on sources
    # a cluster of targets far outside the source box: the whole source tree,
    # root included, is well separated from their batches
    tx[-150:] = 9.0 + 0.3 * g.uniform(150, 0, 1)
    ty[-150:] = -7.0 + 0.3 * g.uniform(150, 0, 1)
    tz[-150:] = 5.0 + 0.3 * g.uniform(150, 0, 1)
    return x, y, z, f, w, tx, ty, tz, tf


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss", "yukawa", "coulomb"])
def test_separate_targets_theta_zero_is_the_direct_sum(kernel):
    x, y, z, f, w, tx, ty, tz, tf = _targets_case()
    u = bltc.treecode(x, y, z, f, w, kernel, 1.1, 0.0, 4, 150, targets=(tx, ty, tz, tf))[0]
    ref, ab = direct_sum(kernel, x, y, z, f, w, tx, ty, tz, tf, kappa=1.1, return_abs=True)
    assert np.max(np.abs(u - ref) / (ab + np.abs(ref))) < 1e-13


def test_separate_targets_equal_to_the_sources_reproduce_the_self_case():
    # a tree built on the sources' own coordinates is the source tree, so its
    # batches, lists and sums are the same, bit for bit
    x, y, z, f, w = uniform_cube(2500, seed=17)
    u0 = bltc.treecode(x, y, z, f, w, "yukawa_ss", 0.9, 0.7, 5, 200)
    u1 = bltc.treecode(x, y, z, f, w, "yukawa_ss", 0.9, 0.7, 5, 200, targets=(x, y, z, f))
    assert np.array_equal(u0, u1)


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
def test_separate_targets_meet_the_treecode_accuracy(kernel):
    x, y, z, f, w, tx, ty, tz, tf = _targets_case()
    u, parts = bltc.treecode(x, y, z, f, w, kernel, 1.1, 0.7, 7, 150, targets=(tx, ty, tz, tf),
                             return_parts=True)
    ref = direct_sum(kernel, x, y, z, f, w, tx, ty, tz, tf, kappa=1.1)
    err = np.linalg.norm(u[0] - ref) / np.linalg.norm(ref)
    assert err < 1e-6, err
    # the far-away targets take the whole source tree through the root's charges
    bt = parts["batch_tree"]
    far_targets = [fl for B, fl in zip(parts["batches"], parts["far"]) if bt.lo[B][0] > 8.0]
    assert far_targets and all(fl == [0] for fl in far_targets)
    # every batch covers every source exactly once
    t = parts["tree"]
    for fl, nl in zip(parts["far"], parts["near"]):
        cover = np.zeros(x.size, dtype=np.int64)
        for C in fl + nl:
            cover[t.begin[C]:t.end[C]] += 1
        assert np.all(cover == 1)
