"""Pins of the learned-list oracle (oracle/learned.py) on the CPU.

Networks with all weights zero output their last-layer biases whatever the
input, so a decision can be worked out by hand: the chosen degree is the lowest
n with (n+1)^3 < N_S and b[n-4] + s <= budget, with the pair scale s and the
batch budget computed here from the geometry and charges directly. Three such
networks reduce the learned traversal to known lists: one that predicts tiny
errors everywhere accepts every candidate at degree 4 (the fixed MAC at
(theta_max, 4)); one that predicts huge errors opens everything (the direct sum);
and features outside the training range give the fallback MAC."""
import numpy as np
import pytest

from oracle import bltc, learned
from oracle.direct import direct_sum
from workloads.configs import uniform_cube
from workloads.rng import SplitMix64

N_PARAM = (5 * 64 + 64) + 2 * (64 * 64 + 64) + (64 * 9 + 9)
OPEN_RANGE = np.concatenate([np.zeros(5), np.ones(5), np.full(5, -1e30), np.full(5, 1e30)])


def bias_network(b):
    """Zero weights, zero hidden biases, output biases b (9,)."""
    p = np.zeros(N_PARAM)
    p[-9:] = b
    return p


def _case(n=3000, leaf=150, seed=7):
    x, y, z, f, w = uniform_cube(n, seed=seed)
    g = SplitMix64(seed + 100)
    F = np.stack([f, g.uniform(n, 0.0, 2.0)])
    t = bltc.build_tree(x, y, z, leaf)
    p = t.perm
    return t, x[p], y[p], z[p], F[:, p], w[p], (x, y, z, F, w)


def _run(t, X, Y, Z, F, W, params, norm, kernel="yukawa_ss", kappa=(0.8, 2.0), log_tol=(-6, -6),
         theta_max=0.8, theta_fb=0.6, degree_fb=8):
    return learned.learned_lists(t, X, Y, Z, F, W, kernel, np.array(kappa), params, norm,
                                 np.array(log_tol, float), theta_max, theta_fb, degree_fb)


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
def test_network_accepting_everything_gives_the_fixed_mac_at_degree_4(kernel):
    t, X, Y, Z, F, W, orig = _case()
    far, near, ties = _run(t, X, Y, Z, F, W, bias_network(np.full(9, -100.0)), OPEN_RANGE,
                           kernel=kernel)
    _, far_ref, near_ref = bltc.interaction_lists(t, 0.8, 4)
    assert far == [[(C, 4) for C in fl] for fl in far_ref]
    assert near == near_ref and not ties
    assert sum(map(len, far)) > 0
    # the sum over these lists is the fixed-MAC treecode at (0.8, 4)
    U = learned.lists_treecode(t, X, Y, Z, F, W, kernel, [0.8, 2.0], far, near)
    ref = bltc.treecode(*orig, kernel, [0.8, 2.0], 0.8, 4, 150, tree=t)[:, t.perm]
    np.testing.assert_allclose(U, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_network_rejecting_everything_gives_the_direct_sum():
    t, X, Y, Z, F, W, orig = _case()
    far, near, ties = _run(t, X, Y, Z, F, W, bias_network(np.full(9, 100.0)), OPEN_RANGE)
    assert all(not fl for fl in far) and not ties
    U = learned.lists_treecode(t, X, Y, Z, F, W, "yukawa_ss", [0.8, 2.0], far, near)
    x, y, z, Fo, w = orig
    for o, kap in enumerate((0.8, 2.0)):
        ref, ab = direct_sum("yukawa_ss", x, y, z, Fo[o], w, kappa=kap, return_abs=True)
        u = np.empty_like(ref)
        u[t.perm] = U[o]
        assert np.max(np.abs(u - ref) / (ab + np.abs(ref))) < 1e-13


def test_features_out_of_range_give_the_fallback_mac():
    t, X, Y, Z, F, W, orig = _case()
    norm = OPEN_RANGE.copy()
    norm[10:15] = 1e30  # every log-feature below its range
    far, near, ties = _run(t, X, Y, Z, F, W, bias_network(np.full(9, -100.0)), norm,
                           theta_max=0.8, theta_fb=0.6, degree_fb=5)
    _, far_ref, near_ref = bltc.interaction_lists(t, 0.6, 5)
    assert far == [[(C, 5) for C in fl] for fl in far_ref]
    assert near == near_ref
    U = learned.lists_treecode(t, X, Y, Z, F, W, "coulomb_ss", [1.0, 1.0], far, near)
    ref = bltc.treecode(*orig, "coulomb_ss", 1.0, 0.6, 5, 150, tree=t)[:, t.perm]
    np.testing.assert_allclose(U, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def _cheb_grid_cluster(centre, copies=2):
    """(4+1)^3 points on the degree-4 Chebyshev grid of [c-1, c+1]^3, each taken
    `copies` times: every point sits on a proxy node, so the degree-4 proxy
    charges are the sums of the charges at each node."""
    s = np.cos(np.pi * np.arange(5) / 4)
    g = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)
    g = np.repeat(g, copies, axis=0)
    return g + np.asarray(centre, float)[None, :]


def _four_cluster_case():
    # four grid clusters of 250 points (N_L = 250: each is a leaf) at y, z in
    # {0, 4}, and a batch of 10 points near x = 30
    g = SplitMix64(5)
    pts = [_cheb_grid_cluster((0.0, cy, cz)) for cy in (0.0, 4.0) for cz in (0.0, 4.0)]
    bat = np.stack([30.0 + 0.3 * g.uniform(10), 2.0 + 0.3 * g.uniform(10),
                    2.0 + 0.3 * g.uniform(10)], axis=1)
    P = np.concatenate(pts + [bat])
    n = P.shape[0]
    f = np.concatenate([g.uniform(1000, 0.1, 1.0), g.uniform(10, -3.0, 3.0)])
    w = g.uniform(n, 0.5, 1.5)
    return P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), f, w


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
@pytest.mark.parametrize("shift", [-0.5, -0.2, -0.05, 0.05, 0.2, 0.5, 1.05])
def test_hand_computed_decisions_with_the_batch_budget(shift, kernel):
    x, y, z, f, w = _four_cluster_case()
    t = bltc.build_tree(x, y, z, 250)
    # root -> (grid clusters' parent, batch); parent -> the four grid clusters
    assert len(t.children[0]) == 2 and len(t.children[t.children[0][0]]) == 4
    p = t.perm
    X, Y, Z, F, W = x[p], y[p], z[p], f[p][None, :], w[p]
    B = t.children[0][1]
    grids = t.children[t.children[0][0]]
    kappa, theta_max = 0.7, 0.15
    # decay rate of the pair scale: kappa for Yukawa, 0 for Coulomb (1/r)
    c = kappa if kernel == "yukawa_ss" else 0.0
    b = np.array([-5.0, -6.0, -7.0, -8.0, -9.0, -10.0, -11.0, -12.0, -13.0])
    # by hand: batch geometry, and per grid cluster the features of the decision
    Pb = np.stack([x, y, z], axis=1)[p[t.begin[B]:t.end[B]]]
    cb = 0.5 * (Pb.min(axis=0) + Pb.max(axis=0))
    rb = 0.5 * np.linalg.norm(Pb.max(axis=0) - Pb.min(axis=0))
    fmax = np.abs(F[0, t.begin[B]:t.end[B]]).max()
    # the grid clusters' parent fails theta_max, each grid cluster passes it:
    # M_B = 4 candidate pairs, so the pair budget is tol / 2
    budget = None
    expected = []
    for C in grids:
        s0, s1 = t.begin[C], t.end[C]
        Pc = np.stack([X[s0:s1], Y[s0:s1], Z[s0:s1]], axis=1)
        cc = 0.5 * (Pc.min(axis=0) + Pc.max(axis=0))
        rc = 0.5 * np.linalg.norm(Pc.max(axis=0) - Pc.min(axis=0))
        R = np.linalg.norm(cb - cc)
        assert rb + rc < theta_max * R and rc == pytest.approx(np.sqrt(3.0), abs=1e-15)
        d = R - rb
        # points on the proxy nodes and positive f, w: l1 = sum q + g max|f| sum w,
        # g = 1 for Yukawa-SS and the Gaussian at the least distance for Coulomb-SS
        g = 1.0 if kernel == "yukawa_ss" else np.exp(-max(R - rb - rc, 0.0) ** 2)
        l1 = np.sum(F[0, s0:s1] * W[s0:s1]) + g * fmax * np.sum(W[s0:s1])
        s = np.log10(l1) - c * d / np.log(10.0) - np.log10(d)
        if budget is None:
            # straddle the first cluster's degree-5 threshold (shift 0) and degree-4
            # threshold (shift 1) after the budget's 1/M_B factor
            budget = b[1] + s + np.log10(4.0) + shift
        pair_budget = budget - np.log10(4.0)
        # degrees with (n+1)^3 < 250: 4 and 5
        deg = 4 if b[0] + s <= pair_budget else (5 if b[1] + s <= pair_budget else None)
        expected.append((C, deg))
    far, near, ties = learned.learned_lists(t, X, Y, Z, F, W, kernel, [kappa],
                                            bias_network(b), OPEN_RANGE, [budget], theta_max,
                                            0.1, 8)
    bi = t.leaves().index(B)
    assert far[bi] == [(C, d) for C, d in expected if d is not None]
    assert near[bi] == [C for C, d in expected if d is None] + [B]
    assert expected[0][1] == (None if shift < 0 else (5 if shift < 1 else 4))


def test_subtracted_weight_of_the_l1_feature():
    # the subtracted charges -f_i w^ carry the Gaussian for Coulomb-SS: bounded by
    # its value at the least distance a target and a proxy point can have
    assert learned.subtracted_weight("yukawa_ss", 5.0, 1.0, 1.0, 1.0) == 1.0
    assert learned.subtracted_weight("yukawa", 5.0, 1.0, 1.0, 1.0) == 0.0
    assert learned.subtracted_weight("coulomb", 5.0, 1.0, 1.0, 1.0) == 0.0
    assert learned.subtracted_weight("coulomb_ss", 5.0, 1.0, 1.0, 1.0) == pytest.approx(np.exp(-9.0))
    assert learned.subtracted_weight("coulomb_ss", 5.0, 1.0, 1.0, 2.0) == pytest.approx(np.exp(-9.0 / 4))
    # overlapping spheres: the bound is 1
    assert learned.subtracted_weight("coulomb_ss", 1.5, 1.0, 1.0, 1.0) == 1.0


def test_decay_feature_is_finite_for_coulomb_and_continuous_in_kappa():
    # the third log-feature ln(c + 0.25): Coulomb (c = 0) is the kappa -> 0 end
    # of the Yukawa values
    assert learned.decay("coulomb_ss", 3.0) == 0.0 and learned.decay("coulomb", 3.0) == 0.0
    assert learned.decay("yukawa_ss", 3.0) == 3.0
    f0 = np.log(learned.decay("coulomb_ss", 1.0) + learned.LOG_OFFSET[2])
    f1 = np.log(learned.decay("yukawa_ss", 1e-9) + learned.LOG_OFFSET[2])
    assert np.isfinite(f0) and abs(f0 - f1) < 1e-8
    assert np.all(learned.LOG_OFFSET[[0, 1, 3, 4]] == 0.0)


def test_candidate_counts_are_the_fixed_mac_far_counts():
    t, *_ = _case()
    _, far, _ = bltc.interaction_lists(t, 0.7, 4)
    assert list(learned.candidate_counts(t, 0.7)) == [len(fl) for fl in far]


def test_cluster_l1_on_grid_points_is_the_sum_of_charges():
    # sources on the proxy nodes: the charges are the per-node sums (Kronecker
    # basis), so for positive charges their l1 norm is the plain sum
    x, y, z, f, w = _four_cluster_case()
    t = bltc.build_tree(x, y, z, 250)
    p = t.perm
    F = np.abs(f[p])[None, :]
    for C in t.children[t.children[0][0]]:
        s0, s1 = t.begin[C], t.end[C]
        l1 = learned.cluster_l1(t, x[p], y[p], z[p], F, w[p], C)
        np.testing.assert_allclose(l1, [np.sum(F[0, s0:s1] * w[p][s0:s1]), np.sum(w[p][s0:s1])],
                                   rtol=1e-14)
