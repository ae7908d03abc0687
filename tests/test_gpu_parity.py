"""GPU path vs the CPU oracle, element by element, through the C ABI.

Tolerances. FP64 sums of m terms carry a rounding error of at most about
m * 2^-53 * sum|term| and typically sqrt(m) times less; the device exp and
rsqrt are within a few ulp. The GPU forms a1 - f_i a2 for the subtracted
kernels where the oracle sums (f_j - f_i) G w_j, so both are compared against
the scale S_i = sum_j G |f_j| w_j + |f_i| sum_j G w_j + |s f_i| (what the
terms can cancel down from): |u_gpu - u_ref| <= 1e-12 S_i for sums over up to
~4e4 sources. Integer stages (tree, lists) must agree exactly.
"""
import numpy as np
import pytest
import torch

from oracle import bltc
from oracle.direct import direct_sum
from workloads.configs import atom_mesh, uniform_cube
from workloads.rng import SplitMix64

pytestmark = pytest.mark.gpu

KAPPA = 1.3


def _tag():
    import paper_2003_01833_amd as tagi
    return tagi


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def _scale(kernel, x, y, z, f, w, kappa, alpha=1.0, idx=None):
    """S_i: sum_j |K1| |f_j| w_j + |f_i| sum_j |K2| w_j + |s f_i| by the oracle's
    plain kernels (all terms non-negative)."""
    tx = ty = tz = tf = None
    if idx is not None:
        tx, ty, tz, tf = x[idx], y[idx], z[idx], f[idx]
    fi = np.abs(f if idx is None else f[idx])
    if kernel.startswith("yukawa"):
        a = direct_sum("yukawa", x, y, z, np.abs(f), w, tx, ty, tz, tf, kappa=kappa)
        s = a
        if kernel == "yukawa_ss":
            s = s + fi * direct_sum("yukawa", x, y, z, np.ones_like(f), w, tx, ty, tz, tf, kappa=kappa)
            s = s + 4 * np.pi / kappa ** 2 * fi
        return s
    a = direct_sum("coulomb", x, y, z, np.abs(f), w, tx, ty, tz, tf)
    if kernel == "coulomb_ss":
        a = a + fi * direct_sum("coulomb", x, y, z, np.ones_like(f), w, tx, ty, tz, tf) + 2 * np.pi * alpha ** 2 * fi
    return a


def _ragged_case(n=7777, seed=12):
    x, y, z, f, w = uniform_cube(n, seed=seed)
    # half the points squeezed toward a corner: uneven leaves and deep branches
    x = np.where(np.arange(n) % 3 == 0, -1.0 + 0.05 * (x + 1.0), x)
    y = np.where(np.arange(n) % 3 == 0, -1.0 + 0.05 * (y + 1.0), y)
    return x, y, z, f, w


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss", "yukawa", "coulomb"])
def test_direct_matches_oracle(kernel):
    tagi = _tag()
    x, y, z, f, w = _ragged_case(5003)
    ref = direct_sum(kernel, x, y, z, f, w, kappa=KAPPA)
    dx, dy, dz, df, dw = _dev(x, y, z, f, w)
    u = tagi.direct(kernel, dx, dy, dz, df, dw, kappa=KAPPA).cpu().numpy()
    S = _scale(kernel, x, y, z, f, w, KAPPA)
    assert np.all(np.abs(u - ref) <= 1e-12 * S), np.max(np.abs(u - ref) / S)


def test_direct_separate_targets_and_coincident_points():
    tagi = _tag()
    x, y, z, f, w = uniform_cube(1000, seed=3)
    g = SplitMix64(8)
    tx, ty, tz, tf = g.uniform(130, -1, 1), g.uniform(130, -1, 1), g.uniform(130, -1, 1), g.uniform(130, -1, 1)
    tx[:5], ty[:5], tz[:5] = x[:5], y[:5], z[:5]  # targets sitting on sources
    for kernel in ("yukawa_ss", "coulomb_ss"):
        ref = direct_sum(kernel, x, y, z, f, w, tx, ty, tz, tf, kappa=0.8)
        d = _dev(x, y, z, f, w, tx, ty, tz, tf)
        u = tagi.direct(kernel, *d[:5], d[5], d[6], d[7], d[8], kappa=0.8).cpu().numpy()
        np.testing.assert_allclose(u, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.fixture(scope="module")
def ragged_tree():
    tagi = _tag()
    x, y, z, f, w = _ragged_case()
    t = tagi.Tree(*_dev(x, y, z), leaf_size=200)
    ref = bltc.build_tree(x, y, z, 200)
    return dict(tagi=tagi, x=x, y=y, z=z, f=f, w=w, t=t, ref=ref)


def test_tree_matches_oracle_exactly(ragged_tree):
    t, ref = ragged_tree["t"], ragged_tree["ref"]
    e = t.export()
    assert np.array_equal(e["perm"], ref.perm)
    assert np.array_equal(e["begin"], ref.begin) and np.array_equal(e["end"], ref.end)
    assert np.array_equal(e["level"], ref.level) and np.array_equal(e["parent"], ref.parent)
    assert np.array_equal(e["n_child"], np.array([len(c) for c in ref.children]))
    assert np.array_equal(e["lo"], ref.lo) and np.array_equal(e["hi"], ref.hi)


def test_tree_with_domain_box_matches_oracle():
    tagi = _tag()
    d = atom_mesh(tol_m=1e-9)  # ~700k-point Be-like mesh in [-20, 20]^3
    x, y, z = d["x"], d["y"], d["z"]
    box = (-20, -20, -20, 20, 20, 20)
    t = tagi.Tree(*_dev(x, y, z), leaf_size=500, box=box)
    ref = bltc.build_tree(x, y, z, 500, domain=((-20, -20, -20), (20, 20, 20)))
    e = t.export()
    assert np.array_equal(e["perm"], ref.perm)
    assert np.array_equal(e["begin"], ref.begin) and np.array_equal(e["end"], ref.end)
    assert np.array_equal(e["lo"], ref.lo) and np.array_equal(e["hi"], ref.hi)
    # Fejer cells of 8^3 points split at their centres into leaves of 64
    sizes = e["end"][e["n_child"] == 0] - e["begin"][e["n_child"] == 0]
    assert sizes.max() <= 500


@pytest.mark.parametrize("theta,degree", [(0.7, 6), (0.5, 3), (0.0, 4)])
def test_lists_match_oracle_exactly(ragged_tree, theta, degree):
    t, ref = ragged_tree["t"], ragged_tree["ref"]
    batches, far, near = bltc.interaction_lists(ref, theta, degree)
    L = t.lists(theta, degree)
    for b in range(len(batches)):
        assert list(L["far_id"][L["far_off"][b]:L["far_off"][b + 1]]) == far[b]
        assert list(L["near_id"][L["near_off"][b]:L["near_off"][b + 1]]) == near[b]


def test_lists_on_a_deep_adaptive_mesh_match_oracle_exactly():
    # a small Be-like mesh refined toward the nucleus (10,800 points in cells of
    # 27) with leaves of at most 8 points: nine levels of clusters, the deepest
    # traversals of the list tests, over a thousand batches
    tagi = _tag()
    d = atom_mesh(tol_m=1e-3, p=2, uniform_levels=1)
    x, y, z = d["x"], d["y"], d["z"]
    t = tagi.Tree(*_dev(x, y, z), leaf_size=8, box=(-20, -20, -20, 20, 20, 20))
    ref = bltc.build_tree(x, y, z, 8, domain=((-20, -20, -20), (20, 20, 20)))
    assert int(np.max(ref.level)) >= 9
    e = t.export()
    assert np.array_equal(e["begin"], ref.begin) and np.array_equal(e["end"], ref.end)
    for theta, degree in ((0.7, 1), (0.5, 2)):
        batches, far, near = bltc.interaction_lists(ref, theta, degree)
        assert len(batches) > 1000
        L = t.lists(theta, degree)
        assert L["far_id"].tolist() == [C for fl in far for C in fl]
        assert L["near_id"].tolist() == [C for nl in near for C in nl]
        assert np.array_equal(L["far_off"], np.cumsum([0] + [len(fl) for fl in far]))
        assert np.array_equal(L["near_off"], np.cumsum([0] + [len(nl) for nl in near]))


def test_upward_matches_oracle(ragged_tree):
    c = ragged_tree
    t, ref = c["t"], c["ref"]
    g = SplitMix64(31)
    F = np.stack([c["f"], g.uniform(c["f"].size, -2, 1)])
    dF, dw = _dev(F, c["w"])
    deg = 5
    t.upward(dF, dw, deg)
    P = t.proxies()
    perm = ref.perm
    X, Y, Z, W = c["x"][perm], c["y"][perm], c["z"][perm], c["w"][perm]
    Q = F[:, perm] * W[None, :]
    K = (deg + 1) ** 3
    approx = [cl for cl in range(1, ref.n_nodes) if ref.count(cl) > K]
    assert list(P["cluster"]) == approx
    for s, cl in enumerate(approx):
        b, e = ref.begin[cl], ref.end[cl]
        nodes, ch = bltc.proxy_charges(X[b:e], Y[b:e], Z[b:e], np.vstack([Q[:, b:e], W[None, b:e]]),
                                       ref.lo[cl], ref.hi[cl], deg)
        np.testing.assert_allclose(P["nodes"][s], nodes, rtol=0, atol=1e-15 * np.abs(nodes).max())
        scale_q = np.abs(Q[:, b:e]).sum(axis=1)
        for o in range(2):
            assert np.abs(P["qhat"][o, s] - ch[o].reshape(-1)).max() <= 1e-13 * scale_q[o]
        assert np.abs(P["what"][s] - ch[2].reshape(-1)).max() <= 1e-13 * W[b:e].sum()


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss", "yukawa", "coulomb"])
def test_treecode_matches_oracle_treecode(ragged_tree, kernel):
    c = ragged_tree
    t = c["t"]
    g = SplitMix64(77)
    F = np.stack([c["f"], g.uniform(c["f"].size, -1, 1), g.uniform(c["f"].size, 0, 3)])
    kap = np.array([0.6, 1.3, 3.1])
    deg, theta = 5, 0.65
    dF, dw = _dev(F, c["w"])
    t.upward(dF, dw, deg)
    u = t.convolve(kernel, kap, theta, deg).cpu().numpy()
    ref = bltc.treecode(c["x"], c["y"], c["z"], F, c["w"], kernel, kap, theta, deg, 200, tree=c["ref"])
    for o in range(3):
        S = _scale(kernel, c["x"], c["y"], c["z"], F[o], c["w"], kap[o])
        assert np.all(np.abs(u[o] - ref[o]) <= 1e-12 * S), (o, np.max(np.abs(u[o] - ref[o]) / S))


def test_coulomb_ss_narrow_gaussian_matches_oracle(ragged_tree):
    # alpha = 0.1: about a third of the near work lies in clusters whose boxes are
    # at least 6.12 alpha from the batch, where the kernel sums only the 1/d part
    # (every Gaussian term there is below 2^-54); the oracle sums every term
    c = ragged_tree
    t = c["t"]
    deg, theta, alpha = 5, 0.65, 0.1
    dF, dw = _dev(c["f"], c["w"])
    t.upward(dF, dw, deg)
    u = t.convolve("coulomb_ss", 1.0, theta, deg, alpha=alpha).cpu().numpy()[0]
    ref = bltc.treecode(c["x"], c["y"], c["z"], c["f"], c["w"], "coulomb_ss", 1.0, theta, deg,
                        200, alpha=alpha, tree=c["ref"])[0]
    S = _scale("coulomb_ss", c["x"], c["y"], c["z"], c["f"], c["w"], 1.0, alpha=alpha)
    assert np.all(np.abs(u - ref) <= 1e-12 * S), np.max(np.abs(u - ref) / S)


@pytest.mark.parametrize("kernel,n_orb,degree,theta", [
    ("coulomb_ss", 9, 8, 0.8),   # orbital blocks of 8 and a ragged last block; separable Gaussian
    ("yukawa_ss", 5, 9, 0.8),    # blocks of 4 and 1; proxy rows taken in steps
    ("coulomb_ss", 2, 11, 0.9),  # 12 proxy points per dimension
    ("yukawa", 3, 3, 0.6),       # a degree without a compiled loop (run-time trip counts)
])
def test_treecode_orbital_blocks_and_degrees(ragged_tree, kernel, n_orb, degree, theta):
    c = ragged_tree
    t = c["t"]
    g = SplitMix64(90 + n_orb)
    F = np.stack([g.uniform(c["f"].size, -1, 1) for _ in range(n_orb)])
    kap = np.array([0.5 + 0.4 * o for o in range(n_orb)])
    dF, dw = _dev(F, c["w"])
    t.upward(dF, dw, degree)
    u = t.convolve(kernel, kap, theta, degree).cpu().numpy()
    assert t.stats()["n_far_pairs"] > 0
    ref = bltc.treecode(c["x"], c["y"], c["z"], F, c["w"], kernel, kap, theta, degree, 200,
                        tree=c["ref"])
    for o in range(n_orb):
        S = _scale(kernel, c["x"], c["y"], c["z"], F[o], c["w"], kap[o])
        assert np.all(np.abs(u[o] - ref[o]) <= 1e-12 * S), (o, np.max(np.abs(u[o] - ref[o]) / S))


@pytest.mark.parametrize("kernel,ob", [("coulomb_ss", 8), ("yukawa_ss", 4)])
def test_degree_12_matches_oracle(kernel, ob):
    # degree 12 (13 proxy points per dimension, the highest compiled loop; the
    # learned selector's top degree) in blocks of `ob` orbitals over 3 orbitals
    # (a ragged block): FP64 to the 1e-12 S_i bar, and the mixed far field (whose
    # Coulomb-SS blocks of 8 take the run-time loop at this width) within 1e-6
    tagi = _tag()
    x, y, z, _, w = uniform_cube(20000, seed=31)
    g = SplitMix64(91)
    F = np.stack([g.uniform(x.size, -1, 1) for _ in range(3)])
    kap = np.array([0.5, 0.9, 1.3])
    t = tagi.Tree(*_dev(x, y, z), leaf_size=400)
    dF, dw = _dev(F, w)
    t.upward(dF, dw, 12)
    t.set_orbital_block(ob)
    u = t.convolve(kernel, kap, 0.9, 12).cpu().numpy()
    assert t.stats()["n_far_pairs"] > 0
    um = t.convolve(kernel, kap, 0.9, 12, precision="mixed").cpu().numpy()
    t.close()
    ref = bltc.treecode(x, y, z, F, w, kernel, kap, 0.9, 12, 400)
    for o in range(3):
        S = _scale(kernel, x, y, z, F[o], w, kap[o])
        assert np.all(np.abs(u[o] - ref[o]) <= 1e-12 * S), (o, np.max(np.abs(u[o] - ref[o]) / S))
        assert np.linalg.norm(um[o] - ref[o]) / np.linalg.norm(ref[o]) < 1e-6
        assert np.abs(um[o] - ref[o]).max() / np.abs(ref[o]).max() < 1e-6


def test_theta_zero_equals_direct_and_is_repeatable(ragged_tree):
    c = ragged_tree
    tagi, t = c["tagi"], c["t"]
    dx, dy, dz, df, dw = _dev(c["x"], c["y"], c["z"], c["f"], c["w"])
    t.upward(df, dw, 4)
    u0 = t.convolve("yukawa_ss", KAPPA, 0.0, 4)
    u1 = t.convolve("yukawa_ss", KAPPA, 0.0, 4)
    assert torch.equal(u0, u1)
    ud = tagi.direct("yukawa_ss", dx, dy, dz, df, dw, kappa=KAPPA)
    S = _scale("yukawa_ss", c["x"], c["y"], c["z"], c["f"], c["w"], KAPPA)
    assert np.all(np.abs(u0[0].cpu().numpy() - ud.cpu().numpy()) <= 1e-12 * S)


def test_uniform_cube_32768_meets_1e6_against_direct_sum():
    # the small uniform workload at full size: N = 32768, kappa = 1, theta = 0.7,
    # degree 6, N_L = 500, against the oracle's full direct sum
    tagi = _tag()
    x, y, z, f, w = uniform_cube(32768, seed=1)
    ref = direct_sum("yukawa_ss", x, y, z, f, w, kappa=1.0)
    dx, dy, dz, df, dw = _dev(x, y, z, f, w)
    u = tagi.treecode(dx, dy, dz, df, dw, "yukawa_ss", 1.0, 0.7, 6, 500)[0].cpu().numpy()
    rel_l2 = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    rel_max = np.abs(u - ref).max() / np.abs(ref).max()
    assert rel_l2 < 1e-6 and rel_max < 1e-6, (rel_l2, rel_max)
    ud = tagi.direct("yukawa_ss", dx, dy, dz, df, dw, kappa=1.0).cpu().numpy()
    np.testing.assert_allclose(ud, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
def test_mixed_precision_far_field_within_1e6(ragged_tree, kernel):
    # FP32 batch-proxy tiles, FP64 everywhere else: per-orbital error against the
    # FP64 oracle treecode (same tree and lists) stays below 1e-6 relative
    c = ragged_tree
    t = c["t"]
    g = SplitMix64(78)
    F = np.stack([c["f"], g.uniform(c["f"].size, 0, 3)])
    kap = np.array([0.6, 3.1])
    deg, theta = 6, 0.7
    dF, dw = _dev(F, c["w"])
    t.upward(dF, dw, deg)
    u = t.convolve(kernel, kap, theta, deg, precision="mixed").cpu().numpy()
    ref = bltc.treecode(c["x"], c["y"], c["z"], F, c["w"], kernel, kap, theta, deg, 200, tree=c["ref"])
    for o in range(2):
        assert np.linalg.norm(u[o] - ref[o]) / np.linalg.norm(ref[o]) < 1e-6
        assert np.abs(u[o] - ref[o]).max() / np.abs(ref[o]).max() < 1e-6


def test_argument_errors():
    tagi = _tag()
    x, y, z, f, w = _dev(*uniform_cube(300, seed=1))
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        tagi.Tree(x, y, z, leaf_size=0)
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        tagi.Tree(x, y, z, leaf_size=50, box=(-0.5, -1, -1, 1, 1, 1))
    t = tagi.Tree(x, y, z, leaf_size=50)
    with pytest.raises(tagi.TagiError, match="E_STATE"):
        t.convolve("yukawa", 1.0, 0.5, 4)
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        t.upward(f, w, 17)
    t.upward(f, w, 4)
    with pytest.raises(tagi.TagiError, match="E_STATE"):
        t.convolve("yukawa", 1.0, 0.5, 5)
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        t.convolve("yukawa", 1.0, 1.0, 4)
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        t.convolve("yukawa_ss", 0.0, 0.5, 4)
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        t.convolve("coulomb_ss", 1.0, 0.5, 4, alpha=0.0)
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        tagi.direct("yukawa_ss", x, y, z, f, w, kappa=-1.0)
    # a single point, a single leaf: only the analytic term remains
    one = _dev(np.zeros(1), np.zeros(1), np.zeros(1), np.full(1, 2.0), np.ones(1))
    t1 = tagi.Tree(one[0], one[1], one[2], leaf_size=10)
    t1.upward(one[3], one[4], 3)
    u = t1.convolve("yukawa_ss", 2.0, 0.5, 3).cpu().numpy()
    assert u[0, 0] == pytest.approx(2.0 * 4 * np.pi / 4.0, rel=1e-15)
