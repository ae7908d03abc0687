"""Separate target sets (Eq. direct-sum with targets x_i distinct from the
sources y_j; Section 6.1 target batches): the GPU treecode through the C ABI
against the oracle treecode with its own tree on the targets, element by
element at <= 1e-12 S_i (S_i as in test_gpu_parity: the sum the terms can cancel
down from), and against the direct sum at theta = 0."""
import numpy as np
import pytest
import torch

from oracle import bltc
from oracle.direct import direct_sum
from workloads.configs import uniform_cube
from workloads.rng import SplitMix64

pytestmark = pytest.mark.gpu

LEAF = 150


def _tag():
    import paper_2003_01833_amd as tagi
    return tagi


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def _scale(kernel, src, tgt, kappa, alpha=1.0):
    """S_i at the targets: sum_j |K1| |f_j| w_j + |f_i| sum_j |K2| w_j + |s f_i|."""
    x, y, z, f, w = src
    tx, ty, tz, tf = tgt
    fi = np.abs(tf)
    if kernel.startswith("yukawa"):
        s = direct_sum("yukawa", x, y, z, np.abs(f), w, tx, ty, tz, tf, kappa=kappa)
        if kernel == "yukawa_ss":
            s = s + fi * direct_sum("yukawa", x, y, z, np.ones_like(f), w, tx, ty, tz, tf, kappa=kappa)
            s = s + 4 * np.pi / kappa ** 2 * fi
        return s
    s = direct_sum("coulomb", x, y, z, np.abs(f), w, tx, ty, tz, tf)
    if kernel == "coulomb_ss":
        s = s + fi * direct_sum("coulomb", x, y, z, np.ones_like(f), w, tx, ty, tz, tf)
        s = s + 2 * np.pi * alpha ** 2 * fi
    return s


def _sources(n=6000, seed=21):
    x, y, z, f, w = uniform_cube(n, seed=seed)
    # a third of the points squeezed toward a corner: uneven leaves
    k = np.arange(n) % 3 == 0
    x = np.where(k, -1.0 + 0.05 * (x + 1.0), x)
    y = np.where(k, -1.0 + 0.05 * (y + 1.0), y)
    return x, y, z, f, w


def _targets(src, n_t, seed, n_on=0, n_out=0):
    """n_t targets: uniform in [-1.2, 1.2]^3, the first n_on copied from sources,
    the last n_out far outside the sources' box (there the root cluster passes
    the MAC); values for n_orb = 3 orbitals."""
    g = SplitMix64(seed)
    tx, ty, tz = (g.uniform(n_t, -1.2, 1.2) for _ in range(3))
    x, y, z = src[:3]
    tx[:n_on], ty[:n_on], tz[:n_on] = x[:n_on], y[:n_on], z[:n_on]
    if n_out:
        tx[n_t - n_out:] = g.uniform(n_out, 6.0, 7.0)
        ty[n_t - n_out:] = g.uniform(n_out, -0.5, 0.5)
    tf = np.stack([g.uniform(n_t, -1.0, 1.0) for _ in range(3)])
    return tx, ty, tz, tf


@pytest.fixture(scope="module")
def case():
    tagi = _tag()
    src = _sources()
    x, y, z, f, w = src
    g = SplitMix64(5)
    F = np.stack([f, g.uniform(f.size, -1, 1), g.uniform(f.size, 0, 2)])
    ref_tree = bltc.build_tree(x, y, z, LEAF)
    t = tagi.Tree(*_dev(x, y, z), leaf_size=LEAF)
    return dict(tagi=tagi, src=src, F=F, t=t, ref_tree=ref_tree)


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss", "yukawa", "coulomb"])
def test_separate_targets_match_oracle_treecode(case, kernel):
    x, y, z, f, w = case["src"]
    F, t = case["F"], case["t"]
    tx, ty, tz, tf = _targets(case["src"], 2345, seed=40, n_on=100, n_out=60)
    kap = np.array([0.7, 1.4, 2.9])
    deg, theta = 5, 0.7
    dF, dw = _dev(F, w)
    t.upward(dF, dw, deg)
    ss = kernel.endswith("_ss")
    dt = _dev(tx, ty, tz, tf)
    u = t.convolve(kernel, kap, theta, deg,
                   targets=(dt[0], dt[1], dt[2], dt[3] if ss else None)).cpu().numpy()
    ref, parts = bltc.treecode(x, y, z, F, w, kernel, kap, theta, deg, LEAF,
                               tree=case["ref_tree"], targets=(tx, ty, tz, tf if ss else None),
                               return_parts=True)
    # the outlying targets accept the root as a far cluster
    assert any(0 in fl for fl in parts["far"])
    for o in range(3):
        S = _scale(kernel, (x, y, z, F[o], w), (tx, ty, tz, tf[o] if ss else np.zeros_like(tx)),
                   kap[o])
        assert np.all(np.abs(u[o] - ref[o]) <= 1e-12 * S), (o, np.max(np.abs(u[o] - ref[o]) / S))


def test_separate_targets_theta_zero_is_the_direct_sum(case):
    tagi = case["tagi"]
    x, y, z, f, w = case["src"]
    t = case["t"]
    tx, ty, tz, tf = _targets(case["src"], 777, seed=41, n_on=50)
    dF, dw = _dev(f, w)
    t.upward(dF, dw, 4)
    dt = _dev(tx, ty, tz, tf[0])
    for kernel in ("yukawa_ss", "coulomb_ss"):
        u = t.convolve(kernel, 1.1, 0.0, 4, targets=tuple(dt)).cpu().numpy()[0]
        ref = direct_sum(kernel, x, y, z, f, w, tx, ty, tz, tf[0], kappa=1.1)
        S = _scale(kernel, (x, y, z, f, w), (tx, ty, tz, tf[0]), 1.1)
        assert np.all(np.abs(u - ref) <= 1e-12 * S), np.max(np.abs(u - ref) / S)
        ds = _dev(x, y, z, f, w)
        ud = tagi.direct(kernel, *ds, *dt, kappa=1.1).cpu().numpy()
        assert np.all(np.abs(u - ud) <= 1e-12 * S)


def test_targets_equal_to_sources_reproduce_the_default_bitwise(case):
    # with the sources passed as targets, the target tree is the source tree (same
    # rule, same bounding box), so lists, schedule and sums are the same
    x, y, z, f, w = case["src"]
    F, t = case["F"], case["t"]
    dF, dw = _dev(F, w)
    t.upward(dF, dw, 6)
    kap = np.array([0.9, 1.5, 3.0])
    u0 = t.convolve("yukawa_ss", kap, 0.65, 6).clone()
    dx, dy, dz = _dev(x, y, z)
    u1 = t.convolve("yukawa_ss", kap, 0.65, 6, targets=(dx, dy, dz, dF))
    assert torch.equal(u0, u1)
    # and the default path is unaffected by a call with targets
    u2 = t.convolve("yukawa_ss", kap, 0.65, 6)
    assert torch.equal(u0, u2)


@pytest.mark.parametrize("n_t", [1, 64, 65, 150, 151])
def test_ragged_target_counts(case, n_t):
    x, y, z, f, w = case["src"]
    t = case["t"]
    tx, ty, tz, tf = _targets(case["src"], n_t, seed=100 + n_t)
    dF, dw = _dev(f, w)
    t.upward(dF, dw, 5)
    dt = _dev(tx, ty, tz, tf[0])
    u = t.convolve("yukawa_ss", 1.3, 0.7, 5, targets=tuple(dt)).cpu().numpy()[0]
    ref = bltc.treecode(x, y, z, f, w, "yukawa_ss", 1.3, 0.7, 5, LEAF, tree=case["ref_tree"],
                        targets=(tx, ty, tz, tf[0]))[0]
    S = _scale("yukawa_ss", (x, y, z, f, w), (tx, ty, tz, tf[0]), 1.3)
    assert u.shape == (n_t,)
    assert np.all(np.abs(u - ref) <= 1e-12 * S), np.max(np.abs(u - ref) / S)


def test_empty_target_set_writes_nothing(case):
    x, y, z, f, w = case["src"]
    t = case["t"]
    dF, dw = _dev(f, w)
    t.upward(dF, dw, 4)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    out = torch.empty((1, 0), dtype=torch.float64, device="cuda")
    u = t.convolve("yukawa_ss", 1.0, 0.7, 4, targets=(e, e, e, e), out=out)
    assert u.numel() == 0


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
def test_separate_targets_mixed_precision_within_1e6(case, kernel):
    x, y, z, f, w = case["src"]
    F, t = case["F"], case["t"]
    tx, ty, tz, tf = _targets(case["src"], 3000, seed=42, n_on=30, n_out=20)
    kap = np.array([0.7, 1.4, 2.9])
    dF, dw = _dev(F, w)
    t.upward(dF, dw, 6)
    dt = _dev(tx, ty, tz, tf)
    u = t.convolve(kernel, kap, 0.7, 6, precision="mixed", targets=tuple(dt)).cpu().numpy()
    ref = bltc.treecode(x, y, z, F, w, kernel, kap, 0.7, 6, LEAF, tree=case["ref_tree"],
                        targets=(tx, ty, tz, tf))
    for o in range(3):
        assert np.linalg.norm(u[o] - ref[o]) / np.linalg.norm(ref[o]) < 1e-6
        assert np.abs(u[o] - ref[o]).max() / np.abs(ref[o]).max() < 1e-6


def test_separate_target_argument_errors(case):
    tagi = case["tagi"]
    x, y, z, f, w = case["src"]
    t = case["t"]
    dF, dw = _dev(f, w)
    t.upward(dF, dw, 4)
    tx, ty, tz, tf = _dev(*_targets(case["src"], 10, seed=9)[:3], np.zeros(10))
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        t.convolve("yukawa_ss", 1.0, 0.7, 4, targets=(tx, ty, tz, None))
    bad = tx.clone()
    bad[3] = float("inf")
    with pytest.raises(tagi.TagiError, match="E_ARG"):
        t.convolve("yukawa", 1.0, 0.7, 4, targets=(bad, ty, tz, None))
