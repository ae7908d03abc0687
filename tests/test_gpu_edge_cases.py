"""Degenerate and extreme inputs through the C ABI against the oracle: one point,
leaves of one point, coincident points, flat (zero-extent) point sets, the
lowest and highest degrees, and the largest orbital count."""
import numpy as np
import pytest
import torch

from oracle import bltc
from oracle.direct import direct_sum
from workloads.configs import uniform_cube
from workloads.rng import SplitMix64

pytestmark = pytest.mark.gpu


def _tag():
    import paper_2003_01833_amd as tagi
    return tagi


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def _scale(kernel, x, y, z, f, w, kappa):
    # sum of the magnitudes the result can cancel down from (as in the parity tests)
    fi = np.abs(f)
    if kernel.startswith("yukawa"):
        s = direct_sum("yukawa", x, y, z, fi, w, kappa=kappa)
        if kernel == "yukawa_ss":
            s = s + fi * direct_sum("yukawa", x, y, z, np.ones_like(f), w, kappa=kappa) + 4 * np.pi / kappa ** 2 * fi
        return s
    s = direct_sum("coulomb", x, y, z, fi, w)
    if kernel == "coulomb_ss":
        s = s + fi * direct_sum("coulomb", x, y, z, np.ones_like(f), w) + 2 * np.pi * fi
    return s


def _check(x, y, z, F, w, kernel, kap, theta, degree, leaf, tol=1e-12):
    tagi = _tag()
    dx, dy, dz, dF, dw = _dev(x, y, z, F, w)
    t = tagi.Tree(dx, dy, dz, leaf)
    t.upward(dF, dw, degree)
    u = t.convolve(kernel, kap, theta, degree).cpu().numpy()
    ref = bltc.treecode(x, y, z, F, w, kernel, kap, theta, degree, leaf)
    for o in range(F.shape[0]):
        S = _scale(kernel, x, y, z, F[o], w, float(np.atleast_1d(kap)[o]))
        assert np.all(np.abs(u[o] - ref[o]) <= tol * S + 1e-300), (o, np.max(np.abs(u[o] - ref[o]) / S))
    st = t.stats()
    t.close()
    return st


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss", "yukawa", "coulomb"])
def test_single_point(kernel):
    # one source: no pair at nonzero distance, only the analytic term remains
    x, y, z = np.array([0.3]), np.array([-0.2]), np.array([0.1])
    F, w = np.array([[1.7]]), np.array([0.5])
    _check(x, y, z, F, w, kernel, np.array([1.1]), 0.7, 3, 4)


def test_leaves_of_one_point():
    x, y, z, f, w = uniform_cube(300, seed=71)
    st = _check(x, y, z, f[None], w, "yukawa_ss", np.array([1.3]), 0.7, 2, 1)
    assert st["n_far_pairs"] > 0


def test_coincident_points():
    # 60 copies of one point among 400 others: pairs at distance zero add nothing
    x, y, z, f, w = uniform_cube(400, seed=72)
    x[:60], y[:60], z[:60] = 0.25, -0.5, 0.125
    for kernel in ("yukawa_ss", "coulomb_ss"):
        _check(x, y, z, f[None], w, kernel, np.array([0.9]), 0.6, 3, 50)


def test_all_points_coincident():
    # the root cannot be divided: one leaf of 100 points, every pair at distance 0
    x = np.full(100, 0.5)
    y = np.full(100, -0.25)
    z = np.full(100, 2.0)
    g = SplitMix64(73)
    F, w = g.uniform(100, -1, 1)[None], g.uniform(100, 0.1, 1.0)
    tagi = _tag()
    dx, dy, dz, dF, dw = _dev(x, y, z, F, w)
    t = tagi.Tree(dx, dy, dz, 10)
    t.upward(dF, dw, 3)
    u = t.convolve("yukawa_ss", 1.5, 0.7, 3).cpu().numpy()
    np.testing.assert_allclose(u[0], 4 * np.pi / 1.5 ** 2 * F[0], rtol=1e-14)
    t.close()


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
def test_flat_point_set(kernel):
    # every point in the plane z = 0: zero-extent boxes in z at every level
    x, y, _, f, w = uniform_cube(3000, seed=74)
    z = np.zeros_like(x)
    st = _check(x, y, z, f[None], w, kernel, np.array([1.2]), 0.7, 4, 100)
    assert st["n_far_pairs"] > 0


def test_lowest_degree():
    x, y, z, f, w = uniform_cube(20000, seed=75)
    st = _check(x, y, z, f[None], w, "yukawa_ss", np.array([0.8]), 0.5, 1, 400)
    assert st["n_far_pairs"] > 0


def test_highest_degree():
    # two separated blobs of 6000 points: each is one cluster, far from the
    # other's batches, holding more than (16+1)^3 = 4913 sources
    x, y, z, f, w = uniform_cube(12000, seed=78)
    x, y, z = 0.5 * x, 0.5 * y, 0.5 * z
    x[6000:] += 10.0
    st = _check(x, y, z, f[None], w, "yukawa_ss", np.array([0.3]), 0.95, 16, 400)
    assert st["n_far_pairs"] > 0


def test_largest_orbital_count():
    # 64 orbitals (the maximum): Coulomb blocks of 8, Yukawa blocks of 8
    x, y, z, _, w = uniform_cube(1500, seed=76)
    g = SplitMix64(77)
    F = np.stack([g.uniform(x.size, -1, 1) for _ in range(64)])
    kap = np.linspace(0.5, 4.0, 64)
    for kernel in ("coulomb_ss", "yukawa_ss"):
        _check(x, y, z, F, w, kernel, kap, 0.7, 4, 100)


def test_timing_reports_each_interaction_launch():
    # the fixed MAC runs one interaction launch per convolution: its own
    # duration (events on its stream around it alone) lies within the phase's;
    # the learned lists run one launch per degree in use plus one for the near
    # pairs, each timed on its own stream
    import os

    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd.selector import Selector
    x, y, z, f, w = uniform_cube(40000, seed=44)
    dx, dy, dz, df, dw = (torch.from_numpy(a).cuda() for a in (x, y, z, f, w))
    t = tagi.Tree(dx, dy, dz, 500)
    t.upward(df, dw, 6)
    t.convolve("yukawa_ss", 1.2, 0.7, 6)
    t.set_timing(True)
    t.convolve("yukawa_ss", 1.2, 0.7, 6)
    tm = t.timing()
    assert tm["interact_launches"] == 1
    assert 0.0 < tm["interact_kernel_ms"] <= tm["interact_ms"] * (1 + 1e-6) + 1e-3
    sel = Selector.load(os.path.join(os.path.dirname(tagi.__file__), "selector_weights.npz"))
    t.upward(df, dw, 1)
    t.set_timing(True)
    t.convolve_learned("yukawa_ss", 1.2, sel, [1e-7])
    tm = t.timing()
    st = t.learned_stats()
    degrees = [d for d, c in st["far_pairs_by_degree"].items() if c > 0]
    assert tm["interact_launches"] == len(degrees) + (st["near_interactions"] > 0)
    assert tm["interact_kernel_ms"] > 0.0 and tm["interact_ms"] > 0.0
    t.close()
