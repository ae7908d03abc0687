"""Learned degree/MAC lists on the GPU against the oracle traversal with the same
network (evaluated there in FP64). The FP32 network on the GPU and the FP64 one
may put a decision whose compared quantity lies within 2e-4 (log10 units) of its
threshold on either side; the oracle reports such ties and never takes the
GPU's decision. Every batch without a tie must have identical lists; batches
with a tie (at most a handful) must still cover every source exactly once."""
import os

import numpy as np
import pytest
import torch

from oracle import bltc
from oracle.learned import learned_lists
from workloads.configs import atom_mesh
from workloads.rng import SplitMix64

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2003_01833_amd", "selector_weights.npz")


def _slater(r, seed):
    g = SplitMix64(seed)
    f = np.zeros_like(r)
    for _ in range(3):
        c = g.uniform(1, -1.0, 1.0)[0]
        z = g.uniform(1, 0.5, 6.0)[0]
        f += c * np.exp(-z * r)
    return f


def _compare(t, ref_tree, far, near, ties):
    """GPU lists (exported) against the oracle's, batch by batch; returns the
    degrees in use."""
    L = t.learned_lists()
    nl = len(ref_tree.leaves())
    assert L["far_off"].size == nl + 1
    tied = {b for b, _, _ in ties}
    assert len(tied) <= 5, ties
    degrees = set()
    for b, B in enumerate(ref_tree.leaves()):
        e0, e1 = L["far_off"][b], L["far_off"][b + 1]
        n0, n1 = L["near_off"][b], L["near_off"][b + 1]
        gfar = list(zip(L["far_id"][e0:e1].tolist(), L["far_degree"][e0:e1].tolist()))
        gnear = L["near_id"][n0:n1].tolist()
        degrees.update(dg for _, dg in gfar)
        if b in tied:
            # still a partition of the sources into the listed clusters
            cover = np.zeros(ref_tree.end[0], np.int32)
            for C in [c for c, _ in gfar] + gnear:
                cover[ref_tree.begin[C]:ref_tree.end[C]] += 1
            assert np.all(cover == 1), b
            continue
        # far entries grouped by degree (stable), near entries in traversal order
        assert gfar == sorted(far[b], key=lambda e: e[1]), b
        assert gnear == near[b], b
    return degrees


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained selector weights")
@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
def test_learned_lists_match_oracle_traversal(kernel):
    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd.selector import Selector
    sel = Selector.load(WEIGHTS)
    d = atom_mesh(tol_m=1e-5, p=5, uniform_levels=2)
    x, y, z, w = d["x"], d["y"], d["z"], d["w"]
    r = np.sqrt(x * x + y * y + z * z)
    if kernel == "yukawa_ss":
        F = np.stack([_slater(r, 51), _slater(r, 52)])
        kap = np.array([0.8, 2.0])
        tol = 1e-8 * 4 * np.pi / kap ** 2 * np.abs(F).max(axis=1)
    else:
        F = np.stack([_slater(r, 53) ** 2])
        kap = np.array([1.0])
        tol = 1e-8 * 2 * np.pi * np.abs(F).max(axis=1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    t = tagi.Tree(dev(x), dev(y), dev(z), 300)
    t.upward(dev(F), dev(w), 1)
    t.convolve_learned(kernel, kap, sel, tol, theta_max=0.9, theta_fb=0.7, degree_fb=8)
    ref_tree = bltc.build_tree(x, y, z, 300)
    p = ref_tree.perm
    far, near, ties = learned_lists(ref_tree, x[p], y[p], z[p], F[:, p], w[p], kernel, kap,
                                    sel.net(kernel).params, sel.net(kernel).norm, np.log10(tol),
                                    0.9, 0.7, 8)
    degrees = _compare(t, ref_tree, far, near, ties)
    assert len(degrees) >= 3, degrees  # the selection is not degenerate
    t.close()


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained selector weights")
def test_learned_precisions_share_lists_and_agree():
    # FP64 and mixed calls on one tree use different orbital blocks (8 and 4 for
    # nine orbitals): each call must run on a schedule built for its own block
    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd.selector import Selector
    sel = Selector.load(WEIGHTS)
    d = atom_mesh(tol_m=1e-5, p=5, uniform_levels=2)
    x, y, z, w = d["x"], d["y"], d["z"], d["w"]
    r = np.sqrt(x * x + y * y + z * z)
    F = np.stack([_slater(r, 60 + o) for o in range(9)])
    kap = np.linspace(0.7, 3.5, 9)
    tol = 3e-9 * 4 * np.pi / kap ** 2 * np.abs(F).max(axis=1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    t = tagi.Tree(dev(x), dev(y), dev(z), 300)
    t.upward(dev(F), dev(w), 1)
    u64 = t.convolve_learned("yukawa_ss", kap, sel, tol).clone()
    u32 = t.convolve_learned("yukawa_ss", kap, sel, tol, precision="mixed").clone()
    u64b = t.convolve_learned("yukawa_ss", kap, sel, tol)
    assert torch.equal(u64, u64b)
    # a stale schedule gives errors of order one; the FP32 far field alone stays
    # far below 1e-4 of max|u| here
    err = ((u32 - u64).abs().amax(dim=1) / u64.abs().amax(dim=1)).cpu().numpy()
    assert err.max() < 1e-4, err
    t.close()


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained selector weights")
def test_learned_lists_follow_new_charges():
    # the lists take their features from the charges: after an upward pass with
    # other values and the same kappa and tol, the result must be that of a
    # fresh tree on the new values, not of the lists cached for the old ones
    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd.selector import Selector
    sel = Selector.load(WEIGHTS)
    d = atom_mesh(tol_m=1e-5, p=5, uniform_levels=2)
    x, y, z, w = d["x"], d["y"], d["z"], d["w"]
    r = np.sqrt(x * x + y * y + z * z)
    F1 = np.stack([_slater(r, 51), _slater(r, 52)])
    F2 = np.stack([_slater(r, 53), 40.0 * _slater(r, 54)])
    kap = np.array([0.8, 2.0])
    tol = np.array([1e-9, 1e-9])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    dx, dy, dz, dw = dev(x), dev(y), dev(z), dev(w)
    t = tagi.Tree(dx, dy, dz, 300)
    t.upward(dev(F1), dw, 1)
    t.convolve_learned("yukawa_ss", kap, sel, tol)
    s1 = t.learned_stats()
    t.upward(dev(F2), dw, 1)
    u = t.convolve_learned("yukawa_ss", kap, sel, tol).clone()
    s2 = t.learned_stats()
    fresh = tagi.Tree(dx, dy, dz, 300)
    fresh.upward(dev(F2), dw, 1)
    ref = fresh.convolve_learned("yukawa_ss", kap, sel, tol)
    assert s1 != fresh.learned_stats()  # the two charge sets select different lists
    assert s2 == fresh.learned_stats()
    assert torch.equal(u, ref)
    t.close()
    fresh.close()
