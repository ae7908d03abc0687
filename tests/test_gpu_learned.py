"""Learned degree/MAC lists on the GPU against the oracle traversal with the same
network (evaluated there in FP64): every decision must agree except ties, where
the FP32 network on the GPU and the FP64 one may fall on either side of a
threshold within 2e-4 (log10 units)."""
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


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained selector weights")
def test_learned_lists_match_oracle_traversal():
    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd.selector import Selector
    sel = Selector.load(WEIGHTS)
    d = atom_mesh(tol_m=1e-5, p=5, uniform_levels=2)
    x, y, z, w = d["x"], d["y"], d["z"], d["w"]
    r = np.sqrt(x * x + y * y + z * z)
    F = np.stack([_slater(r, 51), _slater(r, 52)])
    kap = np.array([0.8, 2.0])
    tol = 3e-9 * 4 * np.pi / kap ** 2 * np.abs(F).max(axis=1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    t = tagi.Tree(dev(x), dev(y), dev(z), 300)
    t.upward(dev(F), dev(w), 1)
    t.convolve_learned("yukawa_ss", kap, sel, tol, theta_max=0.9, theta_fb=0.7, degree_fb=8)
    L = t.learned_lists()
    ref_tree = bltc.build_tree(x, y, z, 300)
    nl = len(ref_tree.leaves())
    assert L["far_off"].size == nl + 1
    gpu = []
    for b in range(nl):
        dct = {}
        for e in range(L["far_off"][b], L["far_off"][b + 1]):
            dct[int(L["far_id"][e])] = ("far", int(L["far_degree"][e]))
        for e in range(L["near_off"][b], L["near_off"][b + 1]):
            dct[int(L["near_id"][e])] = ("near",)
        gpu.append(dct)
    p = ref_tree.perm
    far, near, ties, mism = learned_lists(ref_tree, x[p], y[p], z[p], F[:, p], w[p], kap,
                                          sel.params, sel.norm, np.log10(tol), 0.9, 0.7, 8,
                                          reference=gpu)
    assert not mism, mism[:5]
    assert len(ties) <= 5, ties
    degrees = set()
    for b in range(nl):
        # far entries grouped by degree (stable), near in traversal order
        of = sorted(far[b], key=lambda e: e[1])
        e0, e1 = L["far_off"][b], L["far_off"][b + 1]
        assert [c for c, _ in of] == list(L["far_id"][e0:e1]), b
        assert [dg for _, dg in of] == list(L["far_degree"][e0:e1]), b
        n0, n1 = L["near_off"][b], L["near_off"][b + 1]
        assert near[b] == list(L["near_id"][n0:n1]), b
        degrees.update(dg for _, dg in of)
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
