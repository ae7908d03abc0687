"""A captured Green-iteration step (upward + convolve as a HIP graph) against the
eager calls, replayed several times with eager work and synchronisations in
between and with the input rewritten in place between replays."""
import numpy as np
import pytest
import torch

from workloads.configs import uniform_cube
from workloads.rng import SplitMix64

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kernel,precision", [("yukawa_ss", "fp64"), ("coulomb_ss", "fp64"),
                                              ("yukawa_ss", "mixed")])
def test_graph_replays_equal_eager_calls(kernel, precision):
    import paper_2003_01833_amd as tagi
    x, y, z, f, w = uniform_cube(9000, seed=5)
    g = SplitMix64(17)
    F = np.stack([f, g.uniform(f.size, -1, 1), g.uniform(f.size, 0, 2)])
    kap = [0.7, 1.4, 2.9]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    dx, dy, dz, dw, dF = dev(x), dev(y), dev(z), dev(w), dev(F)
    t = tagi.Tree(dx, dy, dz, 300)
    out = torch.empty_like(dF)
    step = t.graph(dF, dw, 6, kernel, kap, 0.7, out, precision=precision)
    ref_tree = tagi.Tree(dx, dy, dz, 300)
    for rep in range(4):
        # rewrite f in place, replay, and compare with eager calls on a second tree
        dF.mul_(0.5).add_(float(rep) * 0.1)
        step.launch()
        torch.cuda.synchronize()
        got = out.clone()
        ref_tree.upward(dF, dw, 6)
        ref = ref_tree.convolve(kernel, kap, 0.7, 6, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), rep
        _ = torch.linalg.norm(ref)  # unrelated eager work between replays
    step.close()
    t.close()
    ref_tree.close()
