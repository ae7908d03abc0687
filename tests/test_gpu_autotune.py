"""Orbital-block override and the autotuner: the width of the orbital block only
changes how many orbitals share a pair's geometry, never the arithmetic of an
orbital, so every width gives the same bits; the autotuner's pick must be one of
the candidates and reproduce the same result as setting it by hand."""
import numpy as np
import pytest
import torch

from workloads.configs import uniform_cube
from workloads.rng import SplitMix64

pytestmark = pytest.mark.gpu


def _case(n_orb):
    x, y, z, f, w = uniform_cube(12000, seed=21)
    g = SplitMix64(22)
    F = np.stack([f] + [g.uniform(f.size, -1, 1) for _ in range(n_orb - 1)])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    return dev(x), dev(y), dev(z), dev(w), dev(F)


@pytest.mark.parametrize("kernel,precision", [("yukawa_ss", "fp64"), ("coulomb_ss", "fp64"),
                                              ("yukawa_ss", "mixed")])
def test_orbital_block_width_does_not_change_results(kernel, precision):
    import paper_2003_01833_amd as tagi
    dx, dy, dz, dw, dF = _case(9)
    kap = np.linspace(0.6, 3.0, 9)
    t = tagi.Tree(dx, dy, dz, 250)
    t.upward(dF, dw, 7)
    outs = []
    for ob in (1, 2, 4, 8, 0):
        t.set_orbital_block(ob)
        outs.append(t.convolve(kernel, kap, 0.7, 7, precision=precision).clone())
    for ob, u in zip((2, 4, 8, 0), outs[1:]):
        assert torch.equal(u, outs[0]), ob
    t.close()


def test_orbital_block_rejects_other_widths():
    import paper_2003_01833_amd as tagi
    dx, dy, dz, dw, dF = _case(2)
    t = tagi.Tree(dx, dy, dz, 250)
    with pytest.raises(tagi.TagiError):
        t.set_orbital_block(3)
    t.close()


def test_autotune_picks_a_candidate_that_reproduces_the_result():
    import paper_2003_01833_amd as tagi
    dx, dy, dz, dw, dF = _case(5)
    kap = np.linspace(0.8, 2.4, 5)
    (leaf, ob), times = tagi.autotune(dx, dy, dz, dF, dw, "yukawa_ss", kap, 0.7, 6,
                                      leaf_sizes=(150, 400), obs=(1, 4), reps=2)
    assert leaf in (150, 400) and ob in (1, 4)
    assert times.shape == (2, 2) and np.all(times > 0)
    assert times[(150, 400).index(leaf), (1, 4).index(ob)] == times.min()
    t = tagi.Tree(dx, dy, dz, leaf)
    t.set_orbital_block(ob)
    t.upward(dF, dw, 6)
    u = t.convolve("yukawa_ss", kap, 0.7, 6)
    t2 = tagi.Tree(dx, dy, dz, leaf)
    t2.upward(dF, dw, 6)
    assert torch.equal(u, t2.convolve("yukawa_ss", kap, 0.7, 6))
    t.close()
    t2.close()
