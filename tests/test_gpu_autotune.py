"""Orbital-block override, kernel launch variants and the autotuner: the width
of the orbital block only changes how many orbitals share a pair's geometry, and
a launch variant only the register budget or the loop steps, never the
arithmetic of an orbital or its order, so every width and variant gives the
same bits; the autotuner's pick must be one of the candidates and reproduce the
same result as setting it by hand; the same for the autotuner of the learned
lists."""
import os

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


@pytest.mark.parametrize("kernel,precision,ob,degree", [
    ("yukawa_ss", "fp64", 1, 8), ("yukawa_ss", "fp64", 8, 7), ("yukawa_ss", "mixed", 4, 9),
    ("coulomb_ss", "fp64", 1, 8), ("coulomb_ss", "fp64", 4, 10), ("coulomb_ss", "mixed", 1, 6),
    ("yukawa_ss", "fp64", 2, 8), ("coulomb", "fp64", 4, 8)])
def test_kernel_variants_give_the_same_bits(kernel, precision, ob, degree):
    # the last two cases have no compiled variants: every variant runs the defaults
    import paper_2003_01833_amd as tagi
    dx, dy, dz, dw, dF = _case(ob)
    kap = np.linspace(0.7, 2.5, ob)
    t = tagi.Tree(dx, dy, dz, 300)
    t.upward(dF, dw, degree)
    t.set_orbital_block(ob)
    ref = t.convolve(kernel, kap, 0.7, degree, precision=precision).clone()
    for v in (1, 2, 3, 0):
        t.set_kernel_variant(v)
        assert torch.equal(t.convolve(kernel, kap, 0.7, degree, precision=precision), ref), v
    with pytest.raises(tagi.TagiError):
        t.set_kernel_variant(4)
    t.close()


def test_orbital_block_rejects_other_widths():
    import paper_2003_01833_amd as tagi
    dx, dy, dz, dw, dF = _case(2)
    t = tagi.Tree(dx, dy, dz, 250)
    with pytest.raises(tagi.TagiError):
        t.set_orbital_block(3)
    t.close()


def test_autotune_picks_a_candidate_that_reproduces_the_result(tmp_path):
    import paper_2003_01833_amd as tagi
    dx, dy, dz, dw, dF = _case(5)
    kap = np.linspace(0.8, 2.4, 5)
    (leaf, ob, items, var), times = tagi.autotune(dx, dy, dz, dF, dw, "yukawa_ss", kap, 0.7, 6,
                                                  leaf_sizes=(150, 400), obs=(1, 4),
                                                  items=(0, 1024), reps=2, variants=(0, 1))
    assert leaf in (150, 400) and ob in (1, 4) and items in (0, 1024) and var in (0, 1)
    assert times.shape == (2, 2, 2, 2) and np.all(times > 0)
    assert times[(150, 400).index(leaf), (1, 4).index(ob), (0, 1024).index(items),
                 var] == times.min()
    t = tagi.Tree(dx, dy, dz, leaf)
    t.set_orbital_block(ob)
    t.set_schedule_items(items)
    t.set_kernel_variant(var)
    t.upward(dF, dw, 6)
    u = t.convolve("yukawa_ss", kap, 0.7, 6)
    t2 = tagi.Tree(dx, dy, dz, leaf)
    t2.upward(dF, dw, 6)
    u2 = t2.convolve("yukawa_ss", kap, 0.7, 6)
    # the schedule's granularity only regroups the partial sums
    assert torch.allclose(u, u2, rtol=0, atol=1e-13 * float(u2.abs().max()))
    t.close()
    t2.close()
    # the JSON cache: tuned once, read back afterwards
    cache = str(tmp_path / "tuning.json")
    best, hit = tagi.autotune_cached(cache, dx, dy, dz, dF, dw, "yukawa_ss", kap, 0.7, 6,
                                     leaf_sizes=(150, 400), obs=(1, 4))
    assert not hit and best[0] in (150, 400) and best[1] in (1, 4)
    again, hit = tagi.autotune_cached(cache, dx, dy, dz, dF, dw, "yukawa_ss", kap, 0.7, 6,
                                      leaf_sizes=(150, 400), obs=(1, 4))
    assert hit and again == best
    # another candidate set is tuned afresh
    other, hit = tagi.autotune_cached(cache, dx, dy, dz, dF, dw, "yukawa_ss", kap, 0.7, 6,
                                      leaf_sizes=(150, 400), obs=(1, 4), variants=(0, 3))
    assert not hit and other[3] in (0, 3)


def test_schedule_items_change_only_the_grouping_of_partial_sums():
    import paper_2003_01833_amd as tagi
    dx, dy, dz, dw, dF = _case(3)
    kap = np.array([0.7, 1.5, 3.0])
    t = tagi.Tree(dx, dy, dz, 200)
    t.upward(dF, dw, 7)
    ref = t.convolve("coulomb_ss", kap, 0.7, 7).clone()
    for items in (256, 4096, 1 << 20, 0):
        t.set_schedule_items(items)
        u = t.convolve("coulomb_ss", kap, 0.7, 7)
        assert torch.allclose(u, ref, rtol=0, atol=1e-13 * float(ref.abs().max())), items
    with pytest.raises(tagi.TagiError):
        t.set_schedule_items(100)
    t.close()


WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2003_01833_amd", "selector_weights.npz")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained selector weights")
def test_learned_autotune_picks_a_candidate_that_reproduces_the_result():
    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd.selector import Selector
    sel = Selector.load(WEIGHTS)
    dx, dy, dz, dw, dF = _case(5)
    kap = np.linspace(0.8, 2.4, 5)
    tol = 1e-8 * 4 * np.pi / kap ** 2
    (leaf, ob, items, var), times = tagi.autotune_learned(
        dx, dy, dz, dF, dw, "yukawa_ss", kap, sel, tol, leaf_sizes=(150, 400), obs=(4, 8),
        items=(0,), variants=(0, 1), reps=2)
    assert leaf in (150, 400) and ob in (4, 8) and items == 0 and var in (0, 1)
    assert times.shape == (2, 2, 1, 2) and np.all(times > 0)
    assert times[(150, 400).index(leaf), (4, 8).index(ob), 0, var] == times.min()
    # the pick on a tree by hand against the defaults on the same leaf size: the
    # orbital block and the launch variant leave the bits alone
    t = tagi.Tree(dx, dy, dz, leaf)
    t.set_orbital_block(ob)
    t.set_kernel_variant(var)
    t.upward(dF, dw, 1)
    u = t.convolve_learned("yukawa_ss", kap, sel, tol, precision="mixed").clone()
    t2 = tagi.Tree(dx, dy, dz, leaf)
    t2.upward(dF, dw, 1)
    u2 = t2.convolve_learned("yukawa_ss", kap, sel, tol, precision="mixed")
    assert torch.equal(u, u2)
    t.close()
    t2.close()
