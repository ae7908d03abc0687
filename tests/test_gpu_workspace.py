"""The device-memory limit: with TAGI_WORKSPACE_LIMIT set, an allocation beyond
it fails with TAGI_E_OOM before anything that needs it is launched, and the
tree stays usable: the same call once the limit is lifted gives the bits of a
tree that never failed. The limit is swept over the bytes a call allocates, so
that the failure falls on the allocations of the upward pass, the lists, the
schedule, the launch order, the FP32 charge copies, the learned lists and
items, the Green step's buffers and the target tree in turn. Nothing is leaked:
the bytes the library holds return to their start once the trees are closed.
(Failure handling forced from the host: every kernel that runs gets its
buffers.)"""
import os

import numpy as np
import pytest
import torch

from workloads.configs import uniform_cube
from workloads.rng import SplitMix64

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2003_01833_amd", "selector_weights.npz")
LIMIT = "TAGI_WORKSPACE_LIMIT"
FRACTIONS = (0.0, 0.02, 0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.98, 0.995,
             0.999)


def _case():
    x, y, z, f, w = uniform_cube(20000, seed=61)
    g = SplitMix64(62)
    F = np.stack([f, g.uniform(f.size, -1, 1), g.uniform(f.size, 0, 1)])
    tx, ty, tz, tf, _ = uniform_cube(3000, seed=63)
    tF = np.stack([tf, 0.5 * tf, tf * tf])  # the targets' own values, one row per orbital
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    r = np.sqrt(x * x + y * y + z * z)
    return {"x": dev(x), "y": dev(y), "z": dev(z), "w": dev(w), "F": dev(F),
            "t": (dev(1.5 * tx), dev(1.5 * ty), dev(1.5 * tz), dev(tF)),
            "V": dev(-1.0 / (r + 0.3)), "kap": np.array([0.8, 1.6, 2.4])}


def _steps():
    from paper_2003_01833_amd.selector import Selector
    sel = Selector.load(WEIGHTS) if os.path.exists(WEIGHTS) else None

    def fp64(t, c):
        t.upward(c["F"], c["w"], 6)
        return t.convolve("yukawa_ss", c["kap"], 0.7, 6)

    def mixed(t, c):
        t.upward(c["F"], c["w"], 8)
        return t.convolve("coulomb_ss", c["kap"], 0.8, 8, precision="mixed")

    def targets(t, c):
        t.upward(c["F"], c["w"], 6)
        return t.convolve("yukawa_ss", c["kap"], 0.7, 6, targets=c["t"])

    def green(t, c):
        return t.green_step(c["F"], c["V"], c["w"], -0.5 * c["kap"] ** 2, 0.7, 6)[0]

    def learned(t, c):
        t.upward(c["F"], c["w"], 1)
        tol = 1e-8 * 4 * np.pi / c["kap"] ** 2
        return t.convolve_learned("yukawa_ss", c["kap"], sel, tol, precision="mixed")

    steps = {"fp64": fp64, "mixed": mixed, "targets": targets, "green": green}
    if sel is not None:
        steps["learned"] = learned
    return steps


@pytest.mark.parametrize("kind", ["fp64", "mixed", "targets", "green", "learned"])
def test_workspace_limit_fails_cleanly_and_leaves_the_tree_usable(kind, monkeypatch):
    import paper_2003_01833_amd as tagi
    steps = _steps()
    if kind not in steps:
        pytest.skip("no trained selector weights")
    step = steps[kind]
    c = _case()
    monkeypatch.delenv(LIMIT, raising=False)
    start = tagi.binding.workspace_held()
    t = tagi.Tree(c["x"], c["y"], c["z"], 200)
    built = tagi.binding.workspace_held()
    ref = step(t, c).clone()
    need = tagi.binding.workspace_held() - built
    t.close()
    assert need > 0
    failed = 0
    for q in FRACTIONS:
        t = tagi.Tree(c["x"], c["y"], c["z"], 200)
        h0 = tagi.binding.workspace_held()
        monkeypatch.setenv(LIMIT, str(h0 + int(q * need)))
        with pytest.raises(tagi.TagiError, match=LIMIT):
            step(t, c)
        failed += 1
        monkeypatch.delenv(LIMIT)
        u = step(t, c)
        assert torch.equal(u, ref), (kind, q)
        t.close()
    assert failed == len(FRACTIONS)
    assert tagi.binding.workspace_held() == start


def test_workspace_limit_refuses_a_tree_beyond_it(monkeypatch):
    import paper_2003_01833_amd as tagi
    c = _case()
    start = tagi.binding.workspace_held()
    monkeypatch.setenv(LIMIT, "64K")
    with pytest.raises(tagi.TagiError, match=LIMIT):
        tagi.Tree(c["x"], c["y"], c["z"], 200)
    monkeypatch.setenv(LIMIT, "1G")  # suffixes: 2^30 bytes is plenty here
    t = tagi.Tree(c["x"], c["y"], c["z"], 200)
    t.upward(c["F"], c["w"], 5)
    t.convolve("yukawa_ss", c["kap"], 0.7, 5)
    t.close()
    assert tagi.binding.workspace_held() == start
