"""The GPU path at the full sizes and in the launch configurations the benchmark
times, against the oracle's direct sum at seeded sample targets (the oracle
computes each sampled output on its own, over all sources):

* the Be-like atom mesh (1,007,616 points, N_L = 2000): Yukawa-SS and
  Coulomb-SS at the benchmark's stored (theta, n) settings;
* the atom's Hartree (Coulomb-SS) convolution with the learned selector;
* 10,000,000 uniform points, Coulomb kernel, theta 0.7, degree 7 (the accuracy
  the paper reports in Section 6.6, to within a decade);
* the benzene mesh (4,143,104 points, 21 orbitals, N_L = 2000), 10,000 seeded
  targets per orbital against the GPU direct sum, which agrees with the
  oracle's at 300 of them to 1e-12: the batched FP64 step (theta 0.7, n 8), the
  mixed-precision far field (theta 0.8, n 10) and the learned selector in FP64
  and with the mixed far field, which must also need under 60% of the kernel
  evaluations of the fixed MAC it falls back to.

The bar is the accuracy target the settings were chosen for: maximum error over
the samples within 1e-6 of max |u| and relative L2 error within 1e-6, per
orbital. Results must also be bitwise repeatable.
"""
import os

import numpy as np
import pytest
import torch

from oracle.direct import direct_sum
from workloads.configs import DOMAIN, atom_mesh, benzene_mesh, benzene_orbitals, sample_targets
from workloads.settings import load_settings

pytestmark = pytest.mark.gpu

BOX = (*DOMAIN[0], *DOMAIN[1])


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def _errors(u, ref):
    return (np.abs(u - ref).max() / np.abs(ref).max(),
            np.linalg.norm(u - ref) / np.linalg.norm(ref))


def test_atom_mesh_at_the_benchmark_setting():
    import paper_2003_01833_amd as tagi
    d = atom_mesh()
    x, y, z, w = d["x"], d["y"], d["z"], d["w"]
    assert x.size == 1007616
    X, Y, Z, W = _dev(x, y, z, w)
    st = load_settings()["atom"]
    t = tagi.Tree(X, Y, Z, st["leaf_size"], BOX)
    idx = sample_targets(x.size, 200, seed=11)
    for kernel, f, kappa in (("yukawa_ss", d["psi"], d["kappa"]), ("coulomb_ss", d["rho"], 1.0)):
        theta, n = st[kernel]["fp64"]
        (F,) = _dev(f)
        t.upward(F, W, n)
        u = t.convolve(kernel, kappa, theta, n)
        again = t.convolve(kernel, kappa, theta, n)
        assert torch.equal(u, again)
        ref = direct_sum(kernel, x, y, z, f, w, x[idx], y[idx], z[idx], f[idx], kappa=kappa)
        e_max, e_l2 = _errors(u[0].cpu().numpy()[idx], ref)
        assert e_max <= 1e-6 and e_l2 <= 1e-6, (kernel, e_max, e_l2)


def test_atom_hartree_with_the_learned_selector():
    # the Coulomb-SS (Hartree) convolution of the atom's density with the learned
    # degree/MAC selection, at the budget the selector was calibrated for, against
    # the oracle's direct sum; and fewer evaluations than the fixed MAC it falls
    # back to (theta 0.7, n 8)
    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd.selector import Selector
    d = atom_mesh()
    x, y, z, w, rho = d["x"], d["y"], d["z"], d["w"], d["rho"]
    X, Y, Z, W, R = _dev(x, y, z, w, rho)
    t = tagi.Tree(X, Y, Z, 2000, BOX)
    t.upward(R, W, 8)
    u_fix = t.convolve("coulomb_ss", 1.0, 0.7, 8)
    st = t.stats()
    fixed = st["far_interactions"] + st["near_interactions"]
    sel = Selector.load(os.path.join(os.path.dirname(tagi.__file__), "selector_weights.npz"))
    tol = sel.eta("coulomb_ss") * 1e-6 * u_fix.abs().amax(dim=1).cpu().numpy()
    t.upward(R, W, 1)
    u = t.convolve_learned("coulomb_ss", None, sel, tol)
    ls = t.learned_stats()
    idx = sample_targets(x.size, 400, seed=13)
    ref = direct_sum("coulomb_ss", x, y, z, rho, w, x[idx], y[idx], z[idx], rho[idx])
    e_max, e_l2 = _errors(u[0].cpu().numpy()[idx], ref)
    assert e_max <= 1e-6 and e_l2 <= 1e-6, (e_max, e_l2)
    assert len(ls["far_pairs_by_degree"]) >= 2, ls
    assert ls["far_interactions"] + ls["near_interactions"] < fixed, (ls, fixed)


def test_benzene_21_orbitals_batched_mixed_and_learned():
    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd.selector import Selector
    m = benzene_mesh()
    orb = benzene_orbitals(m["x"], m["y"], m["z"])
    x, y, z, w = m["x"], m["y"], m["z"], m["w"]
    psi, kap = orb["psi"], np.asarray(orb["kappa"])
    n_orb = psi.shape[0]
    assert x.size == 4143104 and n_orb == 21
    X, Y, Z, W, F = _dev(x, y, z, w, psi)
    t = tagi.Tree(X, Y, Z, 2000, BOX)
    # 10,000 seeded targets (the benchmark's): the GPU direct sum there, itself
    # checked against the oracle's at 300 of them spread over the sample
    idx = sample_targets(x.size, 10000, seed=4)
    sub = idx[np.linspace(0, idx.size - 1, 300).round().astype(np.int64)]
    pos = np.searchsorted(idx, sub)
    T = [torch.from_numpy(a[idx]).cuda() for a in (x, y, z)]
    refs = []
    for o in range(n_orb):
        g = tagi.direct("yukawa_ss", X, Y, Z, F[o].contiguous(), W, T[0], T[1], T[2],
                        torch.from_numpy(psi[o][idx]).cuda(), kappa=float(kap[o])).cpu().numpy()
        ref = direct_sum("yukawa_ss", x, y, z, psi[o], w, x[sub], y[sub], z[sub], psi[o][sub],
                         kappa=float(kap[o]))
        assert np.abs(g[pos] - ref).max() <= 1e-12 * np.abs(ref).max(), o
        refs.append(g)

    def check(U, label):
        Uh = U.cpu().numpy()[:, idx]
        for o in range(n_orb):
            e_max, e_l2 = _errors(Uh[o], refs[o])
            assert e_max <= 1e-6 and e_l2 <= 1e-6, (label, o, e_max, e_l2)

    t.upward(F, W, 8)
    U64 = t.convolve("yukawa_ss", kap, 0.7, 8)
    check(U64, "batched fp64")
    st = t.stats()
    fixed = st["far_interactions"] + st["near_interactions"]
    t.upward(F, W, 10)
    Um = t.convolve("yukawa_ss", kap, 0.8, 10, precision="mixed")
    check(Um, "batched mixed")
    weights = os.path.join(os.path.dirname(tagi.__file__), "selector_weights.npz")
    sel = Selector.load(weights)
    tol = sel.eta("yukawa_ss") * 1e-6 * U64.abs().amax(dim=1).cpu().numpy()
    t.upward(F, W, 1)
    Ul = t.convolve_learned("yukawa_ss", kap, sel, tol, precision="fp64")
    check(Ul, "learned fp64")
    Ul = t.convolve_learned("yukawa_ss", kap, sel, tol, precision="mixed")
    again = t.convolve_learned("yukawa_ss", kap, sel, tol, precision="mixed")
    assert torch.equal(Ul, again)
    check(Ul, "learned mixed")
    # what the trained network gains over the fixed MAC it falls back to
    # (theta 0.7, n 8), at the same 1e-6 bar: far fewer kernel evaluations
    ls = t.learned_stats()
    learned = ls["far_interactions"] + ls["near_interactions"]
    print(f"benzene learned/fixed kernel evaluations: {learned / fixed:.3f}")
    assert learned < 0.6 * fixed, (learned, fixed)


def test_uniform_10m_coulomb_accuracy_anchor():
    # Section 6.6: 10,000,000 points uniformly random in a cube, Coulomb kernel,
    # theta 0.7, degree 7; the paper reports a relative L2 error of 2.31e-6 against
    # the direct sum. Its charges and N_L are not stated (here f ~ U[-1, 1],
    # w = 8/N on [-1, 1]^3, N_L 2000), so the error has to land within a decade
    # of it; measured against the oracle at 1000 seeded targets.
    import paper_2003_01833_amd as tagi
    from workloads.configs import uniform_cube
    x, y, z, f, w = uniform_cube(10_000_000, seed=6)
    u = tagi.treecode(*_dev(x, y, z, f, w), "coulomb", 1.0, 0.7, 7, 2000)[0]
    idx = sample_targets(x.size, 1000, seed=7)
    ref = direct_sum("coulomb", x, y, z, f, w, x[idx], y[idx], z[idx], f[idx])
    e_max, e_l2 = _errors(u.cpu().numpy()[idx], ref)
    print(f"10M uniform Coulomb theta 0.7 n 7: rel L2 {e_l2:.3e} (paper 2.31e-6), rel max {e_max:.3e}")
    assert 2.31e-7 <= e_l2 <= 2.31e-5, e_l2
