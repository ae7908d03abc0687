"""Trains the degree/MAC selector on the GPU and stores it beside this file.

    python -m paper_2003_01833_amd.train_selector [--pairs 50000] [--epochs 60] [--margin 2]
    python -m paper_2003_01833_amd.train_selector --recalibrate [--margin 2]

1. Samples: the Be-like atom mesh (1,007,616 points), seeds 1..5, each a Slater
   mixture at the nucleus with four kappa values log-uniform in [0.5, 5]
   (Yukawa-SS), and the square of another mixture under the Coulomb-SS kernel;
   per case up to --pairs candidate pairs, each labelled at degrees 4..12
   (about 9 labels per pair). Trees with N_L = 2000, the leaf size of the
   workloads the selector serves (samples, calibration and use alike).
2. Training: one network per kernel family (Yukawa, Coulomb) on that family's
   samples, by tagi_selector_train (FP32 Adam, mini-batches of 4096).
3. Calibration: the budget of one target's sum is tol_o = eta * 1e-6 * max|u_o|
   with u_o the FP64 fixed-MAC result (the list kernel gives each of a batch's
   M_B candidate pairs tol_o / M_B); eta is, per kernel family, the largest of
   a decreasing ladder for which the learned result stays within 1e-6 / 2
   (relative L2 and max) of the direct sum on every held-out case of
   calibration_cases: the atom and a diatomic molecule (every mesh point), and
   two random molecules whose orbital-like functions are built the way the
   benchmark builds its orbitals (20,000 seeded points). None of them is in
   the training data or is the benchmark's molecule.
Writes selector_weights.npz and selector_weights.json (loss history, sample
count, eta, timings).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(HERE, "selector_weights.npz")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


ETAS = (30.0, 10.0, 5.0, 3.0, 2.0, 1.0, 0.5, 0.3, 0.2, 0.1, 0.05, 0.03, 0.02, 0.01, 0.005, 0.003,
        0.001)


MOLECULE_SEEDS = (71, 72)  # held-out random molecules of the calibration
MOLECULE_SAMPLES = 20000   # seeded sample points per molecule for the errors


def calibration_cases(mesh, seed: int = 6, kappas=(0.6, 1.5, 4.0)):
    """The held-out cases of the calibration, none of which the networks were
    trained on: (name, mesh, Yukawa-SS fields [3][n], their kappas, Coulomb-SS
    density [n], sample indices or None for every point).
    * the Be-like atom (the training mesh) and a diatomic molecule (two Be-like
      centres 3 bohr apart): three Slater mixtures about the centres (seed 6) at
      the given kappas, and the square of another as the density; errors at
      every mesh point;
    * random molecules (three carbon-like and three hydrogen-like nuclei at
      seeded positions, their Fejer meshes refined as for benzene): three
      orbital-like functions (sums of signed Slater functions about the nuclei,
      kappa from eps log-spaced in [-10, -0.2]) and the sum of their squares as
      the density; errors at 20,000 seeded points."""
    from paper_2003_01833_amd.selector import centred_field
    from workloads.configs import (diatomic_mesh, molecule_mesh, molecule_orbitals,
                                   random_molecule, sample_targets)
    out = []
    for name, m, centres in (("atom", mesh, [(0.0, 0.0, 0.0)]), ("diatomic", None, None)):
        if m is None:
            m = diatomic_mesh()
            centres = m["centres"]
        F = np.stack([centred_field(m["x"], m["y"], m["z"], centres, 1000 + seed + 10 * k)
                      for k in range(len(kappas))])
        rho = centred_field(m["x"], m["y"], m["z"], centres, 3000 + seed) ** 2
        out.append((name, m, F, np.asarray(kappas, dtype=np.float64), rho, None))
    for ms in MOLECULE_SEEDS:
        m = molecule_mesh(random_molecule(ms))
        orb = molecule_orbitals(m["atoms"], m["x"], m["y"], m["z"], 3, ms + 1)
        rho = (orb["psi"] ** 2).sum(axis=0)
        idx = sample_targets(m["x"].size, MOLECULE_SAMPLES, seed=ms + 2)
        out.append((f"molecule {ms}", m, orb["psi"], orb["kappa"], rho, idx))
    return out


def calibrate(tagi, torch, sel, mesh, leaf: int = 2000, etas=ETAS, target: float = 1e-6,
              margin: float = 2.0):
    """eta per kernel family for the budget tol_o = eta * target * max|u_o| of one
    target's sum (the list kernel divides it by M_B per pair): for each family,
    the largest rung of `etas` at which every held-out case of that family
    (calibration_cases) stays within target / margin (relative L2 and max) of the
    direct sum. The families get their own factor because the networks'
    accuracy differs between them."""
    from workloads.configs import DOMAIN
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    worst = {"yukawa": {e: 0.0 for e in etas}, "coulomb": {e: 0.0 for e in etas}}
    evals = {"yukawa": {e: 0 for e in etas}, "coulomb": {e: 0 for e in etas}}
    names = []
    for name, m, Fh, kap, rhoh, idx_h in calibration_cases(mesh):
        names.append(name)
        x, y, z, w = dev(m["x"]), dev(m["y"]), dev(m["z"]), dev(m["w"])
        F, rho = dev(Fh), dev(rhoh)
        idx = None if idx_h is None else torch.from_numpy(idx_h).cuda()
        pick = (lambda a: a) if idx is None else (lambda a: a[idx].contiguous())  # noqa: E731
        cases = {"yukawa": ("yukawa_ss", F, kap), "coulomb": ("coulomb_ss", rho[None, :].contiguous(), None)}
        t = tagi.Tree(x, y, z, leaf, (*DOMAIN[0], *DOMAIN[1]))
        for fam, (kernel, G, k) in cases.items():
            refs = []
            for o in range(G.shape[0]):
                kw = dict(kappa=1.0 if k is None else float(k[o]))
                if idx is None:
                    refs.append(tagi.direct(kernel, x, y, z, G[o].contiguous(), w, **kw))
                else:
                    refs.append(tagi.direct(kernel, x, y, z, G[o].contiguous(), w, pick(x), pick(y),
                                            pick(z), pick(G[o]), **kw))
            t.upward(G, w, 8)
            um = t.convolve(kernel, 1.0 if k is None else k, 0.7, 8).abs().amax(dim=1).cpu().numpy()
            for eta in etas:
                u = t.convolve_learned(kernel, k, sel, eta * target * um)
                for o in range(G.shape[0]):
                    uo = pick(u[o])
                    worst[fam][eta] = max(
                        worst[fam][eta],
                        float(torch.linalg.norm(uo - refs[o]) / torch.linalg.norm(refs[o])),
                        float((uo - refs[o]).abs().max() / refs[o].abs().max()))
                st = t.learned_stats()
                evals[fam][eta] += st["far_interactions"] + st["near_interactions"]
                _log(f"calibration {name} {fam}: eta {eta}: worst so far {worst[fam][eta]:.3e}")
        t.close()
        del x, y, z, w, F, rho
    log = {fam: [{"eta": e, "worst_rel_err": worst[fam][e], "evaluations": evals[fam][e]}
                 for e in etas] for fam in worst}
    chosen = choose_eta(log, target, margin)
    for fam, e in chosen.items():
        _log(f"calibration {fam}: eta {e}")
    return chosen, log, names


def choose_eta(log, target: float = 1e-6, margin: float = 4.0):
    """Per family, the largest eta of the calibration log whose worst relative
    error over the held-out cases is within target / margin (the smallest eta
    tried if none is)."""
    out = {}
    for fam, rows in log.items():
        ok = [r["eta"] for r in rows if r["worst_rel_err"] <= target / margin]
        out[fam] = max(ok) if ok else min(r["eta"] for r in rows)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=50000)
    ap.add_argument("--kappas-per-seed", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--margin", type=float, default=2.0,
                    help="headroom of the calibration: eta keeps every held-out case within "
                         "1e-6 / margin")
    ap.add_argument("--reselect-eta", type=float, default=None, metavar="MARGIN",
                    help="only recompute eta from the calibration log stored with --out's "
                         "weights, for headroom MARGIN, and rewrite its JSON")
    ap.add_argument("--recalibrate", action="store_true",
                    help="keep --weights' networks and run the calibration again (the cases "
                         "of calibration_cases, headroom --margin); write to --out")
    ap.add_argument("--weights", default=WEIGHTS)
    args = ap.parse_args()
    if args.recalibrate:
        import torch

        import paper_2003_01833_amd as tagi
        from paper_2003_01833_amd.selector import Selector
        from workloads.configs import atom_mesh
        torch.cuda.set_device(0)
        sel = Selector.load(args.weights)
        t0 = time.perf_counter()
        eta, cal, names = calibrate(tagi, torch, sel, atom_mesh(), margin=args.margin)
        sel.meta.update({"eta": eta, "margin": args.margin, "calibration": cal,
                         "calibration_cases": names,
                         "calibration_seconds": time.perf_counter() - t0})
        sel.save(args.out)
        _log(f"saved {args.out} (eta {eta})")
        return
    if args.reselect_eta is not None:
        from paper_2003_01833_amd.selector import Selector
        sel = Selector.load(args.out)
        sel.meta["eta"] = choose_eta(sel.meta["calibration"], 1e-6, args.reselect_eta)
        sel.meta["margin"] = args.reselect_eta
        sel.save(args.out)
        _log(f"eta {sel.meta['eta']} for headroom {args.reselect_eta}")
        return

    import torch

    import paper_2003_01833_amd as tagi
    from paper_2003_01833_amd import selector as S
    from workloads.configs import atom_mesh

    torch.cuda.set_device(0)
    mesh = atom_mesh()
    t0 = time.perf_counter()
    samples = S.make_samples(tagi, torch, pairs=args.pairs, kappas_per_seed=args.kappas_per_seed,
                             mesh=mesh, log=_log)
    t1 = time.perf_counter()
    nets, record = {}, {}
    for fam, (raw, err) in samples.items():
        X, Y, M, norm = S.prepare(raw, err)
        _log(f"samples {fam}: {X.shape[0]} pairs, {int(M.sum())} labels")
        nets[fam], rec = S.train(tagi, torch, X, Y, M, norm, epochs=args.epochs, batch=args.batch,
                                 lr=args.lr, log=_log)
        record[fam] = dict(rec, n_labels=int(M.sum()))
    sel = S.Selector(nets)
    t2 = time.perf_counter()
    held = S.make_samples(tagi, torch, seeds=(6,), kappas_per_seed=2, pairs=args.pairs, mesh=mesh,
                          log=_log)
    rep = {}
    for fam, (raw_h, err_h) in held.items():
        rep[fam] = S.heldout_report(sel.nets[fam], raw_h, err_h)
        _log(f"held-out {fam} pairs (seed 6): predicted - observed log10 error: " +
             ", ".join(f"{k} {v:.3g}" for k, v in rep[fam].items()))
    eta, cal, names = calibrate(tagi, torch, sel, mesh, margin=args.margin)  # per kernel family
    sel.meta.update({"eta": eta, "margin": args.margin, "calibration": cal,
                     "calibration_cases": names, "training": record,
                     "heldout": rep,
                     "sample_seconds": t1 - t0, "train_seconds": t2 - t1,
                     "training_data": "Be-like atom mesh (1,007,616 points), N_L 2000, seeds 1-5: "
                                      f"{args.kappas_per_seed} Yukawa-SS kappas per seed (Yukawa "
                                      "network) and one Coulomb-SS density per seed (Coulomb "
                                      f"network), {args.pairs} pairs per case, theta_max 0.9"})
    sel.save(args.out)
    _log(f"saved {args.out} (eta {eta})")


if __name__ == "__main__":
    main()
