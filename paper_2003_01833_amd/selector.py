"""Learned degree/MAC selector: training data, training and storage.

The network (5 -> 64 -> 64 -> 64 -> 9, tanh) predicts, for a batch-cluster pair,
log10 of the largest absolute error of the barycentric approximation at degrees
4..12. Its training data comes from the method itself (tagi_selector_samples on
Be-like atom meshes with seeded Slater mixtures and kappa values); training runs
on the GPU through tagi_selector_train. tagi_convolve_learned then picks, per
pair, the lowest degree whose predicted error fits the pair's error budget.

Feature transform (both here and in the list kernel): x_k = (ln raw_k - shift_k)
* scale_k with raw = (r_C, R - r_B, kappa, N_S, l1 norm of the degree-4 proxy
charges); shift/scale standardise the training set; lo/hi are the training range
of ln raw, outside which the list kernel falls back to the fixed MAC.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

from workloads.configs import DOMAIN, atom_mesh
from workloads.rng import SplitMix64

N_IN, N_OUT = 5, 9
DEGREES = tuple(range(4, 13))
LOG_FLOOR = -30.0


@dataclass
class Selector:
    params: np.ndarray          # float32 [param_count]
    norm: np.ndarray            # float32 [20] = shift, scale, lo, hi
    meta: dict = field(default_factory=dict)

    def save(self, path: str):
        np.savez(path, params=self.params.astype(np.float32), norm=self.norm.astype(np.float32))
        with open(os.path.splitext(path)[0] + ".json", "w") as fh:
            json.dump(self.meta, fh, indent=1, sort_keys=True)

    @staticmethod
    def load(path: str) -> "Selector":
        with np.load(path, allow_pickle=False) as z:
            params, norm = z["params"].copy(), z["norm"].copy()
        meta = {}
        mp = os.path.splitext(path)[0] + ".json"
        if os.path.exists(mp):
            with open(mp) as fh:
                meta = json.load(fh)
        return Selector(params, norm, meta)


def log_features(raw: np.ndarray) -> np.ndarray:
    """ln of the raw features, with the distance and the l1 norm floored as the
    list kernel floors them."""
    r = np.array(raw, dtype=np.float64, copy=True)
    r[:, 1] = np.maximum(r[:, 1], 1e-12)
    r[:, 4] = np.maximum(r[:, 4], 1e-30)
    return np.log(r).astype(np.float32)


def init_params(n_params: int, seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases, in the library's flat layout."""
    g = SplitMix64(seed)
    sizes = (N_IN, 64, 64, 64, N_OUT)
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        out.append((g.uniform(a * b) * 2.0 - 1.0) * lim)
        out.append(np.zeros(b))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == n_params
    return p


def slater_field(r: np.ndarray, seed: int, terms: int = 3):
    """sum_m c_m exp(-zeta_m r), c ~ U[-1, 1], zeta ~ U[0.5, 6] from SplitMix64(seed)."""
    g = SplitMix64(seed)
    f = np.zeros_like(r)
    for _ in range(terms):
        c = g.uniform(1, -1.0, 1.0)[0]
        z = g.uniform(1, 0.5, 6.0)[0]
        f += c * np.exp(-z * r)
    return f


def make_samples(tagi, torch, seeds=(1, 2, 3, 4, 5), kappas_per_seed: int = 4,
                 pairs: int = 50000, theta_max: float = 0.9, leaf: int = 500, mesh=None,
                 log=print):
    """Training data on the Be-like mesh: per seed a Slater mixture at the nucleus
    and kappa values log-uniform in [0.5, 5]. Returns (raw features, errors)."""
    d = mesh if mesh is not None else atom_mesh()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    x, y, z, w = dev(d["x"]), dev(d["y"]), dev(d["z"]), dev(d["w"])
    r = np.sqrt(d["x"] ** 2 + d["y"] ** 2 + d["z"] ** 2)
    t = tagi.Tree(x, y, z, leaf, (*DOMAIN[0], *DOMAIN[1]))
    feats, errs = [], []
    for seed in seeds:
        f = dev(slater_field(r, 1000 + seed))
        g = SplitMix64(2000 + seed)
        for _ in range(kappas_per_seed):
            kappa = float(np.exp(g.uniform(1, np.log(0.5), np.log(5.0))[0]))
            fe, er = t.selector_samples(f, w, kappa, theta_max, pairs)
            feats.append(fe)
            errs.append(er)
            log(f"selector samples: seed {seed} kappa {kappa:.3f}: {fe.shape[0]} pairs")
    t.close()
    return np.concatenate(feats), np.concatenate(errs)


def prepare(raw: np.ndarray, errors: np.ndarray):
    """(X, Y, M, norm): standardised log features, log10 errors, mask of existing labels."""
    L = log_features(raw)
    shift = L.mean(axis=0)
    scale = 1.0 / np.maximum(L.std(axis=0), 1e-6)
    lo, hi = L.min(axis=0), L.max(axis=0)
    X = ((L - shift) * scale).astype(np.float32)
    M = np.isfinite(errors).astype(np.float32)
    Y = np.where(M > 0, np.log10(np.maximum(np.nan_to_num(errors, nan=1.0), 1e-30)), 0.0)
    Y = np.maximum(Y, LOG_FLOOR).astype(np.float32)
    norm = np.concatenate([shift, scale, lo, hi]).astype(np.float32)
    return X, Y, M, norm


def train(tagi, torch, X, Y, M, norm, epochs: int = 30, batch: int = 4096, lr: float = 2e-3,
          seed: int = 7, log=print) -> Selector:
    n_par = tagi.binding.selector_param_count()
    params = torch.from_numpy(init_params(n_par, seed)).cuda()
    dX, dY, dM = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, Y, M))
    g = SplitMix64(seed + 1)
    order = np.argsort(g.uniform(X.shape[0])).astype(np.int32)
    hist = tagi.binding.selector_train(params, dX, dY, dM, order, epochs, batch, lr)
    log(f"selector training: loss {hist[0]:.4f} -> {hist[-1]:.4f} over {epochs} epochs")
    return Selector(params.cpu().numpy(), norm, {"loss_history": [float(v) for v in hist],
                                                 "n_samples": int(X.shape[0]),
                                                 "epochs": epochs, "batch": batch, "lr": lr})
