"""Learned degree/MAC selector: training data, training and storage.

A network (5 -> 64 -> 64 -> 64 -> 9, tanh) predicts, for a batch-cluster pair,
log10 of the largest absolute error of the barycentric approximation at degrees
4..12. There is one network per kernel family (Yukawa, Coulomb), each trained
on its own family's data, which comes from the method itself
(tagi_selector_samples on Be-like atom meshes with seeded Slater mixtures and
kappa values, and squared mixtures for the Coulomb family); training runs on the
GPU through tagi_selector_train. tagi_convolve_learned then picks, per pair, the
lowest degree whose predicted error fits the pair's error budget.

Feature transform (both here and in the list kernel): x_k = (ln(raw_k + o_k) -
shift_k) * scale_k with raw = (r_C, R - r_B, c, N_S, l1), c the kernel's decay
rate (kappa for Yukawa, 0 for Coulomb: 1/r is the kappa -> 0 limit of
exp(-kappa r)/r), o = (0, 0, 0.25, 0, 0) so that c = 0 stays finite, and l1 the
size of the degree-4 charges q^_k - f_i w^_k the pair's far field carries
(l1(q^) + g max_B |f| l1(w^), g = 1 for Yukawa-SS, the Gaussian at the least
batch-cluster distance for Coulomb-SS); shift/scale standardise the
training set; lo/hi are the training range of the log features, outside which
the list kernel falls back to the fixed MAC.

Target: the network learns the residual log10(error) - s with the pair scale
s = log10(l1) - c d log10(e) - log10(d), d = R - r_B, i.e. the error relative
to the size l1 exp(-c d) / d of the far field the pair contributes; the list
kernel adds s back before comparing with the pair budget.
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
DECAY_OFFSET = 0.25  # added to the decay rate c before its logarithm
RANGE_PAD = 1e-3     # log units added on both sides of the training range


FAMILIES = ("yukawa", "coulomb")


def family(kernel: str) -> str:
    """The kernel family whose network and budget a kernel uses."""
    return "coulomb" if kernel.startswith("coulomb") else "yukawa"


@dataclass
class Network:
    params: np.ndarray          # float32 [param_count]
    norm: np.ndarray            # float32 [20] = shift, scale, lo, hi


@dataclass
class Selector:
    """One network per kernel family (Yukawa, Coulomb), each trained on its own
    family's samples, and the calibrated budget factors (meta["eta"])."""
    nets: dict                  # family -> Network
    meta: dict = field(default_factory=dict)

    @staticmethod
    def single(params, norm, meta=None) -> "Selector":
        """The same network for every family."""
        net = Network(np.asarray(params, np.float32), np.asarray(norm, np.float32))
        return Selector({f: net for f in FAMILIES}, meta or {})

    def net(self, kernel: str) -> Network:
        return self.nets[family(kernel)]

    def save(self, path: str):
        arrays = {}
        for f, n in self.nets.items():
            arrays[f"params_{f}"] = n.params.astype(np.float32)
            arrays[f"norm_{f}"] = n.norm.astype(np.float32)
        np.savez(path, **arrays)
        with open(os.path.splitext(path)[0] + ".json", "w") as fh:
            json.dump(self.meta, fh, indent=1, sort_keys=True)

    def eta(self, kernel: str) -> float:
        """The calibrated budget factor for a kernel family: tol_o = eta * 1e-6 *
        max|u_o| is the error budget of one target's sum."""
        return float(self.meta["eta"][family(kernel)])

    @staticmethod
    def load(path: str) -> "Selector":
        with np.load(path, allow_pickle=False) as z:
            nets = {f: Network(z[f"params_{f}"].copy(), z[f"norm_{f}"].copy())
                    for f in FAMILIES if f"params_{f}" in z}
        meta = {}
        mp = os.path.splitext(path)[0] + ".json"
        if os.path.exists(mp):
            with open(mp) as fh:
                meta = json.load(fh)
        return Selector(nets, meta)


def log_features(raw: np.ndarray) -> np.ndarray:
    """ln of the raw features, with the distance and the l1 norm floored as the
    list kernel floors them."""
    r = np.array(raw, dtype=np.float64, copy=True)
    r[:, 1] = np.maximum(r[:, 1], 1e-12)
    r[:, 2] = r[:, 2] + DECAY_OFFSET
    r[:, 4] = np.maximum(r[:, 4], 1e-30)
    return np.log(r).astype(np.float32)


def pair_scale(raw: np.ndarray) -> np.ndarray:
    """log10 of l1 exp(-c d) / d, d = R - r_B, c the decay rate, per sample
    (floored as in log_features)."""
    d = np.maximum(np.asarray(raw[:, 1], dtype=np.float64), 1e-12)
    l1 = np.maximum(np.asarray(raw[:, 4], dtype=np.float64), 1e-30)
    c = np.asarray(raw[:, 2], dtype=np.float64)
    return np.log10(l1) - c * d * np.log10(np.e) - np.log10(d)


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


def centred_field(x, y, z, centres, seed: int):
    """A Slater mixture (slater_field) about each centre, seed + 97 c for centre c,
    summed: a multi-centre orbital-like function."""
    f = np.zeros_like(x)
    for c, (cx, cy, cz) in enumerate(centres):
        r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
        f += slater_field(r, seed + 97 * c)
    return f


def make_samples(tagi, torch, seeds=(1, 2, 3, 4, 5), kappas_per_seed: int = 4,
                 pairs: int = 50000, theta_max: float = 0.9, leaf: int = 2000, mesh=None,
                 coulomb: bool = True, log=print):
    """Training data on the Be-like mesh: per seed a Slater mixture at the nucleus
    with kappa values log-uniform in [0.5, 5] (Yukawa-SS), and, with `coulomb`,
    the square of another mixture (a density) under the Coulomb-SS kernel with
    the Gaussian width 1. Returns {family: (raw features, errors)}."""
    d = mesh if mesh is not None else atom_mesh()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    x, y, z, w = dev(d["x"]), dev(d["y"]), dev(d["z"]), dev(d["w"])
    r = np.sqrt(d["x"] ** 2 + d["y"] ** 2 + d["z"] ** 2)
    t = tagi.Tree(x, y, z, leaf, (*DOMAIN[0], *DOMAIN[1]))
    feats, errs, cf, ce = [], [], [], []
    for seed in seeds:
        f = dev(slater_field(r, 1000 + seed))
        g = SplitMix64(2000 + seed)
        for _ in range(kappas_per_seed):
            kappa = float(np.exp(g.uniform(1, np.log(0.5), np.log(5.0))[0]))
            fe, er = t.selector_samples(f, w, kappa, theta_max, pairs)
            feats.append(fe)
            errs.append(er)
            log(f"selector samples: seed {seed} kappa {kappa:.3f}: {fe.shape[0]} pairs")
        if coulomb:
            rho = dev(slater_field(r, 3000 + seed) ** 2)
            fe, er = t.selector_samples(rho, w, 0.0, theta_max, pairs, kernel="coulomb_ss",
                                        alpha=1.0)
            cf.append(fe)
            ce.append(er)
            log(f"selector samples: seed {seed} Coulomb-SS density: {fe.shape[0]} pairs")
    t.close()
    out = {"yukawa": (np.concatenate(feats), np.concatenate(errs))}
    if cf:
        out["coulomb"] = (np.concatenate(cf), np.concatenate(ce))
    return out


def prepare(raw: np.ndarray, errors: np.ndarray):
    """(X, Y, M, norm): standardised log features, residual log10 errors (over
    pair_scale), mask of the labels that exist and are nonzero."""
    L = log_features(raw)
    shift = L.mean(axis=0)
    sd = L.std(axis=0)
    # a feature constant over the training set (the decay rate of the Coulomb
    # family) gets scale 0: the network sees 0 there whatever its rounding
    scale = np.where(sd > 1e-3, 1.0 / np.maximum(sd, 1e-3), 0.0)
    # the training range, widened by RANGE_PAD so that the extreme values of the
    # training set itself (the Coulomb decay rate 0 is the lower end of the third
    # feature) lie inside it whether the list kernel rounds them in FP32 or the
    # FP64 reference does
    lo, hi = L.min(axis=0) - RANGE_PAD, L.max(axis=0) + RANGE_PAD
    X = ((L - shift) * scale).astype(np.float32)
    err = np.nan_to_num(np.asarray(errors, dtype=np.float64), nan=0.0)
    M = (np.isfinite(errors) & (err > 0.0)).astype(np.float32)
    Y = np.log10(np.maximum(err, 1e-300)) - pair_scale(raw)[:, None]
    Y = np.where(M > 0, np.maximum(Y, LOG_FLOOR), 0.0).astype(np.float32)
    norm = np.concatenate([shift, scale, lo, hi]).astype(np.float32)
    return X, Y, M, norm


def predict_log_error(sel: "Network", raw: np.ndarray) -> np.ndarray:
    """log10 error the list kernel would predict at degrees 4..12 for raw features
    (network output plus pair_scale), evaluated in FP64 on the host; for reports."""
    n_in = N_IN
    norm = sel.norm.astype(np.float64)
    h = (log_features(raw).astype(np.float64) - norm[:n_in]) * norm[n_in:2 * n_in]
    p = sel.params.astype(np.float64)
    off = 0
    sizes = (N_IN, 64, 64, 64, N_OUT)
    for li, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
        W = p[off:off + a * b].reshape(b, a)
        off += a * b
        bias = p[off:off + b]
        off += b
        h = h @ W.T + bias
        if li < len(sizes) - 2:
            h = np.tanh(h)
    return h + pair_scale(raw)[:, None]


def heldout_report(sel: "Network", raw: np.ndarray, errors: np.ndarray) -> dict:
    """How the predicted log10 error compares with the observed one on held-out pairs:
    quantiles of predicted - observed, and the fraction under-predicted by more
    than 2x and 10x."""
    pred = predict_log_error(sel, raw)
    err = np.nan_to_num(np.asarray(errors, dtype=np.float64), nan=0.0)
    ok = np.isfinite(errors) & (err > 0.0)
    d = (pred - np.log10(np.maximum(err, 1e-300)))[ok]
    q = np.quantile(d, [0.001, 0.01, 0.1, 0.5, 0.9]) if d.size else np.zeros(5)
    return {"labels": int(d.size), "q0.001": float(q[0]), "q0.01": float(q[1]),
            "q0.1": float(q[2]), "median": float(q[3]), "q0.9": float(q[4]),
            "under_2x": float(np.mean(d < -np.log10(2.0))) if d.size else 0.0,
            "under_10x": float(np.mean(d < -1.0)) if d.size else 0.0}


def train(tagi, torch, X, Y, M, norm, epochs: int = 30, batch: int = 4096, lr: float = 2e-3,
          seed: int = 7, log=print):
    """(Network, training record) from mini-batch Adam on the GPU."""
    n_par = tagi.binding.selector_param_count()
    params = torch.from_numpy(init_params(n_par, seed)).cuda()
    dX, dY, dM = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, Y, M))
    g = SplitMix64(seed + 1)
    order = np.argsort(g.uniform(X.shape[0])).astype(np.int32)
    hist = tagi.binding.selector_train(params, dX, dY, dM, order, epochs, batch, lr)
    log(f"selector training: loss {hist[0]:.4f} -> {hist[-1]:.4f} over {epochs} epochs")
    return Network(params.cpu().numpy(), norm), {"loss_history": [float(v) for v in hist],
                                                 "n_samples": int(X.shape[0]),
                                                 "epochs": epochs, "batch": batch, "lr": lr}
