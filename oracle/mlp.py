"""ORACLE (test infrastructure only): the degree/MAC selector network in plain
numpy FP64, to check the GPU training and inference kernels against.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this.

Network: 5 inputs -> three hidden layers of 64 tanh units -> 9 linear outputs.
Layer l computes h_{l+1} = tanh(W_l h_l + b_l) (the last layer without tanh).
Loss of a mini-batch of m samples with targets y (m, 9) and a mask M (m, 9) of
the entries that exist, with residual r = out - y and weight a(r) = 1 for r >= 0
and UNDER = 4 for r < 0 (predicting below the observed error costs more):
  L = sum(M a(r) r^2) / (2 sum(M)).
Adam (Kingma and Ba, 2015): with gradient g at step t,
  m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
  p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

SIZES = (5, 64, 64, 64, 9)
UNDER = 4.0


def init_params(seed_uniform, sizes=SIZES):
    """Weights W_l (out, in) ~ U[-1, 1] * sqrt(6 / (in + out)) (Glorot), b_l = 0.
    seed_uniform(n) must return n uniforms in [0, 1)."""
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        W = (seed_uniform(a * b).reshape(b, a) * 2.0 - 1.0) * lim
        params += [W, np.zeros(b)]
    return params


def forward(params, X):
    """Returns the output (m, 9) and the activations needed by backward."""
    acts = [np.asarray(X, dtype=np.float64)]
    h = acts[0]
    n_layers = len(params) // 2
    for l in range(n_layers):
        W, b = params[2 * l], params[2 * l + 1]
        z = h @ W.T + b
        h = np.tanh(z) if l < n_layers - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grads(params, X, Y, M):
    out, acts = forward(params, X)
    cnt = M.sum()
    r = (out - Y) * M
    a = np.where(r < 0.0, UNDER, 1.0)
    loss = 0.5 * np.sum(a * r * r) / cnt
    g = a * r / cnt  # dL/dout
    grads = [None] * len(params)
    n_layers = len(params) // 2
    for l in range(n_layers - 1, -1, -1):
        W = params[2 * l]
        h_in = acts[l]
        grads[2 * l] = g.T @ h_in
        grads[2 * l + 1] = g.sum(axis=0)
        if l > 0:
            g = (g @ W) * (1.0 - h_in * h_in)  # tanh' = 1 - tanh^2
    return loss, grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update; state = dict(t=int, m=list, v=list)."""
    if not state:
        state.update(t=0, m=[np.zeros_like(p) for p in params], v=[np.zeros_like(p) for p in params])
    state["t"] += 1
    t = state["t"]
    for p, g, m, v in zip(params, grads, state["m"], state["v"]):
        m *= b1
        m += (1 - b1) * g
        v *= b2
        v += (1 - b2) * g * g
        p -= lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return params
