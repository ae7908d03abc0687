"""ORACLE (test infrastructure only): one block step of Green Iteration in plain
numpy FP64.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this.

Algorithm 2 (Section 3) takes one wavefunction at a time; the block step applies
its iteration body to every wavefunction of a block at once, in the paper's
order:

1. psi'_o = G(eps_o) psi_o (Eq. integral_operator with the Green's function of
   Eq. Hemlholtz_Greens_Function): the Yukawa convolution of f_o = V_eff psi_o
   with kappa_o = sqrt(-2 eps_o), scaled by -1/(2 pi). `convolve(f, kappa)`
   supplies the singularity-subtracted sum of Eq. direct-sum_2 (the oracle's
   direct sum, or its treecode), which approximates the integral of
   exp(-kappa |r - r'|) / |r - r'| f(r') dr';
2. the gradient-free eigenvalue update (Eq. gradient-free):
   eps'_o = eps_o - <V_eff psi_o, psi_o - psi'_o> / <psi'_o, psi'_o>, taken with
   psi'_o before orthogonalization;
3. orthogonalize psi'_o against the block's earlier wavefunctions (classical
   Gram-Schmidt, applied twice), in block order;
4. normalize;
5. residual_o = || psi'_o - psi_o ||.

Inner products and norms are the mesh quadrature <a, b> = sum_j w_j a_j b_j
(Eq. quadrature-example).
"""
from __future__ import annotations

import numpy as np


def dot(w, a, b):
    return float(np.sum(w * a * b))


def green_step(w, psi, veff, eps, convolve):
    """psi (n_orb, N), veff (N,), eps (n_orb,); convolve(f, kappa) -> (N,) array.
    Returns (psi_new (n_orb, N), eps_new (n_orb,), residual (n_orb,))."""
    psi = np.atleast_2d(np.asarray(psi, np.float64))
    w = np.asarray(w, np.float64)
    veff = np.asarray(veff, np.float64)
    eps = np.asarray(eps, np.float64)
    n_orb = psi.shape[0]
    new = np.empty_like(psi)
    eps_new = np.empty(n_orb)
    for o in range(n_orb):
        f = veff * psi[o]
        kappa = np.sqrt(-2.0 * eps[o])
        new[o] = -convolve(f, kappa) / (2.0 * np.pi)
        eps_new[o] = eps[o] - dot(w, f, psi[o] - new[o]) / dot(w, new[o], new[o])
    for o in range(n_orb):
        for _ in range(2):
            c = [dot(w, new[j], new[o]) for j in range(o)]
            for j in range(o):
                new[o] -= c[j] * new[j]
        new[o] /= np.sqrt(dot(w, new[o], new[o]))
    resid = np.array([np.sqrt(dot(w, new[o] - psi[o], new[o] - psi[o])) for o in range(n_orb)])
    return new, eps_new, resid
