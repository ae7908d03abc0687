"""ORACLE (test infrastructure only): a plain CPU FP64 barycentric Hermite treecode.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this.

The paper's conclusions (Section 8) propose a treecode based on barycentric Hermite
interpolation (Krasny and Wang, 2019) for the high-accuracy regime, without giving
its form. The form taken here replaces the Lagrange interpolation of Section 6.2
by Hermite interpolation on the same points and keeps everything else of
Algorithm 3 (tree, MAC, near field, subtraction by linearity):

* One dimension, nodes s_0..s_n (Chebyshev points of the second kind mapped to
  the cluster box, as in the Lagrange treecode): the interpolant of g matching
  g and g' at every node is p(t) = sum_k [g(s_k) A_k(t) + g'(s_k) B_k(t)] with
      A_k(t) = (1 - 2 c_k (t - s_k)) L_k(t)^2,   B_k(t) = (t - s_k) L_k(t)^2,
      c_k = L_k'(s_k) = sum_{m != k} 1 / (s_k - s_m),
  L_k the Lagrange basis on the same nodes; it reproduces polynomials of degree
  at most 2n + 1.
* Three dimensions, the tensor product over beta in {0, 1}^3 (H^0 = A, H^1 = B):
      G(x, y) ~ sum_k sum_beta d^beta_y G(x, s_k) prod_d H^{beta_d}_{k_d}(y_d),
  so a cluster's sum becomes sum_k sum_beta d^beta_y G(x_i, s_k) q^_{k,beta} with
  the Hermite proxy charges q^_{k,beta} = sum_j prod_d H^{beta_d}_{k_d}(y_{j,d}) q_j.
* Derivatives with respect to the source point of a radial kernel g(r),
  r = |y - x|, along distinct coordinates:
      d^beta_y g = D_{|beta|}(r) prod_{d in beta} (y_d - x_d),
      D_0 = g,  D_{m+1}(r) = (1/r) dD_m/dr.
  `radial_derivatives` holds D_0..D_3 of e^{-k r}/r, 1/r and e^{-r^2/a^2}/r,
  obtained by applying that recursion by hand.
* The size part of the MAC counts charges: a cluster is approximated only if
  8 (n+1)^3 < N_S, so that the approximation never carries more charges than the
  direct sum has sources (Algorithm 3 compares the (n+1)^3 Lagrange charges with
  N_S the same way).

Here the Lagrange basis is the product formula prod_{m != k} (t - s_m)/(s_k - s_m)
(the plain definition; the GPU uses the barycentric form), and the proxy charges
are formed directly from the particles.
"""
from __future__ import annotations

import numpy as np

from oracle import bltc

# beta index b: bit 0 = derivative in x, bit 1 = in y, bit 2 = in z
BETAS = [((b >> 0) & 1, (b >> 1) & 1, (b >> 2) & 1) for b in range(8)]


def lagrange_product(t, s):
    """L_k(t_j) by the product formula; (len(t), len(s))."""
    t = np.asarray(t, np.float64)
    n1 = s.size
    L = np.ones((t.size, n1))
    for k in range(n1):
        for m in range(n1):
            if m != k:
                L[:, k] *= (t - s[m]) / (s[k] - s[m])
    return L


def hermite_basis(t, s):
    """A_k(t_j), B_k(t_j): each (len(t), len(s)). A zero-extent dimension puts
    all mass on node 0 (A_0 = 1, the rest 0)."""
    t = np.asarray(t, np.float64)
    if s[0] == s[-1]:
        A = np.zeros((t.size, s.size))
        A[:, 0] = 1.0
        return A, np.zeros((t.size, s.size))
    L = lagrange_product(t, s)
    c = np.array([sum(1.0 / (s[k] - s[m]) for m in range(s.size) if m != k)
                  for k in range(s.size)])
    dt = t[:, None] - s[None, :]
    A = (1.0 - 2.0 * c[None, :] * dt) * L * L
    B = dt * L * L
    return A, B


def proxy_charges(px, py, pz, q, lo, hi, n):
    """Hermite proxy charges q^_{k1 k2 k3, beta} for q of shape (m, N_S).
    Returns nodes (3, n+1) and charges (m, n+1, n+1, n+1, 8)."""
    sx, sy, sz = (bltc.cheb2_nodes(lo[d], hi[d], n) for d in range(3))
    H = [hermite_basis(px, sx), hermite_basis(py, sy), hermite_basis(pz, sz)]
    q = np.atleast_2d(q)
    out = np.empty((q.shape[0], n + 1, n + 1, n + 1, 8))
    for b, (bx, by, bz) in enumerate(BETAS):
        out[..., b] = np.einsum("ja,jb,jc,mj->mabc", H[0][bx], H[1][by], H[2][bz], q,
                                optimize=True)
    return np.stack([sx, sy, sz]), out


def radial_derivatives(kind, r, kappa=0.0, alpha=1.0):
    """D_0..D_3 (each shaped like r) of g = e^{-k r}/r ('yukawa'), 1/r ('coulomb')
    or e^{-r^2/a^2}/r ('gauss'), with D_{m+1} = (1/r) dD_m/dr."""
    r = np.asarray(r, np.float64)
    if kind == "yukawa":
        p = kappa * r
        e = np.exp(-p)
        return (e / r,
                -(1.0 + p) * e / r ** 3,
                (3.0 + 3.0 * p + p * p) * e / r ** 5,
                -(15.0 + 15.0 * p + 6.0 * p * p + p ** 3) * e / r ** 7)
    if kind == "coulomb":
        return 1.0 / r, -1.0 / r ** 3, 3.0 / r ** 5, -15.0 / r ** 7
    b = 1.0 / (alpha * alpha)
    E = np.exp(-r * r * b)
    return (E / r,
            -E * (1.0 / r ** 3 + 2.0 * b / r),
            E * (3.0 / r ** 5 + 4.0 * b / r ** 3 + 4.0 * b * b / r),
            -E * (15.0 / r ** 7 + 18.0 * b / r ** 5 + 12.0 * b * b / r ** 3
                  + 8.0 * b ** 3 / r))


def kernel_derivatives(kind, tx, ty, tz, sx, sy, sz, kappa=0.0, alpha=1.0):
    """d^beta_y g(|y - x|) at x = targets, y = sources, for the 8 beta: (8, T, S)."""
    dx = sx[None, :] - tx[:, None]
    dy = sy[None, :] - ty[:, None]
    dz = sz[None, :] - tz[:, None]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    D = radial_derivatives(kind, r, kappa, alpha)
    out = np.empty((8,) + r.shape)
    for b, (bx, by, bz) in enumerate(BETAS):
        f = D[bx + by + bz].copy()
        if bx:
            f *= dx
        if by:
            f *= dy
        if bz:
            f *= dz
        out[b] = f
    return out


def treecode(x, y, z, f, w, kernel: str, kappa, theta: float, degree: int, leaf_size: int,
             alpha: float = 1.0, domain=None, tree=None):
    """u (n_orb, N) in the caller's order, the far field by Hermite interpolation."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    f = np.atleast_2d(np.asarray(f, np.float64))
    w = np.asarray(w, np.float64)
    n_orb, N = f.shape
    kap = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (n_orb,))
    ss = kernel in ("yukawa_ss", "coulomb_ss")
    k1_kind = "yukawa" if kernel.startswith("yukawa") else "coulomb"
    k2_kind = "yukawa" if kernel == "yukawa_ss" else "gauss"
    if tree is None:
        tree = bltc.build_tree(x, y, z, leaf_size, domain)
    perm = tree.perm
    X, Y, Zs, W = x[perm], y[perm], z[perm], w[perm]
    F = f[:, perm]
    Q = F * W[None, :]
    ncoef = 8 * (degree + 1) ** 3
    nodes, fhat, what = {}, {}, {}
    for c in range(tree.n_nodes):
        if tree.count(c) > ncoef:
            b, e = tree.begin[c], tree.end[c]
            qs = np.vstack([Q[:, b:e], W[None, b:e]])
            nd, ch = proxy_charges(X[b:e], Y[b:e], Zs[b:e], qs, tree.lo[c], tree.hi[c], degree)
            nodes[c] = nd
            fhat[c] = ch[:n_orb].reshape(n_orb, -1, 8)
            what[c] = ch[n_orb].reshape(-1, 8)
    batches, far, near = bltc.interaction_lists(tree, theta, degree, ncoef)
    U = np.zeros((n_orb, N))
    for B, fl, nl in zip(batches, far, near):
        b0, b1 = tree.begin[B], tree.end[B]
        tx, ty, tz = X[b0:b1], Y[b0:b1], Zs[b0:b1]
        for o in range(n_orb):
            acc = np.zeros(b1 - b0)
            fi = F[o, b0:b1]
            for C in fl:
                sx, sy, sz = nodes[C]
                gx, gy, gz = (g.reshape(-1) for g in np.meshgrid(sx, sy, sz, indexing="ij"))
                G1 = kernel_derivatives(k1_kind, tx, ty, tz, gx, gy, gz, kap[o], alpha)
                acc += np.einsum("bts,sb->t", G1, fhat[C][o])
                if ss:
                    G2 = kernel_derivatives(k2_kind, tx, ty, tz, gx, gy, gz, kap[o], alpha)
                    acc -= fi * np.einsum("bts,sb->t", G2, what[C])
            for C in nl:
                s0, s1 = tree.begin[C], tree.end[C]
                dx = tx[:, None] - X[None, s0:s1]
                dy = ty[:, None] - Y[None, s0:s1]
                dz = tz[:, None] - Zs[None, s0:s1]
                d2 = dx * dx + dy * dy + dz * dz
                d = np.sqrt(d2)
                zero = d == 0.0
                dsafe = np.where(zero, 1.0, d)
                k1, k2 = bltc._pair_kernel(kernel, dsafe, d2, kap[o], alpha)
                acc += np.where(zero, 0.0, k1) @ Q[o, s0:s1]
                if ss:
                    acc -= fi * (np.where(zero, 0.0, k2) @ W[s0:s1])
            if kernel == "yukawa_ss":
                acc += 4.0 * np.pi * fi / (kap[o] * kap[o])
            elif kernel == "coulomb_ss":
                acc += 2.0 * np.pi * alpha * alpha * fi
            U[o, b0:b1] = acc
    out = np.empty_like(U)
    out[:, perm] = U
    return out
