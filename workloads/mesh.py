"""Adaptive cuboid-cell meshes with tensor Fejer quadrature (paper Section 4.2).

Quadrature nodes in each cell are Chebyshev points of the first kind,
x_i = cos((2i+1) pi / (2p+2)), i = 0..p (paper Eq. Chebyshev_points), and the
weights are Fejer's first rule on those p+1 nodes,

    w_i = (2/N) [1 - 2 sum_{m=1}^{floor(N/2)} cos(2 m t_i) / (4 m^2 - 1)],
    N = p + 1, t_i = (2i+1) pi / (2N)

(Waldvogel, BIT 46 (2006)). The rule integrates degree-p polynomials exactly on
[-1, 1]; the tests check that property.

Refinement (paper Section 4.2, Eq. refinement_criterion): starting from the
domain cube, a number of uniform bisection levels is applied; afterwards a cell C
is split into its eight children whenever

    | int_C t  -  sum_i int_{C_i} t | >= tol_m

with both integrals taken by the Fejer rule. After refinement, cells that hold an
atom in their interior are split at the atom so that every atom sits on cell
vertices, and cells whose aspect ratio exceeds ``max_aspect`` are halved along
their longest side until it does not.

This module only builds inputs (points and weights); it holds none of the
treecode arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def cheb1_nodes(p: int) -> np.ndarray:
    i = np.arange(p + 1, dtype=np.float64)
    return np.cos((2.0 * i + 1.0) * np.pi / (2.0 * p + 2.0))


def fejer_weights(p: int) -> np.ndarray:
    n = p + 1
    t = (2.0 * np.arange(n, dtype=np.float64) + 1.0) * np.pi / (2.0 * n)
    s = np.zeros(n)
    for m in range(1, n // 2 + 1):
        s += np.cos(2.0 * m * t) / (4.0 * m * m - 1.0)
    return (2.0 / n) * (1.0 - 2.0 * s)


def cell_points(lo: np.ndarray, hi: np.ndarray, p: int):
    """Tensor Fejer points/weights of cells. lo, hi: (C, 3). Returns x, y, z, w of
    shape (C, (p+1)^3), ordered with the x index slowest."""
    nd = cheb1_nodes(p)
    wd = fejer_weights(p)
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo)
    px = c[:, 0:1] + h[:, 0:1] * nd[None, :]  # (C, p+1)
    py = c[:, 1:2] + h[:, 1:2] * nd[None, :]
    pz = c[:, 2:3] + h[:, 2:3] * nd[None, :]
    wx = h[:, 0:1] * wd[None, :]
    wy = h[:, 1:2] * wd[None, :]
    wz = h[:, 2:3] * wd[None, :]
    q = p + 1
    C = lo.shape[0]
    x = np.broadcast_to(px[:, :, None, None], (C, q, q, q)).reshape(C, -1)
    y = np.broadcast_to(py[:, None, :, None], (C, q, q, q)).reshape(C, -1)
    z = np.broadcast_to(pz[:, None, None, :], (C, q, q, q)).reshape(C, -1)
    w = (wx[:, :, None, None] * wy[:, None, :, None] * wz[:, None, None, :]).reshape(C, -1)
    return x, y, z, w


def _children(lo: np.ndarray, hi: np.ndarray):
    """Eight bisection children of each cell; returns (8C, 3) arrays, children of
    cell c at rows 8c..8c+7."""
    mid = 0.5 * (lo + hi)
    los, his = [], []
    for b in range(8):
        bx, by, bz = (b >> 2) & 1, (b >> 1) & 1, b & 1
        sel = np.array([bx, by, bz], dtype=bool)
        clo = np.where(sel[None, :], mid, lo)
        chi = np.where(sel[None, :], hi, mid)
        los.append(clo)
        his.append(chi)
    lo8 = np.stack(los, axis=1).reshape(-1, 3)
    hi8 = np.stack(his, axis=1).reshape(-1, 3)
    return lo8, hi8


def _integrate(fn, lo, hi, p, chunk=4096):
    out = np.empty(lo.shape[0])
    for s in range(0, lo.shape[0], chunk):
        x, y, z, w = cell_points(lo[s:s + chunk], hi[s:s + chunk], p)
        out[s:s + chunk] = np.sum(fn(x, y, z) * w, axis=1)
    return out


@dataclass
class Mesh:
    lo: np.ndarray  # (C, 3) cell lower corners
    hi: np.ndarray  # (C, 3) cell upper corners
    p: int
    domain: tuple   # (lo3, hi3)

    @property
    def n_cells(self) -> int:
        return self.lo.shape[0]

    @property
    def n_points(self) -> int:
        return self.n_cells * (self.p + 1) ** 3

    def points(self):
        """Flat x, y, z, w arrays (cell-major order)."""
        x, y, z, w = cell_points(self.lo, self.hi, self.p)
        return (np.ascontiguousarray(x.reshape(-1)), np.ascontiguousarray(y.reshape(-1)),
                np.ascontiguousarray(z.reshape(-1)), np.ascontiguousarray(w.reshape(-1)))


def refine_mesh(test_fn, domain_lo, domain_hi, p: int, tol_m: float,
                uniform_levels: int = 3, max_level: int = 40, atoms=(),
                max_aspect: float = 2.0) -> Mesh:
    lo = np.array([domain_lo], dtype=np.float64)
    hi = np.array([domain_hi], dtype=np.float64)
    for _ in range(uniform_levels):
        lo, hi = _children(lo, hi)
    done_lo, done_hi = [], []
    level = uniform_levels
    while lo.shape[0] and level < max_level:
        parent_int = _integrate(test_fn, lo, hi, p)
        clo, chi = _children(lo, hi)
        child_int = _integrate(test_fn, clo, chi, p).reshape(-1, 8).sum(axis=1)
        refine = np.abs(parent_int - child_int) >= tol_m
        done_lo.append(lo[~refine])
        done_hi.append(hi[~refine])
        sel = np.repeat(refine, 8)
        lo, hi = clo[sel], chi[sel]
        level += 1
    done_lo.append(lo)
    done_hi.append(hi)
    lo = np.concatenate(done_lo)
    hi = np.concatenate(done_hi)
    # atoms on cell vertices: a cell whose closed box holds an atom is split at the
    # atom along every dimension in which the atom is strictly interior
    for a in atoms:
        a = np.asarray(a, dtype=np.float64)
        touch = np.all((lo <= a[None, :]) & (a[None, :] <= hi), axis=1)
        interior = (lo < a[None, :]) & (a[None, :] < hi)  # (C, 3)
        m = touch & np.any(interior, axis=1)
        if not np.any(m):
            continue
        new_lo, new_hi = [lo[~m]], [hi[~m]]
        for c in np.nonzero(m)[0]:
            dims = [d for d in range(3) if interior[c, d]]
            for b in range(1 << len(dims)):
                clo, chi = lo[c].copy(), hi[c].copy()
                for k, d in enumerate(dims):
                    if (b >> k) & 1:
                        clo[d] = a[d]
                    else:
                        chi[d] = a[d]
                new_lo.append(clo[None, :])
                new_hi.append(chi[None, :])
        lo = np.concatenate(new_lo)
        hi = np.concatenate(new_hi)
    # aspect-ratio repair: halve the longest side while the ratio is too large
    while True:
        ext = hi - lo
        ratio = ext.max(axis=1) / ext.min(axis=1)
        bad = ratio > max_aspect
        if not np.any(bad):
            break
        d = np.argmax(ext[bad], axis=1)
        blo, bhi = lo[bad], hi[bad]
        mid = 0.5 * (blo[np.arange(d.size), d] + bhi[np.arange(d.size), d])
        a_lo, a_hi = blo.copy(), bhi.copy()
        b_lo, b_hi = blo.copy(), bhi.copy()
        a_hi[np.arange(d.size), d] = mid
        b_lo[np.arange(d.size), d] = mid
        lo = np.concatenate([lo[~bad], a_lo, b_lo])
        hi = np.concatenate([hi[~bad], a_hi, b_hi])
    # deterministic order: sort cells by (lo z, lo y, lo x, hi ...)
    order = np.lexsort((hi[:, 2], hi[:, 1], hi[:, 0], lo[:, 2], lo[:, 1], lo[:, 0]))
    return Mesh(lo=lo[order].copy(), hi=hi[order].copy(), p=p,
                domain=(tuple(domain_lo), tuple(domain_hi)))
