"""ORACLE (test infrastructure only): adaptive cuboid cells with tensor Fejer
quadrature (Section 4.2), cell by cell in plain Python and numpy FP64.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this.

Steps in the paper's order:

1. Level 0 is the domain box; `uniform_levels` rounds bisect every cell in x, y
   and z into eight children (child b has the upper half in x iff bit 2 of b is
   set, in y iff bit 1, in z iff bit 0).
2. Adaptive rounds: for each cell C of the current level, the eight children
   C_i are formed and C is replaced by them iff
   |int_C t - sum_i int_{C_i} t| >= tol_m (Eq. refinement_criterion), both sides
   by the Fejer rule; otherwise C is final. Rounds stop when no cell is split or
   at `max_level`.
3. A final cell holding an atom strictly inside along some dimension is split at
   the atom along those dimensions, so the atom lies on cell vertices.
4. A cell whose longest side exceeds `max_aspect` times its shortest is halved
   along its longest side, repeatedly.

Quadrature (Eq. Chebyshev_points, and Fejer's first rule, Waldvogel, BIT 46
(2006)): on [-1, 1] the nodes are s_i = cos((2i+1) pi / (2p+2)), i = 0..p, with
weights v_i = (2/N) (1 - 2 sum_{m=1}^{floor(N/2)} cos(2 m t_i) / (4 m^2 - 1)),
N = p + 1, t_i = (2i+1) pi / (2N); a cell [lo, hi] maps them to
c + h s_i with weight h v_i per dimension (c = (lo+hi)/2, h = (hi-lo)/2), the
x index slowest. Test functions: `density_test` (sum of hydrogenic 1s densities
Z^3/pi exp(-2 Z d)) and `paper_test` (Eq. test_function with that density as
rho0 and V_ext = -sum_a Z_a / d_a).
"""
from __future__ import annotations

import math

import numpy as np


def nodes_weights(p):
    N = p + 1
    s = np.array([math.cos((2 * i + 1) * math.pi / (2 * p + 2)) for i in range(N)])
    v = np.empty(N)
    for i in range(N):
        t = (2 * i + 1) * math.pi / (2 * N)
        acc = 0.0
        for m in range(1, N // 2 + 1):
            acc += math.cos(2 * m * t) / (4 * m * m - 1)
        v[i] = (2.0 / N) * (1.0 - 2.0 * acc)
    return s, v


def cell_rule(lo, hi, p):
    """Points (q^3,) x, y, z and weights of one cell, x index slowest."""
    s, v = nodes_weights(p)
    c = [0.5 * (lo[d] + hi[d]) for d in range(3)]
    h = [0.5 * (hi[d] - lo[d]) for d in range(3)]
    px, py, pz = (c[d] + h[d] * s for d in range(3))
    wx, wy, wz = (h[d] * v for d in range(3))
    q = p + 1
    x = np.repeat(px, q * q)
    y = np.tile(np.repeat(py, q), q)
    z = np.tile(pz, q * q)
    w = ((wx[:, None] * wy[None, :])[:, :, None] * wz[None, None, :]).reshape(-1)
    return x, y, z, w


def density_test(atoms):
    def t(x, y, z):
        out = np.zeros_like(x)
        for (ax, ay, az), Z in atoms:
            d = np.sqrt((x - ax) ** 2 + (y - ay) ** 2 + (z - az) ** 2)
            out += Z ** 3 / np.pi * np.exp(-2.0 * Z * d)
        return out
    return t


def paper_test(atoms):
    def t(x, y, z):
        rho0 = np.zeros_like(x)
        vext = np.zeros_like(x)
        for (ax, ay, az), Z in atoms:
            d = np.sqrt((x - ax) ** 2 + (y - ay) ** 2 + (z - az) ** 2)
            rho0 += Z ** 3 / np.pi * np.exp(-2.0 * Z * d)
            vext -= Z / d
        return np.sqrt(rho0) * vext
    return t


def integral(t, lo, hi, p):
    x, y, z, w = cell_rule(lo, hi, p)
    return float(np.sum(t(x, y, z) * w))


def children(lo, hi):
    mid = [0.5 * (lo[d] + hi[d]) for d in range(3)]
    out = []
    for b in range(8):
        bits = ((b >> 2) & 1, (b >> 1) & 1, b & 1)
        clo = tuple(mid[d] if bits[d] else lo[d] for d in range(3))
        chi = tuple(hi[d] if bits[d] else mid[d] for d in range(3))
        out.append((clo, chi))
    return out


def build(t, domain_lo, domain_hi, p, tol_m, uniform_levels=3, max_level=40, atoms=(),
          max_aspect=2.0):
    """Final cells as a list of (lo, hi) tuples, sorted by (lo x, lo y, lo z, hi x, ...)."""
    level_cells = [(tuple(map(float, domain_lo)), tuple(map(float, domain_hi)))]
    for _ in range(uniform_levels):
        level_cells = [ch for lo, hi in level_cells for ch in children(lo, hi)]
    final = []
    level = uniform_levels
    while level_cells and level < max_level:
        nxt = []
        for lo, hi in level_cells:
            kids = children(lo, hi)
            whole = integral(t, lo, hi, p)
            parts = sum(integral(t, clo, chi, p) for clo, chi in kids)
            if abs(whole - parts) >= tol_m:
                nxt.extend(kids)
            else:
                final.append((lo, hi))
        level_cells = nxt
        level += 1
    final.extend(level_cells)
    for a in atoms:
        a = tuple(map(float, a))
        out = []
        for lo, hi in final:
            inside = all(lo[d] <= a[d] <= hi[d] for d in range(3))
            dims = [d for d in range(3) if lo[d] < a[d] < hi[d]]
            if not (inside and dims):
                out.append((lo, hi))
                continue
            for b in range(1 << len(dims)):
                clo, chi = list(lo), list(hi)
                for k, d in enumerate(dims):
                    if (b >> k) & 1:
                        clo[d] = a[d]
                    else:
                        chi[d] = a[d]
                out.append((tuple(clo), tuple(chi)))
        final = out
    changed = True
    while changed:
        changed = False
        out = []
        for lo, hi in final:
            ext = [hi[d] - lo[d] for d in range(3)]
            if max(ext) / min(ext) > max_aspect:
                d = int(np.argmax(ext))
                mid = 0.5 * (lo[d] + hi[d])
                a_hi, b_lo = list(hi), list(lo)
                a_hi[d] = mid
                b_lo[d] = mid
                out.append((lo, tuple(a_hi)))
                out.append((tuple(b_lo), hi))
                changed = True
            else:
                out.append((lo, hi))
        final = out
    final.sort(key=lambda c: (c[0][0], c[0][1], c[0][2], c[1][0], c[1][1], c[1][2]))
    return final


def points(cells, p):
    """Flat x, y, z, w of all cells in order."""
    parts = [cell_rule(lo, hi, p) for lo, hi in cells]
    return tuple(np.concatenate([q[k] for q in parts]) for k in range(4))
