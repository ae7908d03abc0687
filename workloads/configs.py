"""Seeded synthetic workloads shaped like the paper's (Sections 4.2, 6.5, 6.6, 7).

Each function returns plain numpy FP64 arrays; nothing here evaluates the
convolution. Recipes:

* ``uniform_cube``: N points uniform in [-1, 1]^3 from SplitMix64(seed); the
  stream is consumed as x_0, y_0, z_0, x_1, ... (3N draws), then f_0..f_{N-1}
  uniform in [-1, 1]; weights w = 8 / N (the cube volume shared equally).
* ``atom_mesh``: Be-like nucleus Z = 4 at the origin in [-20, 20]^3, p = 7 Fejer
  cells (8^3 points per cell), three uniform levels then adaptive refinement on
  the hydrogenic 1s density Z^3/pi exp(-2 Z r) with tol_m = 3e-11 (1968 cells,
  1,007,616 points). Fields: psi_1s + psi_2s for the Yukawa convolution and
  rho = 2 psi_1s^2 + 2 psi_2s^2 for the Hartree (Coulomb) convolution.
* ``benzene_mesh``: C6H6 nuclei at the coordinates printed in the paper
  (Section 7), [-20, 20]^3, p = 7, four uniform levels then refinement with
  tol_m = 5e-4 (8092 cells, 4,143,104 points) on sqrt(rho0) V_ext with a
  hydrogenic stand-in rho0 = sum_a Z_a^3/pi exp(-2 Z_a |r - R_a|) (the paper's
  radial atomic data is not available), atoms moved onto cell vertices.
  Orbitals: for orbital o and atom a, c_{o,a} ~ U[-1, 1] and zeta_{o,a} ~
  U[0.5, 6] from SplitMix64(seed), drawn in the order (o, a, c then zeta);
  psi_o = sum_a c_{o,a} exp(-zeta_{o,a} |r - R_a|). eps_o = -10 (0.02)^(o/20),
  kappa_o = sqrt(-2 eps_o).
"""
from __future__ import annotations

import numpy as np

from .mesh import refine_mesh
from .rng import SplitMix64

DOMAIN = ((-20.0, -20.0, -20.0), (20.0, 20.0, 20.0))


def uniform_cube(n: int = 32768, seed: int = 1):
    g = SplitMix64(seed)
    xyz = g.uniform(3 * n, -1.0, 1.0).reshape(n, 3)
    f = g.uniform(n, -1.0, 1.0)
    w = np.full(n, 8.0 / n)
    return (np.ascontiguousarray(xyz[:, 0]), np.ascontiguousarray(xyz[:, 1]),
            np.ascontiguousarray(xyz[:, 2]), f, w)


def hydrogenic_1s(r, Z):
    return Z ** 1.5 / np.sqrt(np.pi) * np.exp(-Z * r)


def hydrogenic_2s(r, Z):
    return Z ** 1.5 / (2.0 * np.sqrt(2.0 * np.pi)) * (1.0 - Z * r / 2.0) * np.exp(-Z * r / 2.0)


def atom_mesh(Z: float = 4.0, tol_m: float = 3e-11, p: int = 7, uniform_levels: int = 3,
              domain=DOMAIN):
    def rho1s(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        return Z ** 3 / np.pi * np.exp(-2.0 * Z * r)

    mesh = refine_mesh(rho1s, domain[0], domain[1], p, tol_m, uniform_levels=uniform_levels,
                       atoms=[(0.0, 0.0, 0.0)])
    x, y, z, w = mesh.points()
    r = np.sqrt(x * x + y * y + z * z)
    p1, p2 = hydrogenic_1s(r, Z), hydrogenic_2s(r, Z)
    return dict(x=x, y=y, z=z, w=w, psi=p1 + p2, rho=2.0 * p1 * p1 + 2.0 * p2 * p2,
                kappa=float(np.sqrt(0.4)), mesh=mesh, Z=Z)


def diatomic_mesh(Z: float = 4.0, half_sep: float = 1.5, tol_m: float = 1e-10, p: int = 7,
                  uniform_levels: int = 3, domain=DOMAIN):
    """Two Be-like nuclei (charge Z) at (+-half_sep, 0, 0) in [-20, 20]^3, p = 7
    Fejer cells, three uniform levels then refinement on the sum of their
    hydrogenic 1s densities with tol_m, atoms moved onto cell vertices. A small
    multi-centre mesh (about 1.3M points at the defaults) apart from the
    single-atom and benzene workloads."""
    centres = [(-half_sep, 0.0, 0.0), (half_sep, 0.0, 0.0)]

    def rho(x, y, z):
        out = np.zeros_like(x)
        for cx, cy, cz in centres:
            r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
            out += Z ** 3 / np.pi * np.exp(-2.0 * Z * r)
        return out

    mesh = refine_mesh(rho, domain[0], domain[1], p, tol_m, uniform_levels=uniform_levels,
                       atoms=centres)
    x, y, z, w = mesh.points()
    return dict(x=x, y=y, z=z, w=w, mesh=mesh, centres=centres)


BENZENE_C = [(-0.682781, 2.548170, 0.0), (0.682781, -2.548170, 0.0),
             (2.548230, -0.682767, 0.0), (-2.548230, 0.682767, 0.0),
             (1.86544, 1.86541, 0.0), (-1.86544, -1.86541, 0.0)]
BENZENE_H = [(-1.21247, 4.52502, 0.0), (1.21247, -4.52502, 0.0),
             (4.52548, -1.21333, 0.0), (-4.52548, 1.21333, 0.0),
             (3.31252, 3.31351, 0.0), (-3.31252, -3.31351, 0.0)]


def benzene_atoms():
    return [(np.array(c), 6.0) for c in BENZENE_C] + [(np.array(h), 1.0) for h in BENZENE_H]


def molecule_mesh(atoms, tol_m: float = 5e-4, p: int = 7, uniform_levels: int = 4,
                  domain=DOMAIN):
    """Fejer mesh for the nuclei `atoms` ([(R, Z)]) in the domain: refinement on
    sqrt(rho0) v_ext (rho0 the sum of the atoms' hydrogenic 1s densities, v_ext
    their Coulomb potential) with tol_m, nuclei moved onto cell vertices."""
    def test_fn(x, y, z):
        rho0 = np.zeros_like(x)
        vext = np.zeros_like(x)
        for R, Za in atoms:
            d = np.sqrt((x - R[0]) ** 2 + (y - R[1]) ** 2 + (z - R[2]) ** 2)
            rho0 += Za ** 3 / np.pi * np.exp(-2.0 * Za * d)
            vext -= Za / d
        return np.sqrt(rho0) * vext

    mesh = refine_mesh(test_fn, domain[0], domain[1], p, tol_m, uniform_levels=uniform_levels,
                       atoms=[R for R, _ in atoms])
    x, y, z, w = mesh.points()
    return dict(x=x, y=y, z=z, w=w, mesh=mesh, atoms=atoms)


def benzene_mesh(tol_m: float = 5e-4, p: int = 7, uniform_levels: int = 4, domain=DOMAIN):
    return molecule_mesh(benzene_atoms(), tol_m, p, uniform_levels, domain)


def random_molecule(seed: int, n_heavy: int = 3, n_light: int = 3, spread: float = 3.0,
                    min_sep: float = 1.8):
    """n_heavy nuclei of charge 6 and n_light of charge 1 at SplitMix64(seed)
    positions, uniform in [-spread, spread]^3 and at least min_sep apart (draws
    closer to an earlier nucleus are redrawn)."""
    g = SplitMix64(seed)
    atoms = []
    for Z in [6.0] * n_heavy + [1.0] * n_light:
        while True:
            R = g.uniform(3, -spread, spread)
            if all(np.linalg.norm(R - Q) >= min_sep for Q, _ in atoms):
                break
        atoms.append((R, Z))
    return atoms


def molecule_orbitals(atoms, x, y, z, n_orb: int, seed: int):
    """n_orb orbital-like functions on the points: each a sum over the nuclei of
    c exp(-zeta d) with c ~ U[-1, 1] and zeta ~ U[0.5, 6] from SplitMix64(seed),
    and decay rates kappa_o = sqrt(-2 eps_o) with eps log-spaced in [-10, -0.2]."""
    g = SplitMix64(seed)
    coef = np.empty((n_orb, len(atoms)))
    zeta = np.empty((n_orb, len(atoms)))
    for o in range(n_orb):
        for a in range(len(atoms)):
            coef[o, a] = g.uniform(1, -1.0, 1.0)[0]
            zeta[o, a] = g.uniform(1, 0.5, 6.0)[0]
    psi = np.zeros((n_orb, x.size))
    for a, (R, _) in enumerate(atoms):
        d = np.sqrt((x - R[0]) ** 2 + (y - R[1]) ** 2 + (z - R[2]) ** 2)
        for o in range(n_orb):
            psi[o] += coef[o, a] * np.exp(-zeta[o, a] * d)
    eps = -10.0 * 0.02 ** (np.arange(n_orb) / max(n_orb - 1, 1))
    kappa = np.sqrt(-2.0 * eps)
    return dict(psi=psi, kappa=kappa, eps=eps, coef=coef, zeta=zeta)


def benzene_orbitals(x, y, z, n_orb: int = 21, seed: int = 3):
    return molecule_orbitals(benzene_atoms(), x, y, z, n_orb, seed)


def sample_targets(n_total: int, k: int, seed: int = 4) -> np.ndarray:
    """k distinct target indices (sorted) drawn by SplitMix64(seed)."""
    return np.sort(SplitMix64(seed).choice_without_replacement(n_total, k))
