"""ORACLE (test infrastructure only): closed-form convolutions that pin the oracle.

All are exact values of the continuous integrals u(r) = int G(|r - r'|) f(r') dr'
for radial f, which the discrete sums of Section 6 (Eq. direct-sum) approximate
to within the mesh's discretization error.

* Hartree potential of the hydrogenic density rho = Z^3/pi exp(-2 Z r)
  (Coulomb kernel): V(r) = 1/r - (1/r + Z) exp(-2 Z r), V(0) = Z.
* Yukawa convolution of exp(-a r) with G = exp(-k r)/r (k != a): u solves
  (-Laplacian + k^2) u = 4 pi exp(-a r) and stays bounded at the origin, giving
      u(r) = 4 pi e^{-a r} / D + 8 pi a (e^{-k r} - e^{-a r}) / (D^2 r),  D = k^2 - a^2,
  u(0) = 4 pi / (a + k)^2.
* Yukawa convolution of r exp(-a r): minus the a-derivative of the previous one.
* Yukawa convolution of exp(-a r) / r: from the radial formula below,
      u(r) = 4 pi (e^{-a r} - e^{-k r}) / (r (k^2 - a^2)),
  with the limit 2 pi e^{-a r} / a at k = a and 4 pi / (a + k) at r = 0.
* ``radial_convolution``: any radial f by the one-dimensional formulas
      Yukawa:  u(r) = 4 pi / (k r) [e^{-k r} int_0^r sinh(k s) f(s) s ds
                                      + sinh(k r) int_r^inf e^{-k s} f(s) s ds]
      Coulomb: u(r) = 4 pi [ (1/r) int_0^r f(s) s^2 ds + int_r^inf f(s) s ds ]
  by adaptive quadrature; an independent route to the same numbers.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def hydrogenic_hartree(r, Z):
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r < 1e-8
    rs = np.where(small, 1.0, r)
    out[:] = 1.0 / rs - (1.0 / rs + Z) * np.exp(-2.0 * Z * rs)
    out[small] = Z
    return out


def yukawa_of_exp(r, a, k):
    r = np.asarray(r, dtype=np.float64)
    D = k * k - a * a
    small = r < 1e-8
    rs = np.where(small, 1.0, r)
    u = 4.0 * np.pi * np.exp(-a * rs) / D + 8.0 * np.pi * a * (np.exp(-k * rs) - np.exp(-a * rs)) / (D * D * rs)
    return np.where(small, 4.0 * np.pi / (a + k) ** 2, u)


def yukawa_of_r_exp(r, a, k):
    """Yukawa convolution of r exp(-a r) = -d/da of yukawa_of_exp (r > 0)."""
    r = np.asarray(r, dtype=np.float64)
    D = k * k - a * a
    ea, ek = np.exp(-a * r), np.exp(-k * r)
    d_t1 = 4.0 * np.pi * (-r * ea / D + ea * 2.0 * a / (D * D))
    d_t2 = 8.0 * np.pi * ((ek - ea) / (D * D * r) + a * ea / (D * D)
                          + a * (ek - ea) * 4.0 * a / (D ** 3 * r))
    return -(d_t1 + d_t2)


def yukawa_of_exp_over_r(r, a, k):
    """Yukawa convolution of exp(-a r) / r."""
    r = np.asarray(r, dtype=np.float64)
    small = r < 1e-8
    rs = np.where(small, 1.0, r)
    if abs(k - a) < 1e-12 * max(a, k):
        u = 2.0 * np.pi * np.exp(-a * rs) / a
    else:
        u = 4.0 * np.pi * (np.exp(-a * rs) - np.exp(-k * rs)) / (rs * (k * k - a * a))
    return np.where(small, 4.0 * np.pi / (a + k), u)


def radial_convolution(f, r, kernel: str, k: float = 0.0, rmax: float = 60.0):
    """u(r) for a radial function f(s) by one-dimensional adaptive quadrature."""
    r = float(r)
    opts = dict(limit=400, epsabs=1e-14, epsrel=1e-13)
    if kernel == "coulomb":
        inner = integrate.quad(lambda s: f(s) * s * s, 0.0, r, **opts)[0] if r > 0 else 0.0
        outer = integrate.quad(lambda s: f(s) * s, r, rmax, **opts)[0]
        return 4.0 * np.pi * ((inner / r if r > 0 else 0.0) + outer)
    if r == 0.0:
        return 4.0 * np.pi * integrate.quad(lambda s: np.exp(-k * s) * f(s) * s, 0.0, rmax, **opts)[0]
    inner = integrate.quad(lambda s: np.sinh(k * s) * np.exp(-k * r) * f(s) * s, 0.0, r, **opts)[0]
    outer = integrate.quad(lambda s: np.exp(-k * (s - r)) * f(s) * s, r, rmax, **opts)[0]
    # sinh(k r) e^{-k s} = (e^{-k (s - r)} - e^{-k (s + r)}) / 2
    outer2 = integrate.quad(lambda s: np.exp(-k * (s + r)) * f(s) * s, r, rmax, **opts)[0]
    return 4.0 * np.pi / (k * r) * (inner + 0.5 * (outer - outer2))
