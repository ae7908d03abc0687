"""Pins of the Green-iteration step oracle (oracle/green.py) against closed forms.

For V = -Z/r and psi = exp(-a r) with eps = -a^2/2, the modified Helmholtz
equation (1/2 Laplacian + eps) psi' = V psi of Eq. Helmholtz_Form is solved by
psi' = (Z/a) psi, since (1/2 Laplacian - a^2/2) exp(-a r) = -(a/r) exp(-a r).
With <V psi, psi> = -Z pi / a^2 and <psi, psi> = pi / a^3, the gradient-free
update (Eq. gradient-free) then gives eps' = -a^2/2 + a^2 (a - Z) / Z, and a = Z
is the hydrogenic fixed point (psi' = psi, eps' = -Z^2/2). The convolution is the
exact continuous one (closed form of the Yukawa convolution of exp(-a r)/r), so
the step's own arithmetic is what is checked; inner products use the Be-like
mesh quadrature.
"""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle.green import dot, green_step
from workloads.configs import atom_mesh

Z = 4.0


@pytest.fixture(scope="module")
def mesh():
    d = atom_mesh()
    d["r"] = np.sqrt(d["x"] ** 2 + d["y"] ** 2 + d["z"] ** 2)
    return d


def _convolve_exponentials(r, rates):
    """convolve(f, kappa) for f = -c Z exp(-a r)/r with a in `rates` and any
    constant c (the density the step must form from V and psi; checked)."""
    def conv(f, kappa):
        for a in rates:
            g = -Z * np.exp(-a * r) / r
            c = f[0] / g[0]
            if np.allclose(f, c * g, rtol=1e-13, atol=0.0):
                return -c * Z * cf.yukawa_of_exp_over_r(r, a, kappa)
        raise AssertionError("convolve called with an unexpected density")
    return conv


def test_hydrogenic_fixed_point(mesh):
    r, w = mesh["r"], mesh["w"]
    psi = np.exp(-Z * r)
    psi /= np.sqrt(dot(w, psi, psi))
    new, eps, res = green_step(w, psi[None], -Z / r, np.array([-Z * Z / 2]),
                               _convolve_exponentials(r, [Z]))
    assert eps[0] == pytest.approx(-Z * Z / 2, rel=1e-5)
    assert np.abs(new[0] - psi).max() < 1e-5 * np.abs(psi).max()
    assert res[0] < 1e-5


@pytest.mark.parametrize("a", [3.0, 5.0])
def test_eigenvalue_update_off_the_fixed_point(mesh, a):
    r, w = mesh["r"], mesh["w"]
    psi = np.exp(-a * r)
    psi /= np.sqrt(dot(w, psi, psi))
    new, eps, res = green_step(w, psi[None], -Z / r, np.array([-a * a / 2]),
                               _convolve_exponentials(r, [a]))
    assert eps[0] == pytest.approx(-a * a / 2 + a * a * (a - Z) / Z, rel=1e-4)
    # psi' = (Z/a) psi before normalization: the same direction
    assert np.abs(new[0] - psi).max() < 1e-5 * np.abs(psi).max()


def test_block_orthonormalization(mesh):
    # two exponentials: eigenvalues updated independently, then psi'_1 loses its
    # component along psi'_0 (continuous overlaps <e^{-ar}, e^{-br}> = 8 pi/(a+b)^3)
    r, w = mesh["r"], mesh["w"]
    rates = [3.0, 1.5]
    psi = np.stack([np.exp(-a * r) for a in rates])
    for o in range(2):
        psi[o] /= np.sqrt(dot(w, psi[o], psi[o]))
    eps0 = np.array([-a * a / 2 for a in rates])
    new, eps, res = green_step(w, psi, -Z / r, eps0, _convolve_exponentials(r, rates))
    for o, a in enumerate(rates):
        assert eps[o] == pytest.approx(-a * a / 2 + a * a * (a - Z) / Z, rel=1e-4)
    G = np.array([[dot(w, new[i], new[j]) for j in range(2)] for i in range(2)])
    assert np.abs(G - np.eye(2)).max() < 1e-12
    ov = lambda a, b: 8 * np.pi / (a + b) ** 3  # noqa: E731
    n0 = np.exp(-3.0 * r) / np.sqrt(ov(3.0, 3.0))
    c = ov(1.5, 3.0) / np.sqrt(ov(3.0, 3.0))
    v1 = np.exp(-1.5 * r) - c * n0
    v1 /= np.sqrt(ov(1.5, 1.5) - c * c)
    assert np.abs(new[1] - v1).max() < 1e-4 * np.abs(v1).max()
