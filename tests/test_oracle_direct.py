"""Pins of the direct-sum oracle against things other than itself: analytic special
cases, closed-form convolutions on a Fejer mesh, one-dimensional radial
integrals, and invariances of the kernels."""
import numpy as np
import pytest
from scipy import integrate

from oracle import closed_forms as cf
from oracle.direct import direct_sum
from workloads.configs import atom_mesh, sample_targets, uniform_cube

LN2 = np.log(2.0)


def _two_points():
    x = np.array([0.0, 1.0])
    y = np.zeros(2)
    z = np.zeros(2)
    f = np.array([1.0, 3.0])
    w = np.array([0.25, 0.5])
    return x, y, z, f, w


def test_two_point_worked_example():
    # d = 1 and kappa = ln 2 make exp(-kappa d) = 1/2 exactly on paper.
    x, y, z, f, w = _two_points()
    c = 4.0 * np.pi / LN2 ** 2
    u = direct_sum("yukawa_ss", x, y, z, f, w, kappa=LN2)
    np.testing.assert_allclose(u, [(3 - 1) * 0.5 * 0.5 + 1 * c, (1 - 3) * 0.5 * 0.25 + 3 * c], rtol=1e-15)
    u = direct_sum("coulomb_ss", x, y, z, f, w, alpha=1.0)
    e = np.exp(-1.0)
    np.testing.assert_allclose(u, [(3 - e) * 0.5 + 2 * np.pi, (1 - 3 * e) * 0.25 + 6 * np.pi], rtol=1e-15)
    u = direct_sum("yukawa", x, y, z, f, w, kappa=LN2)
    np.testing.assert_allclose(u, [0.5 * 3 * 0.5, 0.5 * 1 * 0.25], rtol=1e-15)
    u = direct_sum("coulomb", x, y, z, f, w)
    np.testing.assert_allclose(u, [3 * 0.5, 1 * 0.25], rtol=1e-15)


@pytest.mark.parametrize("kappa", [0.3, 1.0, 4.47])
def test_yukawa_subtraction_constant_is_the_kernel_integral(kappa):
    # a lone target sees only the analytic term f * int exp(-k r)/r d^3r
    radial = 4.0 * np.pi * integrate.quad(lambda r: np.exp(-kappa * r) * r, 0, np.inf,
                                          epsabs=1e-15, epsrel=1e-13)[0]
    one = np.zeros(1)
    u = direct_sum("yukawa_ss", one, one, one, np.array([2.5]), np.array([1.0]), kappa=kappa)
    assert u[0] == pytest.approx(2.5 * radial, rel=1e-13)


@pytest.mark.parametrize("alpha", [0.5, 1.0, 2.0])
def test_coulomb_subtraction_constant_is_the_gaussian_integral(alpha):
    radial = 4.0 * np.pi * integrate.quad(lambda r: np.exp(-r * r / alpha ** 2) * r, 0, np.inf,
                                          epsabs=1e-15, epsrel=1e-13)[0]
    one = np.zeros(1)
    u = direct_sum("coulomb_ss", one, one, one, np.array([-1.5]), np.array([1.0]), alpha=alpha)
    assert u[0] == pytest.approx(-1.5 * radial, rel=1e-13)


def test_constant_density_invariant():
    # f == c makes every (f_j - f_i) vanish: Yukawa-SS gives exactly 4 pi c / k^2
    x, y, z, _, w = uniform_cube(700, seed=11)
    c, k = 0.75, 1.3
    u = direct_sum("yukawa_ss", x, y, z, np.full(x.size, c), w, kappa=k)
    np.testing.assert_allclose(u, 4 * np.pi * c / k ** 2, rtol=1e-15)


def test_self_pair_is_skipped_and_duplicates_contribute_zero():
    x, y, z, f, w = _two_points()
    xs = np.concatenate([x, x[:1]])
    ys, zs = np.zeros(3), np.zeros(3)
    fs = np.concatenate([f, [5.0]])
    ws = np.concatenate([w, [7.0]])
    u3 = direct_sum("coulomb", xs, ys, zs, fs, ws)
    u2 = direct_sum("coulomb", x, y, z, f, w)
    assert u3[0] == u2[0] and u3[1] == pytest.approx(u2[1] + 5.0 * 7.0, rel=1e-15)


def test_kernel_homogeneity_and_rigid_motions():
    x, y, z, f, w = uniform_cube(400, seed=5)
    s = 2.5
    u = direct_sum("coulomb", x, y, z, f, w)
    us = direct_sum("coulomb", s * x, s * y, s * z, f, w)
    np.testing.assert_allclose(us, u / s, rtol=0, atol=1e-13 * np.abs(u).max())
    u = direct_sum("yukawa", x, y, z, f, w, kappa=1.7)
    us = direct_sum("yukawa", s * x, s * y, s * z, f, w, kappa=1.7 / s)
    np.testing.assert_allclose(us, u / s, rtol=0, atol=1e-13 * np.abs(u).max())
    # axis permutation and translation leave the sums unchanged
    for k in ("yukawa_ss", "coulomb_ss"):
        a = direct_sum(k, x, y, z, f, w, kappa=0.9)
        b = direct_sum(k, z + 3.0, x - 1.0, y, f, w, kappa=0.9)
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * np.abs(a).max())


def test_threads_do_not_change_bits():
    x, y, z, f, w = uniform_cube(900, seed=2)
    a = direct_sum("yukawa_ss", x, y, z, f, w, kappa=1.0, threads=1)
    b = direct_sum("yukawa_ss", x, y, z, f, w, kappa=1.0, threads=7)
    assert np.array_equal(a, b)


def test_closed_forms_against_radial_quadrature():
    k = np.sqrt(0.4)
    for r in (0.0, 0.02, 0.3, 1.0, 4.0):
        assert cf.yukawa_of_exp(np.array([r]), 4.0, k)[0] == pytest.approx(
            cf.radial_convolution(lambda s: np.exp(-4.0 * s), r, "yukawa", k), rel=1e-11)
        assert cf.hydrogenic_hartree(np.array([r]), 4.0)[0] == pytest.approx(
            cf.radial_convolution(lambda s: 64.0 / np.pi * np.exp(-8.0 * s), r, "coulomb"), rel=1e-11)
    for r in (0.02, 0.3, 1.0, 4.0):
        assert cf.yukawa_of_r_exp(np.array([r]), 2.0, k)[0] == pytest.approx(
            cf.radial_convolution(lambda s: s * np.exp(-2.0 * s), r, "yukawa", k), rel=1e-10)
    for a, kk in ((3.0, k), (2.0, 2.0)):
        for r in (0.0, 0.02, 0.3, 1.0, 4.0):
            assert cf.yukawa_of_exp_over_r(np.array([r]), a, kk)[0] == pytest.approx(
                cf.radial_convolution(lambda s: np.exp(-a * s) / s, r, "yukawa", kk), rel=1e-9)


@pytest.fixture(scope="module")
def be_mesh():
    d = atom_mesh()
    d["idx"] = sample_targets(d["x"].size, 48, seed=7)
    return d


def test_hydrogenic_hartree_on_mesh(be_mesh):
    # Coulomb convolution of Z^3/pi exp(-2Zr) vs 1/r - (1/r + Z) exp(-2Zr):
    # the subtracted sum lands within the mesh's discretization error, the plain
    # sum (singularity skipped) is far worse -- the synthetic analogue of the
    # paper's Table 2.
    d, Z = be_mesh, be_mesh["Z"]
    x, y, z, w, i = d["x"], d["y"], d["z"], d["w"], d["idx"]
    r = np.sqrt(x * x + y * y + z * z)
    rho = Z ** 3 / np.pi * np.exp(-2 * Z * r)
    ex = cf.hydrogenic_hartree(r[i], Z)
    u_ss = direct_sum("coulomb_ss", x, y, z, rho, w, x[i], y[i], z[i], rho[i], alpha=1.0)
    u_pl = direct_sum("coulomb", x, y, z, rho, w, x[i], y[i], z[i], rho[i])
    e_ss = np.abs(u_ss - ex).max() / np.abs(ex).max()
    e_pl = np.abs(u_pl - ex).max() / np.abs(ex).max()
    assert e_ss < 2e-5
    assert e_pl > 20 * e_ss


def test_yukawa_of_exponential_on_mesh(be_mesh):
    d = be_mesh
    x, y, z, w, i = d["x"], d["y"], d["z"], d["w"], d["idx"]
    r = np.sqrt(x * x + y * y + z * z)
    k = d["kappa"]
    for a in (4.0, 2.0):
        f = np.exp(-a * r)
        ex = cf.yukawa_of_exp(r[i], a, k)
        u = direct_sum("yukawa_ss", x, y, z, f, w, x[i], y[i], z[i], f[i], kappa=k)
        assert np.abs(u - ex).max() / np.abs(ex).max() < 2e-3
        # the subtracted constant alone is 4 pi f / k^2 ~ 31 f here; dropping or
        # mis-signing it moves the result by orders of magnitude more
        assert np.linalg.norm(u - ex) / np.linalg.norm(ex) < 1e-3


def test_green_iteration_fixed_point_on_mesh(be_mesh):
    # psi = exp(-Z r), V = -Z/r, kappa = Z: -(1/2pi) int G_kappa V psi = psi
    d = be_mesh
    x, y, z, w, i = d["x"], d["y"], d["z"], d["w"], d["idx"]
    Z = 4.0
    r = np.sqrt(x * x + y * y + z * z)
    psi = np.exp(-Z * r)
    f = -Z / r * psi
    u = direct_sum("yukawa_ss", x, y, z, f, w, x[i], y[i], z[i], f[i], kappa=Z)
    got = -u / (2 * np.pi)
    assert np.abs(got - psi[i]).max() / psi.max() < 5e-3
