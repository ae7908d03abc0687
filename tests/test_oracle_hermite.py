"""Pins of the Hermite treecode oracle: the 1-D Hermite basis reproduces
polynomials of degree 2n + 1 and no more, the Hermite proxy charges reproduce the
particle moments to that degree, the radial derivatives agree with finite
differences of the kernels, theta = 0 is the direct sum, and the error falls with
the degree and stays below the Lagrange treecode's at the same (theta, n)."""
import numpy as np
import pytest

from oracle import bltc, hermite
from oracle.direct import direct_sum
from workloads.configs import uniform_cube
from workloads.rng import SplitMix64


@pytest.mark.parametrize("n", [1, 3, 4, 6])
def test_hermite_basis_reproduces_degree_2n_plus_1(n):
    s = bltc.cheb2_nodes(-0.4, 1.1, n)
    t = SplitMix64(7 + n).uniform(60, -0.4, 1.1)
    A, B = hermite.hermite_basis(t, s)
    c = 0.35
    for m in range(2 * n + 3):
        P = (t - c) ** m
        Ps = (s - c) ** m
        dPs = m * (s - c) ** (m - 1) if m > 0 else np.zeros_like(s)
        err = np.max(np.abs(A @ Ps + B @ dPs - P))
        if m <= 2 * n + 1:
            assert err < 1e-12, (m, err)
        else:
            assert err > 1e-6, (m, err)  # degree 2n + 2 is not reproduced
    # at the nodes: A_k(s_m) = delta_km, B_k(s_m) = 0
    A, B = hermite.hermite_basis(s, s)
    np.testing.assert_allclose(A, np.eye(n + 1), atol=1e-13)
    np.testing.assert_allclose(B, 0.0, atol=1e-13)


def test_hermite_basis_derivatives_at_nodes():
    # A_k'(s_m) = 0 and B_k'(s_m) = delta_km, by central differences
    n = 5
    s = bltc.cheb2_nodes(0.0, 2.0, n)
    h = 1e-6
    Ap, Bp = hermite.hermite_basis(s + h, s)
    Am, Bm = hermite.hermite_basis(s - h, s)
    np.testing.assert_allclose((Ap - Am) / (2 * h), 0.0, atol=1e-6)
    np.testing.assert_allclose((Bp - Bm) / (2 * h), np.eye(n + 1), atol=1e-6)


@pytest.mark.parametrize("n", [2, 4])
def test_hermite_proxy_charges_reproduce_moments(n):
    # sum_k sum_beta d^beta P(s_k) q^_{k,beta} = sum_j P(y_j) q_j for every monomial
    # P = x^a y^b z^c with a, b, c <= 2n + 1
    g = SplitMix64(300 + n)
    N = 300
    px, py, pz = g.uniform(N, 0.2, 1.0), g.uniform(N, -1.0, -0.3), g.uniform(N, 3.0, 3.5)
    q = g.uniform(N, -1, 1)
    lo = np.array([px.min(), py.min(), pz.min()])
    hi = np.array([px.max(), py.max(), pz.max()])
    nodes, ch = hermite.proxy_charges(px, py, pz, q, lo, hi, n)
    ch = ch[0]
    c = 0.5 * (lo + hi)
    sx, sy, sz = (nodes[d] - c[d] for d in range(3))

    def mono(v, e, der):
        if der == 0:
            return v ** e
        return e * v ** (e - 1) if e > 0 else np.zeros_like(v)

    top = 2 * n + 1
    for a, b, cc in [(0, 0, 0), (1, 2, 0), (top, 0, 1), (top, top, top), (n + 1, top - 1, 2)]:
        lhs = 0.0
        for bi, (bx, by, bz) in enumerate(hermite.BETAS):
            lhs += np.einsum("abc,a,b,c->", ch[..., bi], mono(sx, a, bx), mono(sy, b, by),
                             mono(sz, cc, bz))
        rhs = np.sum((px - c[0]) ** a * (py - c[1]) ** b * (pz - c[2]) ** cc * q)
        scale = np.sum(np.abs(q)) * np.max(hi - lo) ** (a + b + cc)
        assert abs(lhs - rhs) <= 1e-11 * scale, (a, b, cc, lhs, rhs)


def _fd_derivative(g, x, y, beta, h):
    """d^beta_y g(|y - x|) by nested central differences in the source point."""
    dims = [d for d in range(3) if beta[d]]
    total = 0.0
    for signs in np.ndindex(*([2] * len(dims))):
        yy = y.copy()
        coef = 1.0
        for d, sgn in zip(dims, signs):
            yy[d] += h if sgn == 0 else -h
            coef *= 1.0 if sgn == 0 else -1.0
        total += coef * g(np.linalg.norm(yy - x))
    return total / (2 * h) ** len(dims)


@pytest.mark.parametrize("kind,kappa,alpha", [("yukawa", 1.7, 1.0), ("coulomb", 0.0, 1.0),
                                              ("gauss", 0.0, 0.8)])
def test_kernel_derivatives_match_finite_differences(kind, kappa, alpha):
    g = {"yukawa": lambda r: np.exp(-kappa * r) / r,
         "coulomb": lambda r: 1.0 / r,
         "gauss": lambda r: np.exp(-r * r / (alpha * alpha)) / r}[kind]
    x = np.array([0.1, -0.2, 0.3])
    ys = [np.array([0.9, 0.5, -0.4]), np.array([-0.6, 0.7, 1.1])]
    for y in ys:
        D = hermite.kernel_derivatives(kind, x[:1], x[1:2], x[2:], y[:1], y[1:2], y[2:],
                                       kappa, alpha)[:, 0, 0]
        for b, beta in enumerate(hermite.BETAS):
            fd = _fd_derivative(g, x, y, beta, 1e-3)
            tol = [1e-6, 1e-5, 1e-4, 1e-4][sum(beta)]
            assert abs(D[b] - fd) <= tol * (abs(fd) + abs(D[0])), (kind, beta, D[b], fd)


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss", "yukawa", "coulomb"])
def test_hermite_theta_zero_is_the_direct_sum(kernel):
    x, y, z, f, w = uniform_cube(1500, seed=22)
    u = hermite.treecode(x, y, z, f, w, kernel, 1.3, 0.0, 3, 200)[0]
    ref, ab = direct_sum(kernel, x, y, z, f, w, kappa=1.3, return_abs=True)
    assert np.max(np.abs(u - ref) / (ab + np.abs(ref))) < 1e-13


def test_hermite_constant_density_invariant():
    # f = c: every subtracted pair term vanishes (f^ = c w^ in the far field)
    x, y, z, _, w = uniform_cube(3000, seed=23)
    f = np.full(x.size, 0.75)
    u = hermite.treecode(x, y, z, f, w, "yukawa_ss", 1.1, 0.7, 3, 150)[0]
    np.testing.assert_allclose(u, 4 * np.pi * 0.75 / 1.1 ** 2, rtol=1e-13)


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
def test_hermite_error_falls_with_degree_and_beats_lagrange(kernel):
    x, y, z, f, w = uniform_cube(4000, seed=3)
    ref = direct_sum(kernel, x, y, z, f, w, kappa=1.0)
    tree = bltc.build_tree(x, y, z, 100)
    errs = []
    for n in (1, 2, 3, 4):
        u = hermite.treecode(x, y, z, f, w, kernel, 1.0, 0.7, n, 100, tree=tree)[0]
        e = np.linalg.norm(u - ref) / np.linalg.norm(ref)
        ul = bltc.treecode(x, y, z, f, w, kernel, 1.0, 0.7, n, 100, tree=tree)[0]
        el = np.linalg.norm(ul - ref) / np.linalg.norm(ref)
        assert e < el, (n, e, el)
        errs.append(e)
    assert all(a > b for a, b in zip(errs[:-1], errs[1:])), errs
    assert errs[-1] < 1e-6, errs
