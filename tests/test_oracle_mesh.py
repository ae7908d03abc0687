"""Pins of the adaptive-mesh oracle (oracle/mesh.py): the Fejer rule's exactness,
the mesh quadrature of polynomials and of the hydrogenic density, the cell rules
(atoms on vertices, bounded aspect ratio), and agreement with the independent
input generator of workloads/mesh.py on the Be-like and benzene meshes."""
import numpy as np
import pytest

from oracle import mesh as om
from workloads.configs import DOMAIN, atom_mesh, benzene_atoms, benzene_mesh

Z = 4.0


@pytest.mark.parametrize("p", [3, 5, 7])
def test_fejer_rule_is_exact_to_degree_p(p):
    s, v = om.nodes_weights(p)
    for k in range(p + 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.sum(v * s ** k) == pytest.approx(exact, abs=1e-14)
    # and not beyond: degree p+2 (even) is missed
    k = p + 2 if (p + 2) % 2 == 0 else p + 3
    assert abs(np.sum(v * s ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.fixture(scope="module")
def atom_cells():
    return om.build(om.density_test([((0.0, 0.0, 0.0), Z)]), DOMAIN[0], DOMAIN[1], 7, 3e-11, 3,
                    atoms=[(0.0, 0.0, 0.0)])


def test_mesh_quadrature_of_polynomials_and_density(atom_cells):
    x, y, z, w = om.points(atom_cells, 7)
    L = 20.0
    assert w.sum() == pytest.approx((2 * L) ** 3, rel=1e-13)
    # int x^2 y^2 z^4 over [-L, L]^3 = (2 L^3/3)^2 (2 L^5/5), exact cell by cell
    exact = (2 * L ** 3 / 3) ** 2 * (2 * L ** 5 / 5)
    assert np.sum(w * x ** 2 * y ** 2 * z ** 4) == pytest.approx(exact, rel=1e-12)
    r = np.sqrt(x * x + y * y + z * z)
    assert np.sum(w * Z ** 3 / np.pi * np.exp(-2 * Z * r)) == pytest.approx(1.0, abs=1e-8)


def test_cell_rules(atom_cells):
    lo = np.array([c[0] for c in atom_cells])
    hi = np.array([c[1] for c in atom_cells])
    ext = hi - lo
    assert np.all(ext.max(axis=1) / ext.min(axis=1) <= 2.0)
    interior = np.all((lo < 0.0) & (0.0 < hi), axis=1)
    assert not np.any(interior)  # the nucleus lies on vertices only
    assert np.sum(np.prod(ext, axis=1)) == pytest.approx(64000.0, rel=1e-13)


def test_smaller_tolerance_refines_more():
    t = om.density_test([((0.0, 0.0, 0.0), Z)])
    n1 = len(om.build(t, DOMAIN[0], DOMAIN[1], 5, 1e-6, 2, atoms=[(0.0, 0.0, 0.0)]))
    n2 = len(om.build(t, DOMAIN[0], DOMAIN[1], 5, 1e-8, 2, atoms=[(0.0, 0.0, 0.0)]))
    assert n2 > n1


def test_agrees_with_the_input_generator(atom_cells):
    m = atom_mesh()["mesh"]
    assert np.array_equal(np.array([c[0] for c in atom_cells]), m.lo)
    assert np.array_equal(np.array([c[1] for c in atom_cells]), m.hi)
    atoms = benzene_atoms()
    cells = om.build(om.paper_test([(tuple(R), Za) for R, Za in atoms]), DOMAIN[0], DOMAIN[1], 7,
                     5e-4, 4, atoms=[R for R, _ in atoms])
    mb = benzene_mesh()["mesh"]
    assert np.array_equal(np.array([c[0] for c in cells]), mb.lo)
    assert np.array_equal(np.array([c[1] for c in cells]), mb.hi)
