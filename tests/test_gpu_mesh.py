"""The adaptive mesh built on the GPU (tagi_mesh_build) against the oracle's:
the same cells and the same quadrature points and weights for the Be-like atom
(1s-density test function) and benzene (Eq. test_function) meshes."""
import numpy as np
import pytest

from oracle import mesh as om
from workloads.configs import DOMAIN, benzene_atoms

pytestmark = pytest.mark.gpu


def _compare(cells, got, p):
    x, y, z, w, lo, hi = got
    assert lo.shape[0] == len(cells)
    np.testing.assert_array_equal(lo, np.array([c[0] for c in cells]))
    np.testing.assert_array_equal(hi, np.array([c[1] for c in cells]))
    rx, ry, rz, rw = om.points(cells, p)
    for a, b in ((x, rx), (y, ry), (z, rz)):
        np.testing.assert_array_equal(a.cpu().numpy(), b)
    np.testing.assert_allclose(w.cpu().numpy(), rw, rtol=1e-15, atol=0)


def test_atom_mesh_matches_oracle():
    import paper_2003_01833_amd as tagi
    atoms = [((0.0, 0.0, 0.0), 4.0)]
    cells = om.build(om.density_test(atoms), DOMAIN[0], DOMAIN[1], 7, 3e-11, 3,
                     atoms=[a for a, _ in atoms])
    got = tagi.mesh(DOMAIN[0], DOMAIN[1], 7, 3e-11, 3, atoms=atoms, test="density")
    assert len(cells) == 1968
    _compare(cells, got, 7)


def test_benzene_mesh_matches_oracle():
    import paper_2003_01833_amd as tagi
    atoms = [(tuple(R), Z) for R, Z in benzene_atoms()]
    cells = om.build(om.paper_test(atoms), DOMAIN[0], DOMAIN[1], 7, 5e-4, 4,
                     atoms=[a for a, _ in atoms])
    got = tagi.mesh(DOMAIN[0], DOMAIN[1], 7, 5e-4, 4, atoms=atoms, test="root_density_vext")
    assert len(cells) == 8092
    _compare(cells, got, 7)
    # the weights tile the domain: their sum is its volume, 40^3
    w = got[3].cpu().numpy()
    assert abs(w.sum() / 64000.0 - 1.0) < 1e-12
    assert (w > 0).all()


def test_small_mesh_and_argument_checks():
    import paper_2003_01833_amd as tagi
    atoms = [((0.3, -0.2, 0.1), 2.0)]
    cells = om.build(om.density_test(atoms), (-5, -5, -5), (5, 5, 5), 4, 1e-6, 1,
                     atoms=[a for a, _ in atoms], max_aspect=1.5)
    got = tagi.mesh((-5, -5, -5), (5, 5, 5), 4, 1e-6, 1, atoms=atoms, max_aspect=1.5)
    _compare(cells, got, 4)
    with pytest.raises(tagi.TagiError):
        tagi.mesh(DOMAIN[0], DOMAIN[1], 7, -1.0)
    with pytest.raises(tagi.TagiError):
        tagi.mesh(DOMAIN[0], DOMAIN[1], 16, 1e-6)
