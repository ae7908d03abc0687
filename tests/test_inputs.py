"""The seeded input generators: the random molecules the selector's calibration
holds out are reproducible, keep their nuclei apart, and their orbital-like
functions are built exactly as the benchmark's benzene orbitals are."""
import numpy as np

from workloads.configs import (benzene_atoms, benzene_orbitals, molecule_orbitals,
                               random_molecule)


def test_random_molecules_are_seeded_and_keep_nuclei_apart():
    for seed in (71, 72, 5):
        a, b = random_molecule(seed), random_molecule(seed)
        assert [Z for _, Z in a] == [6.0, 6.0, 6.0, 1.0, 1.0, 1.0]
        for (R, _), (Q, _) in zip(a, b):
            assert np.array_equal(R, Q)
        for i in range(len(a)):
            assert np.all(np.abs(a[i][0]) <= 3.0)
            for j in range(i):
                assert np.linalg.norm(a[i][0] - a[j][0]) >= 1.8
    assert not np.array_equal(random_molecule(71)[0][0], random_molecule(72)[0][0])


def test_molecule_orbitals_follow_their_definition():
    g = np.random.default_rng(0)
    x, y, z = g.uniform(-4, 4, (3, 500))
    atoms = random_molecule(71)
    orb = molecule_orbitals(atoms, x, y, z, 3, 72)
    # each function: sum over nuclei of c exp(-zeta d), c in [-1, 1], zeta in [0.5, 6]
    assert np.all(np.abs(orb["coef"]) <= 1.0)
    assert np.all((orb["zeta"] >= 0.5) & (orb["zeta"] <= 6.0))
    for o in range(3):
        ref = sum(orb["coef"][o, a] * np.exp(-orb["zeta"][o, a] * np.linalg.norm(
            np.stack([x, y, z]) - R[:, None], axis=0)) for a, (R, _) in enumerate(atoms))
        assert np.allclose(orb["psi"][o], ref, rtol=1e-14, atol=1e-300)
    # eps log-spaced in [-10, -0.2], kappa = sqrt(-2 eps)
    assert np.allclose(orb["eps"], [-10.0, -10.0 * 0.02 ** 0.5, -0.2])
    assert np.allclose(orb["kappa"], np.sqrt(-2.0 * orb["eps"]))
    # the benchmark's orbitals are the same construction on the benzene nuclei
    b = benzene_orbitals(x, y, z, 4, 3)
    m = molecule_orbitals(benzene_atoms(), x, y, z, 4, 3)
    assert np.array_equal(b["psi"], m["psi"]) and np.array_equal(b["kappa"], m["kappa"])
