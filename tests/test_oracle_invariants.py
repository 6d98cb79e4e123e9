"""Invariants and exact symmetries of the oracle's H, rho and force.

H^loc, rho(r_g) and F^{loc,Pulay} of Sec. 3.3.1 at the Gamma point.
"""
import numpy as np
import pytest

import gint_inputs as gi


@pytest.fixture(scope="module")
def si8(oracle_mod):
    w = gi.si8_sz()
    o = oracle_mod.Oracle.from_workload(w)
    return w, o, o.H(w.V), o.H(np.ones(w.ngrid))


def test_H_symmetric(si8):
    w, o, H, S = si8
    assert np.max(np.abs(H - H.T)) <= 1e-14 * np.max(np.abs(H))


def test_constant_potential_gives_scaled_overlap(si8, oracle_mod):
    w, o, H, S = si8
    Hc = o.H(np.full(w.ngrid, -2.5))
    # equal up to summation roundoff over ~1e4 mesh points
    assert np.max(np.abs(Hc - (-2.5) * S)) <= 1e-13 * np.max(np.abs(Hc))


def test_density_integrates_to_trace_DS(si8):
    w, o, H, S = si8
    rho = o.rho(w.D)
    lhs = o.dV * rho.sum()
    rhs = np.sum(w.D * S)
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


def test_adjoint_identity_energy_equals_trace_DH(si8):
    w, o, H, S = si8
    E = o.energy(w.V, w.D)
    assert abs(E - np.sum(w.D * H)) <= 1e-13 * np.sum(np.abs(w.D * H))


def test_rank_one_density_is_orbital_squared(si8):
    w, o, H, S = si8
    rng = np.random.default_rng(0)
    idx = rng.choice(w.ngrid, 40, replace=False)
    N = np.array(w.grid)
    for mu in (0, 5, 31):
        D = np.zeros((o.norb, o.norb))
        D[mu, mu] = 1.0
        rho = o.rho(D, idx)
        for q, g in enumerate(idx):
            n = np.array(np.unravel_index(g, w.grid))
            r = (n / N) @ w.lattice
            assert abs(rho[q] - o.phi(r)[mu] ** 2) <= 1e-15


def test_nonsymmetric_density_matrix(si8):
    # rho uses D as given; a quadratic form only sees the symmetric part
    w, o, H, S = si8
    rng = np.random.default_rng(1)
    D = rng.standard_normal((o.norb, o.norb))
    idx = rng.choice(w.ngrid, 30, replace=False)
    N = np.array(w.grid)
    rho = o.rho(D, idx)
    for q, g in enumerate(idx):
        r = (np.array(np.unravel_index(g, w.grid)) / N) @ w.lattice
        p = o.phi(r)
        assert abs(rho[q] - p @ D @ p) <= 1e-12 * (1 + abs(rho[q]))
    np.testing.assert_allclose(o.rho(D.T, idx), rho, rtol=1e-12, atol=1e-14)


def test_lattice_translation_of_one_atom(oracle_mod):
    w = gi.si8_sz()
    o = oracle_mod.Oracle.from_workload(w)
    H0, rho0, F0 = o.H(w.V), o.rho(w.D), o.force(w.V, w.D)
    pos = w.positions.copy()
    pos[3] += w.lattice[1] - 2 * w.lattice[2]
    o.set_positions(pos)
    np.testing.assert_allclose(o.H(w.V), H0, rtol=0, atol=1e-13 * np.abs(H0).max())
    np.testing.assert_allclose(o.rho(w.D), rho0, rtol=0, atol=1e-13 * np.abs(rho0).max())
    np.testing.assert_allclose(o.force(w.V, w.D), F0, rtol=0, atol=1e-12 * np.abs(F0).max())


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_shift_by_mesh_step_rolls_rho(oracle_mod, axis):
    w = gi.si8_sz()
    o = oracle_mod.Oracle.from_workload(w)
    H0, rho0, F0 = o.H(w.V), o.rho(w.D), o.force(w.V, w.D)
    step = w.lattice[axis] / w.grid[axis]
    o.set_positions(w.positions + step)
    V1 = np.roll(w.V.reshape(w.grid), 1, axis=axis).reshape(-1)
    scale = np.abs(H0).max()
    np.testing.assert_allclose(o.H(V1), H0, rtol=0, atol=1e-13 * scale)
    rho1 = o.rho(w.D)
    np.testing.assert_allclose(rho1, np.roll(rho0.reshape(w.grid), 1, axis=axis).reshape(-1),
                               rtol=0, atol=1e-13 * np.abs(rho0).max())
    np.testing.assert_allclose(o.force(V1, w.D), F0, rtol=0, atol=1e-12 * np.abs(F0).max())


def test_atom_permutation_permutes_blocks(oracle_mod):
    w = gi.si8_sz()
    o = oracle_mod.Oracle.from_workload(w)
    H0 = o.H(w.V)
    F0 = o.force(w.V, w.D)
    perm = np.array([5, 2, 7, 0, 1, 6, 3, 4])
    n = 4
    orb = np.concatenate([np.arange(n * p, n * p + n) for p in perm])
    o2 = oracle_mod.Oracle(w.lattice, w.grid, w.species, w.species_of_atom[perm], w.positions[perm])
    H1 = o2.H(w.V)
    np.testing.assert_allclose(H1, H0[np.ix_(orb, orb)], rtol=0, atol=1e-14 * np.abs(H0).max())
    D1 = w.D[np.ix_(orb, orb)]
    np.testing.assert_allclose(o2.force(w.V, D1), F0[perm], rtol=0, atol=1e-13 * np.abs(F0).max())
    np.testing.assert_allclose(o2.rho(D1), o.rho(w.D), rtol=0, atol=1e-14)


def test_support_stats_si8(oracle_mod):
    # every point of the 8-atom cell sees at least one atom; the mean number
    # of atom-images within rc = 6 is 8/a^3 * 4/3 pi rc^3 = 6.70 (folding
    # can only lower the count of distinct atoms)
    w = gi.si8_sz()
    o = oracle_mod.Oracle.from_workload(w)
    s1, s2 = o.support_stats()
    mean_atoms = s1 / w.ngrid / 4
    assert 4.0 < mean_atoms <= 8.0
    assert s2 >= s1 * s1 / w.ngrid  # Cauchy-Schwarz


def test_point_subsets_add_up(oracle_mod):
    # the sampled forms are the same mesh sums restricted to a point subset
    w = gi.si8_sz()
    o = oracle_mod.Oracle.from_workload(w)
    rng = np.random.default_rng(2)
    perm = rng.permutation(w.ngrid)
    a, b = np.sort(perm[: w.ngrid // 3]), np.sort(perm[w.ngrid // 3:])
    Hfull = o.H_rows(w.V, 2, 5)
    np.testing.assert_allclose(o.H_rows(w.V, 2, 5, a) + o.H_rows(w.V, 2, 5, b), Hfull,
                               rtol=0, atol=1e-14 * np.abs(Hfull).max())
    Ffull = o.force(w.V, w.D, [1, 6])
    np.testing.assert_allclose(o.force(w.V, w.D, [1, 6], a) + o.force(w.V, w.D, [1, 6], b), Ffull,
                               rtol=0, atol=1e-13 * np.abs(Ffull).max())
