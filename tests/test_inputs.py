"""The seeded workload generators: shapes, determinism and the recipe."""
import numpy as np

import gint_inputs as gi


def test_si8_recipe():
    w = gi.si8_sz()
    assert w.natom == 8 and w.norb == 32 and w.grid == (24, 24, 24)
    assert w.V.shape == (24**3,) and w.D.shape == (32, 32)
    assert np.allclose(w.D, w.D.T)
    assert len(w.pw_amp) == 8 and np.all(np.abs(w.pw_amp) <= 1)
    G = 2 * np.pi * w.pw_m / gi.A_SI
    assert np.all(np.linalg.norm(G, axis=1) <= 3 * 2 * np.pi / gi.A_SI + 1e-12)
    w2 = gi.si8_sz()
    assert np.array_equal(w.V, w2.V) and np.array_equal(w.D, w2.D)


def test_dzp_species_layout():
    sp = gi.dzp_species()
    assert sp.norb == 13
    assert [r.l for r in sp.radials] == [0, 0, 1, 1, 2]
    assert all(r.nr == 801 and abs(r.rc - 8.0) < 1e-15 for r in sp.radials)


def test_si512_recipe_small_parts():
    lat, pos = gi.si_supercell((4, 4, 4))
    assert pos.shape == (512, 3) and np.allclose(np.diag(lat), 41.04)
    # the displaced positions are the lattice sites plus N(0, 0.05)
    rng = np.random.Generator(np.random.PCG64(5))
    disp = rng.normal(0.0, 0.05, size=pos.shape)
    assert 0.04 < disp.std() < 0.06


def test_batched_cells_sizes():
    cells = gi.batched_cells(n_cells=6)
    for c in cells:
        assert c.natom in (8, 16, 32, 64)
        spacing = np.diag(c.lattice) / np.array(c.grid)
        assert np.allclose(spacing, spacing[0])
