"""The oracle's analytic gradient vs central differences of its own FP64
energy E = dV sum_g V_g rho_g (F^{loc,Pulay} equation of Sec. 3.3.1), plus
the approximate translation (egg-box) sum rule."""
import numpy as np

import gint_inputs as gi


def _displaced_si8(seed=3):
    w = gi.si8_sz()
    rng = np.random.default_rng(seed)
    pos = w.positions + rng.normal(0, 0.1, w.positions.shape)
    return gi.small_cell(pos, w.lattice, w.grid, w.species, n_waves=8, nocc=16, seed=seed)


def test_force_matches_central_differences(oracle_mod):
    w = _displaced_si8()
    o = oracle_mod.Oracle.from_workload(w)
    F = o.force(w.V, w.D)
    h = 1e-4
    scale = np.max(np.abs(F))
    for I in (0, 3, 6):
        for k in range(3):
            p = w.positions.copy()
            p[I, k] += h
            o.set_positions(p)
            Ep = o.energy(w.V, w.D)
            p[I, k] -= 2 * h
            o.set_positions(p)
            Em = o.energy(w.V, w.D)
            o.set_positions(w.positions)
            fd = (Ep - Em) / (2 * h)
            assert abs(F[I, k] - fd) <= 1e-6 * scale


def test_dzp_force_matches_central_differences(oracle_mod):
    sp = gi.dzp_species(rc=5.0)
    lat = np.eye(3) * 8.0
    pos = np.array([[0.5, 0.7, 1.1], [3.9, 4.4, 3.6], [6.1, 1.2, 5.5]])
    w = gi.small_cell(pos, lat, (16, 16, 16), [sp], n_waves=6, nocc=5, seed=21)
    o = oracle_mod.Oracle.from_workload(w)
    F = o.force(w.V, w.D)
    h = 1e-4
    scale = np.max(np.abs(F))
    for I in range(3):
        for k in range(3):
            p = w.positions.copy()
            p[I, k] += h
            o.set_positions(p)
            Ep = o.energy(w.V, w.D)
            p[I, k] -= 2 * h
            o.set_positions(p)
            Em = o.energy(w.V, w.D)
            o.set_positions(w.positions)
            assert abs(F[I, k] - (Ep - Em) / (2 * h)) <= 1e-6 * scale


def test_translation_sum_rule(oracle_mod):
    # moving every atom by delta is moving V by -delta, so
    # sum_I dE/dR_I ~ integral rho grad V (mesh-aliasing error only)
    w = _displaced_si8(5)
    o = oracle_mod.Oracle.from_workload(w)
    F = o.force(w.V, w.D)
    rho = o.rho(w.D)
    N = np.array(w.grid)
    n = np.stack(np.meshgrid(*[np.arange(k) for k in N], indexing="ij"), -1).reshape(-1, 3)
    B = np.linalg.inv(w.lattice).T
    G = 2 * np.pi * (w.pw_m @ B)
    phase = 2 * np.pi * (n / N) @ w.pw_m.T
    gradV = -(np.sin(phase) * w.pw_amp) @ G
    rhs = o.dV * (rho[:, None] * gradV).sum(0)
    assert np.max(np.abs(F.sum(0) - rhs)) <= 1e-3 * np.max(np.abs(F))


def test_nonsymmetric_D_force(oracle_mod):
    # E depends on D only through D + D^T; the gradient must use both
    sp = gi.dzp_species(rc=5.0)
    lat = np.eye(3) * 8.0
    pos = np.array([[0.5, 0.7, 1.1], [3.9, 4.4, 3.6]])
    w = gi.small_cell(pos, lat, (14, 14, 14), [sp], n_waves=6, nocc=5, seed=4)
    rng = np.random.default_rng(8)
    D = rng.standard_normal((w.norb, w.norb)) * 0.1
    o = oracle_mod.Oracle.from_workload(w)
    F = o.force(w.V, D)
    np.testing.assert_allclose(F, o.force(w.V, 0.5 * (D + D.T)), rtol=0, atol=1e-12 * np.abs(F).max())
    h = 1e-4
    for I in range(2):
        for k in range(3):
            p = w.positions.copy()
            p[I, k] += h
            o.set_positions(p)
            Ep = o.energy(w.V, D)
            p[I, k] -= 2 * h
            o.set_positions(p)
            Em = o.energy(w.V, D)
            o.set_positions(w.positions)
            assert abs(F[I, k] - (Ep - Em) / (2 * h)) <= 1e-6 * np.abs(F).max()
