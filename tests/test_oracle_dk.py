"""Pins of the oracle's moving-basis matrix (Sec. 2.3, Ehrenfest dynamics,
D_K equation, at k = 0 on the mesh):

    DK[c, mu, nu] = <phit_mu | W | d phit_nu / d tau_K>_c,  K = atom of nu
                  = -dV sum_g W_g phit_mu(r_g) d_c phit_nu(r_g).

Pinned against references other than itself:
  * closed forms: for pure Gaussian s radials DK with W = 1 is the analytic
    derivative of the overlap with respect to the second centre, and with
    the plane-wave W the analytic derivative of <A|cos(G.r)|B>;
  * central differences of the mesh overlap S_grid (the oracle's H with
    V = 1) in the atom positions, on a DZP cell with p and d orbitals:
    dS_mu,nu/dtau_K = DK[., nu, mu] [mu on K] + DK[., mu, nu] [nu on K];
  * the grid force of Sec. 3.3.1 (pinned elsewhere by closed forms and
    finite differences): dE/dR_I = sum_{mu on I} sum_nu (D + D^T)_mu,nu
    DK_V[., nu, mu] with W = V.
"""
import numpy as np
import pytest

import gint_inputs as gi
from tests.test_oracle_closed_forms import ALPHAS, _cell, _images, _pw_G, closed_form


def closed_form_DK(w, W_kind):
    """Analytic <A_a | W | d B_b / dB> for s-only Gaussians: the derivative
    of the overlap (W = 1) or of the plane-wave matrix element with respect
    to the centre B of the right orbital."""
    T = _images(w.lattice)
    orbs = [(I, a) for I in range(w.natom) for a in ALPHAS]
    n = len(orbs)
    out = np.zeros((3, n, n))
    G = _pw_G(w)
    for i, (I, a) in enumerate(orbs):
        for j, (J, b) in enumerate(orbs):
            p = a + b
            mu = a * b / p
            A = w.positions[I]
            Bs = w.positions[J] + T
            dAB = A - Bs
            base = (1 / (4 * np.pi)) * (np.pi / p) ** 1.5 * np.exp(-mu * np.sum(dAB**2, axis=1))
            if W_kind == "one":
                out[:, i, j] = (2 * mu * dAB * base[:, None]).sum(0)
            else:
                P = (a * A + b * Bs) / p
                for k in range(len(w.pw_amp)):
                    t = base * w.pw_amp[k] * np.exp(-G[k] @ G[k] / (4 * p))
                    ph = P @ G[k]
                    d = (2 * mu * dAB * np.cos(ph)[:, None] - np.sin(ph)[:, None] * G[k] * (b / p)) * t[:, None]
                    out[:, i, j] += d.sum(0)
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_dk_overlap_closed_form(oracle_mod, seed):
    w = _cell(seed)
    o = oracle_mod.Oracle.from_workload(w)
    DK = o.DK(None)
    ref = closed_form_DK(w, "one")
    # The gradient comes from the spline's slope.  The blocks of an atom
    # with itself vanish analytically but keep ~3e-10 of slope error on the
    # mesh, so the bound is set on the scale of the overlap itself (~0.3),
    # far below the size of any entry a sign, transposition or image error
    # would change (>= 1e-6 here)
    S = closed_form(w, "one")
    assert np.max(np.abs(DK - ref)) <= 1e-8 * np.max(np.abs(S))
    off = np.abs(ref) > 1e-6
    assert np.max(np.abs(DK - ref)[off] / np.abs(ref)[off]) <= 1e-6


def test_dk_plane_wave_closed_form(oracle_mod):
    w = _cell(3)
    o = oracle_mod.Oracle.from_workload(w)
    DK = o.DK(w.V)
    ref = closed_form_DK(w, "pw")
    assert np.max(np.abs(DK - ref)) <= 5e-8 * np.max(np.abs(ref))


def _dzp_cell():
    # triclinic, two species (DZP and SZ), rc large enough for self-images
    sp = gi.Species([gi.nao_like_radial(0, 0.4, 5.0), gi.nao_like_radial(0, 1.0, 5.0),
                     gi.nao_like_radial(1, 0.5, 5.0), gi.nao_like_radial(1, 1.0, 5.0),
                     gi.nao_like_radial(2, 0.7, 5.0)])
    lat = np.array([[6.0, 0.0, 0.0], [0.7, 6.5, 0.0], [-0.4, 0.3, 7.0]])
    pos = np.array([[0.3, 0.2, 0.1], [3.1, 2.7, 3.9], [5.0, 5.5, 0.2]])
    return gi.small_cell(pos, lat, (14, 15, 16), [sp, gi.sz_species(4.0)], species_of_atom=[0, 1, 0],
                         n_waves=6, nocc=3, seed=7)


def test_dk_finite_difference_of_grid_overlap(oracle_mod):
    w = _dzp_cell()
    o = oracle_mod.Oracle.from_workload(w)
    one = np.ones(w.ngrid)
    DK = o.DK(None)
    h = 1e-4
    atom_of = np.repeat(np.arange(w.natom), np.diff(o.atom_orb0))
    worst = 0.0
    for K in range(w.natom):
        onK = atom_of == K
        for c in range(3):
            p = w.positions.copy()
            p[K, c] += h
            o.set_positions(p)
            Sp = o.H(one)
            p[K, c] -= 2 * h
            o.set_positions(p)
            Sm = o.H(one)
            fd = (Sp - Sm) / (2 * h)
            ref = np.zeros_like(fd)
            ref[onK, :] += DK[c].T[onK, :]
            ref[:, onK] += DK[c][:, onK]
            worst = max(worst, np.max(np.abs(fd - ref)) / np.max(np.abs(ref)))
    o.set_positions(w.positions)
    # central differences: O(h^2) truncation and ~eps/h roundoff
    assert worst <= 1e-6, worst


def test_dk_weighted_gives_grid_force(oracle_mod):
    w = _dzp_cell()
    o = oracle_mod.Oracle.from_workload(w)
    DKV = o.DK(w.V)
    S2 = w.D + w.D.T
    F = o.force(w.V, w.D)
    ref = np.zeros_like(F)
    for I in range(w.natom):
        rows = slice(o.atom_orb0[I], o.atom_orb0[I + 1])
        for c in range(3):
            ref[I, c] = np.sum(S2[rows, :] * DKV[c][:, rows].T)
    assert np.max(np.abs(F - ref)) <= 1e-12 * np.max(np.abs(F))


def test_dk_rows_and_points_add_up(oracle_mod):
    # the row form and the point-subset form are the same sums
    w = _dzp_cell()
    o = oracle_mod.Oracle.from_workload(w)
    full = o.DK(w.V)
    r0, r1 = o.atom_orb0[1], o.atom_orb0[3]
    np.testing.assert_array_equal(o.DK_rows(w.V, 1, 3), full[:, r0:r1])
    perm = np.random.default_rng(4).permutation(w.ngrid)
    a, b = np.sort(perm[: w.ngrid // 2]), np.sort(perm[w.ngrid // 2:])
    np.testing.assert_allclose(o.DK_rows(w.V, 0, 3, a) + o.DK_rows(w.V, 0, 3, b), full, rtol=0,
                               atol=1e-14 * np.abs(full).max())
