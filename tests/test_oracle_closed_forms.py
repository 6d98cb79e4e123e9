"""Closed-form pins: Gaussian s-orbital overlaps, plane-wave potential
matrix elements and their analytic position derivatives.

With pure Gaussian radials f = exp(-a r^2) and a cutoff where the tails are
negligible, the mesh sums of Sec. 3.3.1 equal the continuous integrals up to
aliasing (spectrally small on these meshes) and spline interpolation error:

  S_AB = sum_T (1/4pi) (pi/p)^{3/2} exp(-mu |A - B - T|^2),
  <A| cos(G.r) |B> = sum_T (1/4pi) (pi/p)^{3/2} exp(-mu|A-B-T|^2)
                     exp(-|G|^2/4p) cos(G.P_T),
  p = a + b, mu = a b / p, P_T = (a A + b (B + T)) / p.
"""
import math

import numpy as np
import pytest

import gint_inputs as gi

ALPHAS = (0.6, 1.1)  # two s radials per atom (zeta = 1, 2)
RC = 10.0


def _cell(seed=0, L=9.0, N=28):
    rng = np.random.default_rng(seed)
    sp = gi.Species([gi.nao_like_radial(0, a, RC, 0.01, smooth_cutoff=False) for a in ALPHAS])
    pos = rng.uniform(0, L, (3, 3))
    lat = np.diag([L, L * 1.1, L * 0.95])
    w = gi.small_cell(pos, lat, (N, int(N * 1.1), int(N * 0.95)), [sp], n_waves=5, nocc=3, seed=seed)
    return w


def _images(lat, n=3):
    r = range(-n, n + 1)
    return np.array([i * lat[0] + j * lat[1] + k * lat[2] for i in r for j in r for k in r])


def _pw_G(w):
    B = np.linalg.inv(w.lattice).T
    return 2 * np.pi * (w.pw_m @ B)


def closed_form(w, V_kind):
    """Analytic H (s-only Gaussians) for V = 1 or the workload's plane waves."""
    T = _images(w.lattice)
    orbs = [(I, a) for I in range(w.natom) for a in ALPHAS]
    n = len(orbs)
    H = np.zeros((n, n))
    G = _pw_G(w)
    for i, (I, a) in enumerate(orbs):
        for j, (J, b) in enumerate(orbs):
            p = a + b
            mu = a * b / p
            A = w.positions[I]
            Bs = w.positions[J] + T
            R2 = np.sum((A - Bs) ** 2, axis=1)
            base = (1 / (4 * np.pi)) * (np.pi / p) ** 1.5 * np.exp(-mu * R2)
            if V_kind == "one":
                H[i, j] = base.sum()
            else:
                P = (a * A + b * Bs) / p
                tot = 0.0
                for k in range(len(w.pw_amp)):
                    tot += w.pw_amp[k] * np.sum(base * np.exp(-G[k] @ G[k] / (4 * p)) * np.cos(P @ G[k]))
                H[i, j] = tot
    return H


def closed_form_energy_gradient(w, D):
    """dE/dR for E = sum_ij D_ij <i|V|j> with the plane-wave V (analytic)."""
    T = _images(w.lattice)
    orbs = [(I, a) for I in range(w.natom) for a in ALPHAS]
    G = _pw_G(w)
    grad = np.zeros((w.natom, 3))
    for i, (I, a) in enumerate(orbs):
        for j, (J, b) in enumerate(orbs):
            p = a + b
            mu = a * b / p
            A = w.positions[I]
            Bs = w.positions[J] + T
            dAB = A - Bs
            R2 = np.sum(dAB**2, axis=1)
            base = (1 / (4 * np.pi)) * (np.pi / p) ** 1.5 * np.exp(-mu * R2)
            P = (a * A + b * Bs) / p
            for k in range(len(w.pw_amp)):
                c = w.pw_amp[k] * np.exp(-G[k] @ G[k] / (4 * p)) * D[i, j]
                ph = P @ G[k]
                t = base * c
                # d/dA and d/dB of exp(-mu|A-B|^2) cos(G.P)
                dA = (-2 * mu * dAB * np.cos(ph)[:, None] - np.sin(ph)[:, None] * G[k] * (a / p)) * t[:, None]
                dB = (2 * mu * dAB * np.cos(ph)[:, None] - np.sin(ph)[:, None] * G[k] * (b / p)) * t[:, None]
                grad[I] += dA.sum(0)
                grad[J] += dB.sum(0)
    return grad


@pytest.mark.parametrize("seed", [0, 1])
def test_gaussian_overlap_closed_form(oracle_mod, seed):
    w = _cell(seed)
    o = oracle_mod.Oracle.from_workload(w)
    S = o.H(np.ones(w.ngrid))
    S_ref = closed_form(w, "one")
    assert np.max(np.abs(S - S_ref)) <= 1e-8 * np.max(np.abs(S_ref))


@pytest.mark.parametrize("seed", [0, 3])
def test_plane_wave_matrix_elements_closed_form(oracle_mod, seed):
    w = _cell(seed)
    o = oracle_mod.Oracle.from_workload(w)
    H = o.H(w.V)
    H_ref = closed_form(w, "pw")
    assert np.max(np.abs(H - H_ref)) <= 1e-8 * np.max(np.abs(H_ref))


def test_force_closed_form(oracle_mod):
    w = _cell(2)
    o = oracle_mod.Oracle.from_workload(w)
    F = o.force(w.V, w.D)
    F_ref = closed_form_energy_gradient(w, w.D)
    # the radial derivative comes from the spline, whose slope error is
    # O(dr^3 max|f''''|); measured agreement is ~5e-9 relative
    assert np.max(np.abs(F - F_ref)) <= 5e-8 * np.max(np.abs(F_ref))
    # and the energy itself matches the closed form sum_ij D_ij H_ij
    H_ref = closed_form(w, "pw")
    assert abs(o.energy(w.V, w.D) - np.sum(w.D * H_ref)) <= 1e-8 * np.sum(np.abs(w.D * H_ref))
