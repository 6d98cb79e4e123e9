"""Pins of the oracle's lattice-vector blocks H(R) (Sec. 3.3.1, H^loc(R)
equation; Sec. 2.1, H(k) equation) and of rho from lattice-vector density
matrices D(R) (Sec. 3.3.1, rho(r_g) equation with its sums over R, R').

* brute force: every crystal mesh point enumerated as a cell point shifted by
  a lattice vector, unfolded orbitals from scipy's spline and harmonics;
* the Gamma point: sum over all R of H(R) is the folded H of the oracle's
  Gamma path (a different image search and loop);
* a 3x1x1 supercell: its Gamma-point blocks between copy c1 of atom I and
  copy c2 of atom J are the sum of H(R) over n1 = c2 - c1 mod 3 and all
  n2, n3 (the supercell runs through the folded Gamma path);
* Hermiticity H(R)_IJ = H(-R)_JI^T, and the lattice-translation rule for
  positions given outside the cell;
* rho(D(R)): brute force; D(R) = D for every R gives the folded Gamma-point
  rho of D; the energy identity dV sum_g V_g rho_g = sum_R <D(R), H(R)>
  against the oracle's H(R) (random, non-symmetric D(R));
* dE/dR for D(R): central differences of that energy, and the Gamma-point
  force for D(R) = D.
"""
import numpy as np
import pytest

import gint_inputs as gi
from tests.bruteforce import BruteCell
from tests.test_oracle_bruteforce import _tiny_long_range, _two_atom_dzp


def _box(n):
    r = range(-n, n + 1)
    return np.array([(a, b, c) for a in r for b in r for c in r], dtype=np.int32)


def _index(R):
    return {tuple(int(x) for x in r): i for i, r in enumerate(R)}


@pytest.mark.parametrize("make", [_two_atom_dzp, _tiny_long_range])
def test_hr_bruteforce(oracle_mod, make):
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(2)
    HR = o.HR(w.V, R)
    bf = BruteCell(w).HR(w.V, [tuple(r) for r in R])
    scale = max(1.0, np.abs(bf).max())
    assert np.abs(bf).max() > 1e-3
    assert np.abs(HR - bf).max() <= 1e-13 * scale


@pytest.mark.parametrize("make", [gi.si8_sz, _two_atom_dzp, _tiny_long_range])
def test_hr_sum_is_gamma(oracle_mod, make):
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(4)
    HR = o.HR(w.V, R)
    # the outer shell of the box is empty, so no R was dropped
    idx = _index(R)
    shell = [i for r, i in idx.items() if max(abs(x) for x in r) == 4]
    assert np.abs(HR[shell]).max() == 0.0
    H = o.H(w.V)
    assert np.abs(HR.sum(0) - H).max() <= 1e-13 * max(1.0, np.abs(H).max())


@pytest.mark.parametrize("make", [gi.si8_sz, _two_atom_dzp])
def test_hr_transpose(oracle_mod, make):
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(3)
    HR = o.HR(w.V, R)
    idx = _index(R)
    for r, i in idx.items():
        j = idx[tuple(-x for x in r)]
        assert np.abs(HR[i] - HR[j].T).max() <= 1e-15 * max(1.0, np.abs(HR).max())


def test_hr_translation(oracle_mod):
    # atom J moved by the lattice vector L: H'(R)_IJ = H(R + L)_IJ,
    # H'(R)_JI = H(R - L)_JI, other blocks unchanged
    w = _two_atom_dzp()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(3)
    idx = _index(R)
    HR = o.HR(w.V, R)
    L = np.array([1, -2, 1])
    pos = np.array(w.positions, dtype=np.float64)
    pos[1] += L @ np.asarray(w.lattice)
    o.set_positions(pos)
    HR2 = o.HR(w.V, R)
    a0, a1 = o.atom_orb0[1], o.atom_orb0[2]
    I = slice(0, a0)
    J = slice(a0, a1)
    checked = 0
    for r, i in idx.items():
        rp = tuple(int(x) for x in np.array(r) + L)
        rm = tuple(int(x) for x in np.array(r) - L)
        # (positions change by a lattice vector: equal up to rounding of d)
        assert np.abs(HR2[i][I, I] - HR[i][I, I]).max() <= 1e-14
        assert np.abs(HR2[i][J, J] - HR[i][J, J]).max() <= 1e-14
        if rp in idx:
            assert np.abs(HR2[i][I, J] - HR[idx[rp]][I, J]).max() <= 1e-14
            checked += np.abs(HR[idx[rp]][I, J]).max() > 0
        if rm in idx:
            assert np.abs(HR2[i][J, I] - HR[idx[rm]][J, I]).max() <= 1e-14
    assert checked > 0


def test_hr_supercell(oracle_mod):
    w = _two_atom_dzp()
    lat = np.asarray(w.lattice, dtype=np.float64)
    N = w.grid
    # 3x1x1 supercell: copies c = 0, 1, 2 of every atom at tau + c a1, the
    # same periodic V on the tripled mesh
    pos_sc = np.concatenate([np.asarray(w.positions) + c * lat[0] for c in range(3)])
    spc_sc = np.concatenate([w.species_of_atom] * 3)
    lat_sc = lat.copy()
    lat_sc[0] *= 3
    V3 = np.asarray(w.V).reshape(N)
    V_sc = np.concatenate([V3] * 3, axis=0).reshape(-1)
    o_sc = oracle_mod.Oracle(lat_sc, (3 * N[0], N[1], N[2]), w.species, spc_sc, pos_sc)
    H_sc = o_sc.H(V_sc)
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(4)
    HR = o.HR(w.V, R)
    nb = o.norb
    for c1 in range(3):
        for c2 in range(3):
            want = sum(HR[i] for i, r in enumerate(R) if (int(r[0]) - (c2 - c1)) % 3 == 0)
            got = H_sc[c1 * nb:(c1 + 1) * nb, c2 * nb:(c2 + 1) * nb]
            assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max())


def _random_DR(rng, nR, norb):
    return rng.normal(size=(nR, norb, norb)) / norb


@pytest.mark.parametrize("make", [_two_atom_dzp, _tiny_long_range])
def test_rhoR_bruteforce(oracle_mod, make):
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(2)
    DR = _random_DR(np.random.default_rng(1), len(R), o.norb)
    rho = o.rhoR(R, DR)
    bf = BruteCell(w).rhoR([tuple(r) for r in R], DR)
    assert np.abs(bf).max() > 1e-3
    assert np.abs(rho - bf).max() <= 1e-13 * max(1.0, np.abs(bf).max())


@pytest.mark.parametrize("make", [gi.si8_sz, _two_atom_dzp, _tiny_long_range])
def test_rhoR_constant_is_gamma(oracle_mod, make):
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(4)
    DR = np.broadcast_to(w.D, (len(R),) + w.D.shape).copy()
    rho = o.rhoR(R, DR)
    ref = o.rho(w.D)
    assert np.abs(rho - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("make", [gi.si8_sz, _two_atom_dzp])
def test_rhoR_energy_identity(oracle_mod, make):
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(3)
    DR = _random_DR(np.random.default_rng(2), len(R), o.norb)
    E1 = o.dV * float(np.dot(w.V, o.rhoR(R, DR)))
    E2 = float(np.sum(DR * o.HR(w.V, R)))
    assert abs(E1 - E2) <= 1e-12 * max(1.0, np.sum(np.abs(DR * o.HR(w.V, R))))


def test_hk_pins(oracle_mod):
    # H(k) of Sec. 2.1 from the oracle's H(R): k = 0 is the Gamma-point H,
    # H(k + G) = H(k), H(k) Hermitian, and the 3x1x1 supercell's Gamma-point
    # blocks are (1/3) sum_m e^{-i 2 pi m c / 3} H(k_m), k_m = (m/3, 0, 0)
    w = _two_atom_dzp()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(4)
    HR = o.HR(w.V, R)
    H = o.H(w.V)
    ks = np.array([[0.0, 0.0, 0.0], [0.25, -0.1, 0.4], [1.25, 0.9, -0.6], [1 / 3, 0, 0], [2 / 3, 0, 0]])
    Hk = oracle_mod.Hk_from_HR(R, HR, ks)
    scale = np.abs(H).max()
    assert np.abs(Hk[0] - H).max() <= 1e-13 * scale
    assert np.abs(Hk[1] - Hk[2]).max() <= 1e-12 * scale
    for h in Hk:
        assert np.abs(h - h.conj().T).max() <= 1e-13 * scale
    lat = np.asarray(w.lattice, dtype=np.float64)
    N = w.grid
    pos_sc = np.concatenate([np.asarray(w.positions) + c * lat[0] for c in range(3)])
    lat_sc = lat.copy()
    lat_sc[0] *= 3
    V_sc = np.concatenate([np.asarray(w.V).reshape(N)] * 3, axis=0).reshape(-1)
    o_sc = oracle_mod.Oracle(lat_sc, (3 * N[0], N[1], N[2]), w.species,
                             np.concatenate([w.species_of_atom] * 3), pos_sc)
    H_sc = o_sc.H(V_sc)
    nb = o.norb
    km = [Hk[0], Hk[3], Hk[4]]
    for c in range(3):
        want = sum(np.exp(-2j * np.pi * m * c / 3) * km[m] for m in range(3)) / 3
        got = H_sc[0:nb, c * nb:(c + 1) * nb]
        assert np.abs(want.imag).max() <= 1e-12 * scale
        assert np.abs(got - want.real).max() <= 1e-12 * scale


@pytest.mark.parametrize("make", [_two_atom_dzp, _tiny_long_range])
def test_forceR_by_differences(oracle_mod, make):
    # dE/dR of E = dV sum V rho(D(R)) against central differences of E
    # computed with rhoR (positions as given; R fixed)
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(3)
    DR = _random_DR(np.random.default_rng(3), len(R), o.norb)
    F = o.forceR(w.V, R, DR)
    pos0 = np.array(w.positions, dtype=np.float64)
    h = 1e-4
    for I in range(len(pos0)):
        for k in range(3):
            e = []
            for sgn in (1, -1):
                pos = pos0.copy()
                pos[I, k] += sgn * h
                o.set_positions(pos)
                e.append(o.dV * float(np.dot(w.V, o.rhoR(R, DR))))
            fd = (e[0] - e[1]) / (2 * h)
            assert abs(F[I, k] - fd) <= 1e-6 * max(1.0, np.abs(F).max()), (I, k, F[I, k], fd)
    o.set_positions(pos0)


@pytest.mark.parametrize("make", [gi.si8_sz, _two_atom_dzp])
def test_forceR_constant_is_gamma(oracle_mod, make):
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    R = _box(4)
    DR = np.broadcast_to(w.D, (len(R),) + w.D.shape).copy()
    F = o.forceR(w.V, R, DR)
    ref = o.force(w.V, w.D)
    assert np.abs(F - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
