"""Brute force on tiny cells vs the oracle (image logic, folding, p/d).

The brute force (tests/bruteforce.py) uses scipy's clamped spline, scipy's
spherical harmonics and all lattice images in a generous cube, with no
neighbour search.  Cells are chosen so several images of one atom reach the
same mesh point (rc > L/2), which is where folding matters.
"""
import numpy as np
import pytest

import gint_inputs as gi
from tests.bruteforce import BruteCell


def _two_atom_dzp(rc=5.0):
    sp = gi.Species([
        gi.nao_like_radial(0, 0.4, rc, 0.01),
        gi.nao_like_radial(1, 0.9, rc, 0.01),
        gi.nao_like_radial(2, 0.7, rc, 0.01),
    ])
    sp2 = gi.sz_species(rc=4.0)
    lat = np.array([[6.0, 0.0, 0.0], [0.7, 6.5, 0.0], [-0.4, 0.3, 7.0]])  # triclinic
    pos = np.array([[0.3, 0.2, 0.1], [3.1, 2.7, 3.9]])
    return gi.small_cell(pos, lat, (10, 11, 12), [sp, sp2], species_of_atom=[0, 1],
                         n_waves=6, nocc=3, seed=7)


def _tiny_long_range():
    # rc = 5.5 > L = 4: images two cells away still carry weight (slow decay)
    sp = gi.Species([gi.nao_like_radial(0, 0.08, 5.5, 0.01), gi.nao_like_radial(1, 0.1, 5.5, 0.01),
                     gi.nao_like_radial(2, 0.12, 5.5, 0.01)])
    lat = np.array([[4.0, 0.0, 0.0], [0.0, 4.4, 0.0], [0.5, 0.0, 4.2]])
    pos = np.array([[0.2, 0.3, 0.1], [2.1, 2.4, 1.9]])
    return gi.small_cell(pos, lat, (7, 8, 8), [sp], n_waves=5, nocc=4, seed=9)


def _si8_coarse():
    w = gi.si8_sz()
    w2 = gi.small_cell(w.positions, w.lattice, (12, 12, 12), w.species, n_waves=8, nocc=8, seed=11)
    return w2


@pytest.mark.parametrize("make", [_two_atom_dzp, _tiny_long_range, _si8_coarse])
def test_bruteforce_H_rho(oracle_mod, make):
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    bf = BruteCell(w)
    phi = bf.phi_all()
    H_bf = bf.H(w.V, phi)
    H = o.H(w.V)
    assert np.max(np.abs(H - H_bf)) <= 1e-13 * max(1.0, np.max(np.abs(H_bf)))
    rho_bf = bf.rho(w.D, phi)
    rho = o.rho(w.D)
    assert np.max(np.abs(rho - rho_bf)) <= 1e-13 * max(1.0, np.max(np.abs(rho_bf)))


@pytest.mark.parametrize("make", [_two_atom_dzp, _tiny_long_range])
def test_bruteforce_force_by_differences(oracle_mod, make):
    # the brute force has no analytic gradient: differentiate its energy
    w = make()
    o = oracle_mod.Oracle.from_workload(w)
    bf = BruteCell(w)
    F = o.force(w.V, w.D)
    h = 1e-5
    for I in range(w.natom):
        for k in range(3):
            p1 = w.positions.copy()
            p1[I, k] += h
            p2 = w.positions.copy()
            p2[I, k] -= h
            fd = (bf.energy(w.V, w.D, p1) - bf.energy(w.V, w.D, p2)) / (2 * h)
            assert abs(F[I, k] - fd) <= 1e-7 * max(1.0, np.max(np.abs(F)))


@pytest.mark.parametrize("make", [_two_atom_dzp, _tiny_long_range, _si8_coarse])
def test_support_stats_bruteforce(oracle_mod, make):
    # the work counts behind the roofline (sum_g n_g, sum_g n_g^2) are exact
    # integers: the oracle's count equals the brute-force count
    w = make()
    s1, s2 = oracle_mod.Oracle.from_workload(w).support_stats()
    b1, b2 = BruteCell(w).support_stats()
    assert (s1, s2) == (b1, b2)
