"""GPU parity of the spherical-grid projector overlaps (gint_psibeta_*;
Sec. 3.3.2) against the FP64 oracle:

    Q[p, mu] = <phit_mu | e^{-i A.r} | beta_p>

on the 110-point Lebedev x Gauss-Legendre product grid around each
projector atom.  FP64 bar: max|dQ| / max|Q| <= 1e-10 on whole matrices of
small cells (a triclinic two-species cell, Si-8, a cell smaller than the
orbitals' reach, an atom in vacuum), after the atoms move, and on the rows
of sampled projector atoms at Si-64 and Si-512; repeatable bits; Q(0) real.
"""
import sys

import numpy as np
import pytest

import gint_inputs as gi
from tests.test_gpu_parity import _long_range_tiny, _vacuum_single_atom

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_21835_amd as g

    g.load_library()
    return torch, torch.device("cuda:0")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _triclinic():
    sp = gi.Species([gi.nao_like_radial(0, 0.4, 5.0), gi.nao_like_radial(1, 0.9, 5.0),
                     gi.nao_like_radial(2, 0.7, 5.0)])
    lat = np.array([[6.0, 0.0, 0.0], [0.7, 6.5, 0.0], [-0.4, 0.3, 7.0]])
    pos = np.array([[0.3, 0.2, 0.1], [3.1, 2.7, 3.9], [5.0, 5.5, 0.2]])
    w = gi.small_cell(pos, lat, (12, 12, 12), [sp, gi.sz_species(4.0)], species_of_atom=[0, 1, 0],
                      n_waves=4, nocc=3, seed=7)
    return w, [gi.si_projector_species(), gi.Species([gi.nao_like_radial(0, 1.2, 1.8)])]


def _si8():
    return gi.si8_sz(), [gi.si_projector_species()]


def _long_range():
    w = _long_range_tiny()
    return w, [gi.Species([gi.nao_like_radial(0, 0.9, 2.5), gi.nao_like_radial(2, 0.9, 2.5)])]


def _vacuum():
    return _vacuum_single_atom(), [gi.si_projector_species()]


def _run(torch, w, proj, A, nrq=140, plan=None):
    import paper_2603_21835_amd as g

    plan = plan or g.GintPlan.from_workload(w)
    pb = g.GintPsiBeta(plan, proj, gi.lebedev_110(), gi.gauss_legendre_01(nrq))
    Q = pb.overlap(A).cpu().numpy()
    return plan, pb, Q


@pytest.mark.parametrize("make", [_triclinic, _si8, _long_range, _vacuum])
def test_psibeta_full(oracle_mod, torch_dev, make):
    torch, dev = torch_dev
    w, proj = make()
    A = gi.vector_potential(11)
    _say(f"case psibeta {w.name} natom {w.natom}")
    plan, pb, Q = _run(torch, w, proj, A)
    ref = oracle_mod.Oracle.from_workload(w).psibeta(proj, gi.lebedev_110(), gi.gauss_legendre_01(140), A)
    e = _rel(Q, ref)
    _say(f"  {Q.shape[0]} projectors: rel {e:.2e}")
    assert Q.shape == ref.shape and e <= TOL
    assert np.array_equal(Q, pb.overlap(A).cpu().numpy())  # repeatable bits
    Q0 = pb.overlap(np.zeros(3)).cpu().numpy()
    assert np.all(Q0.imag == 0.0)


def test_psibeta_after_moving_atoms(oracle_mod, torch_dev):
    torch, dev = torch_dev
    w, proj = _triclinic()
    A = gi.vector_potential(12)
    plan, pb, Q = _run(torch, w, proj, A)
    rng = np.random.default_rng(5)
    w.positions = w.positions + rng.normal(0, 0.4, w.positions.shape) + w.lattice[2]
    plan.set_positions(w.positions)
    _say("case psibeta moved atoms")
    Q2 = pb.overlap(A).cpu().numpy()
    ref = oracle_mod.Oracle.from_workload(w).psibeta(proj, gi.lebedev_110(), gi.gauss_legendre_01(140), A)
    e = _rel(Q2, ref)
    _say(f"  rel {e:.2e}")
    assert e <= TOL


def _sampled(oracle_mod, torch, w, atoms):
    proj = [gi.si_projector_species()]
    A = gi.vector_potential(13, 0.05)
    plan, pb, Q = _run(torch, w, proj, A)
    o = oracle_mod.Oracle.from_workload(w)
    for I in atoms:
        ref = o.psibeta(proj, gi.lebedev_110(), gi.gauss_legendre_01(140), A, I, I + 1)
        got = Q[9 * I:9 * I + 9]
        e = _rel(got, ref)
        _say(f"  rows of atom {I}: rel {e:.2e}")
        assert e <= TOL


def test_psibeta_si64_sampled(oracle_mod, torch_dev):
    torch, dev = torch_dev
    _say("case psibeta si64 sampled")
    _sampled(oracle_mod, torch, gi.si64_dzp(), [0, 45])


@pytest.mark.timeout(600)
def test_psibeta_si512_sampled(oracle_mod, torch_dev):
    torch, dev = torch_dev
    w = gi.si512_dzp()
    _say("case psibeta si512 sampled")
    _sampled(oracle_mod, torch, w, [int(w.fd_atoms[2])])
