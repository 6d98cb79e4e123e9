"""GPU parity of the moving-basis matrix (gint_build_DK; Sec. 2.3, D_K
equation at k = 0 on the mesh) against the FP64 oracle.

    DK[c, mu, nu] = <phit_mu | W | d phit_nu / d tau_K>_c,  K = atom of nu.

FP64 bar: max|dDK| / max|DK| <= 1e-10 (W = 1 and W = V), on Si-8 and the
four small cells of the Gamma-point parity tests (whole matrices), on
sampled rows at Si-64 and Si-512, for 32- and 16-point batches; repeatable
bits; and the grid force from DK(W = V) equals gint_force's.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gint_inputs as gi
from tests.test_gpu_parity import (TOL, _dev, _long_range_tiny, _ragged_five_atoms, _rel_max,
                                   _triclinic_two_species, _vacuum_single_atom)

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("make", [gi.si8_sz, _triclinic_two_species, _long_range_tiny, _ragged_five_atoms,
                                  _vacuum_single_atom])
def test_dk_full(oracle_mod, torch_dev, make):
    torch, dev = torch_dev
    import paper_2603_21835_amd as g

    w = make()
    _say(f"case DK {w.name} grid {w.grid} natom {w.natom}")
    plan = g.GintPlan.from_workload(w)
    o = oracle_mod.Oracle.from_workload(w)
    V = _dev(torch, dev, w.V)
    for W, Wh, tag in ((None, None, "W=1"), (V, w.V, "W=V")):
        DK = plan.build_DK(W).cpu().numpy()
        ref = o.DK(Wh)
        e = _rel_max(DK, ref)
        _say(f"  {tag}: rel {e:.2e}")
        assert e <= TOL
        assert np.array_equal(DK, plan.build_DK(W).cpu().numpy())  # repeatable bits


@pytest.mark.parametrize("batch", [(2, 4, 4), (2, 2, 4)])
def test_dk_batch_shapes(oracle_mod, torch_dev, batch):
    torch, dev = torch_dev
    import paper_2603_21835_amd as g

    w = _ragged_five_atoms()
    _say(f"case DK batch {batch}")
    plan = g.GintPlan.from_workload(w)
    plan.tune(batch)
    DK = plan.build_DK(_dev(torch, dev, w.V)).cpu().numpy()
    assert _rel_max(DK, oracle_mod.Oracle.from_workload(w).DK(w.V)) <= TOL


def test_dk_gives_grid_force(torch_dev):
    # dE/dR_I = sum_{mu on I} sum_nu (D + D^T)_mu,nu DK_V[., nu, mu], both on the GPU
    torch, dev = torch_dev
    import paper_2603_21835_amd as g

    w = _triclinic_two_species()
    plan = g.GintPlan.from_workload(w)
    V, D = _dev(torch, dev, w.V), _dev(torch, dev, w.D)
    DK = plan.build_DK(V).cpu().numpy()
    F = plan.force(V, D).cpu().numpy()
    S2 = w.D + w.D.T
    o0 = np.concatenate([[0], np.cumsum([w.species[s].norb for s in w.species_of_atom])])
    ref = np.array([[np.sum(S2[o0[I]:o0[I + 1], :] * DK[c][:, o0[I]:o0[I + 1]].T) for c in range(3)]
                    for I in range(w.natom)])
    e = _rel_max(ref, F)
    _say(f"case DK -> force identity: rel {e:.2e}")
    assert e <= 1e-12


def _sampled_rows(oracle_mod, torch, dev, w, atoms):
    import paper_2603_21835_amd as g

    plan = g.GintPlan.from_workload(w)
    V = _dev(torch, dev, w.V)
    DK1 = plan.build_DK(None).cpu().numpy()
    DKV = plan.build_DK(V).cpu().numpy()
    plan.close()
    o = oracle_mod.Oracle.from_workload(w)
    jobs = [(None, I) for I in atoms] + [(w.V, I) for I in atoms]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        refs = list(ex.map(lambda j: o.DK_rows(j[0], j[1], j[1] + 1), jobs))
    for (Wh, I), ref in zip(jobs, refs):
        r0 = o.atom_orb0[I]
        got = (DK1 if Wh is None else DKV)[:, r0:r0 + ref.shape[1]]
        e = _rel_max(got, ref)
        _say(f"  rows of atom {I} ({'W=1' if Wh is None else 'W=V'}): rel {e:.2e}")
        assert e <= TOL


def test_dk_si64_sampled(oracle_mod, torch_dev):
    torch, dev = torch_dev
    w = gi.si64_dzp()
    _say("case DK si64 sampled rows")
    _sampled_rows(oracle_mod, torch, dev, w, [0, 21, 63])


@pytest.mark.timeout(600)
def test_dk_si512_sampled(oracle_mod, torch_dev):
    torch, dev = torch_dev
    w = gi.si512_dzp()
    _say("case DK si512 sampled rows")
    _sampled_rows(oracle_mod, torch, dev, w, [int(w.fd_atoms[1]), int(w.fd_atoms[5])])
