"""The benchmark's call, gint_H_rho_force, at the benchmark's size (Si-512
DZP, 192^3 mesh) against the FP64 oracle, element by element on sampled
outputs (Sec. 3.3.1: the H^loc, rho(r_g) and F^{loc,Pulay} equations).

Sampled outputs:
  * H rows of four atoms: the first and the last atom of the plan's internal
    (Morton) processing order and two of the workload's FD atoms;
  * rho at 20 000 random mesh points;
  * dE/dR of the same four atoms.
FP64 bar: relative error <= 1e-10 (max|dH|/max|H| over the sampled rows,
relative L2 over the rho sample, max|dF|/max|F| over the atoms).
FP32 and FP16 hi/lo (3 products) bar: max|dH| <= 1e-6 Ha absolute (the
mixed-precision target), rho relative L2 and force relative max <= 1e-6.
BF16 hi/lo misses the 1e-6 Ha target at this size (about 1.4e-5 Ha); it is
kept only as a regression pin at 3e-5 Ha and meets no target.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gint_inputs as gi

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def si512(oracle_mod):
    """Si-512 inputs, the sampled atoms and points, and the oracle's values
    for them (computed once for the module)."""
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_21835_amd as g

    g.load_library()
    dev = torch.device("cuda:0")
    w = gi.si512_dzp()
    plan = g.GintPlan.from_workload(w)
    order = plan.atom_order()
    plan.close()
    atoms = [int(order[0]), int(order[-1]), int(w.fd_atoms[0]), int(w.fd_atoms[3])]
    assert len(set(atoms)) == 4, atoms
    idx = np.sort(np.random.default_rng(20).choice(w.ngrid, 20000, replace=False))
    _say(f"si512 oracle: H rows and dE/dR of atoms {atoms} (first/last internal, 2 FD atoms), "
         f"rho at {idx.size} points")
    o = oracle_mod.Oracle.from_workload(w)
    # one single-atom H-row call per thread (each call is parallel over its atoms)
    with ThreadPoolExecutor(max_workers=4) as ex:
        rows = list(ex.map(lambda I: o.H_rows(w.V, I, I + 1), atoms))
    _say("  oracle H rows done")
    ref = {"rows": rows, "rho": o.rho(w.D, idx)}
    _say("  oracle rho done")
    ref["F"] = o.force(w.V, w.D, atoms)
    _say("si512 oracle done")
    return torch, dev, w, o, atoms, idx, ref


def _errors(w, o, atoms, idx, ref, H, rho, F):
    eH_abs, Hmax = 0.0, 0.0
    for I, rows in zip(atoms, ref["rows"]):
        r0 = o.atom_orb0[I]
        eH_abs = max(eH_abs, float(np.abs(H[r0:r0 + rows.shape[0]] - rows).max()))
        Hmax = max(Hmax, float(np.abs(rows).max()))
    er = float(np.linalg.norm(rho[idx] - ref["rho"]) / np.linalg.norm(ref["rho"]))
    eF = float(np.abs(F[atoms] - ref["F"]).max() / np.abs(ref["F"]).max())
    return eH_abs, eH_abs / Hmax, er, eF


def _run(torch, dev, w, precision):
    import paper_2603_21835_amd as g

    plan = g.GintPlan.from_workload(w, precision=precision)
    V = torch.from_numpy(w.V).to(dev)
    D = torch.from_numpy(w.D).to(dev)
    H, rho, F = (t.cpu().numpy() for t in plan.H_rho_force(V, D))
    work = plan.work()
    plan.close()
    return H, rho, F, work


@pytest.mark.timeout(900)
def test_H_rho_force_si512_fp64(si512):
    torch, dev, w, o, atoms, idx, ref = si512
    _say("case H_rho_force si512 fp64 (the benchmark's call and configuration)")
    H, rho, F, work = _run(torch, dev, w, "fp64")
    assert work["nslab"] == 1  # the benchmark's launch configuration: one H slab
    eH_abs, eH, er, eF = _errors(w, o, atoms, idx, ref, H, rho, F)
    _say(f"  H rows rel {eH:.2e} (abs {eH_abs:.2e} Ha)  rho rel-L2 {er:.2e}  dE/dR rel {eF:.2e}")
    assert eH <= TOL and er <= TOL and eF <= TOL
    assert np.array_equal(H, H.T)
    E = o.dV * float(np.dot(w.V, rho))
    assert abs(E - np.sum(w.D * H)) <= 1e-11 * np.sum(np.abs(w.D * H))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_H_rho_force_si512_mixed(si512, precision):
    torch, dev, w, o, atoms, idx, ref = si512
    _say(f"case H_rho_force si512 {precision}")
    H, rho, F, _ = _run(torch, dev, w, precision)
    eH_abs, eH, er, eF = _errors(w, o, atoms, idx, ref, H, rho, F)
    _say(f"  {precision}: max|dH| {eH_abs:.2e} Ha  rho rel-L2 {er:.2e}  dE/dR rel {eF:.2e}")
    assert eH_abs <= 1e-6 and er <= 1e-6 and eF <= 1e-6


@pytest.mark.timeout(900)
def test_H_rho_force_si512_bf16x3_regression_pin(si512):
    # BF16 hi/lo does NOT meet the 1e-6 Ha target; this only pins its level
    torch, dev, w, o, atoms, idx, ref = si512
    _say("case H_rho_force si512 bf16x3 (regression pin, misses the target)")
    H, rho, F, _ = _run(torch, dev, w, "bf16x3")
    eH_abs, eH, er, eF = _errors(w, o, atoms, idx, ref, H, rho, F)
    _say(f"  bf16x3: max|dH| {eH_abs:.2e} Ha  rho rel-L2 {er:.2e}  dE/dR rel {eF:.2e}")
    assert eH_abs <= 3e-5 and er <= 1e-6 and eF <= 1e-6
