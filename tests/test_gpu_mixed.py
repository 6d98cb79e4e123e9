"""Mixed-precision modes against the FP64 oracle.

FP32 mode (and rho and the force in the other 16-bit modes): orbital tiles,
packed D and per-batch H block partials in FP32 on v_mfma_f32_16x16x4; every
cross-batch sum and every dot product stays FP64.  16-bit modes: H operands
in BF16 or FP16 (single or hi/lo split) on v_mfma_f32_16x16x32; in the FP16
hi/lo mode the rho / force contraction T = (D + D^T) phi runs as three FP16
hi/lo products on v_mfma_f32_16x16x16f16 as well.
The accuracy target for the mixed path is max|dH| <= 1e-6 Ha (absolute);
the rho relative-L2 and force errors are reported beside it.
"""
import sys

import numpy as np
import pytest

import gint_inputs as gi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tdev():
    import torch

    assert torch.cuda.is_available()
    import paper_2603_21835_amd as g

    g.load_library()
    return torch, torch.device("cuda:0")


def _run(torch, dev, w, prec):
    import paper_2603_21835_amd as g

    plan = g.GintPlan.from_workload(w, precision=prec)
    V = torch.from_numpy(w.V).to(dev)
    D = torch.from_numpy(w.D).to(dev)
    H = plan.build_H(V).cpu().numpy()
    rho = plan.build_rho(D).cpu().numpy()
    F = plan.force(V, D).cpu().numpy()
    return H, rho, F


def test_fp32_si8_full(tdev, oracle_mod):
    torch, dev = tdev
    w = gi.si8_sz()
    H, rho, F = _run(torch, dev, w, "fp32")
    o = oracle_mod.Oracle.from_workload(w)
    Ho, ro, Fo = o.H(w.V), o.rho(w.D), o.force(w.V, w.D)
    dH = np.abs(H - Ho).max()
    er = np.linalg.norm(rho - ro) / np.linalg.norm(ro)
    eF = np.abs(F - Fo).max() / np.abs(Fo).max()
    _say(f"  fp32 si8: max|dH| {dH:.2e} Ha  rho rel-L2 {er:.2e}  F rel {eF:.2e}")
    assert dH <= 1e-6 and er <= 1e-5 and eF <= 1e-4
    assert np.array_equal(H, H.T)


def test_fp32_si64_sampled(tdev, oracle_mod):
    torch, dev = tdev
    w = gi.si64_dzp()
    H, rho, F = _run(torch, dev, w, "fp32")
    o = oracle_mod.Oracle.from_workload(w)
    dH = 0.0
    for I in (0, 42):
        rows = o.H_rows(w.V, I, I + 1)
        r0 = o.atom_orb0[I]
        dH = max(dH, np.abs(H[r0:r0 + rows.shape[0]] - rows).max())
    idx = np.random.default_rng(0).choice(w.ngrid, 20000, replace=False)
    ro = o.rho(w.D, idx)
    er = np.linalg.norm(rho[idx] - ro) / np.linalg.norm(ro)
    Fo = o.force(w.V, w.D, [5, 60])
    eF = np.abs(F[[5, 60]] - Fo).max() / np.abs(Fo).max()
    _say(f"  fp32 si64: max|dH| {dH:.2e} Ha  rho rel-L2 {er:.2e}  F rel {eF:.2e}")
    assert dH <= 1e-6 and er <= 1e-5 and eF <= 1e-4


# max|dH| bounds per mode (Ha) on Si-64 DZP.  FP16 hi/lo keeps 22 bits of
# each operand and meets the 1e-6 Ha target (measured 6.6e-8).  BF16 hi/lo
# keeps only 16 bits (8 + 8), and misses it (measured 4.0e-6 here, 1.4e-5 at
# Si-512); single-pass 16-bit operands (unit roundoff 2^-9 / 2^-12) miss it
# by more.  Those bounds are loose pins of the measured error, not targets.
MODES16 = {"fp16x3": 1e-6, "bf16x3": 2e-5, "bf16": 2e-3, "fp16": 5e-4}


@pytest.mark.parametrize("prec", list(MODES16))
def test_16bit_H_si64_sampled(tdev, oracle_mod, prec):
    torch, dev = tdev
    w = gi.si64_dzp()
    _say(f"case {prec} si64")
    H, rho, F = _run(torch, dev, w, prec)
    o = oracle_mod.Oracle.from_workload(w)
    dH = 0.0
    for I in (0, 42):
        rows = o.H_rows(w.V, I, I + 1)
        r0 = o.atom_orb0[I]
        dH = max(dH, np.abs(H[r0:r0 + rows.shape[0]] - rows).max())
    idx = np.random.default_rng(0).choice(w.ngrid, 20000, replace=False)
    ro = o.rho(w.D, idx)
    er = np.linalg.norm(rho[idx] - ro) / np.linalg.norm(ro)
    # gint_force of the mode (FP16 hi/lo: T on FP16 matrix cores as well)
    Fo = o.force(w.V, w.D, [5, 60])
    eF = np.abs(F[[5, 60]] - Fo).max() / np.abs(Fo).max()
    _say(f"  {prec} si64: max|dH| {dH:.2e} Ha  rho rel-L2 {er:.2e}  F rel {eF:.2e}")
    assert np.array_equal(H, H.T)
    assert dH <= MODES16[prec] and er <= 1e-5 and eF <= 1e-4


def test_16bit_modes_need_32_point_batches(tdev):
    import paper_2603_21835_amd as g

    w = gi.si8_sz()
    plan = g.GintPlan.from_workload(w, precision="bf16x3")
    with pytest.raises(g.GintError):
        plan.tune((2, 2, 4))
    plan.tune((2, 4, 4))
