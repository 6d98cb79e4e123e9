"""GPU batched cells: one call (one captured hipGraph replay) for many cells of
uneven size must give, cell by cell, exactly the single-cell results, and
those match the FP64 oracle."""
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


def _select():
    k = gi.batched_kinds()
    small = [i for i in range(k.size) if k[i] < 2][:6]
    mid = [i for i in range(k.size) if k[i] == 2][:1]
    return sorted(small + mid)


@pytest.fixture(scope="module")
def cells():
    return gi.batched_cells(select=_select())


def _inputs(torch, dev, cells):
    V = [torch.from_numpy(c.V).to(dev) for c in cells]
    D = [torch.from_numpy(c.D).to(dev) for c in cells]
    return V, D


def _single(torch, dev, c):
    import paper_2603_21835_amd as g

    p = g.GintPlan.from_workload(c)
    V, D = torch.from_numpy(c.V).to(dev), torch.from_numpy(c.D).to(dev)
    out = (p.build_H(V).cpu().numpy(), p.build_rho(D).cpu().numpy(), p.force(V, D).cpu().numpy())
    return p, out


def _batched(b, V, D, outs=None):
    if outs is None:
        H, rho, F = b.build_H(V), b.build_rho(D), b.force(V, D)
    else:
        H, rho, F = b.build_H(V, out=outs[0]), b.build_rho(D, out=outs[1]), b.force(V, D, out=outs[2])
    b.sync()
    return [(H[i].cpu().numpy(), rho[i].cpu().numpy(), F[i].cpu().numpy()) for i in range(b.ncell)], (H, rho, F)


def test_batched_equals_single_cells(tdev, cells):
    torch, dev = tdev
    import paper_2603_21835_amd as g

    _say(f"case batched {len(cells)} cells natom {[c.natom for c in cells]}")
    b = g.GintBatch(cells, cells[0].species)
    V, D = _inputs(torch, dev, cells)
    res, outs = _batched(b, V, D)
    for i, c in enumerate(cells):
        p, ref = _single(torch, dev, c)
        assert b.cells[i].work()["nslab"] == p.work()["nslab"]
        for x, y in zip(res[i], ref):
            assert np.array_equal(x, y), f"cell {i} differs from its single-cell result"
    # replay of the captured graphs (same pointers), then a re-capture
    # (new output tensors): identical bits
    res2, _ = _batched(b, V, D, outs)
    res3, _ = _batched(b, V, D)
    for i in range(len(cells)):
        for x, y, z in zip(res[i], res2[i], res3[i]):
            assert np.array_equal(x, y) and np.array_equal(x, z)
    b.close()


def test_batched_vs_oracle_and_moved_atoms(tdev, cells, oracle_mod):
    torch, dev = tdev
    import paper_2603_21835_amd as g

    b = g.GintBatch(cells, cells[0].species)
    V, D = _inputs(torch, dev, cells)
    outs = [b.build_H(V), b.build_rho(D), b.force(V, D)]
    b.sync()
    # move the atoms of the smallest cell: the graphs are re-captured
    i = int(np.argmin([c.ngrid for c in cells]))
    c = cells[i]
    rng = np.random.default_rng(11)
    c.positions = c.positions + rng.normal(0, 0.2, c.positions.shape)
    _say(f"case batched moved cell {i} ({c.natom} atoms) vs oracle")
    b.cells[i].set_positions(c.positions)
    res, _ = _batched(b, V, D, outs)
    o = oracle_mod.Oracle.from_workload(c)
    H, rho, F = res[i]
    Ho, rho_o, Fo = o.H(c.V), o.rho(c.D), o.force(c.V, c.D)
    eH = np.abs(H - Ho).max() / np.abs(Ho).max()
    er = np.linalg.norm(rho - rho_o) / np.linalg.norm(rho_o)
    eF = np.abs(F - Fo).max() / np.abs(Fo).max()
    _say(f"  H {eH:.2e} rho {er:.2e} F {eF:.2e}")
    assert eH <= 1e-10 and er <= 1e-10 and eF <= 1e-10
    b.close()


def test_batched_rejects_timing(tdev, cells):
    torch, dev = tdev
    import paper_2603_21835_amd as g

    sel = cells[:2]
    b = g.GintBatch(sel, sel[0].species)
    V, _ = _inputs(torch, dev, sel)
    b.cells[0].set_timing(True)
    with pytest.raises(g.GintError) as ei:
        b.build_H(V)
    assert ei.value.status == g.GINT_ESTATE
    b.cells[0].set_timing(False)
    b.build_H(V)
    b.sync()
    b.close()


def test_autotune_keeps_results(tdev, cells, oracle_mod):
    torch, dev = tdev
    import paper_2603_21835_amd as g

    sel = [c for c in cells if c.natom <= 16][:3]
    _say(f"case autotune {len(sel)} cells")
    b = g.GintBatch(sel, sel[0].species)
    V, D = _inputs(torch, dev, sel)
    outs = [b.build_H(V), b.build_rho(D), b.force(V, D)]
    shapes = b.autotune(V, D, *outs, reps=1)
    _say(f"  chosen {shapes}")
    for s in shapes:
        assert int(np.prod(s)) in (16, 32)
    res, _ = _batched(b, V, D, outs)
    c = sel[0]
    o = oracle_mod.Oracle.from_workload(c)
    Ho = o.H(c.V)
    assert np.abs(res[0][0] - Ho).max() / np.abs(Ho).max() <= 1e-10
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16x3"])
def test_batched_H_rho_force_matches_single_cells(tdev, cells, oracle_mod, precision):
    # one graph replay for H, rho and dE/dR of every cell: bit for bit the
    # single-cell gint_H_rho_force of each cell (twice: capture, then replay),
    # and the FP64 oracle within 1e-10 (FP64) or 1e-6 Ha / 1e-6 (mixed)
    torch, dev = tdev
    import paper_2603_21835_amd as g

    _say(f"case batched H_rho_force {precision}: {len(cells)} cells")
    b = g.GintBatch(cells, cells[0].species, precision=precision)
    V, D = _inputs(torch, dev, cells)
    for rep in range(2):
        H, rho, F = b.H_rho_force(V, D)
        torch.cuda.synchronize()
        for i, c in enumerate(cells):
            p = g.GintPlan.from_workload(c, precision=precision)
            Hs, rs, Fs = (t.cpu().numpy() for t in p.H_rho_force(V[i], D[i]))
            assert np.array_equal(H[i].cpu().numpy(), Hs), (rep, i)
            assert np.array_equal(rho[i].cpu().numpy(), rs), (rep, i)
            assert np.array_equal(F[i].cpu().numpy(), Fs), (rep, i)
            p.close()
    i = 0  # the first cell against the oracle
    o = oracle_mod.Oracle.from_workload(cells[i])
    Ho, ro, Fo = o.H(cells[i].V), o.rho(cells[i].D), o.force(cells[i].V, cells[i].D)
    Hn, rn, Fn = H[i].cpu().numpy(), rho[i].cpu().numpy(), F[i].cpu().numpy()
    eH = np.abs(Hn - Ho).max()
    er = np.linalg.norm(rn - ro) / np.linalg.norm(ro)
    eF = np.abs(Fn - Fo).max() / np.abs(Fo).max()
    _say(f"  cell 0 vs oracle: max|dH| {eH:.2e}  rho {er:.2e}  F {eF:.2e}")
    if precision == "fp64":
        assert eH <= 1e-10 * np.abs(Ho).max() and er <= 1e-10 and eF <= 1e-10
    else:
        assert eH <= 1e-6 and er <= 1e-6 and eF <= 1e-6
    b.close()
