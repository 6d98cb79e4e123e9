"""GPU adjoint: gradcheck of the autograd binding and central finite
differences of the FP64 energy E = dV sum_g V_g rho_g (F^{loc,Pulay}
equation of Sec. 3.3.1), on a tiny cell and on the Si-512 workload."""
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


def _tiny():
    sp = gi.Species([gi.nao_like_radial(0, 0.5, 3.5), gi.nao_like_radial(1, 0.6, 3.5),
                     gi.nao_like_radial(2, 0.7, 3.5)])
    lat = np.diag([5.0, 5.5, 6.0])
    pos = np.array([[0.4, 0.7, 1.1], [2.6, 3.1, 3.4]])
    return gi.small_cell(pos, lat, (8, 9, 10), [sp], n_waves=4, nocc=3, seed=3)


def test_gradcheck_tiny_cell(tdev):
    torch, dev = tdev
    import paper_2603_21835_amd as g
    from paper_2603_21835_amd.autograd import gint_rho

    w = _tiny()
    _say(f"case gradcheck tiny norb {w.norb} grid {w.grid}")
    plan = g.GintPlan.from_workload(w)
    D = torch.from_numpy(w.D).to(dev).requires_grad_(True)
    R = torch.from_numpy(w.positions.copy()).to(dev).requires_grad_(True)
    # a fixed random projection keeps the Jacobian check cheap and complete
    proj = torch.from_numpy(np.random.default_rng(0).standard_normal((w.ngrid, 3))).to(dev)

    def f(D_, R_):
        return gint_rho(plan, D_, R_) @ proj

    assert torch.autograd.gradcheck(f, (D, R), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_energy_backward_equals_force(tdev, oracle_mod):
    torch, dev = tdev
    import paper_2603_21835_amd as g
    from paper_2603_21835_amd.autograd import gint_rho

    w = _tiny()
    _say("case E.backward vs oracle dE/dR and H")
    plan = g.GintPlan.from_workload(w)
    V = torch.from_numpy(w.V).to(dev)
    D = torch.from_numpy(w.D).to(dev).requires_grad_(True)
    R = torch.from_numpy(w.positions.copy()).to(dev).requires_grad_(True)
    E = plan.dV * torch.dot(V, gint_rho(plan, D, R))
    E.backward()
    o = oracle_mod.Oracle.from_workload(w)
    Fo = o.force(w.V, w.D)
    Ho = o.H(w.V)
    np.testing.assert_allclose(R.grad.cpu().numpy(), Fo, rtol=0, atol=1e-10 * np.abs(Fo).max())
    np.testing.assert_allclose(D.grad.cpu().numpy(), Ho, rtol=0, atol=1e-10 * np.abs(Ho).max())


def test_si512_force_vs_finite_differences(tdev):
    torch, dev = tdev
    import paper_2603_21835_amd as g

    w = gi.si512_dzp()
    _say(f"case si512 FD on atoms {list(w.fd_atoms)}")
    plan = g.GintPlan.from_workload(w)
    V = torch.from_numpy(w.V).to(dev)
    D = torch.from_numpy(w.D).to(dev)
    F = plan.force(V, D).cpu().numpy()
    h = 1e-4

    def energy(pos):
        plan.set_positions(pos)
        rho = plan.build_rho(D)
        return plan.dV * float(torch.dot(V, rho))

    errs = []
    for I in w.fd_atoms:
        for k in range(3):
            p = w.positions.copy()
            p[I, k] += h
            Ep = energy(p)
            p[I, k] -= 2 * h
            Em = energy(p)
            fd = (Ep - Em) / (2 * h)
            errs.append(abs(F[I, k] - fd))
    plan.set_positions(w.positions)
    scale = np.abs(F[w.fd_atoms]).max()
    _say(f"  max |F - FD| = {max(errs):.3e} (scale {scale:.3e})")
    assert max(errs) <= max(1e-6 * scale, 1e-8)


def test_si512_force_sampled_vs_oracle(tdev, oracle_mod):
    torch, dev = tdev
    import paper_2603_21835_amd as g

    w = gi.si512_dzp()
    atoms = list(w.fd_atoms[:2])
    _say(f"case si512 force vs oracle on atoms {atoms}")
    plan = g.GintPlan.from_workload(w)
    F = plan.force(torch.from_numpy(w.V).to(dev), torch.from_numpy(w.D).to(dev)).cpu().numpy()
    o = oracle_mod.Oracle.from_workload(w)
    Fo = o.force(w.V, w.D, atoms)
    e = np.abs(F[atoms] - Fo).max() / np.abs(Fo).max()
    _say(f"  rel err {e:.2e}")
    assert e <= 1e-10
