"""Pins of the oracle's spherical-grid projector overlaps (Sec. 3.3.2,
"Spherical Grid Integration for Nonlocal Potentials"):

    Q[p, mu] = <phit_mu | e^{-i A.r} | beta_p>
             ~ sum_ij rb q_i r_i^2 w_j phit_mu(tau_I + r_i u_j) e^{-i A.(tau_I + r_i u_j)} beta_p(r_i u_j)

on the 110-point Lebedev-Laikov x 140-point Gauss-Legendre product grid
around each projector's atom.  Pinned against references other than
itself:
  * the quadrature rules: the angular rule integrates products of real
    harmonics (from SciPy) up to total degree 16 exactly, the radial rule
    monomials up to degree 279;
  * closed forms for Gaussian s and p projectors against a Gaussian s
    orbital (in a regime where the degree-17 angular rule is exact to
    ~1e-15 and the tables' spline error is ~1e-12);
  * exact symmetries: Q(-A) = conj Q(A), Q(0) real; moving an atom by a
    lattice vector L multiplies its own projector rows by e^{-i A.L} and
    leaves every other row unchanged (its orbitals are folded);
  * brute force with SciPy splines and harmonics and all lattice images of
    a cube, at the same quadrature points, on a triclinic two-species cell
    whose orbitals reach further than the cell.
"""
import numpy as np
import pytest

import gint_inputs as gi
from tests.bruteforce import BruteCell, real_ylm

Y00 = 0.28209479177387814
C1 = 0.4886025119029199


def test_angular_rule_integrates_harmonics():
    ang = gi.lebedev_110()
    u, wq = ang[:, :3], ang[:, 3]
    assert abs(wq.sum() - 4 * np.pi) <= 1e-13
    Y = [real_ylm(l, m, u) for l in range(9) for m in range(-l, l + 1)]
    G = np.array([[np.sum(wq * a * b) for b in Y] for a in Y])
    assert np.max(np.abs(G - np.eye(len(Y)))) <= 1e-13


def test_radial_rule_integrates_monomials():
    rq = gi.gauss_legendre_01(140)
    x, q = rq[:, 0], rq[:, 1]
    for k in range(0, 280, 7):
        assert abs(np.sum(q * x**k) - 1.0 / (k + 1)) <= 1e-14


def _gauss_pair(A, d=(0.3, -0.25, 0.3), alpha=0.2, gamma=1.5):
    """Atom 0 (projectors: Gaussian s and p, no cutoff polynomial) at C,
    atom 1 (one Gaussian s orbital, no projectors) at C + d, in a box large
    enough for single images."""
    L = 40.0
    C = np.array([12.0, 13.0, 11.0])
    B = C + np.asarray(d)
    orb = gi.Species([gi.nao_like_radial(0, alpha, 12.0, 0.01, smooth_cutoff=False)])
    w = gi.small_cell(np.array([C, B]), np.diag([L, L, L]), (8, 8, 8), [orb, orb], species_of_atom=[0, 1],
                      n_waves=2, nocc=1, seed=3)
    proj = [gi.Species([gi.nao_like_radial(0, gamma, 5.0, 0.002, smooth_cutoff=False),
                        gi.nao_like_radial(1, gamma, 5.0, 0.002, smooth_cutoff=False)]),
            gi.Species([])]
    return w, proj, C, B


def _closed_form(A, C, B, alpha, gamma):
    """s orbital at B against s and p Gaussian projectors at C:
    F = int e^{-alpha|r-B|^2} e^{-iA.r} e^{-gamma|r-C|^2} dr and
    int e^{-alpha|r-B|^2} e^{-iA.r} (r-C) e^{-gamma|r-C|^2} dr = (1/2 gamma) dF/dC."""
    p = alpha + gamma
    mu = alpha * gamma / p
    P = (alpha * B + gamma * C) / p
    F = (np.pi / p) ** 1.5 * np.exp(-mu * np.sum((B - C) ** 2)) * np.exp(-A @ A / (4 * p)) * np.exp(-1j * A @ P)
    dF = F * (2 * mu * (B - C) - 1j * gamma * A / p)
    s = Y00 * Y00 * F
    pv = Y00 * C1 * dF / (2 * gamma)
    return np.array([s, pv[1], pv[2], pv[0]])  # projector order s, p(m=-1: y, 0: z, 1: x)


@pytest.mark.parametrize("A", [np.array([0.1, -0.05, 0.04]), np.array([0.0, 0.0, 0.0])])
def test_gaussian_closed_forms(oracle_mod, A):
    alpha, gamma = 0.2, 1.5
    w, proj, C, B = _gauss_pair(A, alpha=alpha, gamma=gamma)
    o = oracle_mod.Oracle.from_workload(w)
    Q = o.psibeta(proj, gi.lebedev_110(), gi.gauss_legendre_01(140), A)
    assert Q.shape == (4, 2)
    ref_far = _closed_form(A, C, B, alpha, gamma)  # orbital of atom 1
    ref_self = _closed_form(A, C, C, alpha, gamma)  # orbital of atom 0 (same centre)
    scale = np.abs(ref_self).max()
    assert np.max(np.abs(Q[:, 1] - ref_far)) <= 1e-9 * scale
    assert np.max(np.abs(Q[:, 0] - ref_self)) <= 1e-9 * scale


def _dzp_cell():
    sp = gi.Species([gi.nao_like_radial(0, 0.4, 5.0), gi.nao_like_radial(1, 0.9, 5.0),
                     gi.nao_like_radial(2, 0.7, 5.0)])
    lat = np.array([[6.0, 0.0, 0.0], [0.7, 6.5, 0.0], [-0.4, 0.3, 7.0]])
    pos = np.array([[0.3, 0.2, 0.1], [3.1, 2.7, 3.9], [5.0, 5.5, 0.2]])
    w = gi.small_cell(pos, lat, (12, 12, 12), [sp, gi.sz_species(4.0)], species_of_atom=[0, 1, 0],
                      n_waves=4, nocc=3, seed=7)
    proj = [gi.si_projector_species(), gi.Species([gi.nao_like_radial(0, 1.2, 1.8)])]
    return w, proj


def test_exact_symmetries(oracle_mod):
    w, proj = _dzp_cell()
    o = oracle_mod.Oracle.from_workload(w)
    ang, rq = gi.lebedev_110(), gi.gauss_legendre_01(60)
    A = gi.vector_potential(8)
    Q = o.psibeta(proj, ang, rq, A)
    np.testing.assert_allclose(o.psibeta(proj, ang, rq, -A), np.conj(Q), rtol=0, atol=1e-15 * np.abs(Q).max())
    Q0 = o.psibeta(proj, ang, rq, np.zeros(3))
    assert np.all(Q0.imag == 0.0)
    # projector atom 2 moved by a lattice vector: its rows pick up e^{-i A.L}
    r0, r1 = 9 + 1, 9 + 1 + 9  # rows of atom 2 (atom 0: 9 projectors, atom 1: 1)
    assert Q.shape[0] == r1
    L = w.lattice[0] - 2 * w.lattice[2]
    pos = w.positions.copy()
    pos[2] += L
    o.set_positions(pos)
    Q2 = o.psibeta(proj, ang, rq, A)
    ph = np.exp(-1j * A @ L)
    np.testing.assert_allclose(Q2[r0:r1], Q[r0:r1] * ph, rtol=0, atol=1e-13 * np.abs(Q).max())
    np.testing.assert_allclose(Q2[:r0], Q[:r0], rtol=0, atol=1e-13 * np.abs(Q).max())
    # moving atom 1 by -a2: its own projector row picks up e^{+i A.a2}; the
    # other atoms' rows see its orbitals unchanged (folded over images)
    pos = w.positions.copy()
    pos[1] -= w.lattice[1]
    o.set_positions(pos)
    Q3 = o.psibeta(proj, ang, rq, A)
    keep = np.r_[0:9, 10:19]
    np.testing.assert_allclose(Q3[keep], Q[keep], rtol=0, atol=1e-13 * np.abs(Q).max())
    np.testing.assert_allclose(Q3[9], Q[9] * np.exp(1j * A @ w.lattice[1]), rtol=0, atol=1e-13 * np.abs(Q).max())


def _brute_psibeta(w, proj, ang, rq, A):
    """phit from scipy splines and harmonics over a cube of images (BruteCell)
    at the quadrature points of every projector atom; beta likewise."""
    from scipy.interpolate import CubicSpline

    bc = BruteCell(w)
    rows = []
    for I, s in enumerate(w.species_of_atom):
        rads = proj[s].radials
        if not rads:
            continue
        rb = max(r.rc for r in rads)
        r = rb * rq[:, 0]
        wr = rb * rq[:, 1] * r * r
        x = (r[:, None, None] * ang[None, :, :3]).reshape(-1, 3)
        W = (wr[:, None] * ang[None, :, 3]).reshape(-1)
        pts = w.positions[I] + x
        bc.points = pts
        phi = bc.phi_all()
        ph = W * np.exp(-1j * (pts @ A))
        rr = np.linalg.norm(x, axis=1)
        u = x / rr[:, None]
        for l in range(3):
            for rad in rads:
                if rad.l != l:
                    continue
                cs = CubicSpline(np.arange(rad.nr) * rad.dr, rad.f, bc_type=((1, rad.dfdr0), (1, rad.dfdrc)))
                b = np.where(rr < rad.rc, cs(np.minimum(rr, rad.rc)), 0.0)
                for m in range(-l, l + 1):
                    rows.append((ph * b * real_ylm(l, m, u)) @ phi)
    return np.array(rows)


def test_bruteforce_triclinic(oracle_mod):
    w, proj = _dzp_cell()
    ang, rq = gi.lebedev_110(), gi.gauss_legendre_01(40)
    A = gi.vector_potential(9)
    Q = oracle_mod.Oracle.from_workload(w).psibeta(proj, ang, rq, A)
    ref = _brute_psibeta(w, proj, ang, rq, A)
    assert np.max(np.abs(Q - ref)) <= 1e-12 * np.abs(ref).max()
