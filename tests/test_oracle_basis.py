"""Pins of the oracle's basis functions: spline, real Ylm, gradients, r = 0.

Each check compares the oracle with something other than itself: a library
spline, a library spherical harmonic, exact polynomials, quadrature, finite
differences or the analytic radial function within the spline error bound.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import gint_inputs as gi
from tests.bruteforce import real_ylm


def _oracle_for(oracle_mod, species, pos=((0.0, 0.0, 0.0),), L=30.0, grid=(4, 4, 4)):
    return oracle_mod.Oracle(np.eye(3) * L, grid, species, np.zeros(len(pos), np.int32), np.array(pos))


def test_spline_matches_scipy_clamped(oracle_mod):
    sp = gi.dzp_species()
    o = _oracle_for(oracle_mod, [sp])
    rng = np.random.default_rng(0)
    rs = np.concatenate([rng.uniform(0, 8.0, 400), np.arange(0, 8.0, 0.01)[::37], [0.0, 7.999999]])
    for k, rad in enumerate(sp.radials):
        x = np.arange(rad.nr) * rad.dr
        cs = CubicSpline(x, rad.f, bc_type=((1, rad.dfdr0), (1, rad.dfdrc)))
        for r in rs:
            v, d = o.radial(k, r)
            assert abs(v - cs(r)) <= 1e-13 * (1 + abs(cs(r)))
            assert abs(d - cs(r, 1)) <= 1e-11 * (1 + abs(cs(r, 1)))


def test_spline_reproduces_cubic_exactly(oracle_mod):
    # a clamped cubic spline through samples of a cubic with its exact end
    # slopes is that cubic
    dr, nr = 0.05, 121
    x = np.arange(nr) * dr
    c = (0.3, -1.2, 0.7, -0.11)
    f = c[0] + c[1] * x + c[2] * x**2 + c[3] * x**3
    df = lambda t: c[1] + 2 * c[2] * t + 3 * c[3] * t**2
    rad = gi.Radial(0, dr, f, df(0.0), df(x[-1]))
    o = _oracle_for(oracle_mod, [gi.Species([rad])])
    for r in np.linspace(0, x[-1] - 1e-9, 97):
        v, d = o.radial(0, r)
        exact = c[0] + c[1] * r + c[2] * r**2 + c[3] * r**3
        assert abs(v - exact) < 1e-12
        assert abs(d - df(r)) < 1e-10


def test_spline_error_within_bound(oracle_mod):
    # |f - s| <= 5/384 dr^4 max|f''''| for a clamped cubic spline
    alpha, rc, dr = 0.6, 6.0, 0.01
    rad = gi.nao_like_radial(0, alpha, rc, dr)
    o = _oracle_for(oracle_mod, [gi.Species([rad])])
    t = np.linspace(0, rc, 20001)
    f = lambda r: np.exp(-alpha * r * r) * (1 - (r / rc) ** 2) ** 2
    h = 1e-3
    f4 = (f(t + 2 * h) - 4 * f(t + h) + 6 * f(t) - 4 * f(t - h) + f(t - 2 * h)) / h**4
    bound = 5.0 / 384.0 * dr**4 * np.max(np.abs(f4[2:-2])) * 1.05
    err = max(abs(o.radial(0, r)[0] - f(r)) for r in np.linspace(0, rc - 1e-9, 3001))
    assert err <= bound


@pytest.mark.parametrize("l", [0, 1, 2])
def test_ylm_matches_scipy(oracle_mod, l):
    rng = np.random.default_rng(l)
    u = rng.standard_normal((200, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for v in u:
        got = oracle_mod.ylm(l, v)
        want = np.array([real_ylm(l, m, v[None, :])[0] for m in range(-l, l + 1)])
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_ylm_orthonormal(oracle_mod):
    # Gauss-Legendre in cos(theta) x trapezoid in phi is exact for these
    # polynomials of degree <= 4
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 16
    ph = np.arange(nphi) * 2 * np.pi / nphi
    Y = []
    W = []
    for ct, w in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for p in ph:
            u = np.array([st * math.cos(p), st * math.sin(p), ct])
            Y.append(np.concatenate([oracle_mod.ylm(l, u) for l in range(3)]))
            W.append(w * 2 * np.pi / nphi)
    Y = np.array(Y)
    W = np.array(W)
    G = (Y * W[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(9), atol=1e-13)


def test_phi_is_radial_times_ylm(oracle_mod):
    sp = gi.dzp_species()
    o = _oracle_for(oracle_mod, [sp], pos=((3.0, 4.0, 5.0),))
    rng = np.random.default_rng(3)
    for _ in range(50):
        d = rng.uniform(-5, 5, 3)
        r = np.linalg.norm(d)
        phi = o.phi(np.array([3.0, 4.0, 5.0]) + d)
        k = 0
        for l in range(3):
            for irad, rad in enumerate(sp.radials):
                if rad.l != l:
                    continue
                alpha = [0.4, 1.0, 0.4, 1.0, 0.7][irad]
                fa = r**l * math.exp(-alpha * r * r) * (1 - (r / 8.0) ** 2) ** 2 if r < 8 else 0.0
                for m in range(-l, l + 1):
                    Y = real_ylm(l, m, (d / r)[None, :])[0]
                    assert abs(phi[k] - fa * Y) < 1e-9
                    k += 1


def test_gradient_matches_central_difference(oracle_mod):
    sp = gi.dzp_species()
    lat = np.eye(3) * 9.0  # images overlap (rc = 8 > L/2): folded gradients
    pos = np.array([[1.0, 2.0, 3.0], [4.5, 4.0, 6.0]])
    o = oracle_mod.Oracle(lat, (6, 6, 6), [sp], np.zeros(2, np.int32), pos)
    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(20):
        r = rng.uniform(0, 9, 3)
        _, g = o.phi(r, grad=True)
        fd = np.zeros_like(g)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd[:, k] = (o.phi(r + e) - o.phi(r - e)) / (2 * h)
        np.testing.assert_allclose(g, fd, atol=2e-8, rtol=0)


def test_limits_at_atom_position(oracle_mod):
    sp = gi.dzp_species()
    o = _oracle_for(oracle_mod, [sp], pos=((1.0, 1.0, 1.0),))
    phi, g = o.phi(np.array([1.0, 1.0, 1.0]), grad=True)
    Y00 = 0.28209479177387814
    # s: f(0) Y00, zero gradient (f'(0) = 0); p and d vanish at the centre
    assert abs(phi[0] - 1.0 * Y00) < 1e-15 and abs(phi[1] - 1.0 * Y00) < 1e-15
    assert np.all(phi[2:] == 0.0)
    assert np.all(g[0:2] == 0.0) and np.all(g[8:] == 0.0)
    # p: grad phi_{1m}(0) = f'(0) C1 e_m with e = (y, z, x) for m = (-1, 0, 1)
    C1 = math.sqrt(3.0 / (4.0 * math.pi))
    for zeta in range(2):
        blk = g[2 + 3 * zeta: 5 + 3 * zeta]
        want = C1 * np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], dtype=float)
        np.testing.assert_allclose(blk, want, atol=1e-15)
    # and the limit agrees with the value just off the centre
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1e-7
        _, g2 = o.phi(np.array([1.0, 1.0, 1.0]) + e, grad=True)
        np.testing.assert_allclose(g2[2:8], g[2:8], atol=1e-6)
