"""Brute-force grid integrals for tiny cells (independent of the C oracle).

Everything here is built from library primitives and the definitions, with
no neighbour lists, no batching and no code shared with either the oracle
or the GPU library:

* radial: ``scipy.interpolate.CubicSpline`` with clamped ends, i.e. the same
  mathematical spline (Sec. 2.1 NAO decomposition; cubic-spline tables);
* angular: real harmonics assembled from ``scipy.special.sph_harm_y``
  (complex, Condon-Shortley phase), not from the closed forms;
* images: every lattice vector in [-n, n]^3, n = ceil(rc / L_min) + 1;
* the sums of Sec. 3.3.1 (rho(r_g), H^loc) as explicit loops;
* H^loc(R): the crystal's mesh enumerated as the cell's points shifted by
  every lattice vector of a cube, with unfolded (per-image) orbitals.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.interpolate import CubicSpline
from scipy.special import sph_harm_y


def real_ylm(l: int, m: int, u: np.ndarray) -> np.ndarray:
    """Real Y_lm (no Condon-Shortley phase) at unit vectors u (..., 3)."""
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    Y = sph_harm_y(l, abs(m), theta, phi)
    sgn = (-1.0) ** abs(m)
    if m > 0:
        return math.sqrt(2.0) * sgn * np.real(Y)
    return math.sqrt(2.0) * sgn * np.imag(Y)


class BruteCell:
    def __init__(self, w):
        self.w = w
        self.lat = np.asarray(w.lattice, dtype=np.float64)
        self.N = np.asarray(w.grid)
        self.splines = []
        self.orbs = []  # per species: list of (spline, rc, l, m)
        for sp in w.species:
            lst = []
            for l in range(0, 3):
                for r in sp.radials:
                    if r.l != l:
                        continue
                    x = np.arange(r.nr) * r.dr
                    cs = CubicSpline(x, r.f, bc_type=((1, r.dfdr0), (1, r.dfdrc)))
                    for m in range(-l, l + 1):
                        lst.append((cs, (r.nr - 1) * r.dr, l, m))
            self.orbs.append(lst)
        n = np.stack(np.meshgrid(*[np.arange(k) for k in self.N], indexing="ij"), -1).reshape(-1, 3)
        self.points = (n / self.N) @ self.lat  # r_g = sum_i (n_i/N_i) a_i
        self.dV = abs(np.linalg.det(self.lat)) / np.prod(self.N)

    def phi_all(self, positions=None):
        """Folded orbital values, shape (ngrid, norb)."""
        w = self.w
        pos = np.asarray(w.positions if positions is None else positions, dtype=np.float64)
        rcmax = max(o[1] for lst in self.orbs for o in lst)
        nimg = int(math.ceil(rcmax / np.min(np.linalg.norm(self.lat, axis=1)))) + 1
        cols = []
        for I, s in enumerate(w.species_of_atom):
            vals = np.zeros((len(self.points), len(self.orbs[s])))
            for n1 in range(-nimg, nimg + 1):
                for n2 in range(-nimg, nimg + 1):
                    for n3 in range(-nimg, nimg + 1):
                        T = n1 * self.lat[0] + n2 * self.lat[1] + n3 * self.lat[2]
                        d = self.points - pos[I] - T
                        r = np.sqrt(np.sum(d * d, axis=1))
                        safe = np.where(r > 0, r, 1.0)
                        u = d / safe[:, None]
                        for k, (cs, rc, l, m) in enumerate(self.orbs[s]):
                            inside = r < rc
                            f = np.where(inside, cs(np.minimum(r, rc)), 0.0)
                            if l == 0:
                                Y = real_ylm(0, 0, u)
                            else:
                                Y = np.where(r > 1e-12, real_ylm(l, m, u), 0.0)
                            vals[:, k] += f * Y
            cols.append(vals)
        return np.concatenate(cols, axis=1)

    def phi_image(self, n, positions=None):
        """Unfolded orbital values phi_mu(r_g - tau_I - T), T = n . (a1, a2, a3),
        at the cell's mesh points: shape (ngrid, norb)."""
        w = self.w
        pos = np.asarray(w.positions if positions is None else positions, dtype=np.float64)
        T = n[0] * self.lat[0] + n[1] * self.lat[1] + n[2] * self.lat[2]
        cols = []
        for I, s in enumerate(w.species_of_atom):
            d = self.points - pos[I] - T
            r = np.sqrt(np.sum(d * d, axis=1))
            safe = np.where(r > 0, r, 1.0)
            u = d / safe[:, None]
            vals = np.zeros((len(self.points), len(self.orbs[s])))
            for k, (cs, rc, l, m) in enumerate(self.orbs[s]):
                f = np.where(r < rc, cs(np.minimum(r, rc)), 0.0)
                if l == 0:
                    Y = real_ylm(0, 0, u)
                else:
                    Y = np.where(r > 1e-12, real_ylm(l, m, u), 0.0)
                vals[:, k] = f * Y
            cols.append(vals)
        return np.concatenate(cols, axis=1)

    def HR(self, V, Rlist):
        """H(R)_mu,nu = dV sum over crystal points r of phi_mu(r - tau_I) V(r)
        phi_nu(r - tau_J - R): crystal points r = r_g - T for every T of a
        cube big enough that no orbital pair is missed.  Returns [n][norb][norb]."""
        rcmax = max(o[1] for lst in self.orbs for o in lst)
        nimg = int(math.ceil(rcmax / np.min(np.linalg.norm(self.lat, axis=1)))) + 1
        cache = {}

        def img(n):
            if n not in cache:
                cache[n] = self.phi_image(n)
            return cache[n]

        out = np.zeros((len(Rlist), self.w.norb, self.w.norb))
        rng = range(-nimg, nimg + 1)
        for T in [(a, b, c) for a in rng for b in rng for c in rng]:
            A = img(T) * V[:, None]
            if not np.any(A):
                continue
            for q, R in enumerate(Rlist):
                out[q] += self.dV * A.T @ img((T[0] + R[0], T[1] + R[1], T[2] + R[2]))
        return out

    def rhoR(self, Rlist, DR):
        """rho(r_g) = sum_T sum_q phi_T(r_g)^T DR[q] phi_{T + R_q}(r_g): the
        sums over R' (= T) and R of the rho(r_g) equation, T over a cube big
        enough that no orbital pair is missed."""
        rcmax = max(o[1] for lst in self.orbs for o in lst)
        nimg = int(math.ceil(rcmax / np.min(np.linalg.norm(self.lat, axis=1)))) + 1
        cache = {}

        def img(n):
            if n not in cache:
                cache[n] = self.phi_image(n)
            return cache[n]

        out = np.zeros(len(self.points))
        rng = range(-nimg, nimg + 1)
        for T in [(a, b, c) for a in rng for b in rng for c in rng]:
            A = img(T)
            if not np.any(A):
                continue
            for q, R in enumerate(Rlist):
                B = img((T[0] + R[0], T[1] + R[1], T[2] + R[2]))
                out += np.einsum("gm,mn,gn->g", A, DR[q], B)
        return out

    def H(self, V, phi=None):
        phi = self.phi_all() if phi is None else phi
        return self.dV * (phi * V[:, None]).T @ phi

    def rho(self, D, phi=None):
        phi = self.phi_all() if phi is None else phi
        return np.einsum("gm,mn,gn->g", phi, D, phi)

    def energy(self, V, D, positions=None):
        phi = self.phi_all(positions)
        return self.dV * float(np.dot(V, self.rho(D, phi)))

    def support_stats(self):
        """sum_g n_g and sum_g n_g^2, n_g = orbitals of the atoms with at
        least one image strictly inside the atom's cutoff (its largest
        radial cutoff) at mesh point g: every lattice vector of a cube."""
        w = self.w
        pos = np.asarray(w.positions, dtype=np.float64)
        rcmax = max(o[1] for lst in self.orbs for o in lst)
        nimg = int(math.ceil(rcmax / np.min(np.linalg.norm(self.lat, axis=1)))) + 1
        n = np.zeros(len(self.points), dtype=np.int64)
        for I, s in enumerate(w.species_of_atom):
            rc = max(o[1] for o in self.orbs[s])
            hit = np.zeros(len(self.points), dtype=bool)
            for n1 in range(-nimg, nimg + 1):
                for n2 in range(-nimg, nimg + 1):
                    for n3 in range(-nimg, nimg + 1):
                        T = n1 * self.lat[0] + n2 * self.lat[1] + n3 * self.lat[2]
                        d = self.points - pos[I] - T
                        hit |= np.sqrt(np.sum(d * d, axis=1)) < rc
            n += hit * len(self.orbs[s])
        return float(n.sum()), float((n * n).sum())
