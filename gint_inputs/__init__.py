"""Seeded synthetic workloads for the real-space grid-integration path.

This module only *prepares inputs*: cells, tabulated radial functions, a
potential sampled on the mesh and a density matrix.  It holds none of the
grid-integration arithmetic (no spline, no spherical harmonics, no grid sums),
so both the CPU oracle and the GPU library can consume what it returns without
sharing any of the method's code.

The workloads stand in for the bulk-silicon supercell family of the paper's
system-size scaling test (Sec. 4.3.1, Table 1: supercells built from the
8-atom cubic diamond cell, radial cutoff 8 bohr, Gamma point).  The paper's
SIAB orbitals and pseudopotentials are not available, so the radials are
analytic and the local potential is a smooth random plane-wave sum.

Random draws use ``numpy.random.Generator(PCG64(seed))`` in a fixed order:
displacements, plane-wave set, plane-wave amplitudes, wavefunction
coefficients C, finite-difference atoms.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

A_SI = 10.26  # bohr, cubic diamond-Si lattice constant of the 8-atom cell

# Fractional positions of the 8-atom conventional diamond cell.
DIAMOND_FRAC = np.array(
    [
        [0.00, 0.00, 0.00],
        [0.00, 0.50, 0.50],
        [0.50, 0.00, 0.50],
        [0.50, 0.50, 0.00],
        [0.25, 0.25, 0.25],
        [0.25, 0.75, 0.75],
        [0.75, 0.25, 0.75],
        [0.75, 0.75, 0.25],
    ]
)


@dataclass
class Radial:
    """One radial function f(r) tabulated at r_i = i*dr, i < nr; rc=(nr-1)*dr.

    ``dfdr0``/``dfdrc`` are the end slopes used for the clamped cubic spline.
    """

    l: int
    dr: float
    f: np.ndarray
    dfdr0: float
    dfdrc: float

    @property
    def nr(self) -> int:
        return int(self.f.shape[0])

    @property
    def rc(self) -> float:
        return (self.nr - 1) * self.dr


@dataclass
class Species:
    """Radials of one species; orbital order is l ascending, zeta, then m."""

    radials: List[Radial]

    @property
    def norb(self) -> int:
        return sum(2 * r.l + 1 for r in self.radials)


@dataclass
class Workload:
    name: str
    lattice: np.ndarray  # (3,3) rows a1, a2, a3 (bohr)
    grid: tuple  # (N1, N2, N3)
    species: List[Species]
    species_of_atom: np.ndarray  # (natom,) int32
    positions: np.ndarray  # (natom, 3) cartesian bohr
    V: Optional[np.ndarray] = None  # (N1*N2*N3,) float64, i3 fastest (Ha)
    D: Optional[np.ndarray] = None  # (norb, norb) float64
    C: Optional[np.ndarray] = None
    pw_m: Optional[np.ndarray] = None  # (K,3) integer reciprocal indices
    pw_amp: Optional[np.ndarray] = None  # (K,)
    fd_atoms: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def natom(self) -> int:
        return int(self.positions.shape[0])

    @property
    def norb(self) -> int:
        return int(sum(self.species[s].norb for s in self.species_of_atom))

    @property
    def ngrid(self) -> int:
        return int(np.prod(self.grid))


# --------------------------------------------------------------------------
# radial tables


def nao_like_radial(l: int, alpha: float, rc: float, dr: float = 0.01,
                    smooth_cutoff: bool = True) -> Radial:
    """f(r) = r^l exp(-alpha r^2) (1-(r/rc)^2)^2 for r<rc (configs' analytic form).

    With ``smooth_cutoff=False`` the polynomial factor is dropped (pure
    Gaussian-type radial, used for the closed-form overlap pins).
    End slopes are the analytic ones: f'(0) = 1 for l = 1 and 0 otherwise;
    f'(rc) = 0 with the smooth cutoff, else the Gaussian's own slope.
    """
    nr = int(round(rc / dr)) + 1
    r = np.arange(nr, dtype=np.float64) * dr
    f = r**l * np.exp(-alpha * r * r)
    if smooth_cutoff:
        f = f * (1.0 - (r / rc) ** 2) ** 2
        f[-1] = 0.0
        drc = 0.0
    else:
        rcv = (nr - 1) * dr
        drc = (l * rcv ** (l - 1) if l > 0 else 0.0) * np.exp(-alpha * rcv * rcv) \
            - 2.0 * alpha * rcv ** (l + 1) * np.exp(-alpha * rcv * rcv)
    d0 = 1.0 if l == 1 else 0.0
    return Radial(l=l, dr=dr, f=f, dfdr0=d0, dfdrc=float(drc))


def sz_species(rc: float = 6.0, dr: float = 0.01) -> Species:
    """1s + 1p single-zeta Si basis of the 8-atom workload (4 orbitals/atom)."""
    return Species([nao_like_radial(0, 0.6, rc, dr), nao_like_radial(1, 0.6, rc, dr)])


def dzp_species(rc: float = 8.0, dr: float = 0.01) -> Species:
    """2s2p1d double-zeta-polarised Si basis (13 orbitals/atom).

    Exponents 0.4 (zeta 1) and 1.0 (zeta 2) for s and p, 0.7 for d.
    """
    return Species(
        [
            nao_like_radial(0, 0.4, rc, dr),
            nao_like_radial(0, 1.0, rc, dr),
            nao_like_radial(1, 0.4, rc, dr),
            nao_like_radial(1, 1.0, rc, dr),
            nao_like_radial(2, 0.7, rc, dr),
        ]
    )


def si_projector_species(rb: float = 2.2, gamma: float = 0.9, dr: float = 0.01) -> Species:
    """Synthetic nonlocal projectors of one Si atom: one radial each for
    l = 0, 1, 2, b_l(r) = r^l exp(-gamma r^2) (1 - (r/rb)^2)^2 for r < rb
    (9 projectors per atom), in the same tabulated form as the orbitals."""
    return Species([nao_like_radial(l, gamma, rb, dr) for l in (0, 1, 2)])


def lebedev_110() -> np.ndarray:
    """The 110-point Lebedev-Laikov rule on the unit sphere (degree 17),
    from SciPy: rows (x, y, z, w), weights summing to 4 pi."""
    from scipy.integrate import lebedev_rule

    x, w = lebedev_rule(17)
    out = np.ascontiguousarray(np.concatenate([x.T, w[:, None]], axis=1), dtype=np.float64)
    assert out.shape == (110, 4)
    return out


def gauss_legendre_01(n: int = 140) -> np.ndarray:
    """n-point Gauss-Legendre rule mapped to [0, 1]: rows (x, q)."""
    t, w = np.polynomial.legendre.leggauss(n)
    return np.ascontiguousarray(np.stack([(t + 1.0) / 2.0, w / 2.0], axis=1), dtype=np.float64)


def vector_potential(seed: int = 6, scale: float = 0.5) -> np.ndarray:
    """A seeded vector potential A (bohr^-1), components U(-scale, scale)."""
    return np.random.default_rng(seed).uniform(-scale, scale, 3)


# --------------------------------------------------------------------------
# cells


def si_supercell(rep: Sequence[int], a: float = A_SI):
    """Diamond-Si supercell: lattice rows and cartesian positions (bohr)."""
    rep = np.asarray(rep, dtype=np.int64)
    lattice = np.diag(a * rep.astype(np.float64))
    frac = []
    for i in range(rep[0]):
        for j in range(rep[1]):
            for k in range(rep[2]):
                for f in DIAMOND_FRAC:
                    frac.append((f + np.array([i, j, k])) / rep)
    frac = np.array(frac)
    return lattice, frac @ lattice


def plane_wave_potential(grid, lattice, n_waves: int, rng: np.random.Generator,
                         gmax: float = 3.0 * 2.0 * np.pi / A_SI):
    """V(r) = sum_k A_k cos(G_k . r) sampled on the mesh.

    G_k are drawn without replacement from the non-zero reciprocal-lattice
    vectors of the cell with |G| <= gmax; A_k ~ U(-1, 1) Ha.  Mesh point
    n has fractional coordinates n/N, so G.r = 2 pi m.(n/N) for G = 2 pi B m.
    Returns (V flattened with i3 fastest, m vectors, amplitudes).
    """
    lattice = np.asarray(lattice, dtype=np.float64)
    B = np.linalg.inv(lattice).T  # rows b_i, a_i . b_j = delta_ij
    mmax = [int(np.ceil(gmax / (2 * np.pi) * np.linalg.norm(lattice[i]))) + 1 for i in range(3)]
    cand = []
    for m1 in range(-mmax[0], mmax[0] + 1):
        for m2 in range(-mmax[1], mmax[1] + 1):
            for m3 in range(-mmax[2], mmax[2] + 1):
                if m1 == 0 and m2 == 0 and m3 == 0:
                    continue
                G = 2 * np.pi * (m1 * B[0] + m2 * B[1] + m3 * B[2])
                if np.linalg.norm(G) <= gmax + 1e-12:
                    cand.append((m1, m2, m3))
    cand = np.array(cand, dtype=np.int64)
    pick = rng.choice(len(cand), size=n_waves, replace=False)
    m = cand[pick]
    amp = rng.uniform(-1.0, 1.0, size=n_waves)
    N = np.asarray(grid)
    n1 = np.arange(N[0])[:, None, None] / N[0]
    n2 = np.arange(N[1])[None, :, None] / N[1]
    n3 = np.arange(N[2])[None, None, :] / N[2]
    V = np.zeros(tuple(N), dtype=np.float64)
    for k in range(n_waves):
        V += amp[k] * np.cos(2 * np.pi * (m[k, 0] * n1 + m[k, 1] * n2 + m[k, 2] * n3))
    return V.reshape(-1), m, amp


def density_matrix(norb: int, nocc: int, rng: np.random.Generator):
    """D = C C^T with C ~ N(0,1)/sqrt(norb), shape (norb, nocc)."""
    C = rng.standard_normal((norb, nocc)) / np.sqrt(norb)
    return C @ C.T, C


# --------------------------------------------------------------------------
# the named workloads


def si8_sz(seed: int = 1) -> Workload:
    """Si-8 cubic cell, SZ basis (rc = 6), 24^3 mesh, 8 plane waves, C 32x16."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lat, pos = si_supercell((1, 1, 1))
    sp = [sz_species()]
    w = Workload("si8_sz", lat, (24, 24, 24), sp, np.zeros(8, np.int32), pos)
    w.V, w.pw_m, w.pw_amp = plane_wave_potential(w.grid, lat, 8, rng)
    w.D, w.C = density_matrix(w.norb, 16, rng)
    return w


def si_dzp(rep, grid, n_waves: int, nocc: int, seed: int, displace: float = 0.0,
           n_fd: int = 0, name: str = "") -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed))
    lat, pos = si_supercell(rep)
    if displace > 0.0:
        pos = pos + rng.normal(0.0, displace, size=pos.shape)
    sp = [dzp_species()]
    w = Workload(name or f"si{len(pos)}_dzp", lat, tuple(grid), sp,
                 np.zeros(len(pos), np.int32), pos)
    w.V, w.pw_m, w.pw_amp = plane_wave_potential(w.grid, lat, n_waves, rng)
    w.D, w.C = density_matrix(w.norb, nocc, rng)
    if n_fd:
        w.fd_atoms = np.sort(rng.choice(w.natom, size=n_fd, replace=False))
    return w


def si64_dzp(seed: int = 2) -> Workload:
    """Si-64 (2x2x2), DZP rc = 8, 96^3 mesh, 32 plane waves, C 832x128."""
    return si_dzp((2, 2, 2), (96, 96, 96), 32, 128, seed, name="si64_dzp")


def si512_dzp(seed: int = 5) -> Workload:
    """Si-512 (4x4x4) displaced N(0, 0.05 bohr), DZP, 192^3, 64 waves, C 6656x1024."""
    return si_dzp((4, 4, 4), (192, 192, 192), 64, 1024, seed, displace=0.05,
                  n_fd=8, name="si512_dzp")


BATCH_REPS = [(1, 1, 1), (1, 1, 2), (1, 2, 2), (2, 2, 2)]


def batched_kinds(n_cells: int = 256, seed: int = 4) -> np.ndarray:
    """Size class (0..3 -> 8, 16, 32, 64 atoms) of each batched cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 4, size=n_cells)


def batched_cells(n_cells: int = 256, seed: int = 4, select=None) -> List[Workload]:
    """Uneven independent cells for the batched launch.

    Sizes are drawn uniformly from {8, 16, 32, 64} atoms with the master seed;
    cell i then uses sub-seed 4000+i for V (16 waves) and C (2 per atom).
    Mesh spacing a/24 for 8/16-atom cells and a/48 for 32/64-atom cells.
    ``select`` (indices) builds only those cells, identical to the full set's.
    """
    kinds = batched_kinds(n_cells, seed)
    cells = []
    for i, k in enumerate(kinds):
        if select is not None and i not in select:
            continue
        rep = BATCH_REPS[int(k)]
        per = 24 if k < 2 else 48
        grid = tuple(per * r for r in rep)
        natom = 8 * int(np.prod(rep))
        cells.append(si_dzp(rep, grid, 16, 2 * natom, 4000 + i,
                            name=f"cell{i}_si{natom}"))
    return cells


def small_cell(positions, lattice, grid, species, species_of_atom=None,
               n_waves: int = 6, nocc: int = 4, seed: int = 0,
               gmax: Optional[float] = None) -> Workload:
    """A free-form small workload for tests (random V and D)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    positions = np.asarray(positions, dtype=np.float64)
    lattice = np.asarray(lattice, dtype=np.float64)
    if species_of_atom is None:
        species_of_atom = np.zeros(len(positions), np.int32)
    w = Workload("small", lattice, tuple(grid), list(species),
                 np.asarray(species_of_atom, np.int32), positions)
    if gmax is None:
        gmax = 3.0 * 2.0 * np.pi / float(np.min(np.linalg.norm(lattice, axis=1)))
    if n_waves:
        w.V, w.pw_m, w.pw_amp = plane_wave_potential(w.grid, lattice, n_waves, rng, gmax=gmax)
    else:
        w.V = np.zeros(w.ngrid)
    w.D, w.C = density_matrix(w.norb, nocc, rng)
    return w
