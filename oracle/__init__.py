"""FP64 CPU oracle for the grid integrals (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library: it has its own spline, spherical harmonics, image search and loops
(``gint_oracle.c``), compiled with gcc into ``liboracle.so``.

Functions follow Sec. 3.3.1 ("Uniform Grid Integration for Usual
Quantities") of the paper: the rho(r_g) equation, the H^loc equation and the
F^{loc,Pulay} equation, at the Gamma point, on the basis of Sec. 2.1; and
the lattice-vector blocks H^loc(R) of the same H^loc equation (``HR``),
whose phase sum is the H(k) equation of Sec. 2.1, and rho from
lattice-vector density-matrix blocks (``rhoR``, the rho(r_g) equation with
its sums over R and R').
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "gint_oracle.c")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           SRC_PATH, "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_long)
    lib.oracle_create.restype = P
    lib.oracle_create.argtypes = [dp, ip, ctypes.c_int, ip, ip, dp, dp, dp, dp,
                                  ctypes.c_int, ip, ctypes.c_int, ip, dp]
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_norb.argtypes = [P]
    lib.oracle_atom_orb0.argtypes = [P, ctypes.c_int]
    lib.oracle_dV.argtypes = [P]
    lib.oracle_dV.restype = ctypes.c_double
    lib.oracle_radial.argtypes = [P, ctypes.c_int, ctypes.c_double, dp]
    lib.oracle_radial.restype = ctypes.c_double
    lib.oracle_ylm.argtypes = [ctypes.c_int, dp, dp]
    lib.oracle_phi.argtypes = [P, dp, dp, dp]
    lib.oracle_H_rows.argtypes = [P, dp, ctypes.c_int, ctypes.c_int, ctypes.c_long, lp, dp]
    lib.oracle_HR_rows.argtypes = [P, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp]
    lib.oracle_HR_rows.restype = ctypes.c_int
    lib.oracle_forceR.argtypes = [P, dp, ctypes.c_int, ip, dp, ctypes.c_int, ip, dp]
    lib.oracle_forceR.restype = ctypes.c_int
    lib.oracle_rhoR.argtypes = [P, ctypes.c_int, ip, dp, ctypes.c_long, lp, dp]
    lib.oracle_rhoR.restype = ctypes.c_int
    lib.oracle_rho.argtypes = [P, dp, ctypes.c_long, lp, dp]
    lib.oracle_force.argtypes = [P, dp, dp, ctypes.c_int, ip, ctypes.c_long, lp, dp]
    lib.oracle_DK_rows.argtypes = [P, dp, ctypes.c_int, ctypes.c_int, ctypes.c_long, lp, dp]
    lib.oracle_proj_create.restype = P
    lib.oracle_proj_create.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp, dp, ctypes.c_int, ip]
    lib.oracle_proj_destroy.argtypes = [P]
    lib.oracle_proj_row0.restype = ctypes.c_int
    lib.oracle_proj_row0.argtypes = [P, P, ctypes.c_int]
    lib.oracle_psibeta.argtypes = [P, P, ctypes.c_int, dp, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_set_positions.argtypes = [P, dp]
    lib.oracle_support_stats.argtypes = [P, dp, dp]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def ylm(l: int, u) -> np.ndarray:
    """Real Y_lm(u), m = -l..l, at a unit vector (closed forms)."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(2 * l + 1)
    lib.oracle_ylm(l, _dp(u), _dp(out))
    return out


def Hk_from_HR(R, HR, kfrac) -> np.ndarray:
    """Bloch sum of Sec. 2.1's H(k) equation: H(k) = sum_R e^{i k.R} H(R),
    k.R = 2 pi kappa . n for fractional reciprocal coordinates kappa and
    lattice multiples n.  Returns complex [nk][norb][norb]."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    kf = np.asarray(kfrac, dtype=np.float64).reshape(-1, 3)
    HR = np.asarray(HR, dtype=np.float64)
    out = np.zeros((kf.shape[0],) + HR.shape[1:], dtype=np.complex128)
    for i, k in enumerate(kf):
        for q in range(R.shape[0]):
            out[i] += np.exp(2j * np.pi * float(k @ R[q])) * HR[q]
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    _load().oracle_set_threads(int(n))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


class Oracle:
    """Oracle context for one cell (geometry, basis, mesh)."""

    def __init__(self, lattice, grid, species, species_of_atom, positions):
        lib = _load()
        self._lib = lib
        rad_l, rad_nr, rad_dr, rad_d0, rad_drc, fs, begin = [], [], [], [], [], [], [0]
        for sp in species:
            for r in sp.radials:
                rad_l.append(r.l)
                rad_nr.append(r.nr)
                rad_dr.append(r.dr)
                rad_d0.append(r.dfdr0)
                rad_drc.append(r.dfdrc)
                fs.append(np.asarray(r.f, dtype=np.float64))
            begin.append(len(rad_l))
        self._keep = [
            np.ascontiguousarray(lattice, dtype=np.float64).reshape(9),
            np.asarray(grid, dtype=np.int32),
            np.asarray(rad_l, dtype=np.int32),
            np.asarray(rad_nr, dtype=np.int32),
            np.asarray(rad_dr, dtype=np.float64),
            np.concatenate(fs),
            np.asarray(rad_d0, dtype=np.float64),
            np.asarray(rad_drc, dtype=np.float64),
            np.asarray(begin, dtype=np.int32),
            np.asarray(species_of_atom, dtype=np.int32),
            np.ascontiguousarray(positions, dtype=np.float64).reshape(-1),
        ]
        k = self._keep
        self.natom = int(len(k[9]))
        self.grid = tuple(int(g) for g in grid)
        self.ngrid = int(np.prod(self.grid))
        self._ctx = lib.oracle_create(_dp(k[0]), _ip(k[1]), len(rad_l), _ip(k[2]), _ip(k[3]), _dp(k[4]),
                                      _dp(k[5]), _dp(k[6]), _dp(k[7]), len(species), _ip(k[8]),
                                      self.natom, _ip(k[9]), _dp(k[10]))
        self.norb = int(lib.oracle_norb(self._ctx))
        self.dV = float(lib.oracle_dV(self._ctx))
        self.atom_orb0 = np.array([lib.oracle_atom_orb0(self._ctx, i) for i in range(self.natom)] + [self.norb])

    @classmethod
    def from_workload(cls, w):
        return cls(w.lattice, w.grid, w.species, w.species_of_atom, w.positions)

    def __del__(self):
        if getattr(self, "_ctx", None):
            self._lib.oracle_destroy(self._ctx)
            self._ctx = None

    # -- pointwise -----------------------------------------------------------
    def radial(self, k: int, r: float):
        d = ctypes.c_double(0.0)
        v = self._lib.oracle_radial(self._ctx, k, float(r), ctypes.byref(d))
        return v, d.value

    def phi(self, r, grad: bool = False):
        r = np.ascontiguousarray(r, dtype=np.float64)
        phi = np.zeros(self.norb)
        g = np.zeros((self.norb, 3)) if grad else None
        self._lib.oracle_phi(self._ctx, _dp(r), _dp(phi), _dp(g) if grad else None)
        return (phi, g) if grad else phi

    def set_positions(self, positions):
        p = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1)
        self._keep[10] = p
        self._lib.oracle_set_positions(self._ctx, _dp(p))

    def support_stats(self):
        a, b = ctypes.c_double(0), ctypes.c_double(0)
        self._lib.oracle_support_stats(self._ctx, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    # -- integrals -------------------------------------------------------------
    @staticmethod
    def _points(points):
        if points is None:
            return 0, None, None
        idx = np.ascontiguousarray(points, dtype=np.int64)
        return idx.size, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), idx

    def H_rows(self, V, I0: int, I1: int, points: Optional[Sequence[int]] = None) -> np.ndarray:
        """Rows of H for atoms I0..I1-1; the mesh sum runs over ``points``
        (all mesh points when None)."""
        V = np.ascontiguousarray(V, dtype=np.float64)
        assert V.size == self.ngrid
        n = int(self.atom_orb0[I1] - self.atom_orb0[I0])
        out = np.zeros((n, self.norb))
        npts, ip_, keep = self._points(points)
        self._lib.oracle_H_rows(self._ctx, _dp(V), int(I0), int(I1), npts, ip_, _dp(out))
        return out

    def H(self, V) -> np.ndarray:
        return self.H_rows(V, 0, self.natom)

    def HR(self, V, R, I0: int = 0, I1: Optional[int] = None) -> np.ndarray:
        """Lattice-vector blocks H(R) for the lattice multiples ``R`` (n x 3
        ints), rows of atoms I0..I1-1: an array [n][rows][norb].  Positions
        are taken as given (not wrapped); contributions to R outside the
        list are dropped."""
        I1 = self.natom if I1 is None else I1
        V = np.ascontiguousarray(V, dtype=np.float64)
        assert V.size == self.ngrid
        Rl = np.ascontiguousarray(np.asarray(R, dtype=np.int32).reshape(-1, 3))
        n = int(self.atom_orb0[I1] - self.atom_orb0[I0])
        out = np.zeros((Rl.shape[0], n, self.norb))
        rc = self._lib.oracle_HR_rows(self._ctx, _dp(V), int(I0), int(I1), int(Rl.shape[0]), _ip(Rl), _dp(out))
        if rc != 0:
            raise RuntimeError("a mesh point sees too many images of one atom")
        return out

    def rhoR(self, R, DR, idx: Optional[Sequence[int]] = None) -> np.ndarray:
        """rho from lattice-vector density-matrix blocks DR [n][norb][norb]
        for the lattice multiples R (n x 3), at mesh points ``idx`` (all when
        None)."""
        Rl = np.ascontiguousarray(np.asarray(R, dtype=np.int32).reshape(-1, 3))
        DR = np.ascontiguousarray(DR, dtype=np.float64)
        assert DR.shape == (Rl.shape[0], self.norb, self.norb)
        if idx is None:
            n, ip_ = self.ngrid, None
        else:
            keep = np.ascontiguousarray(idx, dtype=np.int64)
            n, ip_ = keep.size, keep.ctypes.data_as(ctypes.POINTER(ctypes.c_long))
        out = np.zeros(n)
        rc = self._lib.oracle_rhoR(self._ctx, int(Rl.shape[0]), _ip(Rl), _dp(DR), n, ip_, _dp(out))
        if rc != 0:
            raise RuntimeError("a mesh point sees too many images of one atom")
        return out

    def forceR(self, V, R, DR, atoms: Optional[Sequence[int]] = None) -> np.ndarray:
        """dE/dR_I (not the force) for E = dV sum V rho(D(R)), rho as in
        ``rhoR``, for the chosen atoms."""
        V = np.ascontiguousarray(V, dtype=np.float64)
        Rl = np.ascontiguousarray(np.asarray(R, dtype=np.int32).reshape(-1, 3))
        DR = np.ascontiguousarray(DR, dtype=np.float64)
        assert DR.shape == (Rl.shape[0], self.norb, self.norb)
        sel = np.arange(self.natom, dtype=np.int32) if atoms is None else np.ascontiguousarray(atoms, dtype=np.int32)
        out = np.zeros((sel.size, 3))
        rc = self._lib.oracle_forceR(self._ctx, _dp(V), int(Rl.shape[0]), _ip(Rl), _dp(DR), int(sel.size), _ip(sel),
                                     _dp(out))
        if rc != 0:
            raise RuntimeError("a mesh point sees too many images of one atom")
        return out

    def rho(self, D, idx: Optional[Sequence[int]] = None) -> np.ndarray:
        D = np.ascontiguousarray(D, dtype=np.float64)
        assert D.shape == (self.norb, self.norb)
        if idx is None:
            out = np.zeros(self.ngrid)
            self._lib.oracle_rho(self._ctx, _dp(D), self.ngrid, None, _dp(out))
        else:
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            out = np.zeros(idx.size)
            self._lib.oracle_rho(self._ctx, _dp(D), idx.size,
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out))
        return out

    def force(self, V, D, atoms: Optional[Sequence[int]] = None,
              points: Optional[Sequence[int]] = None) -> np.ndarray:
        """dE/dR_I (not the force) for the chosen atoms, E = dV sum V rho;
        the mesh sum runs over ``points`` (all mesh points when None)."""
        V = np.ascontiguousarray(V, dtype=np.float64)
        D = np.ascontiguousarray(D, dtype=np.float64)
        sel = np.arange(self.natom, dtype=np.int32) if atoms is None else np.ascontiguousarray(atoms, dtype=np.int32)
        out = np.zeros((sel.size, 3))
        npts, ip_, keep = self._points(points)
        self._lib.oracle_force(self._ctx, _dp(V), _dp(D), int(sel.size), _ip(sel), npts, ip_, _dp(out))
        return out

    def DK_rows(self, W, I0: int, I1: int, points: Optional[Sequence[int]] = None) -> np.ndarray:
        """Rows of the moving-basis matrix (Sec. 2.3, D_K equation, Gamma
        point) for the orbitals of atoms I0..I1-1:
        out[c, mu, nu] = <phit_mu | W | d phit_nu / d tau_K>_c with K the
        atom of nu, i.e. -dV sum_g W_g phit_mu d_c phit_nu (W None: W = 1)."""
        Wp = None
        if W is not None:
            W = np.ascontiguousarray(W, dtype=np.float64)
            Wp = _dp(W)
        nrow = int(self.atom_orb0[I1] - self.atom_orb0[I0])
        out = np.zeros((3, nrow, self.norb))
        npts, ip_, keep = self._points(points)
        self._lib.oracle_DK_rows(self._ctx, Wp, int(I0), int(I1), npts, ip_, _dp(out))
        return out

    def DK(self, W=None) -> np.ndarray:
        """The whole 3 x norb x norb moving-basis matrix (see DK_rows)."""
        return self.DK_rows(W, 0, self.natom)

    def psibeta(self, proj_species, ang, rq, A, I0: int = 0, I1: Optional[int] = None) -> np.ndarray:
        """Spherical-grid projector overlaps (Sec. 3.3.2) for the projectors
        of atoms I0..I1-1: Q[p, mu] = <phit_mu | e^{-i A.r} | beta_p> on the
        product grid (angular rule ``ang`` rows (x, y, z, w); radial rule
        ``rq`` rows (x, q) on [0, 1]) centred on each projector's atom.
        ``proj_species``: one Species of projector radials per orbital
        species (may be empty).  Complex (rows, norb)."""
        I1 = self.natom if I1 is None else I1
        l, nr, dr, d0, drc, fs, begin = [], [], [], [], [], [], [0]
        for sp in proj_species:
            for r in sp.radials:
                l.append(r.l)
                nr.append(r.nr)
                dr.append(r.dr)
                d0.append(r.dfdr0)
                drc.append(r.dfdrc)
                fs.append(np.asarray(r.f, dtype=np.float64))
            begin.append(len(l))
        k = [np.asarray(l, dtype=np.int32), np.asarray(nr, dtype=np.int32), np.asarray(dr, dtype=np.float64),
             np.concatenate(fs) if fs else np.zeros(1), np.asarray(d0, dtype=np.float64),
             np.asarray(drc, dtype=np.float64), np.asarray(begin, dtype=np.int32)]
        pp = self._lib.oracle_proj_create(len(l), _ip(k[0]), _ip(k[1]), _dp(k[2]), _dp(k[3]), _dp(k[4]),
                                          _dp(k[5]), len(proj_species), _ip(k[6]))
        try:
            r0 = self._lib.oracle_proj_row0(self._ctx, pp, int(I0))
            r1 = self._lib.oracle_proj_row0(self._ctx, pp, int(I1))
            ang = np.ascontiguousarray(ang, dtype=np.float64)
            rq = np.ascontiguousarray(rq, dtype=np.float64)
            A = np.ascontiguousarray(A, dtype=np.float64)
            out = np.zeros((r1 - r0, self.norb, 2))
            self._lib.oracle_psibeta(self._ctx, pp, int(ang.shape[0]), _dp(ang), int(rq.shape[0]), _dp(rq), _dp(A),
                                     int(I0), int(I1), _dp(out))
        finally:
            self._lib.oracle_proj_destroy(pp)
        return out[..., 0] + 1j * out[..., 1]

    def energy(self, V, D) -> float:
        return float(self.dV * np.dot(np.asarray(V, dtype=np.float64), self.rho(D)))
