"""MI355X (gfx950) grid integration: Python binding over ``libgint.so``.

Argument marshalling only: every step of the computation (splines, binning,
orbital tiles, contractions, reductions) runs in the HIP kernels of the C
library declared in ``include/gint.h``.  PyTorch supplies device memory and
the current stream.  There is no CPU fallback: if the library is missing or
no gfx950 GPU is present, the calls raise.

The computed quantities are those of Sec. 3.3.1 ("Uniform Grid Integration
for Usual Quantities") of arXiv:2603.21835 at the Gamma point: H^loc, rho(r_g)
and the local Pulay force (returned as the gradient dE/dR).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgint.so")

GINT_OK, GINT_EINVAL, GINT_ENOMEM, GINT_EDEVICE, GINT_EUNSUPPORTED, GINT_ESTATE = range(6)
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "bf16x3": 4, "fp16x3": 5}

# Every symbol include/gint.h declares.
EXPORTS = (
    "gint_plan_create", "gint_plan_set_positions", "gint_plan_tune", "gint_plan_set_stream",
    "gint_build_H", "gint_build_H_weighted", "gint_build_rho", "gint_force",
    "gint_force_weighted", "gint_plan_sync", "gint_plan_work", "gint_norb", "gint_natom",
    "gint_dV", "gint_status_string", "gint_last_error", "gint_plan_destroy",
    "gint_plan_set_timing", "gint_plan_timing", "gint_rho_force", "gint_H_rho_force",
    "gint_build_HR", "gint_HR_lattice", "gint_build_rhoR", "gint_HR_to_Hk", "gint_forceR",
    "gint_batch_create", "gint_batch_build_H", "gint_batch_build_rho", "gint_batch_force",
    "gint_batch_sync", "gint_batch_ncell", "gint_batch_cell", "gint_batch_destroy", "gint_batch_autotune",
    "gint_plan_atom_order", "gint_test_fail_rebuilds", "gint_test_DR_gather", "gint_build_DK",
    "gint_psibeta_create", "gint_psibeta_nproj", "gint_psibeta_overlap", "gint_psibeta_destroy",
    "gint_batch_H_rho_force", "gint_HR_to_Hk_noalloc",
)
KERNELS = ("bin", "H_blocks", "H_reduce", "rho", "pack_D", "force", "force_reduce", "H_fill", "rho_force",
           "H_rho_force", "HR", "DK", "psibeta")


class GintError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class _Radial(ctypes.Structure):
    _fields_ = [("l", ctypes.c_int), ("nr", ctypes.c_int), ("dr", ctypes.c_double),
                ("f", ctypes.POINTER(ctypes.c_double)), ("dfdr_0", ctypes.c_double),
                ("dfdr_rc", ctypes.c_double)]


class _Species(ctypes.Structure):
    _fields_ = [("nradial", ctypes.c_int), ("radial", ctypes.POINTER(_Radial))]


class _Cell(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_double * 9), ("grid", ctypes.c_int * 3), ("natom", ctypes.c_int),
                ("species_of_atom", ctypes.POINTER(ctypes.c_int)), ("positions", ctypes.POINTER(ctypes.c_double))]


class Work(ctypes.Structure):
    _fields_ = [("ngrid", ctypes.c_longlong), ("nbatch", ctypes.c_longlong),
                ("nentry", ctypes.c_longlong), ("npair", ctypes.c_longlong),
                ("sum_ng", ctypes.c_double), ("sum_ng2", ctypes.c_double),
                ("batch", ctypes.c_int * 3), ("nslab", ctypes.c_int), ("nblock", ctypes.c_longlong),
                ("mno", ctypes.c_int), ("partial_bytes", ctypes.c_int), ("nblock_hr", ctypes.c_longlong)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgint.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    st = ctypes.c_int
    lib.gint_plan_create.restype = st
    lib.gint_plan_create.argtypes = [dp, ip, ctypes.c_int, ctypes.POINTER(_Species), ctypes.c_int, ip, dp,
                                     ctypes.c_int, P, ctypes.POINTER(P)]
    lib.gint_plan_set_positions.restype = st
    lib.gint_plan_set_positions.argtypes = [P, dp]
    lib.gint_plan_tune.restype = st
    lib.gint_plan_tune.argtypes = [P, ip, ctypes.c_longlong]
    lib.gint_plan_set_stream.restype = st
    lib.gint_plan_set_stream.argtypes = [P, P]
    for name in ("gint_build_H", "gint_build_H_weighted", "gint_build_rho", "gint_build_DK"):
        getattr(lib, name).restype = st
        getattr(lib, name).argtypes = [P, P, P]
    for name in ("gint_force", "gint_force_weighted"):
        getattr(lib, name).restype = st
        getattr(lib, name).argtypes = [P, P, P, P]
    lib.gint_rho_force.restype = st
    lib.gint_rho_force.argtypes = [P, P, P, P, P]
    lib.gint_H_rho_force.restype = st
    lib.gint_H_rho_force.argtypes = [P, P, P, P, P, P]
    lib.gint_plan_sync.restype = st
    lib.gint_build_HR.argtypes = [P, P, ctypes.c_int, ip, P]
    lib.gint_build_HR.restype = ctypes.c_int
    lib.gint_forceR.argtypes = [P, P, ctypes.c_int, ip, P, P]
    lib.gint_forceR.restype = ctypes.c_int
    lib.gint_HR_to_Hk.argtypes = [P, ctypes.c_int, ip, P, ctypes.c_int, dp, P]
    lib.gint_HR_to_Hk.restype = ctypes.c_int
    lib.gint_HR_to_Hk_noalloc.argtypes = [P, ctypes.c_int, ip, P, ctypes.c_int, dp, P]
    lib.gint_HR_to_Hk_noalloc.restype = ctypes.c_int
    lib.gint_build_rhoR.argtypes = [P, ctypes.c_int, ip, P, P]
    lib.gint_build_rhoR.restype = ctypes.c_int
    lib.gint_HR_lattice.argtypes = [P, ctypes.c_int, ip, ip]
    lib.gint_HR_lattice.restype = ctypes.c_int
    lib.gint_plan_sync.argtypes = [P]
    lib.gint_plan_work.restype = st
    lib.gint_plan_work.argtypes = [P, ctypes.POINTER(Work)]
    lib.gint_norb.restype = ctypes.c_int
    lib.gint_norb.argtypes = [P]
    lib.gint_natom.restype = ctypes.c_int
    lib.gint_natom.argtypes = [P]
    lib.gint_dV.restype = ctypes.c_double
    lib.gint_dV.argtypes = [P]
    lib.gint_status_string.restype = ctypes.c_char_p
    lib.gint_status_string.argtypes = [ctypes.c_int]
    lib.gint_last_error.restype = ctypes.c_char_p
    lib.gint_last_error.argtypes = []
    lib.gint_plan_set_timing.restype = st
    lib.gint_plan_set_timing.argtypes = [P, ctypes.c_int]
    lib.gint_plan_timing.restype = st
    lib.gint_plan_timing.argtypes = [P, dp, ip]
    lib.gint_plan_destroy.restype = None
    lib.gint_plan_destroy.argtypes = [P]
    lib.gint_psibeta_create.restype = st
    lib.gint_psibeta_create.argtypes = [P, ctypes.c_int, ctypes.POINTER(_Species), ctypes.c_int, dp, ctypes.c_int,
                                        dp, ctypes.POINTER(P)]
    lib.gint_psibeta_nproj.restype = ctypes.c_int
    lib.gint_psibeta_nproj.argtypes = [P]
    lib.gint_psibeta_overlap.restype = st
    lib.gint_psibeta_overlap.argtypes = [P, dp, P]
    lib.gint_psibeta_destroy.restype = None
    lib.gint_psibeta_destroy.argtypes = [P]
    lib.gint_plan_atom_order.restype = st
    lib.gint_plan_atom_order.argtypes = [P, ip]
    lib.gint_test_fail_rebuilds.restype = st
    lib.gint_test_fail_rebuilds.argtypes = [ctypes.c_int]
    lib.gint_test_DR_gather.restype = st
    lib.gint_test_DR_gather.argtypes = [ctypes.c_int]
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.gint_batch_create.restype = st
    lib.gint_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(_Cell), ctypes.c_int, ctypes.POINTER(_Species),
                                      ctypes.c_int, P, ctypes.POINTER(ctypes.c_void_p)]
    for name in ("gint_batch_build_H", "gint_batch_build_rho"):
        getattr(lib, name).restype = st
        getattr(lib, name).argtypes = [P, PP, PP]
    lib.gint_batch_force.restype = st
    lib.gint_batch_force.argtypes = [P, PP, PP, PP]
    lib.gint_batch_H_rho_force.restype = st
    lib.gint_batch_H_rho_force.argtypes = [P, PP, PP, PP, PP, PP]
    lib.gint_batch_autotune.restype = st
    lib.gint_batch_autotune.argtypes = [P, PP, PP, PP, PP, PP, ctypes.c_int, ip]
    lib.gint_batch_sync.restype = st
    lib.gint_batch_sync.argtypes = [P]
    lib.gint_batch_ncell.restype = ctypes.c_int
    lib.gint_batch_ncell.argtypes = [P]
    lib.gint_batch_cell.restype = P
    lib.gint_batch_cell.argtypes = [P, ctypes.c_int]
    lib.gint_batch_destroy.restype = None
    lib.gint_batch_destroy.argtypes = [P]
    _lib = lib
    return lib


def _check(status: int):
    if status != GINT_OK:
        lib = load_library()
        raise GintError(status, f"{lib.gint_status_string(status).decode()}: {lib.gint_last_error().decode()}")


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _dev_ptr(t, numel: int, what: str):
    import torch

    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{what} must be contiguous float64")
    if t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _species_array(species, keep):
    sp_arr = (_Species * len(species))()
    for s, spc in enumerate(species):
        rads = (_Radial * len(spc.radials))()
        for k, r in enumerate(spc.radials):
            f = np.ascontiguousarray(r.f, dtype=np.float64)
            keep.append(f)
            rads[k] = _Radial(int(r.l), int(f.size), float(r.dr), _dptr(f), float(r.dfdr0), float(r.dfdrc))
        keep.append(rads)
        sp_arr[s] = _Species(len(spc.radials), rads)
    keep.append(sp_arr)
    return sp_arr


class GintPlan:
    """Geometry + mesh + basis of one periodic cell (the GintInfo of Fig. 2).

    ``species`` is a list of objects with ``.radials``, each radial having
    ``l, dr, f (knot values), dfdr0, dfdrc`` (see ``gint_inputs``).
    """

    def __init__(self, lattice, grid, species, species_of_atom, positions, precision: str = "fp64",
                 stream=None):
        lib = load_library()
        self._lib = lib
        self._lat = np.ascontiguousarray(lattice, dtype=np.float64).reshape(9)
        self._grid = np.ascontiguousarray(grid, dtype=np.int32).reshape(3)
        self._keep = []
        sp_arr = _species_array(species, self._keep)
        self._soa = np.ascontiguousarray(species_of_atom, dtype=np.int32)
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1)
        self.natom = int(self._soa.size)
        self.ngrid = int(np.prod(self._grid))
        self.grid = tuple(int(x) for x in self._grid)
        handle = ctypes.c_void_p()
        _check(lib.gint_plan_create(_dptr(self._lat), _iptr(self._grid), len(species), sp_arr, self.natom,
                                    _iptr(self._soa), _dptr(pos), PRECISIONS[precision],
                                    _stream_handle(stream), ctypes.byref(handle)))
        self._h = handle
        self.norb = int(lib.gint_norb(handle))
        self.dV = float(lib.gint_dV(handle))
        self.precision = precision

    @classmethod
    def from_workload(cls, w, precision: str = "fp64", stream=None):
        return cls(w.lattice, w.grid, w.species, w.species_of_atom, w.positions, precision, stream)

    # -- lifecycle -------------------------------------------------------------
    @classmethod
    def _borrowed(cls, handle, lattice, grid, natom, precision):
        """A view of a plan owned by a GintBatch (never destroyed by the view)."""
        self = cls.__new__(cls)
        self._lib = load_library()
        self._owner = False
        self._h = ctypes.c_void_p(handle)
        self.natom = int(natom)
        self.grid = tuple(int(x) for x in grid)
        self.ngrid = int(np.prod(self.grid))
        self.norb = int(self._lib.gint_norb(self._h))
        self.dV = float(self._lib.gint_dV(self._h))
        self.precision = precision
        return self

    def close(self):
        if not getattr(self, "_owner", True):
            self._h = None
            return
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.gint_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _handle(self):
        if self._h is None:
            raise GintError(GINT_ESTATE, "plan is closed")
        return self._h

    # -- geometry ---------------------------------------------------------------
    def set_positions(self, positions):
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1)
        if pos.size != 3 * self.natom:
            raise ValueError("positions must have natom*3 entries")
        _check(self._lib.gint_plan_set_positions(self._handle(), _dptr(pos)))

    def tune(self, batch: Sequence[int], h_budget_bytes: int = 0):
        """Batch shape and the device-memory budget of the H path's block
        partials (0 = automatic); rebuilds the lists."""
        b = np.ascontiguousarray(batch, dtype=np.int32)
        _check(self._lib.gint_plan_tune(self._handle(), _iptr(b), int(h_budget_bytes)))

    def set_stream(self, stream=None):
        _check(self._lib.gint_plan_set_stream(self._handle(), _stream_handle(stream)))

    def sync(self):
        _check(self._lib.gint_plan_sync(self._handle()))

    def work(self) -> dict:
        w = Work()
        _check(self._lib.gint_plan_work(self._handle(), ctypes.byref(w)))
        return {"ngrid": w.ngrid, "nbatch": w.nbatch, "nentry": w.nentry, "npair": w.npair,
                "sum_ng": w.sum_ng, "sum_ng2": w.sum_ng2, "batch": tuple(w.batch), "nslab": w.nslab,
                "nblock": w.nblock, "mno": w.mno, "partial_bytes": w.partial_bytes, "nblock_hr": w.nblock_hr}

    def atom_order(self) -> np.ndarray:
        """Input indices of the atoms in the plan's processing order."""
        order = np.zeros(self.natom, dtype=np.int32)
        _check(self._lib.gint_plan_atom_order(self._handle(), _iptr(order)))
        return order

    def set_timing(self, enable: bool = True):
        _check(self._lib.gint_plan_set_timing(self._handle(), 1 if enable else 0))

    def timing(self) -> dict:
        """{kernel: (total_ms, launches)} since timing was enabled."""
        ms = np.zeros(len(KERNELS))
        n = np.zeros(len(KERNELS), dtype=np.int32)
        _check(self._lib.gint_plan_timing(self._handle(), _dptr(ms), _iptr(n)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}

    # -- the three grid integrals ----------------------------------------------------
    def build_H(self, V, out=None, weighted: bool = False):
        """H^loc (norb x norb). With weighted=True the input is the per-point weight w_g (no dV)."""
        import torch

        vp = _dev_ptr(V, self.ngrid, "V")
        if out is None:
            out = torch.empty((self.norb, self.norb), dtype=torch.float64, device=V.device)
        op = _dev_ptr(out, self.norb * self.norb, "H")
        fn = self._lib.gint_build_H_weighted if weighted else self._lib.gint_build_H
        _check(fn(self._handle(), vp, op))
        return out

    def build_DK(self, W=None, out=None):
        """Moving-basis matrix DK[c, mu, nu] = <phit_mu|W|d phit_nu/d tau_K>_c
        (K the atom of nu; W None: W = 1), a (3, norb, norb) tensor."""
        import torch

        n = self.norb
        wp = ctypes.c_void_p(None) if W is None else _dev_ptr(W, self.ngrid, "W")
        if out is None:
            dev = W.device if W is not None else torch.device("cuda", torch.cuda.current_device())
            out = torch.empty((3, n, n), dtype=torch.float64, device=dev)
        op = _dev_ptr(out, 3 * n * n, "DK")
        _check(self._lib.gint_build_DK(self._handle(), wp, op))
        return out

    def HR_lattice(self):
        """Lattice multiples (n x 3 ints) of every R that can carry a non-zero
        H(R) block (pairs of atom images sharing a mesh batch)."""
        import numpy as np

        n = ctypes.c_int(0)
        self._lib.gint_HR_lattice(self._handle(), 0, ctypes.byref(n), None)
        R = np.zeros((max(n.value, 1), 3), dtype=np.int32)
        _check(self._lib.gint_HR_lattice(self._handle(), n.value, ctypes.byref(n),
                                         R.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return R[: n.value]

    def build_HR(self, V, R=None, out=None):
        """Lattice-vector blocks H(R) (nR x norb x norb) for the lattice
        multiples R (nR x 3 ints; default: HR_lattice()).
        Returns (R, HR)."""
        import numpy as np
        import torch

        if R is None:
            R = self.HR_lattice()
        Rl = np.ascontiguousarray(np.asarray(R, dtype=np.int32).reshape(-1, 3))
        nR = int(Rl.shape[0])
        vp = _dev_ptr(V, self.ngrid, "V")
        if out is None:
            out = torch.empty((nR, self.norb, self.norb), dtype=torch.float64, device=V.device)
        op = _dev_ptr(out, nR * self.norb * self.norb, "HR")
        _check(self._lib.gint_build_HR(self._handle(), vp, nR,
                                       Rl.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), op))
        return Rl, out

    def forceR(self, V, R, DR, out=None):
        """dE/dR (natom x 3) for E = dV sum V rho(D(R)), D(R) blocks DR
        (nR x norb x norb, device) for the lattice multiples R (nR x 3)."""
        import numpy as np
        import torch

        Rl = np.ascontiguousarray(np.asarray(R, dtype=np.int32).reshape(-1, 3))
        nR = int(Rl.shape[0])
        vp = _dev_ptr(V, self.ngrid, "V")
        dp = _dev_ptr(DR, nR * self.norb * self.norb, "DR")
        if out is None:
            out = torch.empty((self.natom, 3), dtype=torch.float64, device=V.device)
        op = _dev_ptr(out, self.natom * 3, "dEdR")
        _check(self._lib.gint_forceR(self._handle(), vp, nR, Rl.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), dp, op))
        return out

    def HR_to_Hk(self, R, HR, kfrac, out=None, noalloc: bool = False):
        """H(k) = sum_q e^{i 2 pi kappa.n_q} H(R_q) for fractional k-points
        kfrac (nk x 3): a complex128 tensor (nk x norb x norb).  noalloc:
        call gint_HR_to_Hk_noalloc (no device allocation in the library;
        ``out`` should then be given)."""
        import numpy as np
        import torch

        Rl = np.ascontiguousarray(np.asarray(R, dtype=np.int32).reshape(-1, 3))
        kf = np.ascontiguousarray(np.asarray(kfrac, dtype=np.float64).reshape(-1, 3))
        nR, nk = int(Rl.shape[0]), int(kf.shape[0])
        hp = _dev_ptr(HR, nR * self.norb * self.norb, "HR")
        if out is None:
            out = torch.empty((nk, self.norb, self.norb), dtype=torch.complex128, device=HR.device)
        if out.dtype != torch.complex128 or not out.is_contiguous() or out.numel() != nk * self.norb * self.norb:
            raise TypeError("out must be a contiguous complex128 tensor of nk*norb*norb elements")
        fn = self._lib.gint_HR_to_Hk_noalloc if noalloc else self._lib.gint_HR_to_Hk
        _check(fn(self._handle(), nR, Rl.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), hp, nk,
                  kf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(out.data_ptr())))
        return out

    def build_rhoR(self, R, DR, out=None):
        """rho (N1*N2*N3) from lattice-vector density-matrix blocks DR
        (nR x norb x norb, device) for the lattice multiples R (nR x 3)."""
        import numpy as np
        import torch

        Rl = np.ascontiguousarray(np.asarray(R, dtype=np.int32).reshape(-1, 3))
        nR = int(Rl.shape[0])
        dp = _dev_ptr(DR, nR * self.norb * self.norb, "DR")
        if out is None:
            out = torch.empty(self.ngrid, dtype=torch.float64, device=DR.device)
        op = _dev_ptr(out, self.ngrid, "rho")
        _check(self._lib.gint_build_rhoR(self._handle(), nR, Rl.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                         dp, op))
        return out

    def build_rho(self, D, out=None):
        import torch

        dp = _dev_ptr(D, self.norb * self.norb, "D")
        if out is None:
            out = torch.empty(self.ngrid, dtype=torch.float64, device=D.device)
        op = _dev_ptr(out, self.ngrid, "rho")
        _check(self._lib.gint_build_rho(self._handle(), dp, op))
        return out

    def force(self, W, D, out=None, weighted: bool = False):
        """dE/dR (natom x 3) for E = dV sum W rho (or sum w rho with weighted=True)."""
        import torch

        wp = _dev_ptr(W, self.ngrid, "W")
        dp = _dev_ptr(D, self.norb * self.norb, "D")
        if out is None:
            out = torch.empty((self.natom, 3), dtype=torch.float64, device=W.device)
        op = _dev_ptr(out, self.natom * 3, "dEdR")
        fn = self._lib.gint_force_weighted if weighted else self._lib.gint_force
        _check(fn(self._handle(), wp, dp, op))
        return out

    def rho_force(self, W, D, rho=None, out=None):
        """(rho, dE/dR) in one pass: E = dV sum W rho."""
        import torch

        wp = _dev_ptr(W, self.ngrid, "W")
        dp = _dev_ptr(D, self.norb * self.norb, "D")
        if rho is None:
            rho = torch.empty(self.ngrid, dtype=torch.float64, device=W.device)
        if out is None:
            out = torch.empty((self.natom, 3), dtype=torch.float64, device=W.device)
        rp = _dev_ptr(rho, self.ngrid, "rho")
        op = _dev_ptr(out, self.natom * 3, "dEdR")
        _check(self._lib.gint_rho_force(self._handle(), wp, dp, rp, op))
        return rho, out

    def H_rho_force(self, V, D, H=None, rho=None, out=None):
        """(H, rho, dE/dR) of one V and D in one call (one pass over the mesh
        batches for all three in the FP64 / FP32 modes)."""
        import torch

        vp = _dev_ptr(V, self.ngrid, "V")
        dp = _dev_ptr(D, self.norb * self.norb, "D")
        if H is None:
            H = torch.empty((self.norb, self.norb), dtype=torch.float64, device=V.device)
        if rho is None:
            rho = torch.empty(self.ngrid, dtype=torch.float64, device=V.device)
        if out is None:
            out = torch.empty((self.natom, 3), dtype=torch.float64, device=V.device)
        hp = _dev_ptr(H, self.norb * self.norb, "H")
        rp = _dev_ptr(rho, self.ngrid, "rho")
        op = _dev_ptr(out, self.natom * 3, "dEdR")
        _check(self._lib.gint_H_rho_force(self._handle(), vp, dp, hp, rp, op))
        return H, rho, out


class GintPsiBeta:
    """Spherical-grid projector overlaps Q[p, mu] = <phit_mu|e^{-iA.r}|beta_p>
    of one plan (gint_psibeta_*): ``proj_species`` holds one Species of
    projector radials per orbital species (may be empty), ``ang`` the
    angular rule rows (x, y, z, w), ``rq`` the radial rule rows (x, q) on
    [0, 1]."""

    def __init__(self, plan: GintPlan, proj_species, ang, rq):
        self._lib = plan._lib
        self.plan = plan
        self._keep = []
        sp_arr = _species_array(proj_species, self._keep)
        self._ang = np.ascontiguousarray(ang, dtype=np.float64).reshape(-1, 4)
        self._rq = np.ascontiguousarray(rq, dtype=np.float64).reshape(-1, 2)
        h = ctypes.c_void_p()
        _check(self._lib.gint_psibeta_create(plan._handle(), len(proj_species), sp_arr, self._ang.shape[0],
                                             _dptr(self._ang), self._rq.shape[0], _dptr(self._rq), ctypes.byref(h)))
        self._h = h
        self.nproj = int(self._lib.gint_psibeta_nproj(h))

    def overlap(self, A, out=None):
        """Q for the vector potential A (3 floats): complex128 (nproj, norb)."""
        import torch

        a = np.ascontiguousarray(A, dtype=np.float64).reshape(3)
        n = self.plan.norb
        if out is None:
            out = torch.empty((self.nproj, n), dtype=torch.complex128,
                              device=torch.device("cuda", torch.cuda.current_device()))
        if out.dtype != torch.complex128 or not out.is_contiguous() or out.numel() != self.nproj * n:
            raise TypeError("out must be a contiguous complex128 tensor of nproj*norb elements")
        _check(self._lib.gint_psibeta_overlap(self._h, _dptr(a), ctypes.c_void_p(out.data_ptr())))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.gint_psibeta_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_H(plan: GintPlan, V, out=None):
    return plan.build_H(V, out)


def build_rho(plan: GintPlan, D, out=None):
    return plan.build_rho(D, out)


def force(plan: GintPlan, W, D, out=None):
    return plan.force(W, D, out)


class GintBatch:
    """Many independent periodic cells (uneven sizes, one basis) behind one
    call per quantity; each call replays one captured hipGraph while the
    geometries and the tensors passed stay the same.

    ``cells``: list of workloads (objects with lattice, grid,
    species_of_atom, positions).  Pass ``out=`` lists to keep the device
    pointers, and so the captured graph, the same from call to call.
    """

    def __init__(self, cells, species, precision: str = "fp64", stream=None):
        lib = load_library()
        self._lib = lib
        self._keep = []
        sp_arr = _species_array(species, self._keep)
        n = len(cells)
        arr = (_Cell * n)()
        self.ngrid, self.natom, self.grid = [], [], []
        for i, c in enumerate(cells):
            lat = np.ascontiguousarray(c.lattice, dtype=np.float64).reshape(9)
            grid = np.ascontiguousarray(c.grid, dtype=np.int32).reshape(3)
            soa = np.ascontiguousarray(c.species_of_atom, dtype=np.int32)
            pos = np.ascontiguousarray(c.positions, dtype=np.float64).reshape(-1)
            self._keep += [soa, pos]
            arr[i].lattice[:] = list(lat)
            arr[i].grid[:] = [int(x) for x in grid]
            arr[i].natom = int(soa.size)
            arr[i].species_of_atom = _iptr(soa)
            arr[i].positions = _dptr(pos)
            self.ngrid.append(int(np.prod(grid)))
            self.natom.append(int(soa.size))
            self.grid.append(tuple(int(x) for x in grid))
        handle = ctypes.c_void_p()
        _check(lib.gint_batch_create(n, arr, len(species), sp_arr, PRECISIONS[precision], _stream_handle(stream),
                                     ctypes.byref(handle)))
        self._h = handle
        self.ncell = n
        self.precision = precision
        self.cells = [GintPlan._borrowed(lib.gint_batch_cell(handle, i), cells[i].lattice, self.grid[i],
                                         self.natom[i], precision) for i in range(n)]
        self.norb = [p.norb for p in self.cells]
        self.dV = [p.dV for p in self.cells]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            for p in self.cells:
                p.close()
            self._lib.gint_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _handle(self):
        if self._h is None:
            raise GintError(GINT_ESTATE, "batch is closed")
        return self._h

    def _ptrs(self, ts, sizes, what):
        if len(ts) != self.ncell:
            raise ValueError(f"{what}: expected {self.ncell} tensors")
        arr = (ctypes.c_void_p * self.ncell)()
        for i, (t, n) in enumerate(zip(ts, sizes)):
            arr[i] = _dev_ptr(t, n, f"{what}[{i}]").value
        return arr

    def _outs(self, out, shapes, like):
        import torch

        if out is None:
            out = [torch.empty(sh, dtype=torch.float64, device=like.device) for sh in shapes]
        return out

    def sync(self):
        _check(self._lib.gint_batch_sync(self._handle()))

    def autotune(self, V, D, H, rho, F, reps: int = 2):
        """Time the candidate batch shapes per class of equal cells (mesh and
        atom count) and keep the fastest; returns each cell's shape."""
        nn = [n * n for n in self.norb]
        chosen = np.zeros(3 * self.ncell, dtype=np.int32)
        _check(self._lib.gint_batch_autotune(self._handle(), self._ptrs(V, self.ngrid, "V"), self._ptrs(D, nn, "D"),
                                             self._ptrs(H, nn, "H"), self._ptrs(rho, self.ngrid, "rho"),
                                             self._ptrs(F, [3 * a for a in self.natom], "dEdR"), int(reps),
                                             _iptr(chosen)))
        return [tuple(int(x) for x in chosen[3 * i:3 * i + 3]) for i in range(self.ncell)]

    def build_H(self, V, out=None):
        nn = [n * n for n in self.norb]
        out = self._outs(out, [(n, n) for n in self.norb], V[0])
        _check(self._lib.gint_batch_build_H(self._handle(), self._ptrs(V, self.ngrid, "V"),
                                            self._ptrs(out, nn, "H")))
        return out

    def build_rho(self, D, out=None):
        nn = [n * n for n in self.norb]
        out = self._outs(out, [(g,) for g in self.ngrid], D[0])
        _check(self._lib.gint_batch_build_rho(self._handle(), self._ptrs(D, nn, "D"),
                                              self._ptrs(out, self.ngrid, "rho")))
        return out

    def H_rho_force(self, V, D, H=None, rho=None, out=None):
        """H, rho and dE/dR of every cell in one graph replay."""
        nn = [n * n for n in self.norb]
        H = self._outs(H, [(n, n) for n in self.norb], V[0])
        rho = self._outs(rho, [(g,) for g in self.ngrid], V[0])
        out = self._outs(out, [(a, 3) for a in self.natom], V[0])
        _check(self._lib.gint_batch_H_rho_force(self._handle(), self._ptrs(V, self.ngrid, "V"),
                                                self._ptrs(D, nn, "D"), self._ptrs(H, nn, "H"),
                                                self._ptrs(rho, self.ngrid, "rho"),
                                                self._ptrs(out, [3 * a for a in self.natom], "dEdR")))
        return H, rho, out

    def force(self, W, D, out=None):
        nn = [n * n for n in self.norb]
        out = self._outs(out, [(a, 3) for a in self.natom], W[0])
        _check(self._lib.gint_batch_force(self._handle(), self._ptrs(W, self.ngrid, "W"), self._ptrs(D, nn, "D"),
                                          self._ptrs(out, [3 * a for a in self.natom], "dEdR")))
        return out
