"""The C-ABI library: it loads, exports every symbol include/gint.h declares,
and rejects invalid arguments on the host before touching any device."""
import ctypes
import os
import re

import numpy as np
import pytest

import gint_inputs as gi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_2603_21835_amd as g

    if not os.path.exists(g.LIB_PATH):
        from paper_2603_21835_amd import build

        build.build(verbose=False)
    return g.load_library()


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "gint.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gint_[a-z_A-Z0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    import paper_2603_21835_amd as g

    declared = _declared_symbols()
    assert declared, "no declarations parsed"
    assert sorted(g.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def _args(w, **over):
    """ctypes arguments of gint_plan_create for workload w, with overrides."""
    import paper_2603_21835_amd as g

    keep = []
    sp = (g._Species * len(w.species))()
    for s, spc in enumerate(w.species):
        rads = (g._Radial * len(spc.radials))()
        for k, r in enumerate(spc.radials):
            f = np.ascontiguousarray(r.f)
            keep.append(f)
            rads[k] = g._Radial(r.l, f.size, r.dr, g._dptr(f), r.dfdr0, r.dfdrc)
        keep.append(rads)
        sp[s] = g._Species(len(spc.radials), rads)
    lat = np.ascontiguousarray(w.lattice, dtype=np.float64).reshape(9)
    grid = np.array(w.grid, dtype=np.int32)
    soa = np.ascontiguousarray(w.species_of_atom, dtype=np.int32)
    pos = np.ascontiguousarray(w.positions, dtype=np.float64).reshape(-1)
    a = dict(lattice=g._dptr(lat), grid=g._iptr(grid), nspecies=len(w.species), species=sp,
             natom=w.natom, soa=g._iptr(soa), pos=g._dptr(pos), prec=0, stream=None)
    a.update(over)
    keep += [lat, grid, soa, pos]
    return a, keep


def _create(lib, a):
    out = ctypes.c_void_p(12345)
    st = lib.gint_plan_create(a["lattice"], a["grid"], a["nspecies"], a["species"], a["natom"], a["soa"],
                              a["pos"], a["prec"], a["stream"], ctypes.byref(out))
    return st, out.value


def test_invalid_arguments_rejected_before_device(lib):
    import paper_2603_21835_amd as g

    w = gi.si8_sz()
    cases = []
    bad_grid = np.array([24, 0, 24], dtype=np.int32)
    cases.append(dict(grid=g._iptr(bad_grid)))
    sing = np.zeros(9)
    cases.append(dict(lattice=g._dptr(sing)))
    cases.append(dict(natom=0))
    cases.append(dict(nspecies=0))
    bad_soa = np.full(8, 3, dtype=np.int32)
    cases.append(dict(soa=g._iptr(bad_soa)))
    nanpos = w.positions.copy().reshape(-1)
    nanpos[5] = np.nan
    cases.append(dict(pos=g._dptr(nanpos)))
    cases.append(dict(pos=None))
    cases.append(dict(prec=9))
    keep = [bad_grid, sing, bad_soa, nanpos]
    for over in cases:
        a, k = _args(w, **over)
        st, out = _create(lib, a)
        assert st == g.GINT_EINVAL, (over, st, lib.gint_last_error())
        assert out == 12345, "output handle must be untouched on error"
    # NULL out pointer
    a, k = _args(w)
    assert lib.gint_plan_create(a["lattice"], a["grid"], a["nspecies"], a["species"], a["natom"], a["soa"],
                                a["pos"], 0, None, None) == g.GINT_EINVAL


def test_unsupported_basis_rejected(lib):
    import paper_2603_21835_amd as g

    w = gi.si8_sz()
    w.species = [gi.Species([gi.nao_like_radial(3, 0.5, 5.0)])]
    a, k = _args(w)
    st, out = _create(lib, a)
    assert st == g.GINT_EUNSUPPORTED and out == 12345
    w.species = [gi.Species([gi.nao_like_radial(2, 0.5, 5.0)] * 4)]  # 20 orbitals
    a, k = _args(w)
    assert _create(lib, a)[0] == g.GINT_EUNSUPPORTED
    short = gi.Radial(0, 0.1, np.ones(3), 0.0, 0.0)
    w.species = [gi.Species([short])]
    a, k = _args(w)
    assert _create(lib, a)[0] == g.GINT_EINVAL


def test_null_plan_calls(lib):
    import paper_2603_21835_amd as g

    assert lib.gint_build_H(None, None, None) == g.GINT_EINVAL
    assert lib.gint_build_rho(None, None, None) == g.GINT_EINVAL
    assert lib.gint_force(None, None, None, None) == g.GINT_EINVAL
    assert lib.gint_plan_sync(None) == g.GINT_EINVAL
    assert lib.gint_norb(None) == -1
    lib.gint_plan_destroy(None)  # accepted
    assert b"GINT_EINVAL" in lib.gint_status_string(1)


def test_valid_plan_without_gpu_reports_device_error(lib):
    import torch

    import paper_2603_21835_amd as g

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    w = gi.si8_sz()
    a, k = _args(w)
    st, out = _create(lib, a)
    assert st == g.GINT_EDEVICE and out == 12345


def test_batch_invalid_arguments(lib):
    import paper_2603_21835_amd as g

    out = ctypes.c_void_p(777)
    assert lib.gint_batch_create(0, None, 0, None, 0, None, ctypes.byref(out)) == g.GINT_EINVAL
    w = gi.si8_sz()
    a, k = _args(w)
    cell = g._Cell()
    cell.lattice[:] = list(np.asarray(w.lattice, dtype=np.float64).reshape(9))
    cell.grid[:] = [24, 0, 24]
    cell.natom = w.natom
    soa = np.zeros(w.natom, dtype=np.int32)
    pos = np.ascontiguousarray(w.positions).reshape(-1)
    cell.species_of_atom = g._iptr(soa)
    cell.positions = g._dptr(pos)
    cells = (g._Cell * 1)(cell)
    assert lib.gint_batch_create(1, cells, a["nspecies"], a["species"], 0, None, ctypes.byref(out)) == g.GINT_EINVAL
    assert out.value == 777
    assert lib.gint_batch_create(1, cells, a["nspecies"], a["species"], 0, None, None) == g.GINT_EINVAL
    assert lib.gint_batch_build_H(None, None, None) == g.GINT_EINVAL
    assert lib.gint_batch_build_rho(None, None, None) == g.GINT_EINVAL
    assert lib.gint_batch_force(None, None, None, None) == g.GINT_EINVAL
    assert lib.gint_batch_sync(None) == g.GINT_EINVAL
    assert lib.gint_batch_ncell(None) == -1
    assert lib.gint_batch_cell(None, 0) is None
    lib.gint_batch_destroy(None)  # accepted


def test_library_resolves_every_symbol(lib):
    # a launcher declared but defined in another namespace shows up only at
    # the first call; binding every symbol at load time catches it on the CPU
    import paper_2603_21835_amd as g

    ctypes.CDLL(g.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)
