"""gint_HR_to_Hk_noalloc (the allocation-free H(k) call, workspace in a fixed
device array) against gint_HR_to_Hk, called through the C ABI: two calls in
a row, the second with fewer k-points and fewer lattice vectors, each within
1e-10 of the allocating call's output (relative to its largest element;
the two form the phases on the device and on the host respectively); sizes
beyond the fixed workspace are rejected on the host."""
import ctypes
import sys

import numpy as np
import pytest

import gint_inputs as gi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cell():
    sp = gi.Species([gi.nao_like_radial(0, 0.4, 5.0), gi.nao_like_radial(1, 0.9, 5.0),
                     gi.nao_like_radial(2, 0.7, 5.0)])
    lat = np.array([[6.0, 0.0, 0.0], [0.7, 6.5, 0.0], [-0.4, 0.3, 7.0]])
    pos = np.array([[0.3, 0.2, 0.1], [3.1, 2.7, 3.9], [5.0, 5.5, 0.2]])
    return gi.small_cell(pos, lat, (15, 17, 18), [sp, gi.sz_species(4.0)], species_of_atom=[0, 1, 0],
                         n_waves=6, nocc=3, seed=7)


def _call(lib, plan, fn, R, HR, kf, out):
    Rl = np.ascontiguousarray(R, dtype=np.int32)
    kfa = np.ascontiguousarray(kf, dtype=np.float64)
    return fn(plan._handle(), len(Rl), Rl.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.c_void_p(HR.data_ptr()),
              len(kfa), kfa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(out.data_ptr()))


def test_hk_noalloc_matches_allocating_call():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_21835_amd as g

    lib = g.load_library()
    dev = torch.device("cuda:0")
    w = _cell()
    plan = g.GintPlan.from_workload(w)
    V = torch.from_numpy(w.V).to(dev)
    R, HR = plan.build_HR(V)
    n = plan.norb
    rng = np.random.default_rng(31)
    cases = [(R, rng.uniform(-1, 1, (11, 3))), (R[: len(R) // 2], rng.uniform(-1, 1, (3, 3)))]
    for i, (Rq, kf) in enumerate(cases):
        HRq = HR[: len(Rq)].contiguous() if len(Rq) < len(R) else HR
        _say(f"case H(k) no-alloc call {i}: nR {len(Rq)} nk {len(kf)}")
        ref = torch.empty((len(kf), n, n), dtype=torch.complex128, device=dev)
        out = torch.full((len(kf), n, n), float("nan"), dtype=torch.complex128, device=dev)
        assert _call(lib, plan, lib.gint_HR_to_Hk, Rq, HRq, kf, ref) == 0
        assert _call(lib, plan, lib.gint_HR_to_Hk_noalloc, Rq, HRq, kf, out) == 0
        plan.sync()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        e = float(np.abs(a - b).max() / np.abs(b).max())
        _say(f"  rel diff {e:.2e}")
        assert np.all(np.isfinite(a)) and e <= 1e-10
    # beyond the fixed workspace: rejected on the host, output untouched
    big_k = np.zeros((9000, 3))
    out = torch.zeros((len(big_k), n, n), dtype=torch.complex128, device=dev)  # room for every k regardless
    assert _call(lib, plan, lib.gint_HR_to_Hk_noalloc, R[:1], HR, big_k, out) == g.GINT_EINVAL
    assert "workspace" in lib.gint_last_error().decode()
    plan.close()
