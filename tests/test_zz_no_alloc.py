"""fams_apply_stage_noalloc (the allocation-free preconditioner application)
against fams_apply_stage on the same handle: two calls in a row, the second
on a smaller system, in both precision forms.  The two entry points run the
same kernels in the same order, so their results are identical."""
import ctypes as C

import numpy as np
import pytest

from tests._cases import small_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _noalloc():
    from paper_1705_05784_amd import fams
    f = fams.lib().fams_apply_stage_noalloc
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    f.restype = C.c_int
    return f


def _solver(name, precision, smoother):
    from paper_1705_05784_amd import fams
    s, spec = small_case(name)
    wb, pr, vx, _ = fams.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    return s, fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=3,
                          precision=precision, alpha=1e-2, smoother=smoother)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_stage_equals_stage(precision):
    f = _noalloc()
    for name, smoother in (("3d", 2), ("2d", 1)):   # the second system is the smaller one
        print(f"[noalloc] {name} precision={precision} smoother={smoother}", flush=True)
        s, g = _solver(name, precision, smoother)
        r = torch.from_numpy(np.random.default_rng(5).standard_normal(s.n)).cuda()
        z_ref = g.apply_stage(r)
        z = torch.full_like(r, np.nan)
        torch.cuda.synchronize()
        assert f(g._h, r.data_ptr(), z.data_ptr()) == 0
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref)
        g.close()


class _PtrAttr(C.Structure):
    _fields_ = [("type", C.c_int), ("device", C.c_int), ("devicePointer", C.c_void_p),
                ("hostPointer", C.c_void_p), ("isManaged", C.c_int), ("allocationFlags", C.c_uint)]


def _runtime_says_addressable(ptr):
    hip = C.CDLL("libamdhip64.so")
    a = _PtrAttr()
    if hip.hipPointerGetAttributes(C.byref(a), C.c_void_p(ptr)) != 0:
        hip.hipGetLastError()
        return False
    return bool(a.devicePointer) or bool(a.isManaged)


def test_noalloc_refuses_host_memory():
    """Pageable host arrays are refused before any work is issued (the
    library asks the runtime what the pointer is; the test first asks the
    same question itself and runs only when the runtime says "host")."""
    f = _noalloc()
    s, g = _solver("2d", 0, 1)
    r = np.zeros(s.n)
    z = np.zeros(s.n)
    if _runtime_says_addressable(r.ctypes.data) or _runtime_says_addressable(z.ctypes.data):
        pytest.skip("the runtime reports this host memory as device-addressable")
    assert f(g._h, r.ctypes.data, z.ctypes.data) == -1
    g.close()
