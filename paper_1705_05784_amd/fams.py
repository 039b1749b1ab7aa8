"""Python binding of libfams.so (include/fams.h): argument marshalling only.

Device arrays are torch tensors on the current HIP device; the library runs
on torch's current stream.  Every computation happens inside libfams.so; if
the library is missing this module raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfams.so")

DECOUPLED, FRAC, ROCK, COUPLED = 0, 1, 2, 3
VARIANTS = {"decoupled": DECOUPLED, "frac": FRAC, "rock": ROCK, "coupled": COUPLED}
FP64, MIXED = 0, 1
RESTRICT_FE, RESTRICT_FV, RESTRICT_MIX = 0, 1, 2
RESTRICTIONS = {"fe": RESTRICT_FE, "fv": RESTRICT_FV, "mix": RESTRICT_MIX}
RICHARDSON, GMRES = 0, 1
OK, NOT_CONVERGED, DIVERGED = 0, 1, 2


class FamsError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        msg = f"{where}: {status_string(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class CSR(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_matrix", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("n_wells", C.c_int64)]


class Grid(C.Structure):
    _fields_ = [("n_coarse", C.c_int64), ("wb_type", C.c_void_p), ("primal", C.c_void_p),
                ("vertex", C.c_void_p)]


class SetupOpts(C.Structure):
    _fields_ = [("variant", C.c_int32), ("precision", C.c_int32), ("trunc_alpha", C.c_double),
                ("merge_cap", C.c_int64), ("smoother", C.c_int32), ("profile", C.c_int32),
                ("restriction", C.c_int32), ("nonsymmetric", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class AllocatorHook(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


def _torch_alloc(ctx, nbytes, stream):
    try:
        import torch
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  int(stream or 0))
    except Exception:   # NULL: the library reports FAMS_ERR_OOM
        return None


def _torch_free(ctx, ptr, stream):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:   # interpreter shutdown: the process returns the memory
        pass


# torch's caching allocator behind the library's allocation hook: a handle's
# buffers go back to torch's cache when it is destroyed and the next handle of
# the same shape takes them from there (measured on MI355X: a 140 GB lock-step
# work space allocated anew after an earlier handle had released its memory
# cost ~4 s of host time on its first solve; taken from the cache, nothing)
TORCH_ALLOCATOR = AllocatorHook(None, _ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free))


class SolveOpts(C.Structure):
    _fields_ = [("outer", C.c_int32), ("restart", C.c_int32), ("rtol", C.c_double),
                ("max_iter", C.c_int32), ("use_initial_guess", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("rel_residual", C.c_double),
                ("ms", C.c_double)]


class SetupInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_matrix", C.c_int64), ("nnz", C.c_int64),
                ("n_coarse", C.c_int64), ("nnz_P", C.c_int64), ("n_blocks", C.c_int64),
                ("max_block", C.c_int64), ("fp32_fallback_blocks", C.c_int64),
                ("ilu_levels_lower", C.c_int64), ("ilu_levels_upper", C.c_int64),
                ("ms_setup", C.c_double), ("device_bytes", C.c_int64),
                ("local_flops", C.c_double), ("local_subst_flops", C.c_double),
                ("peak_device_bytes", C.c_int64), ("long_waits", C.c_int64),
                ("tiled_rows", C.c_int64)]


EXPORTS = {
    "fams_status_string": ([C.c_int], C.c_char_p),
    "fams_last_error": ([], C.c_char_p),
    "fams_footprint": ([C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                        C.POINTER(C.c_size_t)], C.c_int),
    "fams_setup": ([C.POINTER(CSR), C.POINTER(Grid), C.POINTER(SetupOpts),
                    C.POINTER(AllocatorHook), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "fams_update_values": ([C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_int32)],
                           C.c_int),
    "fams_solve": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(SolveOpts),
                    C.POINTER(Info)], C.c_int),
    "fams_reconstruct_flux": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(C.c_double)], C.c_int),
    "fams_get_setup_info": ([C.c_void_p, C.POINTER(SetupInfo)], C.c_int),
    "fams_dense_op": ([C.c_int32, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "fams_destroy": ([C.c_void_p], C.c_int),
    "fams_get_prolongation": ([C.c_void_p, C.POINTER(C.c_int64), C.c_void_p, C.c_void_p,
                               C.c_void_p], C.c_int),
    "fams_get_coarse_matrix": ([C.c_void_p, C.c_void_p], C.c_int),
    "fams_get_ilu": ([C.c_void_p, C.c_void_p], C.c_int),
    "fams_apply_stage": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "fams_apply_stage_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "fams_set_profiling": ([C.c_void_p, C.c_int32], C.c_int),
    "fams_get_kernel_stats": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                               C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                               C.POINTER(C.c_int64)], C.c_int),
    "fams_grid_structured": ([C.c_int32] * 6 + [C.c_void_p, C.c_void_p, C.c_void_p,
                                                C.POINTER(C.c_int64)], C.c_int),
    "fams_grid_fracture": ([C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                            C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.POINTER(C.c_int64)], C.c_int),
}

_lib = None


def lib():
    """Load libfams.so (built by paper_1705_05784_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1705_05784_amd.build` (no fallback exists)")
        # torch first: it ships its own HIP runtime under the same soname as
        # the system's, and the library must bind to the runtime that owns
        # the tensors it is handed
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().fams_status_string(int(s)).decode()


def _check(st, where):
    if st < 0:
        raise FamsError(st, where, lib().fams_last_error().decode())
    return st


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def footprint(n, nnz, n_coarse, precision=FP64, restart=30, max_nrhs=1) -> int:
    out = C.c_size_t()
    _check(lib().fams_footprint(n, nnz, n_coarse, precision, restart, max_nrhs, C.byref(out)),
           "footprint")
    return int(out.value)


class Solver:
    """An F-AMS setup resident on the GPU (one fams_handle_t).

    variant: coupling strategy (0 Decoupled, 1 Frac, 2 Rock, 3 Coupled-AMS, or
    its name); precision: FP64 or MIXED; alpha: truncation threshold of P;
    smoother: 0 none, 1 (or True) ILU(0), 2 ILU(0) plus the per-medium stage;
    restriction: RESTRICT_FE (P^T), RESTRICT_FV or RESTRICT_MIX (or "fe",
    "fv", "mix"); n_wells: the last n_wells unknowns are well pressures (each
    a coarse node of its own); nonsymmetric: A may be non-symmetric (LU local
    solves and coarse inverse; no flux reconstruction); allocator: None
    (hipMallocAsync / hipFreeAsync on the handle's stream), "torch" (torch's
    caching allocator, so that handles created one after another reuse the
    same device memory) or an AllocatorHook of the caller's (kept alive with
    the handle).  Arrays may be numpy or torch; the handle copies them.
    """

    def __init__(self, row_ptr, col, val, n_matrix, wb_type, primal, vertex, variant=DECOUPLED,
                 precision=FP64, alpha=0.0, merge_cap=4096, smoother=True, profile=False,
                 restriction=0, n_wells=0, nonsymmetric=False, allocator=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())

        def on(a, dt):
            t = torch.as_tensor(a)
            return t.to(device=dev, dtype=dt).contiguous()
        self._keep = [on(row_ptr, torch.int64), on(col, torch.int32), on(val, torch.float64),
                      on(wb_type, torch.int8), on(primal, torch.int32), on(vertex, torch.int64)]
        rp, ci, va, wb, pr, vx = self._keep
        self.n = int(rp.numel() - 1)
        self.nnz = int(ci.numel())
        self.n_matrix = int(n_matrix)
        self.n_coarse = int(vx.numel())
        self.n_wells = int(n_wells)
        csr = CSR(self.n, self.n_matrix, self.nnz, _ptr(rp), _ptr(ci), _ptr(va), self.n_wells)
        grid = Grid(self.n_coarse, _ptr(wb), _ptr(pr), _ptr(vx))
        if isinstance(variant, str):
            variant = VARIANTS[variant]
        if isinstance(restriction, str):
            restriction = RESTRICTIONS[restriction]
        opts = SetupOpts(int(variant), int(precision), float(alpha), int(merge_cap),
                         int(smoother), 1 if profile else 0, int(restriction),
                         1 if nonsymmetric else 0)
        if isinstance(allocator, AllocatorHook):
            hook = C.byref(allocator)
        elif allocator in (None, "torch"):
            hook = C.byref(TORCH_ALLOCATOR) if allocator == "torch" else None
        else:
            raise ValueError("allocator must be None, 'torch' or an AllocatorHook, "
                             f"not {allocator!r}")
        self._hook = allocator  # the callbacks must outlive the handle
        h = C.c_void_p()
        self._h = None
        _check(lib().fams_setup(C.byref(csr), C.byref(grid), C.byref(opts), hook, _stream(),
                                C.byref(h)), "fams_setup")
        self._h = h
        self._keep = None   # the handle owns copies of everything it needs
        self.device = dev

    def close(self):
        if getattr(self, "_h", None):
            lib().fams_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, q, p=None, outer=GMRES, restart=30, rtol=1e-6, max_iter=1000,
              use_initial_guess=False):
        """q: [n] or [nrhs, n] float64 (row nrhs-major == column-major [n x nrhs])."""
        import torch
        q = torch.as_tensor(q).to(self.device, torch.float64).contiguous()
        nrhs = 1 if q.dim() == 1 else q.shape[0]
        if p is None:
            p = torch.zeros_like(q)
            use_initial_guess = False
        else:  # the library reads and writes p on the device
            p = torch.as_tensor(p).to(self.device, torch.float64).contiguous()
            if p.shape != q.shape:
                raise ValueError("solve: p must have the shape of q")
        if isinstance(outer, str):
            outer = {"richardson": RICHARDSON, "gmres": GMRES}[outer]
        opts = SolveOpts(int(outer), int(restart), float(rtol), int(max_iter),
                         1 if use_initial_guess else 0)
        infos = (Info * nrhs)()
        st = lib().fams_solve(self._h, _ptr(q), _ptr(p), nrhs, C.byref(opts), infos)
        _check(st, "fams_solve")
        return p, [dict(status=i.status, iterations=i.iterations, rel_residual=i.rel_residual,
                        ms=i.ms) for i in infos]

    def update_values(self, val, threshold=0.0):
        """New values of A on the setup's pattern; True when P was recomputed
        (largest relative change above `threshold`; negative: always)."""
        import torch
        v = torch.as_tensor(val).to(self.device, torch.float64).contiguous()
        if v.numel() != self.nnz:
            raise ValueError("update_values: expected nnz values")
        rec = C.c_int32()
        _check(lib().fams_update_values(self._h, _ptr(v), float(threshold), C.byref(rec)),
               "fams_update_values")
        return bool(rec.value)

    def reconstruct_flux(self, q, p):
        import torch
        q = torch.as_tensor(q).to(self.device, torch.float64).contiguous()
        p = torch.as_tensor(p).to(self.device, torch.float64).contiguous()
        flux = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        pfv = torch.empty(self.n, dtype=torch.float64, device=self.device)
        imb = C.c_double()
        _check(lib().fams_reconstruct_flux(self._h, _ptr(q), _ptr(p), _ptr(flux), _ptr(pfv),
                                           C.byref(imb)), "fams_reconstruct_flux")
        return flux, pfv, float(imb.value)

    def apply_stage(self, r):
        import torch
        r = torch.as_tensor(r).to(self.device, torch.float64).contiguous()
        z = torch.empty_like(r)
        _check(lib().fams_apply_stage(self._h, _ptr(r), _ptr(z)), "fams_apply_stage")
        return z

    def setup_info(self) -> dict:
        si = SetupInfo()
        _check(lib().fams_get_setup_info(self._h, C.byref(si)), "fams_get_setup_info")
        return {k: getattr(si, k) for k, _ in SetupInfo._fields_}

    def prolongation(self):
        """(row_ptr, col, val) of P on the host."""
        nnz = C.c_int64()
        _check(lib().fams_get_prolongation(self._h, C.byref(nnz), None, None, None), "P")
        rp = np.empty(self.n + 1, dtype=np.int64)
        ci = np.empty(nnz.value, dtype=np.int32)
        va = np.empty(nnz.value, dtype=np.float64)
        _check(lib().fams_get_prolongation(self._h, C.byref(nnz), rp.ctypes.data, ci.ctypes.data,
                                           va.ctypes.data), "P")
        return rp, ci, va

    def coarse_matrix(self):
        a = np.empty(self.n_coarse * self.n_coarse, dtype=np.float64)
        _check(lib().fams_get_coarse_matrix(self._h, a.ctypes.data), "A_c")
        return a.reshape(self.n_coarse, self.n_coarse).T.copy()   # column-major -> [I, J]

    def ilu(self):
        a = np.empty(self.nnz, dtype=np.float64)
        _check(lib().fams_get_ilu(self._h, a.ctypes.data), "ILU")
        return a

    def profiling(self, on=True):
        _check(lib().fams_set_profiling(self._h, 1 if on else 0), "profiling")

    def kernel_stats(self) -> dict:
        n = C.c_int32()
        _check(lib().fams_get_kernel_stats(self._h, 0, C.byref(n), None, None, None), "stats")
        k = n.value
        names = (C.c_char_p * k)()
        ms = (C.c_double * k)()
        cnt = (C.c_int64 * k)()
        _check(lib().fams_get_kernel_stats(self._h, k, C.byref(n), names, ms, cnt), "stats")
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(k)}


# ---- coarse-grid host helpers -----------------------------------------------

def grid_structured(nx, ny, nz, cx, cy, cz):
    nc = C.c_int64()
    _check(lib().fams_grid_structured(nx, ny, nz, cx, cy, cz, None, None, None, C.byref(nc)),
           "grid")
    n = nx * ny * nz
    wb = np.empty(n, dtype=np.int8)
    pr = np.empty(n, dtype=np.int32)
    vx = np.empty(nc.value, dtype=np.int64)
    _check(lib().fams_grid_structured(nx, ny, nz, cx, cy, cz, wb.ctypes.data, pr.ctypes.data,
                                      vx.ctypes.data, C.byref(nc)), "grid")
    return wb, pr, vx


def grid_fracture(sysm, n_coarse_matrix, d_min, r_z):
    """Fracture classes/primal/vertices for a workloads.FracturedSystem."""
    nf = sysm.n - sysm.n_matrix - getattr(sysm, "n_wells", 0)
    wb = np.empty(nf, dtype=np.int8)
    pr = np.empty(nf, dtype=np.int32)
    vx = np.empty(max(nf, 1), dtype=np.int64)
    ncf = C.c_int64()
    a = lambda x, dt: np.ascontiguousarray(x, dtype=dt)  # noqa: E731
    rp, ci = a(sysm.row_ptr, np.int64), a(sysm.col, np.int32)
    cc, cz = a(sysm.cell_col, np.int32), a(sysm.cell_z, np.int32)
    cp, cptr, cadj = a(sysm.col_plate, np.int32), a(sysm.col_ptr, np.int64), a(sysm.col_adj, np.int32)
    zlo, zhi = a(sysm.plate_zlo, np.int32), a(sysm.plate_zhi, np.int32)
    _check(lib().fams_grid_fracture(sysm.n_matrix, sysm.n_matrix + nf, rp.ctypes.data,
                                    ci.ctypes.data,
                                    cc.ctypes.data, cz.ctypes.data, len(cp), cp.ctypes.data,
                                    cptr.ctypes.data, cadj.ctypes.data, len(zlo), zlo.ctypes.data,
                                    zhi.ctypes.data, int(d_min), int(r_z), int(n_coarse_matrix),
                                    wb.ctypes.data, pr.ctypes.data, vx.ctypes.data,
                                    C.byref(ncf)), "grid_fracture")
    return wb, pr, vx[:ncf.value]


def full_grid(sysm, coarse, d_min, r_z):
    """Matrix + fracture grid of a workloads.FracturedSystem through the
    library's helpers; each well (the last sysm.n_wells unknowns) is a
    coarse node of its own, appended after the fracture nodes."""
    nw = getattr(sysm, "n_wells", 0)
    wbm, pm, vm = grid_structured(sysm.nx, sysm.ny, sysm.nz, *coarse)
    wbf, pf, vf = grid_fracture(sysm, len(vm), d_min, r_z)
    nc0 = len(vm) + len(vf)
    wbw = np.full(nw, 3, dtype=np.int8)
    pw = np.arange(nc0, nc0 + nw, dtype=np.int32)
    vw = np.arange(sysm.n - nw, sysm.n, dtype=np.int64)
    return (np.concatenate([wbm, wbf, wbw]), np.concatenate([pm, pf, pw]),
            np.concatenate([vm, vf, vw]), len(vm))


def setup(sysm, coarse, d_min, r_z, **kw) -> Solver:
    wb, pr, vx, _ = full_grid(sysm, coarse, d_min, r_z)
    return Solver(sysm.row_ptr, sysm.col, sysm.val, sysm.n_matrix, wb, pr, vx,
                  n_wells=getattr(sysm, "n_wells", 0), **kw)


def dense_op(op: int, a):
    """Run one of the coarse system's dense kernels on a (n x n, float64):
    0 a@a, 1 SPD Gauss-Jordan inverse, 2 pivoted LU inverse, 3 LU-solve
    inverse, 4 packed LU factors (getrf layout).  Returns a torch tensor on
    the current device."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    a = torch.as_tensor(a).to(device=dev, dtype=torch.float64)
    n = a.shape[0]
    ac = a.t().contiguous()            # column-major
    out = torch.empty_like(ac)
    torch.cuda.synchronize()
    _check(lib().fams_dense_op(int(op), int(n), _ptr(ac), _ptr(out)), "fams_dense_op")
    return out.t().contiguous()

