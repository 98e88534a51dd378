"""ctypes binding of libnfvm.so (the C ABI in include/nfvm.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  If the library is missing, loading raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnfvm.so")

NFVM_OK, NFVM_PENDING = 0, 1
NFVM_E_INVAL, NFVM_E_NOMEM, NFVM_E_DEVICE = -1, -2, -3
NFVM_E_DIVERGED, NFVM_E_NOTCONV, NFVM_E_NOTFOUND = -4, -5, -6
NFVM_FP64, NFVM_FP32, NFVM_MIXED = 0, 1, 2

_dp = C.POINTER(C.c_double)

EXPORTS = (
    "nfvm_set_allocator", "nfvm_init_grid", "nfvm_step", "nfvm_step_batch", "nfvm_mg_solve",
    "nfvm_mg_solve_device", "nfvm_mg_solve_device_noalloc", "nfvm_mg_solve_adjoint_device",
    "nfvm_pressure_adjoint_device", "nfvm_explicit_adjoint_device",
    "nfvm_destroy_adjoint_device", "nfvm_step_adjoint_device", "nfvm_tune",
    "nfvm_get_fields", "nfvm_set_fields", "nfvm_lambda2", "nfvm_line_probe",
    "nfvm_grid_footprint",
    "nfvm_reduction_blocks", "nfvm_free_grid",
    "nfvm_server_create", "nfvm_submit", "nfvm_poll", "nfvm_request_times", "nfvm_server_drain",
    "nfvm_server_destroy", "nfvm_profile", "nfvm_profile_read", "nfvm_set_option", "nfvm_tuning_table",
    "nfvm_last_error",
)

KERNELS = ("smooth0", "smooth0_zero", "restrict0", "prolong0", "explicit", "destroy", "rhs",
           "project", "fcg_apply", "fcg_update", "smooth_coarse", "restrict_coarse",
           "prolong_coarse", "bottom", "fcg_start", "finalize", "smooth0_pair")


class nfvm_patch(C.Structure):
    _fields_ = [("face", C.c_int32), ("lo", C.c_int32 * 2), ("hi", C.c_int32 * 2),
                ("kind", C.c_int32), ("U", C.c_double * 3), ("T", C.c_double),
                ("k", C.c_double), ("omega", C.c_double), ("T_wall", C.c_double)]


class nfvm_grid_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double * 3),
                ("nu", C.c_double), ("rho", C.c_double), ("alpha_T", C.c_double),
                ("Pr_t", C.c_double), ("sigma_k", C.c_double), ("sigma_w", C.c_double),
                ("dt", C.c_double), ("physics", C.c_uint32), ("gravity", C.c_double * 3),
                ("T_ref", C.c_double), ("beta_T", C.c_double), ("T_solid", C.c_double),
                ("n_patches", C.c_int32), ("patches", C.POINTER(nfvm_patch)),
                ("solid_mask", C.POINTER(C.c_uint8)), ("precision", C.c_int32),
                ("n_levels", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("omega_jacobi", C.c_double), ("tol", C.c_double), ("max_cycles", C.c_int32),
                ("nu_coarse", C.c_int32), ("coarse_fp32_cells", C.c_int32)]


class nfvm_fields(C.Structure):
    _fields_ = [(n, _dp) for n in ("u", "v", "w", "p", "T", "k", "omega")]


class nfvm_step_stats(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("status", C.c_int32), ("rel_residual", C.c_double),
                ("max_face_div", C.c_double), ("min_k", C.c_double), ("min_omega", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def lib():
    """Load libnfvm.so; raises OSError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: build it with paper_2603_21869_amd/build.py")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        L.nfvm_set_allocator.argtypes = [ALLOC_FN, FREE_FN, C.c_void_p]
        L.nfvm_init_grid.argtypes = [C.POINTER(nfvm_grid_desc), C.POINTER(nfvm_fields), C.c_void_p,
                                     C.POINTER(C.c_void_p)]
        L.nfvm_step.argtypes = [C.c_void_p, C.c_int32, C.POINTER(nfvm_step_stats)]
        L.nfvm_step_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_int32,
                                      C.POINTER(nfvm_step_stats), C.POINTER(C.c_int32)]
        L.nfvm_mg_solve.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int32, C.c_int32,
                                    C.POINTER(nfvm_step_stats)]
        L.nfvm_mg_solve_device.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                           C.c_int32, C.c_int32, C.POINTER(nfvm_step_stats)]
        L.nfvm_mg_solve_device_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p,
                                                   C.c_double, C.c_int32, C.c_int32,
                                                   C.POINTER(nfvm_step_stats)]
        L.nfvm_mg_solve_adjoint_device.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p,
                                                   C.c_double, C.c_int32, C.c_int32,
                                                   C.POINTER(nfvm_step_stats)]
        L.nfvm_pressure_adjoint_device.argtypes = [C.c_void_p] + [C.c_void_p] * 7 + [
            C.c_double, C.c_int32, C.c_int32, C.POINTER(nfvm_step_stats)]
        L.nfvm_get_fields.argtypes = [C.c_void_p, C.POINTER(nfvm_fields)]
        L.nfvm_lambda2.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.nfvm_explicit_adjoint_device.argtypes = [C.c_void_p, C.POINTER(nfvm_fields),
                                                   C.POINTER(nfvm_fields),
                                                   C.POINTER(nfvm_fields)]
        L.nfvm_destroy_adjoint_device.argtypes = [C.c_void_p, C.POINTER(nfvm_fields), C.c_double,
                                                  C.c_void_p, C.c_void_p,
                                                  C.POINTER(nfvm_fields)]
        L.nfvm_step_adjoint_device.argtypes = [C.c_void_p, C.POINTER(nfvm_fields),
                                               C.POINTER(nfvm_fields),
                                               C.POINTER(nfvm_fields), C.c_double, C.c_int32,
                                               C.c_int32, C.POINTER(nfvm_step_stats)]
        L.nfvm_line_probe.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32,
                                      C.POINTER(C.c_double)]
        L.nfvm_set_fields.argtypes = [C.c_void_p, C.POINTER(nfvm_fields)]
        L.nfvm_grid_footprint.argtypes = [C.POINTER(nfvm_grid_desc), C.POINTER(C.c_size_t)]
        L.nfvm_reduction_blocks.argtypes = [C.POINTER(nfvm_grid_desc), C.POINTER(C.c_int32),
                                            C.POINTER(C.c_int32)]
        L.nfvm_free_grid.argtypes = [C.c_void_p]
        L.nfvm_server_create.argtypes = [C.c_double, C.c_int32, C.POINTER(C.c_void_p)]
        L.nfvm_submit.argtypes = [C.c_void_p, C.POINTER(nfvm_grid_desc), C.POINTER(nfvm_fields),
                                  C.c_int32, C.POINTER(C.c_uint64)]
        L.nfvm_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(nfvm_fields),
                                C.POINTER(nfvm_step_stats)]
        L.nfvm_request_times.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_double)]
        L.nfvm_server_drain.argtypes = [C.c_void_p]
        L.nfvm_server_destroy.argtypes = [C.c_void_p]
        L.nfvm_profile.argtypes = [C.c_void_p, C.c_uint32]
        L.nfvm_profile_read.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.nfvm_set_option.argtypes = [C.c_void_p, C.c_int32, C.c_double]
        L.nfvm_tuning_table.argtypes = [C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]
        L.nfvm_tune.argtypes = [C.POINTER(nfvm_grid_desc)]
        L.nfvm_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name != "nfvm_last_error":
                getattr(L, name).restype = st
        _lib = L
    return _lib


class NfvmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"nfvm status {status}: {msg}")
        self.status = status


def _check(st: int, allow=(NFVM_OK,)):
    if st not in allow:
        raise NfvmError(st, lib().nfvm_last_error().decode())
    return st


_torch_alloc = None  # the installed callbacks (kept alive while installed)


def use_torch_allocator(on: bool = True):
    """Route the library's later device allocations through PyTorch's
    caching allocator on the current device (nfvm_set_allocator), or with
    on=False back to hipMalloc / hipFree.  Grids free their memory only after
    their stream has drained, so a block returned to the cache is idle."""
    global _torch_alloc
    L = lib()
    if not on:
        _check(L.nfvm_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _torch_alloc = None
        return
    import torch

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:  # out of memory: the library reports NFVM_E_NOMEM
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    cb = (ALLOC_FN(_alloc), FREE_FN(_free))
    _check(L.nfvm_set_allocator(cb[0], cb[1], None))
    _torch_alloc = cb


def nfvm_last_error() -> str:
    return lib().nfvm_last_error().decode()


class Desc:
    """Owns a filled nfvm_grid_desc and the arrays it points at."""

    def __init__(self, case, precision: Optional[int] = None, tol: Optional[float] = None,
                 max_cycles: Optional[int] = None):
        d = nfvm_grid_desc()
        d.dim = case.dim
        d.n[:] = list(case.n)
        d.h[:] = list(case.h)
        d.nu, d.rho, d.alpha_T, d.Pr_t = case.nu, case.rho, case.alpha_T, case.Pr_t
        d.sigma_k, d.sigma_w, d.dt = case.sigma_k, case.sigma_w, case.dt
        d.physics = case.physics
        d.gravity[:] = list(case.gravity)
        d.T_ref, d.beta_T, d.T_solid = case.T_ref, case.beta_T, case.T_solid
        pats = (nfvm_patch * max(1, len(case.patches)))()
        for q, p in enumerate(case.patches):
            pats[q].face = p.face
            pats[q].lo[:] = list(p.lo)
            pats[q].hi[:] = list(p.hi)
            pats[q].kind = p.kind
            pats[q].U[:] = list(p.U)
            pats[q].T, pats[q].k, pats[q].omega, pats[q].T_wall = p.T, p.k, p.omega, p.T_wall
        self._pats = pats
        d.n_patches = len(case.patches)
        d.patches = C.cast(pats, C.POINTER(nfvm_patch))
        if case.solid is not None:
            self._mask = np.ascontiguousarray(case.solid, dtype=np.uint8)
            d.solid_mask = self._mask.ctypes.data_as(C.POINTER(C.c_uint8))
        else:
            self._mask = None
            d.solid_mask = C.POINTER(C.c_uint8)()
        d.precision = case.precision if precision is None else precision
        d.n_levels, d.nu1, d.nu2 = case.n_levels, case.nu1, case.nu2
        d.omega_jacobi = case.omega_jacobi
        d.tol = case.tol if tol is None else tol
        d.max_cycles = case.max_cycles if max_cycles is None else max_cycles
        d.nu_coarse = case.nu_coarse
        d.coarse_fp32_cells = case.coarse_fp32_cells
        self.d = d


FIELD_ORDER = ("u", "v", "w", "p", "T", "k", "omega")


def _fields_struct(arrs: Dict[str, np.ndarray]) -> nfvm_fields:
    f = nfvm_fields()
    for n in FIELD_ORDER:
        a = arrs[n]
        assert a.dtype == np.float64 and a.flags.c_contiguous
        setattr(f, n, a.ctypes.data_as(_dp))
    return f


def nfvm_init_grid(desc: Desc, fields: Dict[str, np.ndarray], stream: int = 0) -> C.c_void_p:
    arrs = {n: np.ascontiguousarray(fields[n], dtype=np.float64) for n in FIELD_ORDER}
    h = C.c_void_p()
    _check(lib().nfvm_init_grid(C.byref(desc.d), C.byref(_fields_struct(arrs)),
                                C.c_void_p(stream), C.byref(h)))
    return h


def nfvm_step(grid, n_steps: int, allow=(NFVM_OK,)):
    st = (nfvm_step_stats * max(1, n_steps))()
    s = _check(lib().nfvm_step(grid, n_steps, st), allow)
    return s, [st[i].as_dict() for i in range(n_steps)]


def nfvm_step_batch(grids, n_steps: int, allow=(NFVM_OK,)):
    """n_steps time steps of several grids in batched launches; returns the
    call's status, each grid's status and each grid's per-step stats."""
    n = len(grids)
    hs = (C.c_void_p * n)(*[g.value if isinstance(g, C.c_void_p) else g for g in grids])
    st = (nfvm_step_stats * max(1, n * n_steps))()
    sts = (C.c_int32 * n)()
    s = _check(lib().nfvm_step_batch(hs, n, n_steps, st, sts), allow)
    stats = [[st[i * n_steps + j].as_dict() for j in range(n_steps)] for i in range(n)]
    return s, list(sts), stats


def nfvm_mg_solve(grid, b: np.ndarray, x0: Optional[np.ndarray] = None, tol: float = 1e-10,
                  max_cycles: int = 100, forced_cycles: int = -1, allow=(NFVM_OK,)):
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).copy()
    st = nfvm_step_stats()
    s = _check(lib().nfvm_mg_solve(grid, b.ctypes.data_as(_dp), x.ctypes.data_as(_dp), tol,
                                   max_cycles, forced_cycles, C.byref(st)), allow)
    return x, st.as_dict(), s


def nfvm_mg_solve_device(grid, b_ptr: int, x_ptr: int, tol: float = 1e-10, max_cycles: int = 100,
                         forced_cycles: int = -1, allow=(NFVM_OK,)):
    st = nfvm_step_stats()
    s = _check(lib().nfvm_mg_solve_device(grid, C.c_void_p(b_ptr), C.c_void_p(x_ptr), tol,
                                          max_cycles, forced_cycles, C.byref(st)), allow)
    return st.as_dict(), s


def nfvm_mg_solve_adjoint_device(grid, xbar_ptr: int, bbar_ptr: int, tol: float = 1e-10,
                                 max_cycles: int = 100, forced_cycles: int = -1,
                                 allow=(NFVM_OK,)):
    """bbar = A^-T xbar on device FP64 arrays (bbar: initial guess in, result out)."""
    st = nfvm_step_stats()
    s = _check(lib().nfvm_mg_solve_adjoint_device(grid, C.c_void_p(xbar_ptr),
                                                  C.c_void_p(bbar_ptr), tol, max_cycles,
                                                  forced_cycles, C.byref(st)), allow)
    return st.as_dict(), s


def nfvm_pressure_adjoint_device(grid, bars, outs, tol: float = 1e-10, max_cycles: int = 100,
                                 forced_cycles: int = -1, allow=(NFVM_OK,)):
    """Reverse mode of the pressure step on device FP64 arrays: bars = device
    pointers of (ubar, vbar, wbar, pbar), outs = those of (usbar, vsbar, wsbar)."""
    st = nfvm_step_stats()
    s = _check(lib().nfvm_pressure_adjoint_device(grid, *[C.c_void_p(p) for p in bars],
                                                  *[C.c_void_p(p) for p in outs], tol,
                                                  max_cycles, forced_cycles, C.byref(st)), allow)
    return st.as_dict(), s


def _dev_fields(ptrs) -> nfvm_fields:
    f = nfvm_fields()
    for nm in ("u", "v", "w", "p", "T", "k", "omega"):
        q = ptrs.get(nm)
        setattr(f, nm, C.cast(C.c_void_p(q), C.POINTER(C.c_double)) if q else None)
    return f


def nfvm_explicit_adjoint_device(grid, state, bars, outs):
    """Reverse mode of the explicit stage on device FP64 arrays: state, bars
    and outs map field names (u v w p T k omega) to device pointers."""
    s, b, o = _dev_fields(state), _dev_fields(bars), _dev_fields(outs)
    _check(lib().nfvm_explicit_adjoint_device(grid, C.byref(s), C.byref(b), C.byref(o)))


def nfvm_destroy_adjoint_device(grid, state, tau: float, kbar: int, wbar: int, outs):
    """Reverse mode of the destruction step on device FP64 arrays: state and
    outs map u v w k omega to device pointers; kbar, wbar are pointers."""
    s, o = _dev_fields(state), _dev_fields(outs)
    _check(lib().nfvm_destroy_adjoint_device(grid, C.byref(s), tau, C.c_void_p(kbar),
                                             C.c_void_p(wbar), C.byref(o)))


def nfvm_step_adjoint_device(grid, state, bars, outs, tol: float = 1e-12,
                             max_cycles: int = 200, forced_cycles: int = -1,
                             allow=(NFVM_OK,)):
    """Reverse mode of one whole step on device FP64 arrays (name -> device
    pointer maps of the seven fields).  Returns the two solves' stats."""
    s, b, o = _dev_fields(state), _dev_fields(bars), _dev_fields(outs)
    st = (nfvm_step_stats * 2)()
    r = _check(lib().nfvm_step_adjoint_device(grid, C.byref(s), C.byref(b), C.byref(o), tol,
                                              max_cycles, forced_cycles, st), allow)
    return [st[0].as_dict(), st[1].as_dict()], r


def nfvm_mg_solve_device_noalloc(grid, b_ptr: int, x_ptr: int, tol: float = 1e-10,
                                 max_cycles: int = 100, forced_cycles: int = -1,
                                 allow=(NFVM_OK,)):
    """nfvm_mg_solve_device without device allocation (library-held scratch)."""
    st = nfvm_step_stats()
    s = _check(lib().nfvm_mg_solve_device_noalloc(grid, C.c_void_p(b_ptr), C.c_void_p(x_ptr),
                                                  tol, max_cycles, forced_cycles, C.byref(st)),
               allow)
    return st.as_dict(), s


def nfvm_lambda2(grid, shape) -> np.ndarray:
    """The lambda2 vortex criterion of the grid's current velocity, [nz][ny][nx]."""
    out = np.zeros(shape)
    _check(lib().nfvm_lambda2(grid, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def nfvm_line_probe(grid, pts) -> np.ndarray:
    """{V, T, k, omega} at points (metres, shape (n, 3)) of the grid's fields."""
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
    out = np.empty((len(p), 4))
    _check(lib().nfvm_line_probe(grid, p.ctypes.data_as(C.POINTER(C.c_double)), len(p),
                                 out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def line(p0, p1, n: int) -> np.ndarray:
    """n points evenly spaced from p0 to p1 (both included)."""
    t = np.linspace(0.0, 1.0, n)[:, None]
    return (1.0 - t) * np.asarray(p0, dtype=np.float64) + t * np.asarray(p1, dtype=np.float64)


def nfvm_get_fields(grid, shape) -> Dict[str, np.ndarray]:
    out = {n: np.zeros(shape) for n in FIELD_ORDER}
    _check(lib().nfvm_get_fields(grid, C.byref(_fields_struct(out))))
    return out


def nfvm_set_fields(grid, fields: Dict[str, np.ndarray]):
    arrs = {n: np.ascontiguousarray(fields[n], dtype=np.float64) for n in FIELD_ORDER}
    _check(lib().nfvm_set_fields(grid, C.byref(_fields_struct(arrs))))


def nfvm_grid_footprint(desc: Desc) -> int:
    b = C.c_size_t(0)
    _check(lib().nfvm_grid_footprint(C.byref(desc.d), C.byref(b)))
    return b.value


def nfvm_reduction_blocks(desc: Desc):
    """(needed, capacity): the largest reducing launch in workgroups over
    every tile choice, and the workgroups the partial buffer holds."""
    n = C.c_int32(0)
    c = C.c_int32(0)
    _check(lib().nfvm_reduction_blocks(C.byref(desc.d), C.byref(n), C.byref(c)))
    return n.value, c.value


def nfvm_free_grid(grid):
    _check(lib().nfvm_free_grid(grid))


def nfvm_profile(grid, kernel_mask: int):
    _check(lib().nfvm_profile(grid, kernel_mask))


def nfvm_profile_read(grid, kernel: int):
    n = C.c_int64(0)
    s = C.c_double(0.0)
    b = C.c_double(0.0)
    _check(lib().nfvm_profile_read(grid, kernel, C.byref(n), C.byref(s), C.byref(b)))
    return dict(launches=n.value, seconds=s.value, bytes_per_launch=b.value)


NFVM_OPT_GRAPHS, NFVM_OPT_PREDICT, NFVM_OPT_BOTTOM, NFVM_OPT_AUTOTUNE = 0, 1, 2, 3
NFVM_OPT_WARM_START = 4
NFVM_OPT_PROLONG = 5
NFVM_OPT_RK_ORDER = 6
NFVM_OPT_LITERAL = 7
NFVM_OPT_SWEEP_PAIRS = 8


def nfvm_tune(desc: Desc):
    """Tune the tile shapes of a descriptor's shape and precision (no grid kept)."""
    _check(lib().nfvm_tune(C.byref(desc.d)))


def nfvm_tuning_table():
    buf = (C.c_int32 * (7 * 1024))()
    cnt = C.c_int32(0)
    _check(lib().nfvm_tuning_table(buf, 1024, C.byref(cnt)))
    return [tuple(buf[7 * i: 7 * i + 7]) for i in range(cnt.value)]


def nfvm_set_option(grid, option: int, value: float):
    _check(lib().nfvm_set_option(grid, option, value))


def nfvm_server_create(hbm_budget_bytes: float = 0.0, max_slots: int = 4):
    h = C.c_void_p()
    _check(lib().nfvm_server_create(hbm_budget_bytes, max_slots, C.byref(h)))
    return h


def nfvm_submit(server, desc: Desc, fields: Dict[str, np.ndarray], n_steps: int) -> int:
    arrs = {n: np.ascontiguousarray(fields[n], dtype=np.float64) for n in FIELD_ORDER}
    t = C.c_uint64(0)
    _check(lib().nfvm_submit(server, C.byref(desc.d), C.byref(_fields_struct(arrs)), n_steps,
                             C.byref(t)))
    return t.value


def nfvm_poll(server, ticket: int, shape=None, allow=(NFVM_OK, NFVM_PENDING)):
    """Poll a request; with shape None the fields are not copied back."""
    st = nfvm_step_stats()
    if shape is None:
        s = _check(lib().nfvm_poll(server, ticket, None, C.byref(st)), allow)
        return s, None, st.as_dict()
    out = {n: np.zeros(shape) for n in FIELD_ORDER}
    s = _check(lib().nfvm_poll(server, ticket, C.byref(_fields_struct(out)), C.byref(st)), allow)
    return s, (out if s != NFVM_PENDING else None), st.as_dict()


def nfvm_request_times(server, ticket: int):
    t = (C.c_double * 4)()
    _check(lib().nfvm_request_times(server, ticket, t))
    return list(t)


def nfvm_server_drain(server):
    _check(lib().nfvm_server_drain(server))


def nfvm_server_destroy(server):
    _check(lib().nfvm_server_destroy(server))


class Grid:
    """Convenience owner of one grid handle."""

    def __init__(self, case, precision=None, tol=None, max_cycles=None, stream: int = 0,
                 fields=None):
        self.case = case
        self.desc = Desc(case, precision, tol, max_cycles)
        self.shape = (case.n[2], case.n[1], case.n[0])
        self.h = nfvm_init_grid(self.desc, case.fields if fields is None else fields, stream)
        if getattr(case, "prolong", 0):
            nfvm_set_option(self.h, NFVM_OPT_PROLONG, float(case.prolong))
        if getattr(case, "rk_order", 1) != 1:
            nfvm_set_option(self.h, NFVM_OPT_RK_ORDER, float(case.rk_order))
        if getattr(case, "literal", 0):
            nfvm_set_option(self.h, NFVM_OPT_LITERAL, 1.0)

    def step(self, n: int, allow=(NFVM_OK,)):
        return nfvm_step(self.h, n, allow)

    def fields(self):
        return nfvm_get_fields(self.h, self.shape)

    def lambda2(self):
        return nfvm_lambda2(self.h, self.shape)

    def probe(self, pts):
        return nfvm_line_probe(self.h, pts)

    def set_fields(self, f):
        nfvm_set_fields(self.h, f)

    def mg_solve(self, b, x0=None, **kw):
        return nfvm_mg_solve(self.h, b, x0, **kw)

    def close(self):
        if self.h:
            nfvm_free_grid(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
