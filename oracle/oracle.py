"""ctypes front-end of the serial FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares
no code with the HIP path; it only reads the seeded inputs of
``paper_2603_21869_amd.cases``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "nfvm_oracle.c")

_dp = C.POINTER(C.c_double)


class _Patch(C.Structure):
    _fields_ = [("face", C.c_int), ("lo", C.c_int * 2), ("hi", C.c_int * 2), ("kind", C.c_int),
                ("U", C.c_double * 3), ("T", C.c_double), ("k", C.c_double),
                ("omega", C.c_double), ("T_wall", C.c_double)]


class _Case(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double * 3), ("nu", C.c_double),
                ("alpha_T", C.c_double), ("Pr_t", C.c_double), ("sigma_k", C.c_double),
                ("sigma_w", C.c_double), ("dt", C.c_double), ("physics", C.c_int),
                ("gravity", C.c_double * 3), ("T_ref", C.c_double), ("beta_T", C.c_double),
                ("T_solid", C.c_double), ("n_patches", C.c_int), ("patches", C.POINTER(_Patch)),
                ("solid", C.POINTER(C.c_ubyte)), ("n_levels", C.c_int), ("nu1", C.c_int),
                ("nu2", C.c_int), ("omega_jacobi", C.c_double), ("tol", C.c_double),
                ("max_cycles", C.c_int), ("prolong", C.c_int),
                ("rk_order", C.c_int), ("literal", C.c_int), ("nu_coarse", C.c_int)]


class _Fields(C.Structure):
    _fields_ = [(n, _dp) for n in ("u", "v", "w", "p", "T", "k", "omega")]


class _Stats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("status", C.c_int), ("rel_residual", C.c_double),
                ("max_face_div", C.c_double), ("min_k", C.c_double), ("min_omega", C.c_double)]


FIELDS = ("u", "v", "w", "p", "T", "k", "omega")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.orc_mg_create.restype = C.c_void_p
        L.orc_mg_create.argtypes = [C.POINTER(_Case)]
        for name in ("orc_mg_free",):
            getattr(L, name).argtypes = [C.c_void_p]
        L.orc_mg_levels.argtypes = [C.c_void_p]
        L.orc_mg_apply.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_mg_smooth.argtypes = [C.c_void_p, C.c_int, _dp, _dp, C.c_int]
        L.orc_mg_restrict.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_mg_prolong_add.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_mg_vcycle.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_mg_solve.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, C.c_int,
                                   C.POINTER(C.c_int), _dp]
        L.orc_mg_level_shape.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), _dp]
        L.orc_mg_level_active.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_ubyte)]
        L.orc_closure_point.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
        L.orc_pressure_adjoint.argtypes = [C.POINTER(_Case), _dp, _dp, _dp, _dp, C.c_double,
                                           C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp,
                                           C.POINTER(C.c_int), _dp]
        L.orc_ghost_table.argtypes = [C.POINTER(_Case), C.POINTER(C.c_int), _dp, _dp,
                                      C.POINTER(C.c_ubyte)]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


class OracleCase:
    """Marshals a ``cases.Case`` into the oracle's C struct (keeps arrays alive)."""

    def __init__(self, case):
        self.case = case
        pats = (_Patch * max(1, len(case.patches)))()
        for q, p in enumerate(case.patches):
            pats[q].face = p.face
            pats[q].lo[:] = list(p.lo)
            pats[q].hi[:] = list(p.hi)
            pats[q].kind = p.kind
            pats[q].U[:] = list(p.U)
            pats[q].T = p.T
            pats[q].k = p.k
            pats[q].omega = p.omega
            pats[q].T_wall = p.T_wall
        self._pats = pats
        c = _Case()
        c.dim = case.dim
        c.n[:] = list(case.n)
        c.h[:] = list(case.h)
        c.nu = case.nu
        c.alpha_T = case.alpha_T
        c.Pr_t = case.Pr_t
        c.sigma_k = case.sigma_k
        c.sigma_w = case.sigma_w
        c.dt = case.dt
        c.physics = case.physics
        c.gravity[:] = list(case.gravity)
        c.T_ref = case.T_ref
        c.beta_T = case.beta_T
        c.T_solid = case.T_solid
        c.n_patches = len(case.patches)
        c.patches = C.cast(pats, C.POINTER(_Patch))
        if case.solid is not None:
            self._solid = np.ascontiguousarray(case.solid, dtype=np.uint8)
            c.solid = self._solid.ctypes.data_as(C.POINTER(C.c_ubyte))
        else:
            self._solid = None
            c.solid = C.POINTER(C.c_ubyte)()
        c.n_levels = case.n_levels
        c.nu1 = case.nu1
        c.nu2 = case.nu2
        c.omega_jacobi = case.omega_jacobi
        c.tol = case.tol
        c.max_cycles = case.max_cycles
        c.prolong = case.prolong
        c.rk_order = case.rk_order
        c.literal = getattr(case, "literal", 0)
        c.nu_coarse = getattr(case, "nu_coarse", 0)
        self.c = c

    @property
    def ref(self):
        return C.byref(self.c)

    @property
    def shape(self):
        n = self.case.n
        return (n[2], n[1], n[0])


def _fields_struct(f: Dict[str, np.ndarray]):
    s = _Fields()
    for n in FIELDS:
        setattr(s, n, _ptr(f[n]))
    return s


def _fresh(case) -> Dict[str, np.ndarray]:
    return {n: np.ascontiguousarray(case.fields[n], dtype=np.float64).copy() for n in FIELDS}


def step(case, n_steps: Optional[int] = None, forced_cycles: Optional[Sequence[int]] = None,
         fields: Optional[Dict[str, np.ndarray]] = None, warm: bool = False):
    """Run n_steps time steps from the case's initial fields (or ``fields``).
    Each pressure solve starts from zero; with ``warm`` from the previous
    step's increment instead (zero at the first step).

    Returns (fields, stats list, status)."""
    L = lib()
    oc = OracleCase(case)
    n_steps = case.n_steps if n_steps is None else n_steps
    f = _fresh(case) if fields is None else {k: np.ascontiguousarray(v, dtype=np.float64).copy() for k, v in fields.items()}
    fs = _fields_struct(f)
    st = (_Stats * max(1, n_steps))()
    if forced_cycles is not None:
        fc = (C.c_int * n_steps)(*[int(x) for x in forced_cycles])
        fcp = C.cast(fc, C.POINTER(C.c_int))
    else:
        fcp = C.POINTER(C.c_int)()
    status = L.orc_step(oc.ref, C.byref(fs), n_steps, fcp, st, 1 if warm else 0)
    stats = [dict(cycles=st[i].cycles, status=st[i].status, rel_residual=st[i].rel_residual,
                  max_face_div=st[i].max_face_div, min_k=st[i].min_k, min_omega=st[i].min_omega)
             for i in range(n_steps)]
    return f, stats, status


def closure_point(nu: float, k: float, omega: float):
    out = (C.c_double * 4)()
    lib().orc_closure_point(nu, k, omega, out)
    return dict(alpha_star=out[0], nu_t=out[1], alpha=out[2], beta_star=out[3])


def fixed_omega(case, omega: np.ndarray) -> np.ndarray:
    oc = OracleCase(case)
    o = np.ascontiguousarray(omega, dtype=np.float64).copy()
    lib().orc_fixed_omega(oc.ref, _ptr(o))
    return o


def nut(case, k, omega):
    oc = OracleCase(case)
    out = np.zeros(oc.shape)
    lib().orc_nut(oc.ref, _ptr(np.ascontiguousarray(k, dtype=np.float64)),
                  _ptr(np.ascontiguousarray(omega, dtype=np.float64)), _ptr(out))
    return out


def explicit_rhs(case, fields: Dict[str, np.ndarray]):
    oc = OracleCase(case)
    fin = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in fields.items()}
    out = {k: np.zeros(oc.shape) for k in FIELDS}
    lib().orc_explicit_rhs(oc.ref, C.byref(_fields_struct(fin)), C.byref(_fields_struct(out)))
    return out


def explicit(case, fields: Dict[str, np.ndarray]):
    oc = OracleCase(case)
    fin = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in fields.items()}
    out = {k: np.zeros(oc.shape) for k in FIELDS}
    lib().orc_explicit(oc.ref, C.byref(_fields_struct(fin)), C.byref(_fields_struct(out)))
    return out


def destroy(case, u, v, w, k, omega, tau):
    oc = OracleCase(case)
    ko = np.zeros(oc.shape)
    oo = np.zeros(oc.shape)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (u, v, w, k, omega)]
    lib().orc_destroy(oc.ref, *[_ptr(x) for x in a], C.c_double(tau), _ptr(ko), _ptr(oo))
    return ko, oo


def velocity_gradient(case, u, v, w):
    """G[..., a, b] = d u_a / d x_b per cell (central, with boundary ghosts);
    zero on non-fluid cells."""
    oc = OracleCase(case)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (u, v, w)]
    G = np.zeros(oc.shape + (3, 3))
    lib().orc_velocity_gradient(oc.ref, *[_ptr(x) for x in a], _ptr(G))
    return G


def lambda2(case, u, v, w):
    """Vortex criterion of Sec. 3.2 (Jeong and Hussain): the middle
    eigenvalue of S^2 + W^2, S and W the symmetric and antisymmetric parts of
    the velocity gradient (the oracle's central gradient with boundary
    ghosts); zero on non-fluid cells.  The eigenvalues come from numpy's
    symmetric eigensolver."""
    G = velocity_gradient(case, u, v, w)
    S = 0.5 * (G + np.swapaxes(G, -1, -2))
    W = 0.5 * (G - np.swapaxes(G, -1, -2))
    M = S @ S + W @ W
    return np.linalg.eigvalsh(M)[..., 1]


def line_probe(case, fields: Dict[str, np.ndarray], pts) -> np.ndarray:
    """Line probes of Sec. 3.1: the velocity magnitude V, the temperature T,
    k and omega at points (metres, shape (n, 3): x, y, z), as compared with
    the reference solutions along lines there.  The paper does not say how
    values between cell centres are formed; this reading interpolates each
    field trilinearly between the cell centres (centre of cell i at
    (i + 1/2) h), over the fluid cells among the eight around the point with
    their weights renormalised to sum to one (NaN where none is fluid), with
    the point clamped into the box of cell centres; V is the magnitude of the
    interpolated velocity.  fields are dense [nz][ny][nx] arrays with T
    absolute.  Returns (n, 4) columns V, T, k, omega.  Plain loops."""
    n = tuple(case.n)
    dim = case.dim
    h = tuple(case.h)
    fluid = np.ones(n[::-1], dtype=bool) if case.solid is None else case.solid == 0
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.full((len(pts), 4), np.nan)
    names = ("u", "v", "w", "T", "k", "omega")
    for q, x in enumerate(pts):
        lo, t = [0, 0, 0], [0.0, 0.0, 0.0]
        for d in range(dim):
            f = min(max(x[d] / h[d] - 0.5, 0.0), n[d] - 1.0)
            i = min(int(math.floor(f)), max(n[d] - 2, 0))
            lo[d], t[d] = i, f - i
        acc = np.zeros(6)
        wsum = 0.0
        for c in range(8 if dim == 3 else 4):
            idx, wt = [], 1.0
            for d in range(3):
                bit = (c >> d) & 1
                if d >= dim:
                    idx.append(0)
                    continue
                idx.append(min(lo[d] + bit, n[d] - 1))
                wt *= t[d] if bit else 1.0 - t[d]
            i, j, k = idx
            if not fluid[k, j, i]:
                continue
            wsum += wt
            for a, nm in enumerate(names):
                acc[a] += wt * fields[nm][k, j, i]
        if wsum > 0.0:
            val = acc / wsum
            out[q] = (math.sqrt(val[0] ** 2 + val[1] ** 2 + val[2] ** 2), val[3], val[4], val[5])
    return out


def ghost_tables(case):
    """The oracle's boundary classification as arrays over the flattened
    cells: neighbour index per face direction (-1: ghost), the affine ghost
    rule a0 + a1 value_P per direction and field (u, v, w, p, T, k, omega,
    nu_t), and the fixed-omega flag."""
    oc = OracleCase(case)
    n = int(np.prod(oc.shape))
    nidx = np.zeros((n, 6), dtype=np.int32)
    a0 = np.zeros((n, 6, 8))
    a1 = np.zeros((n, 6, 8))
    fixed = np.zeros(n, dtype=np.uint8)
    lib().orc_ghost_table(oc.ref, nidx.ctypes.data_as(C.POINTER(C.c_int)), _ptr(a0), _ptr(a1),
                          fixed.ctypes.data_as(C.POINTER(C.c_ubyte)))
    return nidx, a0, a1, fixed.astype(bool)


def rhs_b(case, us, vs, ws):
    oc = OracleCase(case)
    b = np.zeros(oc.shape)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (us, vs, ws)]
    lib().orc_rhs_b(oc.ref, *[_ptr(x) for x in a], _ptr(b))
    return b


def pressure_adjoint(case, ubar, vbar, wbar, pbar, tol: float = 1e-12, max_cycles: int = 200,
                     forced: int = -1):
    """Reverse mode of the pressure step (rhs_b, the solve, project): the
    adjoints of u*, v*, w* for the adjoints (ubar, vbar, wbar, pbar) of the
    step's velocity and pressure (the adjoint of p^n is pbar).  Returns
    (usbar, vsbar, wsbar, phibar, lambda, cycles, rel_residual, status):
    phibar is the right-hand side of the second solve, lambda its solution."""
    oc = OracleCase(case)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (ubar, vbar, wbar, pbar)]
    out = [np.zeros(oc.shape) for _ in range(5)]
    cyc = C.c_int(0)
    rel = C.c_double(0.0)
    st = lib().orc_pressure_adjoint(oc.ref, *[_ptr(x) for x in a], tol, max_cycles, forced,
                                    *[_ptr(x) for x in out], C.byref(cyc), C.byref(rel))
    return out[0], out[1], out[2], out[3], out[4], cyc.value, rel.value, st


def project(case, phi, us, vs, ws, p):
    oc = OracleCase(case)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (phi, us, vs, ws)]
    pp = np.ascontiguousarray(p, dtype=np.float64).copy()
    u = np.zeros(oc.shape)
    v = np.zeros(oc.shape)
    w = np.zeros(oc.shape)
    md = C.c_double(0.0)
    lib().orc_project(oc.ref, *[_ptr(x) for x in a], _ptr(pp), _ptr(u), _ptr(v), _ptr(w),
                      C.byref(md))
    return pp, u, v, w, md.value


class MG:
    """The oracle's multigrid hierarchy for the pressure operator of a case."""

    def __init__(self, case):
        self.oc = OracleCase(case)
        self.h = lib().orc_mg_create(self.oc.ref)
        if not self.h:
            raise ValueError("oracle multigrid: invalid level count for this grid")
        self.L = lib().orc_mg_levels(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_mg_free(self.h)
            self.h = None

    def shape(self, l: int):
        n = (C.c_int * 3)()
        h = (C.c_double * 3)()
        lib().orc_mg_level_shape(self.h, l, n, h)
        return (n[2], n[1], n[0]), (h[0], h[1], h[2])

    def active(self, l: int) -> np.ndarray:
        sh, _ = self.shape(l)
        a = np.zeros(sh, dtype=np.uint8)
        lib().orc_mg_level_active(self.h, l, a.ctypes.data_as(C.POINTER(C.c_ubyte)))
        return a

    def apply(self, l: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        lib().orc_mg_apply(self.h, l, _ptr(x), _ptr(y))
        return y

    def smooth(self, l: int, x: np.ndarray, b: np.ndarray, sweeps: int) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64).copy()
        lib().orc_mg_smooth(self.h, l, _ptr(x), _ptr(np.ascontiguousarray(b, dtype=np.float64)), sweeps)
        return x

    def restrict(self, l: int, r: np.ndarray) -> np.ndarray:
        sh, _ = self.shape(l + 1)
        bc = np.zeros(sh)
        lib().orc_mg_restrict(self.h, l, _ptr(np.ascontiguousarray(r, dtype=np.float64)), _ptr(bc))
        return bc

    def prolong_add(self, l: int, e: np.ndarray, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64).copy()
        lib().orc_mg_prolong_add(self.h, l, _ptr(np.ascontiguousarray(e, dtype=np.float64)), _ptr(x))
        return x

    def vcycle(self, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64).copy()
        lib().orc_mg_vcycle(self.h, _ptr(x), _ptr(np.ascontiguousarray(b, dtype=np.float64)))
        return x

    def solve(self, b: np.ndarray, x: Optional[np.ndarray] = None, tol: float = 1e-10,
              max_cycles: int = 100, forced: int = -1):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x is None else np.ascontiguousarray(x, dtype=np.float64).copy()
        cyc = C.c_int(0)
        rel = C.c_double(0.0)
        st = lib().orc_mg_solve(self.h, _ptr(b), _ptr(x), tol, max_cycles, forced, C.byref(cyc),
                                C.byref(rel))
        return x, cyc.value, rel.value, st
