"""Seeded synthetic workloads for the NeuralFVM time step.

This module only builds inputs: grid shapes and spacings, boundary patches,
solid masks, fluid properties and initial fields.  It holds none of the
method's arithmetic, so both the HIP library binding and the CPU oracle may
read what it produces.

Geometry follows the paper's test cases: the open channel of the verification
section (Sec. 3.1: 2.56 m x 0.64 m x 0.64 m, inlet 0.1 m/s, nu = 1.46e-5), a
2D channel, and a room with heated blocks standing in for the indoor-airflow
study (Sec. 3.2).  No measured data is used; every array is generated here.

Random numbers: splitmix64 (Steele, Lea, Flood 2014) seeded with
``seed ^ stream``; a uniform double is ``(x >> 11) * 2**-53``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

# face ids: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+
WALL, INLET, OUTLET = 0, 1, 2
KIND_NAMES = {WALL: "wall", INLET: "inlet", OUTLET: "outlet"}

PREC_FP64, PREC_FP32, PREC_MIXED = 0, 1, 2
PROL_LINEAR, PROL_NEAREST = 0, 1

PHYS_KOMEGA, PHYS_ENERGY, PHYS_BUOYANCY = 1, 2, 4

FIELDS = ("u", "v", "w", "p", "T", "k", "omega")

_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """n consecutive splitmix64 outputs for state ``seed ^ stream`` (uint64)."""
    state = np.uint64((seed ^ stream) & _MASK64)
    gamma = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        z = state + gamma * np.arange(1, n + 1, dtype=np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """n doubles in [0, 1) from splitmix64."""
    return (splitmix64(seed, n, stream) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


@dataclasses.dataclass
class Patch:
    """A rectangle of boundary faces on one side of the box.

    ``lo``/``hi`` are half-open cell ranges along the two tangential axes of
    the face (x faces: (j, k); y faces: (i, k); z faces: (i, j)).
    """
    face: int
    lo: Tuple[int, int]
    hi: Tuple[int, int]
    kind: int
    U: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    T: float = math.nan
    k: float = 0.0
    omega: float = 0.0
    T_wall: float = math.nan  # NaN: adiabatic wall


@dataclasses.dataclass
class Case:
    name: str
    dim: int
    n: Tuple[int, int, int]
    h: Tuple[float, float, float]
    nu: float
    rho: float
    alpha_T: float
    dt: float
    physics: int
    patches: List[Patch]
    fields: Dict[str, np.ndarray]
    solid: Optional[np.ndarray] = None  # uint8 [nz][ny][nx], 1 = solid
    Pr_t: float = 0.85
    sigma_k: float = 2.0
    sigma_w: float = 2.0
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.81)
    T_ref: float = 293.0
    beta_T: float = 1.0 / 293.0
    T_solid: float = math.nan
    precision: int = PREC_FP64
    n_levels: int = 1
    nu1: int = 2
    nu2: int = 2
    # pre and post sweeps on the levels below the finest (0: nu1, nu2)
    nu_coarse: int = 0
    # mixed precision: coarse levels with at least this many cells in FP32,
    # the others in BF16 (0: the library's default; 2**31 - 1: all BF16)
    coarse_fp32_cells: int = 0
    omega_jacobi: float = 0.0  # 0: method default for the dimension
    tol: float = 1e-6
    max_cycles: int = 100
    # multigrid prolongation: PROL_LINEAR (eq. prolongation) or PROL_NEAREST
    # (piecewise constant, the plainest reading of Algorithm 1's upsampling)
    prolong: int = 0
    # explicit stage: 1 forward Euler, 2 Heun's method (SSP form); the paper
    # names explicit Runge-Kutta schemes without fixing one (Sec. 2.6)
    rk_order: int = 1
    # 1: the pressure solve as Algorithm 1 prints it (undamped Jacobi with the
    # scalar diagonal, V(0,1) with nearest upsampling and one coarsest sweep,
    # a plain iteration without a Krylov wrapper)
    literal: int = 0
    n_steps: int = 1
    seed: int = 0

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def copy(self, **changes) -> "Case":
        c = dataclasses.replace(self, **changes)
        c.fields = {k: v.copy() for k, v in self.fields.items()}
        if self.solid is not None:
            c.solid = self.solid.copy()
        c.patches = [dataclasses.replace(p) for p in self.patches]
        return c


def inlet_turbulence(U: float, H: float) -> Tuple[float, float]:
    """Inlet k and omega of the channel workloads: k = 1.5 (0.05 U)^2,
    omega = sqrt(k) / (0.09**0.25 * 0.07 H)."""
    k = 1.5 * (0.05 * U) ** 2
    om = math.sqrt(k) / (0.09 ** 0.25 * 0.07 * H)
    return k, om


def max_levels(n: Tuple[int, int, int], dim: int) -> int:
    """Number of levels obtained by halving while every active edge is even."""
    lv = 1
    m = list(n[:dim])
    while all(e % 2 == 0 for e in m):
        m = [e // 2 for e in m]
        lv += 1
    return lv


def _face_full(n, face):
    nx, ny, nz = n
    t = {0: (ny, nz), 1: (ny, nz), 2: (nx, nz), 3: (nx, nz), 4: (nx, ny), 5: (nx, ny)}[face]
    return (0, 0), t


def _noisy_u(n, U, seed, fluid):
    nz_, ny_, nx_ = n[2], n[1], n[0]
    r = uniform01(seed, nx_ * ny_ * nz_, stream=0x75).reshape(nz_, ny_, nx_)
    u = U * (1.0 + 0.01 * (2.0 * r - 1.0))
    return np.where(fluid, u, 0.0)


def _base_fields(n, fluid, T0, k0, om0):
    shape = (n[2], n[1], n[0])
    f = {name: np.zeros(shape) for name in FIELDS}
    f["T"][...] = np.where(fluid, T0, 0.0)
    f["k"][...] = np.where(fluid, k0, 0.0)
    f["omega"][...] = np.where(fluid, om0, 0.0)
    return f


def channel2d(nx: int = 256, ny: int = 64, L: float = 4.0, H: float = 1.0, U: float = 1.0,
              nu: float = 1.5e-5, rho: float = 1.2, dt: float = 1e-3, seed: int = 0,
              n_levels: Optional[int] = None, n_steps: int = 100,
              precision: int = PREC_FP64, tol: float = 1e-6, physics: int = PHYS_KOMEGA) -> Case:
    """2D turbulent channel: plug inlet at x-, zero-gradient outlet at x+, no-slip y walls."""
    n = (nx, ny, 1)
    h = (L / nx, H / ny, 1.0)
    k_in, om_in = inlet_turbulence(U, H)
    patches = [
        Patch(0, *_face_full(n, 0), kind=INLET, U=(U, 0.0, 0.0), T=293.0, k=k_in, omega=om_in),
        Patch(1, *_face_full(n, 1), kind=OUTLET),
    ]
    fluid = np.ones((1, ny, nx), dtype=bool)
    f = _base_fields(n, fluid, 293.0, k_in, om_in)
    f["u"][...] = _noisy_u(n, U, seed, fluid)
    if n_levels is None:
        n_levels = min(6, max_levels(n, 2))
    return Case(name=f"channel2d_{nx}x{ny}", dim=2, n=n, h=h, nu=nu, rho=rho, alpha_T=nu / 0.71,
                dt=dt, physics=physics, patches=patches, fields=f, precision=precision,
                n_levels=n_levels, tol=tol, n_steps=n_steps, seed=seed)


def channel3d(nx: int = 256, ny: int = 64, nz: int = 64, Lx: float = 2.56, Ly: float = 0.64,
              Lz: float = 0.64, U: float = 0.1, nu: float = 1.46e-5, rho: float = 1.2,
              dt: float = 2e-3, T_in: float = 293.0, T_bottom: float = 310.0, seed: int = 0,
              n_levels: Optional[int] = None, n_steps: int = 500, precision: int = PREC_FP64,
              tol: float = 1e-8, buoyancy: bool = True) -> Case:
    """3D heated channel (the paper's open channel at 1 cm): plug inlet x-, outlet x+,
    no-slip walls, bottom wall (z-) held at T_bottom, other walls adiabatic."""
    n = (nx, ny, nz)
    h = (Lx / nx, Ly / ny, Lz / nz)
    k_in, om_in = inlet_turbulence(U, Lz)
    patches = [
        Patch(0, *_face_full(n, 0), kind=INLET, U=(U, 0.0, 0.0), T=T_in, k=k_in, omega=om_in),
        Patch(1, *_face_full(n, 1), kind=OUTLET),
        Patch(4, *_face_full(n, 4), kind=WALL, T_wall=T_bottom),
    ]
    fluid = np.ones((nz, ny, nx), dtype=bool)
    f = _base_fields(n, fluid, T_in, k_in, om_in)
    f["u"][...] = _noisy_u(n, U, seed, fluid)
    phys = PHYS_KOMEGA | PHYS_ENERGY | (PHYS_BUOYANCY if buoyancy else 0)
    if n_levels is None:
        n_levels = min(7, max_levels(n, 3))
    return Case(name=f"channel3d_{nx}x{ny}x{nz}", dim=3, n=n, h=h, nu=nu, rho=rho,
                alpha_T=nu / 0.71, dt=dt, physics=phys, patches=patches, fields=f,
                gravity=(0.0, 0.0, -9.81), T_ref=T_in, beta_T=1.0 / T_in,
                precision=precision, n_levels=n_levels, tol=tol, n_steps=n_steps, seed=seed)


OPEN_CHANNEL_LENGTHS = {128: 0.64, 512: 2.56, 2048: 10.24}


def open_channel(nx: int = 512, ny: int = 128, nz: int = 128, h: float = 5e-3, U: float = 0.1,
                 nu: float = 1.46e-5, rho: float = 1.2, dt: float = 2e-3, T_in: float = 298.15,
                 T_wall: float = 308.15, seed: int = 0, n_levels: Optional[int] = None,
                 n_steps: int = 100, precision: int = PREC_MIXED, tol: float = 1e-6,
                 buoyancy: bool = True) -> Case:
    """The paper's open-channel verification flow on its uniform 5 mm mesh
    (Sec. 3.1: 0.64 x 0.64 m cross-section, U_in = 0.1 m/s, nu = 1.46e-5,
    inlet at 25 C, every wall held at 35 C), with the streamwise length set by
    nx as in the time profiling of Sec. 3.3 (Table 1: nx = 128, 512, 2048 for
    L = 0.64, 2.56, 10.24 m; 100 steps).  Plug inlet x-, zero-gradient outlet
    x+, no-slip walls on the four other faces."""
    n = (nx, ny, nz)
    hh = (h, h, h)
    k_in, om_in = inlet_turbulence(U, nz * h)
    patches = [
        Patch(0, *_face_full(n, 0), kind=INLET, U=(U, 0.0, 0.0), T=T_in, k=k_in, omega=om_in),
        Patch(1, *_face_full(n, 1), kind=OUTLET),
    ] + [Patch(f, *_face_full(n, f), kind=WALL, T_wall=T_wall) for f in (2, 3, 4, 5)]
    fluid = np.ones((nz, ny, nx), dtype=bool)
    f = _base_fields(n, fluid, T_in, k_in, om_in)
    f["u"][...] = _noisy_u(n, U, seed, fluid)
    phys = PHYS_KOMEGA | PHYS_ENERGY | (PHYS_BUOYANCY if buoyancy else 0)
    if n_levels is None:
        n_levels = min(8, max_levels(n, 3))
    return Case(name=f"open_channel_{nx}x{ny}x{nz}", dim=3, n=n, h=hh, nu=nu, rho=rho,
                alpha_T=nu / 0.71, dt=dt, physics=phys, patches=patches, fields=f,
                gravity=(0.0, 0.0, -9.81), T_ref=T_in, beta_T=1.0 / T_in,
                precision=precision, n_levels=n_levels, tol=tol, n_steps=n_steps, seed=seed)


def _reachable_from(fluid: np.ndarray, seeds: List[Tuple[int, int, int]]) -> np.ndarray:
    """Fluid cells face-connected to any seed cell (z, y, x indexing)."""
    from scipy import ndimage
    lab, _ = ndimage.label(fluid, structure=ndimage.generate_binary_structure(fluid.ndim, 1))
    keep = {int(lab[s]) for s in seeds if fluid[s]}
    keep.discard(0)
    if not keep:
        return np.zeros_like(fluid, dtype=bool)
    return np.isin(lab, np.fromiter(keep, dtype=lab.dtype))


def room_boxes(seed: int, size=(10.0, 4.0, 3.0), vents=None, n_range=(8, 24),
               side_range=(0.2, 1.5), clearance=0.5, max_tries=10000):
    """Axis-aligned boxes in metres: list of (x0, x1, y0, y1, z0, z1)."""
    if vents is None:
        vents = []
    r = uniform01(seed, 8 * max_tries + 1, stream=0xB0)
    it = iter(r)
    nb = n_range[0] + int(next(it) * (n_range[1] - n_range[0] + 1))
    boxes = []
    tries = 0
    while len(boxes) < nb and tries < max_tries:
        tries += 1
        s = [side_range[0] + next(it) * (side_range[1] - side_range[0]) for _ in range(3)]
        o = [next(it) * (size[a] - s[a]) for a in range(3)]
        box = (o[0], o[0] + s[0], o[1], o[1] + s[1], o[2], o[2] + s[2])
        ok = True
        for v in vents:
            # distance between two axis-aligned boxes
            d2 = 0.0
            for a in range(3):
                lo, hi = box[2 * a], box[2 * a + 1]
                vlo, vhi = v[2 * a], v[2 * a + 1]
                gap = max(vlo - hi, lo - vhi, 0.0)
                d2 += gap * gap
            if math.sqrt(d2) < clearance:
                ok = False
                break
        if ok:
            boxes.append(box)
    return boxes


def room3d(nx: int = 512, ny: int = 256, nz: int = 128, size=(10.0, 4.0, 3.0), seed: int = 0,
           n_levels: Optional[int] = None, n_steps: int = 200, precision: int = PREC_MIXED,
           tol: float = 1e-6, dt: float = 5e-4, nu: float = 1.5e-5, rho: float = 1.2,
           vent: float = 0.5, U_supply: float = 0.455, T_supply: float = 291.0,
           T_box: float = 308.15, T0: float = 293.0, boxes=None, buoyancy: bool = False,
           side_range=(0.2, 1.5), clearance: float = 0.5) -> Case:
    """Ventilated room: supply vent on x- under the ceiling, exhaust on x+ at the floor,
    seeded solid boxes held at T_box, adiabatic no-slip walls, z vertical.

    The supply speed defaults to 0.455 m/s (the inlet speed of the paper's
    indoor-airflow case) and dt to 5e-4 s, inside the explicit diffusion limit
    of the method on 1.6 cm cells; a 2 m/s supply drives the wall cells (omega
    held at 6 nu / (beta_i d^2)) into exponential k growth within ~6 ms."""
    n = (nx, ny, nz)
    h = (size[0] / nx, size[1] / ny, size[2] / nz)
    yc = 0.5 * size[1]
    sup = (0.0, 0.0, yc - vent / 2, yc + vent / 2, size[2] - vent, size[2])
    exh = (size[0], size[0], yc - vent / 2, yc + vent / 2, 0.0, vent)
    if boxes is None:
        boxes = room_boxes(seed, size=size, vents=[sup, exh], side_range=side_range,
                           clearance=clearance)

    def cells(lo, hi, hh, nn):
        a = int(round(lo / hh))
        b = int(round(hi / hh))
        a = max(0, min(nn, a))
        b = max(a + 1, min(nn, b))
        return a, b

    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    for bx in boxes:
        i0, i1 = cells(bx[0], bx[1], h[0], nx)
        j0, j1 = cells(bx[2], bx[3], h[1], ny)
        k0, k1 = cells(bx[4], bx[5], h[2], nz)
        solid[k0:k1, j0:j1, i0:i1] = 1
    sj0, sj1 = cells(sup[2], sup[3], h[1], ny)
    sk0, sk1 = cells(sup[4], sup[5], h[2], nz)
    ej0, ej1 = cells(exh[2], exh[3], h[1], ny)
    ek0, ek1 = cells(exh[4], exh[5], h[2], nz)
    # fluid pockets that cannot reach the exhaust become solid
    fluid = solid == 0
    seeds = [(k, j, nx - 1) for k in range(ek0, ek1) for j in range(ej0, ej1)]
    reach = _reachable_from(fluid, seeds)
    solid[~reach] = 1
    fluid = solid == 0

    k_in, om_in = inlet_turbulence(U_supply, vent)
    patches = [
        Patch(0, (sj0, sk0), (sj1, sk1), kind=INLET, U=(U_supply, 0.0, 0.0), T=T_supply,
              k=k_in, omega=om_in),
        Patch(1, (ej0, ek0), (ej1, ek1), kind=OUTLET),
    ]
    f = _base_fields(n, fluid, T0, k_in, om_in)
    phys = PHYS_KOMEGA | PHYS_ENERGY | (PHYS_BUOYANCY if buoyancy else 0)
    if n_levels is None:
        n_levels = min(8, max_levels(n, 3))
    return Case(name=f"room_{nx}x{ny}x{nz}", dim=3, n=n, h=h, nu=nu, rho=rho, alpha_T=nu / 0.71,
                dt=dt, physics=phys, patches=patches, fields=f, solid=solid, T_solid=T_box,
                gravity=(0.0, 0.0, -9.81), T_ref=T0, beta_T=1.0 / T0, precision=precision,
                n_levels=n_levels, tol=tol, n_steps=n_steps, seed=seed)


def serve_trace(seed: int = 0, n_requests: int = 256, rate: float = 20.0,
                edges=(64, 96, 128, 192, 256), n_steps: int = 50):
    """Arrival trace of the serving workload: list of dicts with arrival time (s),
    grid edges, geometry template and per-request seed."""
    r = uniform01(seed, 6 * n_requests, stream=0x5E)
    out = []
    t = 0.0
    for q in range(n_requests):
        u = r[6 * q: 6 * q + 6]
        t += -math.log(1.0 - u[0]) / rate
        n = tuple(edges[min(len(edges) - 1, int(u[1 + a] * len(edges)))] for a in range(3))
        geom = "channel" if u[4] < 0.5 else "room"
        out.append(dict(arrival=t, n=n, geometry=geom, seed=int(u[5] * 2 ** 31), n_steps=n_steps))
    return out


def serve_case(req: dict, precision: int = PREC_MIXED, tol: float = 1e-6) -> Case:
    """Build the case for one request of the serving trace."""
    nx, ny, nz = req["n"]
    lv = max_levels((nx, ny, nz), 3)
    if req["geometry"] == "channel":
        hh = 0.01
        return channel3d(nx, ny, nz, Lx=nx * hh, Ly=ny * hh, Lz=nz * hh, seed=req["seed"],
                         n_levels=lv, n_steps=req["n_steps"], precision=precision, tol=tol)
    hh = 0.02
    size = (nx * hh, ny * hh, nz * hh)
    scale = min(1.0, min(size) / 3.0)  # boxes and vents shrink with the room
    return room3d(nx, ny, nz, size=size, seed=req["seed"], n_levels=lv,
                  n_steps=req["n_steps"], precision=precision, tol=tol, vent=0.5 * scale,
                  side_range=(0.2 * scale, 1.5 * scale), clearance=0.5 * scale)


def decaying_box(n=(8, 8, 8), h=0.1, k0=1e-3, om0=5.0, nu=1e-10, dt=1e-2, dim=3) -> Case:
    """Quiescent fluid with uniform k, omega and outlets on every face: only the
    destruction terms act (closed form of decaying turbulence)."""
    nn = (n[0], n[1], n[2] if dim == 3 else 1)
    faces = range(6) if dim == 3 else range(4)
    patches = [Patch(f, *_face_full(nn, f), kind=OUTLET) for f in faces]
    fluid = np.ones((nn[2], nn[1], nn[0]), dtype=bool)
    fl = _base_fields(nn, fluid, 293.0, k0, om0)
    return Case(name="decay", dim=dim, n=nn, h=(h, h, h if dim == 3 else 1.0), nu=nu, rho=1.0,
                alpha_T=nu, dt=dt, physics=PHYS_KOMEGA, patches=patches, fields=fl,
                n_levels=1, tol=1e-12)
