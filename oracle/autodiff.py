"""Reverse mode of the explicit stage and of the destruction step by
automatic differentiation: PyTorch (CPU, FP64) restatements of the oracle's
forward-Euler explicit stage (Sec. 2.3, Algorithms 2 and 4, eqs. ko_mom,
ko_temp, ko_k, ko_o, a_star, k_gen, o_gen, a) and of its semi-implicit
destruction step (Sec. 2.5, Algorithm 3, eqs. k_des_step, o_des_step,
beta_star, o_des), differentiated by torch.autograd.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the product
library.  The boundary classification (which faces take ghost values and
their affine rules) is the C oracle's, read through ``oracle.ghost_tables``;
every formula is written out again here, in the C oracle's order, so each
forward map can be checked against ``oracle.explicit`` / ``oracle.destroy``
and the reverse mode against finite differences of them.
"""
from __future__ import annotations

from typing import Dict

import numpy as np
import torch

from oracle import oracle as O

# model constants of Sec. 2.1 (eqs. a_star, Re_t, a, beta_star; R_beta = 8,
# the standard low-Reynolds value, which the paper does not print)
BETA_I = 0.072
BSTAR_INF, R_BETA = 0.09, 8.0
ASTAR_INF, ASTAR_0, R_K = 1.0, 0.072 / 3.0, 6.0
A_INF, A_0, R_W = 0.52, 1.0 / 9.0, 2.95
EPS = 1e-10
F_U, F_V, F_W, F_P, F_T, F_K, F_OM, F_NUT = range(8)
KOMEGA, ENERGY, BUOYANCY = 1, 2, 4
NAMES = ("u", "v", "w", "p", "T", "k", "omega")


class Stage:
    """The explicit stage of one case as a torch function of its seven
    input fields (flattened, C order)."""

    def __init__(self, case):
        self.case = case
        nidx, a0, a1, fixed = O.ghost_tables(case)
        self.nidx = torch.from_numpy(nidx.astype(np.int64))
        self.a0 = torch.from_numpy(a0)
        self.a1 = torch.from_numpy(a1)
        self.fixed = torch.from_numpy(fixed)
        solid = case.solid if case.solid is not None else np.zeros(case.n[::-1], np.uint8)
        self.fluid = torch.from_numpy(np.ascontiguousarray(solid).reshape(-1) == 0)

    def nb(self, a, fld, d):
        """Neighbour value of field array a across face direction d."""
        idx = self.nidx[:, d]
        ghost = self.a0[:, d, fld] + self.a1[:, d, fld] * a
        return torch.where(idx >= 0, a[idx.clamp(min=0)], ghost)

    @staticmethod
    def omhat(om):
        return torch.where(om > EPS, om, torch.full_like(om, EPS))

    def nut(self, k, om):
        """nu_t = alpha* k / omega-hat (eqs. a_star, Re_t, ko_turb_diff); 0
        on non-fluid cells."""
        c = self.case
        oh = self.omhat(om)
        ret = k / (c.nu * oh)
        ast = ASTAR_INF * (ASTAR_0 + ret / R_K) / (1.0 + ret / R_K)
        return torch.where(self.fluid, ast * k / oh, torch.zeros_like(k))

    def transport(self, x, nut, phi, fld, gamma0, inv_sigma, q):
        """Face-flux divergence of one field (upwind convection, central
        diffusion, the -(p + 2/3 k)_f term on the q-faces of momentum)."""
        c = self.case
        vel = (x["u"], x["v"], x["w"])
        rhs = torch.zeros_like(phi)
        for d in range(c.dim):
            for side in (-1, 1):
                dr = 2 * d + (side > 0)
                Uf = 0.5 * (vel[d] + self.nb(vel[d], F_U + d, dr))
                phN = self.nb(phi, fld, dr)
                lower = phN if side < 0 else phi
                upper = phi if side < 0 else phN
                up = torch.where(Uf >= 0.0, lower, upper)
                nutf = 0.5 * (nut + self.nb(nut, F_NUT, dr))
                gam = gamma0 + nutf * inv_sigma
                F = -Uf * up + gam * (upper - lower) / c.h[d]
                if q == d:
                    pf = 0.5 * (x["p"] + self.nb(x["p"], F_P, dr))
                    kf = (0.5 * (x["k"] + self.nb(x["k"], F_K, dr)) if c.physics & KOMEGA
                          else torch.zeros_like(phi))
                    F = F - (pf + (2.0 / 3.0) * kf)
                rhs = rhs + side * F / c.h[d]
        return rhs

    def forward(self, x: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
        """One forward-Euler step of the rest terms, k and omega clamped at
        eps, omega kept on fixed cells, non-fluid cells unchanged."""
        c = self.case
        komega = c.physics & KOMEGA
        nut = self.nut(x["k"], x["omega"]) if komega else torch.zeros_like(x["u"])
        vel = (x["u"], x["v"], x["w"])
        out = {}
        for a, nm in enumerate(("u", "v", "w")):
            if a < c.dim:
                src = 0.0
                if c.physics & BUOYANCY:
                    src = -c.beta_T * (x["T"] - c.T_ref) * c.gravity[a]
                r = self.transport(x, nut, vel[a], F_U + a, c.nu, 1.0, a) + src
                out[nm] = torch.where(self.fluid, x[nm] + c.dt * r, x[nm])
            else:
                out[nm] = x[nm]
        if c.physics & ENERGY:
            r = self.transport(x, nut, x["T"], F_T, c.alpha_T, 1.0 / c.Pr_t, -1)
            out["T"] = torch.where(self.fluid, x["T"] + c.dt * r, x["T"])
        else:
            out["T"] = x["T"]
        if komega:
            G = [[None] * 3 for _ in range(3)]
            zero = torch.zeros_like(x["u"])
            for a in range(3):
                for b in range(3):
                    if a < c.dim and b < c.dim:
                        G[a][b] = (self.nb(vel[a], F_U + a, 2 * b + 1)
                                   - self.nb(vel[a], F_U + a, 2 * b)) / (2.0 * c.h[b])
                    else:
                        G[a][b] = zero
            S2 = zero
            for a in range(3):
                for b in range(3):
                    Sab = 0.5 * (G[a][b] + G[b][a])
                    S2 = S2 + Sab * Sab
            S2 = 2.0 * S2
            ret = x["k"] / (c.nu * self.omhat(x["omega"]))
            Gk = nut * S2
            Gw = A_INF * (A_0 + ret / R_W) / (1.0 + ret / R_W) * S2
            rk = self.transport(x, nut, x["k"], F_K, c.nu, 1.0 / c.sigma_k, -1) + Gk
            rw = self.transport(x, nut, x["omega"], F_OM, c.nu, 1.0 / c.sigma_w, -1) + Gw
            kn = x["k"] + c.dt * rk
            kn = torch.where(kn > EPS, kn, torch.full_like(kn, EPS))
            wn = x["omega"] + c.dt * rw
            wn = torch.where(wn > EPS, wn, torch.full_like(wn, EPS))
            wn = torch.where(self.fixed, x["omega"], wn)
            out["k"] = torch.where(self.fluid, kn, x["k"])
            out["omega"] = torch.where(self.fluid, wn, x["omega"])
        else:
            out["k"], out["omega"] = x["k"], x["omega"]
        return out


    def destroy(self, x: Dict[str, torch.Tensor], tau: float):
        """Destruction over tau: k / (1 + tau beta* f_beta* omega), omega /
        (1 + tau beta_i f_beta omega) from the input k and omega, central
        gradients with ghosts; fixed cells keep omega, non-fluid cells keep
        both."""
        c = self.case
        k, om = x["k"], x["omega"]
        vel = (x["u"], x["v"], x["w"])
        zero = torch.zeros_like(k)

        def cgrad(a, fld, d):
            if d >= c.dim:
                return zero
            return (self.nb(a, fld, 2 * d + 1) - self.nb(a, fld, 2 * d)) / (2.0 * c.h[d])

        oh = self.omhat(om)
        dkdo = zero
        for d in range(c.dim):
            dkdo = dkdo + cgrad(k, F_K, d) * cgrad(om, F_OM, d)
        chik = dkdo / (oh * oh * oh)
        fbs = torch.where(chik <= 0.0, torch.ones_like(chik),
                          (1.0 + 680.0 * chik * chik) / (1.0 + 400.0 * chik * chik))
        ret = k / (c.nu * oh)
        x4 = torch.pow(ret / R_BETA, 4.0)
        bstar = BSTAR_INF * (4.0 / 15.0 + x4) / (1.0 + x4)
        kn = k / (1.0 + tau * bstar * fbs * om)
        G = [[cgrad(vel[a], F_U + a, b) if a < c.dim else zero for b in range(3)]
             for a in range(3)]
        S = [[0.5 * (G[a][b] + G[b][a]) for b in range(3)] for a in range(3)]
        W = [[0.5 * (G[a][b] - G[b][a]) for b in range(3)] for a in range(3)]
        X = zero
        for a in range(3):
            for b in range(3):
                for e in range(3):
                    X = X + W[a][b] * W[b][e] * S[e][a]
        den = BSTAR_INF * oh
        chiw = torch.abs(X) / (den * den * den)
        fb = (1.0 + 70.0 * chiw) / (1.0 + 80.0 * chiw)
        wn = om / (1.0 + tau * BETA_I * fb * om)
        wn = torch.where(self.fixed, om, wn)
        return (torch.where(self.fluid, kn, k), torch.where(self.fluid, wn, om))


def _stage_map(st: Stage, x: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
    """The explicit stage of the case: one forward-Euler step E, or with
    rk_order = 2 Heun's method as the average of the start and a second
    Euler step from the first, (x + E(E(x))) / 2 (Sec. 2.6 names explicit
    Runge-Kutta schemes without fixing one); the second step takes nu_t from
    the first stage's k and omega and the same p."""
    y1 = st.forward(x)
    if getattr(st.case, "rk_order", 1) != 2:
        return y1
    x1 = dict(y1)
    x1["p"] = x["p"]
    y2 = st.forward(x1)
    return {nm: 0.5 * (x[nm] + y2[nm]) for nm in ("u", "v", "w", "T", "k", "omega")}


def _tensors(fields, grad: bool):
    return {nm: torch.tensor(np.ascontiguousarray(fields[nm], dtype=np.float64).reshape(-1),
                             requires_grad=grad) for nm in NAMES if nm in fields}


def explicit_forward(case, fields) -> Dict[str, np.ndarray]:
    """The explicit stage's outputs (u, v, w, T, k, omega) from dense input
    fields, by the torch restatement."""
    st = Stage(case)
    with torch.no_grad():
        out = _stage_map(st, _tensors(fields, False))
    shape = tuple(case.n[::-1])
    return {nm: out[nm].numpy().reshape(shape) for nm in out}


def explicit_vjp(case, fields, bars) -> Dict[str, np.ndarray]:
    """Reverse mode of the explicit stage at the state `fields` (dense u, v,
    w, p, T, k, omega): the adjoints of the seven inputs from the adjoints
    `bars` of the six outputs (u, v, w, T, k, omega), nu_t taken as the
    closure of each Euler step's input k and omega (so its adjoint is folded
    into theirs); Heun's stage when the case's rk_order is 2."""
    st = Stage(case)
    x = _tensors(fields, True)
    out = _stage_map(st, x)
    ys, gs = [], []
    for nm in ("u", "v", "w", "T", "k", "omega"):
        ys.append(out[nm])
        gs.append(torch.tensor(np.ascontiguousarray(bars[nm], dtype=np.float64).reshape(-1)))
    grads = torch.autograd.grad(ys, [x[nm] for nm in NAMES], gs, allow_unused=True)
    shape = tuple(case.n[::-1])
    res = {}
    for nm, gr in zip(NAMES, grads):
        res[nm] = np.zeros(shape) if gr is None else gr.numpy().reshape(shape)
    return res


def destroy_forward(case, fields, tau: float):
    """k and omega after the destruction step, by the torch restatement."""
    st = Stage(case)
    with torch.no_grad():
        kn, wn = st.destroy(_tensors(fields, False), tau)
    shape = tuple(case.n[::-1])
    return kn.numpy().reshape(shape), wn.numpy().reshape(shape)


def destroy_vjp(case, fields, tau: float, kbar, wbar) -> Dict[str, np.ndarray]:
    """Reverse mode of the destruction step at the state `fields` (dense u,
    v, w, k, omega): the adjoints of u, v, w, k and omega from those of the
    step's k and omega."""
    st = Stage(case)
    x = _tensors(fields, True)
    kn, wn = st.destroy(x, tau)
    gk = torch.tensor(np.ascontiguousarray(kbar, dtype=np.float64).reshape(-1))
    gw = torch.tensor(np.ascontiguousarray(wbar, dtype=np.float64).reshape(-1))
    names = ("u", "v", "w", "k", "omega")
    grads = torch.autograd.grad([kn, wn], [x[nm] for nm in names], [gk, gw], allow_unused=True)
    shape = tuple(case.n[::-1])
    return {nm: (np.zeros(shape) if gr is None else gr.numpy().reshape(shape))
            for nm, gr in zip(names, grads)}


def step_vjp(case, fields, bars, tol: float = 1e-13, max_cycles: int = 200) -> Dict[str, np.ndarray]:
    """Reverse mode of one whole time step (the oracle's step: omega reset
    on wall-adjacent cells, destruction over dt/2, the explicit stage, the
    pressure step, destruction over dt/2; Sec. 2.3 to 2.5) at the state
    `fields`: the adjoints of the seven input fields from those of the seven
    output fields.  The forward stages are the C oracle's (the solve to tol),
    the reverse modes of the destruction and explicit stages this module's,
    that of the pressure step the C oracle's (an exact second solve).  The
    solve is differentiated as the exact A^-1 (implicit differentiation)."""
    c = case
    komega = c.physics & KOMEGA
    f0 = {nm: np.array(fields[nm], dtype=np.float64) for nm in NAMES}
    f0["omega"] = O.fixed_omega(c, f0["omega"])
    half = 0.5 * c.dt
    if komega:
        kd, wd = O.destroy(c, f0["u"], f0["v"], f0["w"], f0["k"], f0["omega"], half)
    else:
        kd, wd = f0["k"], f0["omega"]
    s1 = dict(f0, k=kd, omega=wd)
    t = O.explicit(c, s1)
    b = O.rhs_b(c, t["u"], t["v"], t["w"])
    phi, _, _, _ = O.MG(c).solve(b, tol=tol, max_cycles=max_cycles)
    _, u1, v1, w1, _ = O.project(c, phi, t["u"], t["v"], t["w"], f0["p"])
    ub = {nm: np.array(bars[nm], dtype=np.float64) for nm in ("u", "v", "w")}
    if komega:
        d2 = destroy_vjp(c, dict(u=u1, v=v1, w=w1, k=t["k"], omega=t["omega"]), half, bars["k"],
                         bars["omega"])
        for nm in ub:
            ub[nm] = ub[nm] + d2[nm]
        ksb, wsb = d2["k"], d2["omega"]
    else:
        ksb, wsb = bars["k"], bars["omega"]
    usb, vsb, wsb_vel = O.pressure_adjoint(c, ub["u"], ub["v"], ub["w"], bars["p"], tol=tol,
                                           max_cycles=max_cycles)[:3]
    ex = explicit_vjp(c, s1, dict(u=usb, v=vsb, w=wsb_vel, T=bars["T"], k=ksb, omega=wsb))
    out = dict(ex)
    out["p"] = np.asarray(bars["p"], dtype=np.float64) + ex["p"]
    if komega:
        d1 = destroy_vjp(c, f0, half, ex["k"], ex["omega"])
        for nm in ("u", "v", "w"):
            out[nm] = ex[nm] + d1[nm]
        out["k"], out["omega"] = d1["k"], d1["omega"]
        # the reset holds omega on wall-adjacent cells whatever its input
        held = O.fixed_omega(c, np.full(f0["omega"].shape, np.nan))
        out["omega"] = np.where(np.isnan(held), out["omega"], 0.0)
    return out
