"""Pins of the oracle's semi-implicit destruction (Sec. 2.5, eqs. k_des_step,
o_des_step, Algorithm 3) and of decaying turbulence."""
import math

import numpy as np
import pytest

from paper_2603_21869_amd import cases as C
from tests.boxcase import box, centres

BETA, BSTAR = 0.072, 0.09


def test_decaying_turbulence_omega_exact(oracle):
    """Quiescent uniform turbulence: only destruction acts, f_beta = 1, and the
    semi-implicit update keeps 1/omega linear in time, so after n steps
    omega = 1/(1/omega0 + beta n dt) to round-off."""
    c = C.decaying_box(n=(6, 6, 6), k0=1e-2, om0=5.0, nu=1e-12, dt=1e-2)
    f, st, status = oracle.step(c, 200)
    assert status == 0
    want = 1.0 / (1.0 / 5.0 + BETA * 200 * 1e-2)
    assert np.allclose(f["omega"], want, rtol=1e-13)
    assert all(s["cycles"] == 0 for s in st)  # b == 0: nothing to project


def test_decaying_turbulence_k_discrete_product_and_closed_form(oracle):
    """With Re_t >> R_beta (beta* -> 0.09) k follows the discrete product
    k0 prod[(1 + dt/2 beta* om_a)(1 + dt/2 beta* om_b)]^-1 to round-off, and
    the closed form k0 (1 + beta om0 t)^(-beta*/beta) to first order in dt."""
    k0, om0 = 1e-2, 5.0
    errs = []
    for n_steps, dt in ((100, 4e-2), (400, 1e-2)):
        c = C.decaying_box(n=(4, 4, 4), k0=k0, om0=om0, nu=1e-14, dt=dt)
        f, st, status = oracle.step(c, n_steps)
        inv, k = 1.0 / om0, k0
        for _ in range(n_steps):
            om_a = 1.0 / inv
            k = k / (1 + 0.5 * dt * BSTAR * om_a)
            inv += 0.5 * dt * BETA
            om_b = 1.0 / inv
            k = k / (1 + 0.5 * dt * BSTAR * om_b)
            inv += 0.5 * dt * BETA
        assert np.allclose(f["k"], k, rtol=1e-12)
        t = n_steps * dt
        exact = k0 * (1 + BETA * om0 * t) ** (-BSTAR / BETA)
        errs.append(abs(f["k"][0, 0, 0] - exact) / exact)
    assert errs[1] < errs[0] / 3.0 and errs[1] < 2e-3


def test_destruction_closed_form_with_gradients(oracle):
    """Linear k, omega along x (interior central gradients exact):
    chi_k = k' omega' / omega^3, f_beta* = (1+680 chi^2)/(1+400 chi^2),
    beta* from Re_t (R_beta = 8), k_new = k / (1 + tau beta* f_beta* omega)."""
    nu, tau = 1e-4, 0.3
    c = box((8, 4, 4), (0.1, 0.1, 0.1), physics=C.PHYS_KOMEGA, nu=nu,
            kinds=[C.OUTLET] * 6)
    x, y, z = centres(c)
    k = 0.01 + 0.02 * x
    om = 0.2 + 0.3 * x
    zero = np.zeros_like(x)
    kn, on = oracle.destroy(c, zero, zero, zero, k, om, tau)
    inner = (slice(None), slice(None), slice(1, -1))
    chi = 0.02 * 0.3 / om ** 3
    fbs = (1 + 680 * chi ** 2) / (1 + 400 * chi ** 2)
    Re = k / (nu * om)
    x4 = (Re / 8.0) ** 4
    bst = BSTAR * (4 / 15 + x4) / (1 + x4)
    want = k / (1 + tau * bst * fbs * om)
    assert np.allclose(kn[inner], want[inner], rtol=1e-13)
    # no strain, no rotation: f_beta = 1
    assert np.allclose(on[inner], (om / (1 + tau * BETA * om))[inner], rtol=1e-13)


def test_vortex_stretching_invariant(oracle):
    """Linear 3D velocity with gradient [[-c/2, a, 0], [0, -c/2, 0], [0, 0, c]]:
    Omega_ij Omega_jk S_ki = a^2 c / 4 (rotation about z, stretching along z),
    so chi_omega = |a^2 c/4| / (0.09 omega)^3 and f_beta = (1+70 chi)/(1+80 chi)."""
    a, cc, om0, tau = 0.9, 0.6, 0.4, 0.5
    c = box((6, 6, 6), (0.1, 0.1, 0.1), physics=C.PHYS_KOMEGA, kinds=[C.OUTLET] * 6)
    x, y, z = centres(c)
    u = -cc / 2 * x + a * y
    v = -cc / 2 * y
    w = cc * z
    k = np.full(x.shape, 1e-3)
    om = np.full(x.shape, om0)
    kn, on = oracle.destroy(c, u, v, w, k, om, tau)
    chi = abs(a * a * cc / 4) / (BSTAR * om0) ** 3
    fb = (1 + 70 * chi) / (1 + 80 * chi)
    inner = (slice(1, -1),) * 3
    assert np.allclose(on[inner], om0 / (1 + tau * BETA * fb * om0), rtol=1e-13)
    # pure rotation: f_beta = 1
    kn, on = oracle.destroy(c, a * y, -a * x, np.zeros_like(x), k, om, tau)
    assert np.allclose(on[inner], om0 / (1 + tau * BETA * om0), rtol=1e-13)


def test_destruction_keeps_positivity(oracle):
    """The semi-implicit update is unconditionally positive (Sec. 2.5)."""
    rng = np.random.default_rng(9)
    c = box((7, 6, 5), (0.1, 0.1, 0.1), physics=C.PHYS_KOMEGA, kinds=[C.WALL] * 6)
    sh = (5, 6, 7)
    u, v, w = (rng.standard_normal(sh) * 10 for _ in range(3))
    k = rng.random(sh) * 1e-2 + 1e-12
    om = rng.random(sh) * 1e3 + 1e-10
    for tau in (1e-3, 1.0, 1e6):
        kn, on = oracle.destroy(c, u, v, w, k, om, tau)
        assert (kn > 0).all() and (on > 0).all()
        assert (kn <= k).all() and (on <= om).all()
