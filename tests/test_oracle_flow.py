"""Whole-step pins of the oracle: laminar Poiseuille flow (closed form) and
mirror symmetry of the turbulent channel."""
import math

import numpy as np
import pytest

from paper_2603_21869_amd import cases as C


def _poiseuille_error(oracle, ny):
    H, L, U, nu = 1.0, 4.0, 1.0, 0.1
    nx = 4 * ny
    c = C.channel2d(nx, ny, L=L, H=H, U=U, nu=nu, dt=0.08 / ny ** 2 * 4, physics=0,
                    n_levels=3, tol=1e-10)
    y = (np.arange(ny) + 0.5) / ny * H
    prof = 1.5 * U * (1 - (2 * y / H - 1) ** 2)
    f = dict(c.fields)
    f["u"] = np.broadcast_to(prof[None, :, None], f["u"].shape).copy()
    steps = int(round(6.0 / c.dt))
    out, st, status = oracle.step(c, steps, fields=f)
    assert status == 0
    tail = out["u"][0, :, int(0.75 * nx):]
    return np.abs(tail - prof[:, None]).max() / (1.5 * U), out


@pytest.mark.slow
def test_laminar_poiseuille_profile(oracle):
    """Laminar channel (nu_t = 0) driven by a plug inlet: the developed profile
    downstream is 1.5 U (1 - (2y/H - 1)^2), second order in h."""
    e8, _ = _poiseuille_error(oracle, 8)
    e16, out = _poiseuille_error(oracle, 16)
    assert e16 < 0.01
    assert e8 / e16 > 3.0
    # developed: v vanishes, pressure falls linearly by 12 nu U / H^2 per metre
    assert np.abs(out["v"][0, :, 48:]).max() < 1e-3
    p = out["p"][0, 8, :]
    slope = (p[56] - p[48]) / (8 * 4.0 / 64)
    assert slope == pytest.approx(-12 * 0.1 * 1.0, rel=0.03)


def test_mirror_symmetry_of_turbulent_channel(oracle):
    """A y-mirror-symmetric initial state stays symmetric (u, k, omega, p even,
    v odd) through full turbulent steps, to round-off."""
    c = C.channel2d(64, 16, n_steps=4)
    u = c.fields["u"]
    c.fields["u"] = 0.5 * (u + u[:, ::-1, :])
    out, st, status = oracle.step(c, 4)
    assert status == 0
    for name, sign in (("u", 1), ("p", 1), ("k", 1), ("omega", 1), ("v", -1)):
        a = out[name][0]
        scale = np.abs(a).max()
        assert np.abs(a - sign * a[::-1, :]).max() <= 1e-11 * scale, name
    c3 = C.channel3d(32, 8, 8, n_steps=2, buoyancy=False)
    c3.patches = [p for p in c3.patches if p.face != 4]  # symmetric thermal walls
    u = c3.fields["u"]
    u = 0.5 * (u + u[:, ::-1, :])
    c3.fields["u"] = 0.5 * (u + u[::-1, :, :])
    out, st, status = oracle.step(c3, 2)
    for name, sign, ax in (("u", 1, 1), ("u", 1, 0), ("v", -1, 1), ("w", -1, 0), ("k", 1, 0)):
        a = out[name]
        scale = np.abs(a).max()
        flip = a[:, ::-1, :] if ax == 1 else a[::-1, :, :]
        assert np.abs(a - sign * flip).max() <= 1e-11 * scale, name


def test_warm_and_cold_started_steps_agree_to_tolerance(oracle):
    """Starting each pressure solve from the previous step's increment changes
    only where the iteration stops: after several steps both runs agree to the
    solver tolerance.  (In this start-up transient the increments change a lot
    from step to step, so the warm start saves no cycles here.)"""
    c = C.channel2d(64, 16, n_steps=5, tol=1e-9)
    warm, sw, s1 = oracle.step(c, 5, warm=True)
    cold, sc, s2 = oracle.step(c, 5, warm=False)
    assert s1 == 0 and s2 == 0
    assert sw[0]["cycles"] == sc[0]["cycles"]  # first solve: both from 0
    for k in ("u", "v", "p"):
        scale = np.abs(cold[k]).max()
        assert np.abs(warm[k] - cold[k]).max() <= 1e-6 * scale, k


def test_lambda2_closed_forms(oracle):
    """The lambda2 criterion (Sec. 3.2) on linear velocity fields, where the
    central gradient is exact away from the walls: solid-body rotation gives
    -Omega^2, plane shear 0, axisymmetric strain a^2/4, and rotation plus
    axial strain a^2/4 - Omega^2 (negative, a vortex, only when the
    rotation wins); non-fluid cells hold 0."""
    from tests.boxcase import box, centres
    solid = np.zeros((8, 10, 12), dtype=np.uint8)
    solid[0, 0, 0] = 1
    c = box((12, 10, 8), (0.1, 0.12, 0.09), kinds=[C.WALL] * 6, solid=solid)
    x, y, z = centres(c)
    x, y, z = x - x.mean(), y - y.mean(), z - z.mean()
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    Om, a, gam = 1.7, 0.9, 2.3
    cases = [((-Om * y, Om * x, 0 * z), -Om ** 2),
             ((gam * y, 0 * x, 0 * z), 0.0),
             ((-a * x / 2, -a * y / 2, a * z), a * a / 4),
             ((-a * x / 2 - Om * y, -a * y / 2 + Om * x, a * z), a * a / 4 - Om ** 2)]
    for (u, v, w), want in cases:
        l2 = oracle.lambda2(c, u, v, w)
        assert np.allclose(l2[inner], want, rtol=0, atol=1e-12)
        assert l2[0, 0, 0] == 0.0
