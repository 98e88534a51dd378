"""Pins of the reverse mode of the explicit stage (Sec. 2.3; the solver's
differentiability, Sec. 1 and 4): the autodiff restatement reproduces the C
oracle's forward map, and its vector-Jacobian products match central finite
differences of the C oracle along random directions."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_21869_amd import cases as C


def _cases():
    return [
        ("ch2d", C.channel2d(12, 8, L=1.2, H=0.8, n_levels=2)),
        ("ch3d", C.channel3d(10, 6, 5, Lx=1.0, Ly=0.3, Lz=0.25, n_levels=2)),
        ("room", C.room3d(12, 8, 6, size=(10.0, 4.0, 3.0), seed=5, n_levels=2)),
        ("open", C.open_channel(10, 6, 6, h=0.02, n_levels=2)),
    ]


def _state(case, seed):
    """The case's fields with seeded perturbations that make every term
    active (non-uniform k and omega, mixed-sign velocities, pressure)."""
    rng = np.random.default_rng(seed)
    f = {k: np.array(v, dtype=np.float64) for k, v in case.fields.items()}
    sh = f["u"].shape
    scale = max(np.abs(f["u"]).max(), 0.1)
    for nm in ("u", "v", "w"):
        f[nm] = f[nm] + 0.3 * scale * rng.standard_normal(sh)
    if case.dim == 2:
        f["w"][:] = 0.0
    f["p"] = 0.05 * rng.standard_normal(sh)
    f["T"] = f["T"] + 2.0 * rng.standard_normal(sh)
    f["k"] = f["k"] * (1.0 + 0.5 * rng.random(sh)) + 1e-4
    f["omega"] = f["omega"] * (1.0 + 0.5 * rng.random(sh)) + 1.0
    return f


@pytest.mark.parametrize("name,case", _cases(), ids=[c[0] for c in _cases()])
def test_autodiff_forward_reproduces_the_oracle(name, case):
    from oracle import autodiff as AD
    f = _state(case, 1)
    ref = O.explicit(case, f)
    got = AD.explicit_forward(case, f)
    for nm in ("u", "v", "w", "T", "k", "omega"):
        scale = max(np.abs(ref[nm]).max(), 1e-30)
        assert np.abs(got[nm] - ref[nm]).max() <= 1e-13 * scale, nm


@pytest.mark.parametrize("name,case", _cases(), ids=[c[0] for c in _cases()])
def test_vjp_matches_finite_differences(name, case):
    """<ybar, (E(x + e v) - E(x - e v)) / 2e> = <xbar, v> for random v over
    all seven inputs and random ybar over the six outputs (C oracle forward;
    e small against every branch point of the state)."""
    from oracle import autodiff as AD
    rng = np.random.default_rng(7)
    f = _state(case, 2)
    outs = ("u", "v", "w", "T", "k", "omega")
    ybar = {nm: rng.standard_normal(f["u"].shape) for nm in outs}
    xbar = AD.explicit_vjp(case, f, ybar)
    for trial in range(3):
        v = {nm: rng.standard_normal(f["u"].shape) * max(np.abs(f[nm]).max(), 1e-3)
             for nm in O.FIELDS}
        if case.dim == 2:
            v["w"][:] = 0.0
        e = 1e-6
        fp = {nm: f[nm] + e * v[nm] for nm in O.FIELDS}
        fm = {nm: f[nm] - e * v[nm] for nm in O.FIELDS}
        Ep, Em = O.explicit(case, fp), O.explicit(case, fm)
        lhs = sum((ybar[nm] * (Ep[nm] - Em[nm])).sum() for nm in outs) / (2 * e)
        rhs = sum((xbar[nm] * v[nm]).sum() for nm in O.FIELDS)
        assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs), 1e-12), (name, trial, lhs, rhs)


def test_vjp_of_identity_on_solid_cells_and_terms():
    """Solid cells are left unchanged by the stage, so their output adjoint
    passes straight through; and with a zero output adjoint every input
    adjoint is zero."""
    from oracle import autodiff as AD
    case = C.room3d(12, 8, 6, size=(10.0, 4.0, 3.0), seed=5, n_levels=2)
    f = _state(case, 3)
    outs = ("u", "v", "w", "T", "k", "omega")
    zero = AD.explicit_vjp(case, f, {nm: np.zeros(f["u"].shape) for nm in outs})
    assert all(not zero[nm].any() for nm in O.FIELDS)
    solid = case.solid.astype(bool)
    assert solid.any()
    ybar = {nm: np.where(solid, 1.0, 0.0) for nm in outs}
    xb = AD.explicit_vjp(case, f, ybar)
    for nm in outs:
        np.testing.assert_array_equal(xb[nm][solid], 1.0)


@pytest.mark.parametrize("name,case", _cases(), ids=[c[0] for c in _cases()])
def test_autodiff_destruction_reproduces_the_oracle(name, case):
    from oracle import autodiff as AD
    f = _state(case, 5)
    for tau in (0.5 * case.dt, 40.0 * case.dt):
        ko, oo = O.destroy(case, f["u"], f["v"], f["w"], f["k"], f["omega"], tau)
        kg, og = AD.destroy_forward(case, f, tau)
        assert np.abs(kg - ko).max() <= 1e-13 * np.abs(ko).max()
        assert np.abs(og - oo).max() <= 1e-13 * np.abs(oo).max()


@pytest.mark.parametrize("name,case", _cases(), ids=[c[0] for c in _cases()])
def test_destruction_vjp_matches_finite_differences(name, case):
    """<(kbar, wbar), (D(x + e v) - D(x - e v)) / 2e> = <xbar, v> for the
    destruction step D (C oracle forward) over u, v, w, k, omega; tau large
    enough that the limiter functions f_beta*, f_beta vary."""
    from oracle import autodiff as AD
    rng = np.random.default_rng(8)
    f = _state(case, 6)
    tau = 40.0 * case.dt
    kb, wb = rng.standard_normal(f["u"].shape), rng.standard_normal(f["u"].shape)
    xbar = AD.destroy_vjp(case, f, tau, kb, wb)
    names = ("u", "v", "w", "k", "omega")
    for trial in range(3):
        v = {nm: rng.standard_normal(f["u"].shape) * max(np.abs(f[nm]).max(), 1e-3)
             for nm in names}
        if case.dim == 2:
            v["w"][:] = 0.0
        e = 1e-7  # (the limiters are strongly curved: the central difference's
        # truncation error is 1e-6 relative at e = 1e-6 and falls as e^2)
        args = lambda s: [f[nm] + s * e * v[nm] for nm in names]
        kp, op = O.destroy(case, *args(1.0), tau)
        km, om_ = O.destroy(case, *args(-1.0), tau)
        lhs = ((kb * (kp - km)).sum() + (wb * (op - om_)).sum()) / (2 * e)
        rhs = sum((xbar[nm] * v[nm]).sum() for nm in names)
        assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs), 1e-12), (name, trial, lhs, rhs)


def _step_cases():
    # (every extent even: the two-level pressure solve needs them)
    return [
        ("ch2d", C.channel2d(12, 8, L=1.2, H=0.8, n_levels=2)),
        ("ch3d", C.channel3d(12, 6, 4, Lx=1.0, Ly=0.3, Lz=0.25, n_levels=2)),
        ("room", C.room3d(12, 8, 6, size=(10.0, 4.0, 3.0), seed=5, n_levels=2)),
        ("open", C.open_channel(10, 6, 6, h=0.02, n_levels=2)),
    ]


@pytest.mark.parametrize("name,case", _step_cases(), ids=[c[0] for c in _step_cases()])
def test_step_vjp_matches_finite_differences(name, case):
    """The whole step's reverse mode (destruction, explicit stage, pressure
    step, destruction, each stage's reverse mode composed in reverse order)
    against central differences of the C oracle's time step with its
    pressure solve converged to 1e-13, along random directions over all
    seven fields."""
    from oracle import autodiff as AD
    c = case.copy(tol=1e-13, max_cycles=200)
    rng = np.random.default_rng(12)
    f = _state(c, 7)
    bars = {nm: rng.standard_normal(f["u"].shape) for nm in O.FIELDS}
    if c.dim == 2:
        bars["w"][:] = 0.0
    xbar = AD.step_vjp(c, f, bars)
    for trial in range(2):
        v = {nm: rng.standard_normal(f["u"].shape) * max(np.abs(f[nm]).max(), 1e-3)
             for nm in O.FIELDS}
        if c.dim == 2:
            v["w"][:] = 0.0
        e = 1e-7
        fp, _, sp = O.step(c, 1, fields={nm: f[nm] + e * v[nm] for nm in O.FIELDS})
        fm, _, sm = O.step(c, 1, fields={nm: f[nm] - e * v[nm] for nm in O.FIELDS})
        assert sp == 0 and sm == 0
        lhs = sum((bars[nm] * (fp[nm] - fm[nm])).sum() for nm in O.FIELDS) / (2 * e)
        rhs = sum((xbar[nm] * v[nm]).sum() for nm in O.FIELDS)
        assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs), 1e-12), (name, trial, lhs, rhs)


def _heun(case):
    return case.copy(rk_order=2)


@pytest.mark.parametrize("name,case", _cases(), ids=[c[0] for c in _cases()])
def test_heun_autodiff_forward_reproduces_the_oracle(name, case):
    """Heun's stage, (x + E(E(x))) / 2 with the second Euler step's nu_t from
    the first stage's k and omega, restated in torch reproduces the C
    oracle's rk_order = 2 stage, which differs from one Euler step."""
    from oracle import autodiff as AD
    c = _heun(case)
    f = _state(c, 1)
    ref = O.explicit(c, f)
    got = AD.explicit_forward(c, f)
    euler = O.explicit(case, f)
    moved = 0.0
    for nm in ("u", "v", "w", "T", "k", "omega"):
        scale = max(np.abs(ref[nm]).max(), 1e-30)
        assert np.abs(got[nm] - ref[nm]).max() <= 1e-13 * scale, nm
        moved = max(moved, np.abs(ref[nm] - euler[nm]).max() / scale)
    assert moved > 1e-8


@pytest.mark.parametrize("name,case", _cases()[1:3], ids=[c[0] for c in _cases()[1:3]])
def test_heun_vjp_matches_finite_differences(name, case):
    """The reverse mode of Heun's stage against central differences of the
    C oracle's rk_order = 2 stage along random directions."""
    from oracle import autodiff as AD
    c = _heun(case)
    rng = np.random.default_rng(21)
    f = _state(c, 2)
    outs = ("u", "v", "w", "T", "k", "omega")
    ybar = {nm: rng.standard_normal(f["u"].shape) for nm in outs}
    xbar = AD.explicit_vjp(c, f, ybar)
    for trial in range(2):
        v = {nm: rng.standard_normal(f["u"].shape) * max(np.abs(f[nm]).max(), 1e-3)
             for nm in O.FIELDS}
        e = 1e-6
        Ep = O.explicit(c, {nm: f[nm] + e * v[nm] for nm in O.FIELDS})
        Em = O.explicit(c, {nm: f[nm] - e * v[nm] for nm in O.FIELDS})
        lhs = sum((ybar[nm] * (Ep[nm] - Em[nm])).sum() for nm in outs) / (2 * e)
        rhs = sum((xbar[nm] * v[nm]).sum() for nm in O.FIELDS)
        assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs), 1e-12), (name, trial, lhs, rhs)


@pytest.mark.parametrize("name,case", _step_cases()[1:3], ids=[c[0] for c in _step_cases()[1:3]])
def test_heun_step_vjp_matches_finite_differences(name, case):
    """The whole step's reverse mode with Heun's explicit stage against
    central differences of the C oracle's rk_order = 2 time step (pressure
    solve converged to 1e-13)."""
    from oracle import autodiff as AD
    c = _heun(case).copy(tol=1e-13, max_cycles=200)
    rng = np.random.default_rng(22)
    f = _state(c, 7)
    bars = {nm: rng.standard_normal(f["u"].shape) for nm in O.FIELDS}
    xbar = AD.step_vjp(c, f, bars)
    v = {nm: rng.standard_normal(f["u"].shape) * max(np.abs(f[nm]).max(), 1e-3)
         for nm in O.FIELDS}
    e = 1e-7
    fp, _, sp = O.step(c, 1, fields={nm: f[nm] + e * v[nm] for nm in O.FIELDS})
    fm, _, sm = O.step(c, 1, fields={nm: f[nm] - e * v[nm] for nm in O.FIELDS})
    assert sp == 0 and sm == 0
    lhs = sum((bars[nm] * (fp[nm] - fm[nm])).sum() for nm in O.FIELDS) / (2 * e)
    rhs = sum((xbar[nm] * v[nm]).sum() for nm in O.FIELDS)
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs), 1e-12), (name, lhs, rhs)
