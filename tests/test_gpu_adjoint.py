"""Reverse mode of the pressure solve and of the pressure step on the GPU
(through the C ABI) against the oracle's reverse mode, which is pinned by
its assembled Jacobian and a dot-product test (tests/test_oracle_adjoint.py).
Bars as for the forward parity tests: FP64 1e-10 with the oracle running the
GPU's cycle count, mixed 1e-6 with both solves stopped at 1e-9."""
import numpy as np
import pytest

from paper_2603_21869_amd import cases as C
from tests.parity import fluid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2603_21869_amd import nfvm
    nfvm.lib()
    return nfvm


def _cases():
    return [
        ("ch2d", C.channel2d(96, 18, L=4.0, H=1.0, n_levels=2)),
        ("ch3d", C.channel3d(80, 20, 12, Lx=2.0, Ly=0.5, Lz=0.3, n_levels=3)),
        ("room", C.room3d(64, 24, 16, size=(10.0, 4.0, 3.0), seed=5, n_levels=4)),
        ("open", C.open_channel(48, 16, 16, h=0.02, n_levels=3, precision=C.PREC_FP64)),
    ]


def _rel(a, b, m):
    d = (a - b)[m]
    return (float(np.linalg.norm(d) / max(np.linalg.norm(b[m]), 1e-300)),
            float(np.abs(d).max() / max(np.abs(b[m]).max(), 1e-300)))


def test_mg_solve_adjoint_is_the_transposed_solve(nf, oracle):
    """<A^-1 b, c> = <b, A^-T c> with both solves on the GPU, and A^-T c
    against the oracle's solve run the GPU's cycle count."""
    import torch
    case = C.room3d(64, 32, 16, size=(10.0, 4.0, 3.0), seed=5, n_levels=4,
                    precision=C.PREC_FP64)
    g = nf.Grid(case)
    m = fluid(case)
    rng = np.random.default_rng(11)
    b = rng.standard_normal(g.shape) * m
    c = rng.standard_normal(g.shape) * m
    bd, cd = torch.from_numpy(b).cuda(), torch.from_numpy(c).cuda()
    x, y = torch.zeros_like(bd), torch.zeros_like(cd)
    s1, _ = nf.nfvm_mg_solve_device(g.h, bd.data_ptr(), x.data_ptr(), tol=1e-13, max_cycles=200)
    s2, _ = nf.nfvm_mg_solve_adjoint_device(g.h, cd.data_ptr(), y.data_ptr(), tol=1e-13,
                                            max_cycles=200)
    torch.cuda.synchronize()
    x, y = x.cpu().numpy(), y.cpu().numpy()
    g.close()
    lhs, rhs = float(np.sum(x * c)), float(np.sum(b * y))
    print(f"   <A^-1 b, c> = {lhs:.15e}, <b, A^-T c> = {rhs:.15e}", flush=True)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    yr, cyc, rel, st = oracle.MG(case).solve(c, forced=s2["cycles"])
    assert max(_rel(y, yr, m)) <= 1e-10


@pytest.mark.parametrize("prec", [C.PREC_FP64, C.PREC_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,case", _cases(), ids=[c[0] for c in _cases()])
def test_pressure_adjoint_matches_oracle(nf, oracle, name, case, prec):
    import torch
    case = case.copy(precision=prec)
    g = nf.Grid(case)
    sh = g.shape
    rng = np.random.default_rng(17)
    bars = [rng.standard_normal(sh) for _ in range(4)]
    if case.dim == 2:
        bars[2][:] = 0.0
    dev = [torch.from_numpy(a).cuda() for a in bars]
    outs = [torch.zeros_like(dev[0]) for _ in range(3)]
    tol = 1e-12 if prec == C.PREC_FP64 else 1e-9
    st, s = nf.nfvm_pressure_adjoint_device(g.h, [a.data_ptr() for a in dev],
                                            [o.data_ptr() for o in outs], tol=tol,
                                            max_cycles=200)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    g.close()
    forced = st["cycles"] if prec == C.PREC_FP64 else -1
    ref = oracle.pressure_adjoint(case.copy(precision=C.PREC_FP64), *bars,
                                  tol=1e-12 if forced < 0 else 1e-30, max_cycles=400,
                                  forced=forced)
    bar = 1e-10 if prec == C.PREC_FP64 else 1e-6
    everywhere = np.ones(sh, bool)
    for d in range(3):
        err = _rel(got[d], ref[d], everywhere)
        print(f"   {name} prec={prec} cycles={st['cycles']} component {d}: L2 {err[0]:.2e} "
              f"max {err[1]:.2e}", flush=True)
        assert max(err) <= bar, (d, err)
    # non-fluid cells pass their adjoint through unchanged
    m = fluid(case)
    for d in range(3):
        assert np.array_equal(got[d][~m], bars[d][~m])


def _ex_state(case, seed):
    """The case's fields with seeded perturbations that make every term of
    the explicit stage active (as in the oracle's pins)."""
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
def test_explicit_adjoint_matches_autodiff(nf, name, case):
    """nfvm_explicit_adjoint_device against the autodiff reverse mode of the
    oracle's explicit stage (pinned by finite differences of the C oracle):
    every input adjoint over every cell to 1e-10 of its largest value, on
    grids of each precision (the adjoint's arithmetic is FP64 in all); with
    a k adjoint on a cell whose k the stage clamps, that cell's k adjoint is
    the oracle's too."""
    import torch
    from oracle import autodiff as AD
    f = _ex_state(case, 4)
    rng = np.random.default_rng(9)
    outs = ("u", "v", "w", "T", "k", "omega")
    ybar = {nm: rng.standard_normal(f["u"].shape) for nm in outs}
    ref = AD.explicit_vjp(case, f, ybar)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    st = {nm: dev(f[nm]) for nm in ("u", "v", "w", "p", "T", "k", "omega")}
    yb = {nm: dev(ybar[nm]) for nm in outs}
    for prec in (C.PREC_FP64, C.PREC_MIXED):
        g = nf.Grid(case.copy(precision=prec))
        xb = {nm: torch.full_like(st["u"], float("nan")) for nm in st}
        nf.nfvm_explicit_adjoint_device(g.h, {k: v.data_ptr() for k, v in st.items()},
                                        {k: v.data_ptr() for k, v in yb.items()},
                                        {k: v.data_ptr() for k, v in xb.items()})
        torch.cuda.synchronize()
        g.close()
        for nm in st:
            got = xb[nm].cpu().numpy()
            scale = max(np.abs(ref[nm]).max(), 1e-300)
            err = np.abs(got - ref[nm]).max() / scale
            print(f"[ex-adjoint] {name} prec={prec} {nm} max|ref|={scale:.3e} err={err:.2e}",
                  flush=True)
            assert np.isfinite(got).all() and err <= 1e-10, (name, prec, nm, err)


@pytest.mark.parametrize("name,case", _cases(), ids=[c[0] for c in _cases()])
def test_destroy_adjoint_matches_autodiff(nf, name, case):
    """nfvm_destroy_adjoint_device against the autodiff reverse mode of the
    oracle's destruction step (pinned by finite differences of the C
    oracle), over half a time step and over a long tau where the limiters
    vary: the adjoints of u, v, w, k, omega to 1e-10 of their largest value."""
    import torch
    from oracle import autodiff as AD
    f = _ex_state(case, 5)
    rng = np.random.default_rng(10)
    kb, wb = rng.standard_normal(f["u"].shape), rng.standard_normal(f["u"].shape)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    names = ("u", "v", "w", "k", "omega")
    st = {nm: dev(f[nm]) for nm in names}
    kbd, wbd = dev(kb), dev(wb)
    g = nf.Grid(case.copy(precision=C.PREC_FP64))
    for tau in (0.5 * case.dt, 40.0 * case.dt):
        ref = AD.destroy_vjp(case, f, tau, kb, wb)
        xb = {nm: torch.full_like(st["u"], float("nan")) for nm in names}
        nf.nfvm_destroy_adjoint_device(g.h, {k: v.data_ptr() for k, v in st.items()}, tau,
                                       kbd.data_ptr(), wbd.data_ptr(),
                                       {k: v.data_ptr() for k, v in xb.items()})
        torch.cuda.synchronize()
        for nm in names:
            got = xb[nm].cpu().numpy()
            scale = max(np.abs(ref[nm]).max(), 1e-300)
            err = np.abs(got - ref[nm]).max() / scale
            print(f"[des-adjoint] {name} tau={tau:.2e} {nm} max|ref|={scale:.3e} err={err:.2e}",
                  flush=True)
            assert np.isfinite(got).all() and err <= 1e-10, (name, tau, nm, err)
    g.close()


def _step_cases():
    return [
        ("ch2d", C.channel2d(96, 18, L=4.0, H=1.0, n_levels=2)),
        ("ch3d", C.channel3d(80, 20, 12, Lx=2.0, Ly=0.5, Lz=0.3, n_levels=3)),
        ("room", C.room3d(64, 24, 16, size=(10.0, 4.0, 3.0), seed=5, n_levels=4)),
        ("open", C.open_channel(48, 16, 16, h=0.02, n_levels=3)),
    ]


@pytest.mark.parametrize("name,case", _step_cases(), ids=[c[0] for c in _step_cases()])
def test_step_adjoint_matches_oracle(nf, name, case):
    """nfvm_step_adjoint_device on an FP64 grid against the oracle's reverse
    mode of its time step (the stages' reverse modes composed, pinned by
    finite differences of the C oracle's step): every input adjoint to 1e-8
    of its largest value with both pressure solves to 1e-12; the grid holds
    the forward step's result afterwards, as the oracle's step gives it."""
    import torch
    from oracle import autodiff as AD
    from oracle import oracle as O
    c = case.copy(precision=C.PREC_FP64, tol=1e-12, max_cycles=200)
    f = _ex_state(c, 6)
    rng = np.random.default_rng(13)
    names = ("u", "v", "w", "p", "T", "k", "omega")
    bars = {nm: rng.standard_normal(f["u"].shape) for nm in names}
    if c.dim == 2:
        bars["w"][:] = 0.0
    ref = AD.step_vjp(c, f, bars, tol=1e-12)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    st = {nm: dev(f[nm]) for nm in names}
    bd = {nm: dev(bars[nm]) for nm in names}
    xb = {nm: torch.full_like(st["u"], float("nan")) for nm in names}
    g = nf.Grid(c)
    stats, _ = nf.nfvm_step_adjoint_device(g.h, {k: v.data_ptr() for k, v in st.items()},
                                           {k: v.data_ptr() for k, v in bd.items()},
                                           {k: v.data_ptr() for k, v in xb.items()}, tol=1e-12)
    torch.cuda.synchronize()
    after = g.fields()
    g.close()
    print(f"[step-adjoint] {name} cycles fwd={stats[0]['cycles']} adj={stats[1]['cycles']}",
          flush=True)
    for nm in names:
        got = xb[nm].cpu().numpy()
        scale = max(np.abs(ref[nm]).max(), 1e-300)
        err = np.abs(got - ref[nm]).max() / scale
        print(f"[step-adjoint] {name} {nm} max|ref|={scale:.3e} err={err:.2e}", flush=True)
        assert np.isfinite(got).all() and err <= 1e-8, (name, nm, err)
    fwd, _, s = O.step(c, 1, fields=f)
    assert s == 0
    for nm in names:
        scale = max(np.abs(fwd[nm]).max(), 1e-300)
        assert np.abs(after[nm] - fwd[nm]).max() <= 1e-8 * scale, nm


@pytest.mark.parametrize("name,case", _step_cases()[1:3], ids=[c[0] for c in _step_cases()[1:3]])
def test_step_adjoint_on_a_mixed_grid_matches_oracle(nf, name, case):
    """nfvm_step_adjoint_device on a mixed-precision grid (k, omega and T
    stored in FP32, velocity and pressure in FP64): with the state's k,
    omega and T given at FP32 values, so that loading it rounds nothing, the
    input adjoints match the FP64 oracle's reverse mode to 1e-5 of their
    largest value (the forward step rounds its intermediate k, omega and T
    to FP32, which moves the later stages' linearisation points by about
    1e-7), and the grid holds the forward step to 1e-6."""
    import torch
    from oracle import autodiff as AD
    from oracle import oracle as O
    c = case.copy(precision=C.PREC_FP64, tol=1e-12, max_cycles=200)
    f = _ex_state(c, 6)
    for nm in ("k", "omega"):
        f[nm] = f[nm].astype(np.float32).astype(np.float64)
    f["T"] = c.T_ref + (f["T"] - c.T_ref).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(17)
    names = ("u", "v", "w", "p", "T", "k", "omega")
    bars = {nm: rng.standard_normal(f["u"].shape) for nm in names}
    ref = AD.step_vjp(c, f, bars, tol=1e-12)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    st = {nm: dev(f[nm]) for nm in names}
    bd = {nm: dev(bars[nm]) for nm in names}
    xb = {nm: torch.full_like(st["u"], float("nan")) for nm in names}
    g = nf.Grid(c.copy(precision=C.PREC_MIXED))
    stats, _ = nf.nfvm_step_adjoint_device(g.h, {k: v.data_ptr() for k, v in st.items()},
                                           {k: v.data_ptr() for k, v in bd.items()},
                                           {k: v.data_ptr() for k, v in xb.items()}, tol=1e-12)
    torch.cuda.synchronize()
    after = g.fields()
    g.close()
    for nm in names:
        got = xb[nm].cpu().numpy()
        scale = max(np.abs(ref[nm]).max(), 1e-300)
        err = np.abs(got - ref[nm]).max() / scale
        print(f"[step-adjoint mixed] {name} {nm} max|ref|={scale:.3e} err={err:.2e}", flush=True)
        assert np.isfinite(got).all() and err <= 1e-5, (name, nm, err)
    fwd, _, s = O.step(c, 1, fields=f)
    assert s == 0
    for nm in names:
        scale = max(np.abs(fwd[nm]).max(), 1e-300)
        assert np.abs(after[nm] - fwd[nm]).max() <= 1e-6 * scale, nm


@pytest.mark.parametrize("name,case", _step_cases()[:3], ids=[c[0] for c in _step_cases()[:3]])
def test_step_adjoint_with_the_heun_stage_matches_oracle(nf, name, case):
    """With NFVM_OPT_RK_ORDER = 2 the whole step's reverse mode takes Heun's
    stage, (U + E(E(U))) / 2, back as (b + J1^T J2^T b) / 2: on FP64 grids
    every input adjoint matches the oracle's reverse mode of its rk_order = 2
    step (pinned by finite differences of the C oracle's step) to 1e-8 of
    its largest value, and the grid holds the forward Heun step."""
    import torch
    from oracle import autodiff as AD
    from oracle import oracle as O
    c = case.copy(precision=C.PREC_FP64, tol=1e-12, max_cycles=200, rk_order=2)
    f = _ex_state(c, 8)
    rng = np.random.default_rng(23)
    names = ("u", "v", "w", "p", "T", "k", "omega")
    bars = {nm: rng.standard_normal(f["u"].shape) for nm in names}
    if c.dim == 2:
        bars["w"][:] = 0.0
    ref = AD.step_vjp(c, f, bars, tol=1e-12)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    st = {nm: dev(f[nm]) for nm in names}
    bd = {nm: dev(bars[nm]) for nm in names}
    xb = {nm: torch.full_like(st["u"], float("nan")) for nm in names}
    g = nf.Grid(c)  # (the case's rk_order sets NFVM_OPT_RK_ORDER)
    stats, _ = nf.nfvm_step_adjoint_device(g.h, {k: v.data_ptr() for k, v in st.items()},
                                           {k: v.data_ptr() for k, v in bd.items()},
                                           {k: v.data_ptr() for k, v in xb.items()}, tol=1e-12)
    torch.cuda.synchronize()
    after = g.fields()
    g.close()
    for nm in names:
        got = xb[nm].cpu().numpy()
        scale = max(np.abs(ref[nm]).max(), 1e-300)
        err = np.abs(got - ref[nm]).max() / scale
        print(f"[step-adjoint heun] {name} {nm} max|ref|={scale:.3e} err={err:.2e}", flush=True)
        assert np.isfinite(got).all() and err <= 1e-8, (name, nm, err)
    fwd, _, s = O.step(c, 1, fields=f)
    assert s == 0
    for nm in names:
        scale = max(np.abs(fwd[nm]).max(), 1e-300)
        assert np.abs(after[nm] - fwd[nm]).max() <= 1e-8 * scale, nm
