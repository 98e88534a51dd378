"""Pins of the oracle's pressure solve (Sec. 2.4, eqs. pc_residual to
jacobi_pc, Algorithm 1): eigenmodes, manufactured solutions, brute-force
dense solves, transfer operators and the projection identity."""
import math

import numpy as np
import pytest

from paper_2603_21869_amd import cases as C
from tests.boxcase import box, centres


def test_jacobi_sweep_on_dirichlet_eigenmode(oracle):
    """On a box with zero pressure on every face, v = prod sin(pi m_d (i+1/2)/n_d)
    is an eigenvector of A with lambda = sum 4/h^2 sin^2(pi m/(2n)); one damped
    Jacobi sweep with b = 0 gives v (1 - w lambda / D_P) per cell, with the
    diagonal D_P = sum_d (2 + [first cell] + [last cell]) / h_d^2 (a zero-value
    face counts twice: its ghost is -x_P)."""
    n = (8, 6, 5)
    h = (0.1, 0.13, 0.07)
    c = box(n, h, kinds=[C.OUTLET] * 6)
    mg = oracle.MG(c)
    w = 6.0 / 7.0
    idx = np.meshgrid(np.arange(5), np.arange(6), np.arange(8), indexing="ij")
    for m in ((1, 1, 1), (3, 2, 4), (8, 6, 5)):
        v = np.ones((5, 6, 8))
        lam = 0.0
        D = np.zeros((5, 6, 8))
        for d, (ax, nd) in enumerate(((2, 8), (1, 6), (0, 5))):
            i = idx[ax]
            v = v * np.sin(math.pi * m[d] * (i + 0.5) / nd)
            lam += 4 / h[d] ** 2 * math.sin(math.pi * m[d] / (2 * nd)) ** 2
            D += (2 + (i == 0) + (i == nd - 1)) / h[d] ** 2
        assert np.allclose(mg.apply(0, v), lam * v, rtol=0, atol=1e-10 * lam)
        out = mg.smooth(0, v, np.zeros_like(v), 1)
        assert np.allclose(out, v * (1 - w * lam / D), rtol=0, atol=1e-12)


def _solve_rate(oracle, c, b, cycles=8):
    mg = oracle.MG(c)
    x = np.zeros_like(b)
    r0 = np.linalg.norm(b)
    facs = []
    for _ in range(cycles):
        x = x + mg.vcycle(np.zeros_like(b), b - mg.apply(0, x))
        r = np.linalg.norm(b - mg.apply(0, x))
        facs.append(r / r0)
        r0 = r
    return max(facs[-3:])


@pytest.mark.parametrize("dim", [2, 3])
def test_vcycle_factor_is_textbook_and_mesh_independent(oracle, dim):
    """Plain V(2,2) cycling on a channel-type box (zero-gradient inlet and walls,
    zero-value outlet): the convergence factor stays near the local-mode
    analysis values (mu^4 ~ 0.13 in 2D, 0.26 in 3D) as h halves."""
    rates = []
    sizes = [(32, 32), (64, 64), (128, 128)] if dim == 2 else [(16, 16, 16), (32, 32, 32)]
    for n in sizes:
        nn = tuple(n) + ((1,) if dim == 2 else ())
        c = box(nn, tuple(1.0 / s for s in nn), dim=dim,
                kinds=[C.INLET, C.OUTLET, C.WALL, C.WALL, C.WALL, C.WALL])
        c.n_levels = C.max_levels(c.n, dim) - 2
        b = np.random.default_rng(0).standard_normal((c.n[2], c.n[1], c.n[0]))
        rates.append(_solve_rate(oracle, c, b))
    bound = 0.2 if dim == 2 else 0.27
    assert max(rates) < bound
    assert max(rates) - min(rates) < 0.03


def test_manufactured_poisson_second_order(oracle):
    """phi = cos(pi x/(2Lx)) cos(2 pi y/Ly) cos(2 pi z/Lz) satisfies zero gradient
    at x = 0 and the side walls and phi = 0 at x = Lx; with b = -lap(phi) at
    cell centres the discrete solution converges to phi at O(h^2)."""
    errs = []
    for N in (8, 16, 32):
        n = (N, N, N)
        L = (2.0, 1.0, 1.0)
        c = box(n, tuple(L[d] / N for d in range(3)),
                kinds=[C.INLET, C.OUTLET, C.WALL, C.WALL, C.WALL, C.WALL],
                n_levels=C.max_levels(n, 3) - 2)
        x, y, z = centres(c)
        kx, ky, kz = math.pi / (2 * L[0]), 2 * math.pi / L[1], 2 * math.pi / L[2]
        phi = np.cos(kx * x) * np.cos(ky * y) * np.cos(kz * z)
        b = (kx ** 2 + ky ** 2 + kz ** 2) * phi
        mg = oracle.MG(c)
        sol, cyc, rel, st = mg.solve(b, tol=1e-12)
        assert st == 0 and rel <= 1e-12
        errs.append(np.abs(sol - phi).max())
    assert errs[1] / errs[2] > 3.5 and errs[0] / errs[1] > 3.0


def test_mg_solution_equals_dense_solve_with_mask(oracle):
    """Brute force: assemble A by applying the operator to unit vectors, solve
    densely with numpy, compare with the multigrid solution (vented box with a
    solid block, 4 levels)."""
    n = (16, 8, 8)
    solid = np.zeros((8, 8, 16), dtype=np.uint8)
    solid[0:4, 2:5, 5:9] = 1
    pats = [C.Patch(0, (2, 5), (5, 8), kind=C.INLET, U=(1, 0, 0)),
            C.Patch(1, (3, 0), (6, 2), kind=C.OUTLET)]
    c = box(n, (0.1, 0.12, 0.09), patches=pats, solid=solid, n_levels=4)
    mg = oracle.MG(c)
    act = mg.active(0).astype(bool)
    ids = np.flatnonzero(act)
    A = np.zeros((ids.size, ids.size))
    for col, q in enumerate(ids):
        e = np.zeros(act.size)
        e[q] = 1.0
        A[:, col] = mg.apply(0, e.reshape(act.shape)).ravel()[ids]
    assert np.allclose(A, A.T, rtol=0, atol=1e-9)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(act.shape) * act
    want = np.linalg.solve(A, b.ravel()[ids])
    sol, cyc, rel, st = mg.solve(b, tol=1e-14, max_cycles=200)
    assert st == 0
    assert np.abs(sol.ravel()[ids] - want).max() <= 1e-11 * np.abs(want).max()
    assert not sol[~act].any()


def test_transfer_operators(oracle):
    """RES (mean of children) and PROL (cell-centred trilinear): prolongation
    keeps constants everywhere away from zero-value faces and linear functions
    in the interior; restriction of a linear function is linear, and it keeps
    the volume integral."""
    n = (16, 12, 8)
    h = (0.1, 0.2, 0.3)
    c = box(n, h, kinds=[C.WALL] * 6, n_levels=2)
    mg = oracle.MG(c)
    (nzc, nyc, nxc), hc = mg.shape(1)
    Z, Y, X = np.meshgrid((np.arange(nzc) + 0.5) * hc[2], (np.arange(nyc) + 0.5) * hc[1],
                          (np.arange(nxc) + 0.5) * hc[0], indexing="ij")
    x, y, z = centres(c)
    e = 2.0 - 0.5 * X + 0.25 * Y + 1.5 * Z
    out = mg.prolong_add(0, e, np.zeros((8, 12, 16)))
    lin = 2.0 - 0.5 * x + 0.25 * y + 1.5 * z
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.allclose(out[inner], lin[inner], rtol=0, atol=1e-13)
    const = mg.prolong_add(0, np.full(e.shape, 3.0), np.zeros((8, 12, 16)))
    assert np.allclose(const, 3.0, rtol=0, atol=1e-14)
    r = mg.restrict(0, lin)
    assert np.allclose(r, e, rtol=0, atol=1e-13)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((8, 12, 16))
    assert mg.restrict(0, f).sum() * 8 == pytest.approx(f.sum(), rel=1e-12)


def _vented_box(n_levels, **kw):
    n = (16, 8, 8)
    solid = np.zeros((8, 8, 16), dtype=np.uint8)
    solid[0:4, 2:5, 5:9] = 1
    pats = [C.Patch(0, (2, 5), (5, 8), kind=C.INLET, U=(1, 0, 0)),
            C.Patch(1, (3, 0), (6, 2), kind=C.OUTLET)]
    return box(n, (0.1, 0.12, 0.09), patches=pats, solid=solid, n_levels=n_levels, **kw)


def test_nearest_prolongation_is_scaled_transpose_of_restriction(oracle):
    """Nearest upsampling (the plainest reading of Algorithm 1's upsampling)
    and mean-of-children restriction are adjoint up to the factor 2^d on the
    active cells: <R r, e>_coarse * 2^d = <r, P e>_fine for every r, e.  A
    block-constant field over fully active blocks survives R then P.  The
    linear prolongation fails the adjoint identity, so the option changes
    the operator."""
    for dim in (3, 2):
        if dim == 3:
            c = _vented_box(3, prolong=C.PROL_NEAREST)
            lin = oracle.MG(_vented_box(3))
        else:
            c = box((16, 12, 1), (0.1, 0.1, 1.0), dim=2, kinds=[C.WALL, C.OUTLET, C.WALL, C.WALL],
                    n_levels=3, prolong=C.PROL_NEAREST)
            lin = oracle.MG(box((16, 12, 1), (0.1, 0.1, 1.0), dim=2,
                                kinds=[C.WALL, C.OUTLET, C.WALL, C.WALL], n_levels=3))
        mg = oracle.MG(c)
        rng = np.random.default_rng(11 + dim)
        for l in (0, 1):
            fa, ca = mg.active(l).astype(bool), mg.active(l + 1).astype(bool)
            r = rng.standard_normal(fa.shape) * fa
            e = rng.standard_normal(ca.shape) * ca
            Pe = mg.prolong_add(l, e, np.zeros(fa.shape))
            assert not Pe[~fa].any()
            lhs = (mg.restrict(l, r) * e).sum() * 2 ** dim
            assert lhs == pytest.approx((r * Pe).sum(), rel=1e-12)
            Pl = lin.prolong_add(l, e, np.zeros(fa.shape))
            assert abs(lhs - (r * Pl).sum()) > 1e-3 * abs(lhs)
            # block-constant over blocks whose children are all active
            f = np.repeat(np.repeat(e, 2, axis=-1), 2, axis=-2)
            if dim == 3:
                f = np.repeat(f, 2, axis=0)
            blocks = np.repeat(np.repeat(ca, 2, axis=-1), 2, axis=-2)
            if dim == 3:
                blocks = np.repeat(blocks, 2, axis=0)
            full = fa.copy()
            for idx in np.argwhere(blocks & ~fa):
                I = tuple(i // 2 for i in idx) if dim == 3 else (0, idx[1] // 2, idx[2] // 2)
                sl = tuple(slice(2 * i, 2 * i + 2) for i in I) if dim == 3 else \
                    (slice(0, 1), slice(2 * I[1], 2 * I[1] + 2), slice(2 * I[2], 2 * I[2] + 2))
                full[sl] = False
            back = mg.prolong_add(l, mg.restrict(l, f * fa), np.zeros(fa.shape))
            assert np.allclose(back[full], f[full], rtol=1e-14, atol=0)


def test_nearest_cycles_reach_the_dense_solution(oracle):
    """Brute force: with nearest prolongation, as V(2,2) and as Algorithm 1's
    V(0,1) shape, the preconditioned solve reaches the dense solution of the
    assembled operator (the preconditioner changes the path, not the answer),
    and the linear prolongation needs fewer cycles."""
    lin = _vented_box(4)
    mg0 = oracle.MG(lin)
    act = mg0.active(0).astype(bool)
    ids = np.flatnonzero(act)
    A = np.zeros((ids.size, ids.size))
    for col, q in enumerate(ids):
        e = np.zeros(act.size)
        e[q] = 1.0
        A[:, col] = mg0.apply(0, e.reshape(act.shape)).ravel()[ids]
    rng = np.random.default_rng(5)
    b = rng.standard_normal(act.shape) * act
    want = np.linalg.solve(A, b.ravel()[ids])
    _, cyc_lin, _, st = mg0.solve(b, tol=1e-12, max_cycles=200)
    assert st == 0
    for nu1, nu2 in ((2, 2), (0, 1)):
        mg = oracle.MG(_vented_box(4, prolong=C.PROL_NEAREST, nu1=nu1, nu2=nu2))
        sol, cyc, rel, st = mg.solve(b, tol=1e-12, max_cycles=400)
        assert st == 0 and rel <= 1e-12
        assert np.abs(sol.ravel()[ids] - want).max() <= 1e-9 * np.abs(want).max()
        assert not sol[~act].any()
        assert cyc > cyc_lin


def test_projection_identity_and_divergence_free(oracle):
    """Face fluxes after projection satisfy sum_d D_d F_d = -dt (b - A phi) per
    cell for any phi; with a converged phi the face divergence is round-off
    (Sec. 2.4, eqs. pc_residual, pc_discretized)."""
    c = C.room3d(32, 16, 8, seed=3)
    rng = np.random.default_rng(1)
    fl = (c.solid == 0)
    us, vs, ws = (rng.standard_normal(fl.shape) * fl for _ in range(3))
    b = oracle.rhs_b(c, us, vs, ws)
    mg = oracle.MG(c)
    phi1, cyc, rel, st = mg.solve(b, forced=1)
    _, _, _, _, div1 = oracle.project(c, phi1, us, vs, ws, np.zeros(fl.shape))
    res = np.abs(b - mg.apply(0, phi1)).max() * c.dt
    assert div1 == pytest.approx(res, rel=1e-9)
    phi, cyc, rel, st = mg.solve(b, tol=1e-13, max_cycles=200)
    assert st == 0
    p, u, v, w, div = oracle.project(c, phi, us, vs, ws, np.zeros(fl.shape))
    assert div < 1e-11 * np.abs(b).max() * c.dt
    assert np.array_equal(p, phi)


def test_solve_from_any_initial_guess(oracle):
    """The solve reaches the dense solution from a nonzero initial guess, and
    b = 0 gives exactly x = 0 whatever the guess (A is nonsingular with an
    outlet face, so 0 is the only solution)."""
    n = (16, 8, 8)
    pats = [C.Patch(0, (0, 0), (8, 8), kind=C.INLET, U=(1, 0, 0)),
            C.Patch(1, (0, 0), (8, 8), kind=C.OUTLET)]
    c = box(n, (0.1, 0.12, 0.09), patches=pats, n_levels=4)
    mg = oracle.MG(c)
    act = mg.active(0).astype(bool)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(act.shape) * act
    x0 = rng.standard_normal(act.shape) * act
    cold, _, _, st0 = mg.solve(b, tol=1e-13, max_cycles=200)
    warm, cyc, rel, st1 = mg.solve(b, x0, tol=1e-13, max_cycles=200)
    assert st0 == 0 and st1 == 0 and cyc > 0
    assert np.abs(warm - cold).max() <= 1e-10 * np.abs(cold).max()
    # started at the solution: no cycle is needed and the guess is kept
    again, cyc2, _, _ = mg.solve(b, cold, tol=1e-10, max_cycles=200)
    assert cyc2 == 0 and np.array_equal(again, cold)
    z, cyc3, rel3, st3 = mg.solve(np.zeros_like(b), x0, tol=1e-10, max_cycles=200)
    assert st3 == 0 and cyc3 == 0 and not z.any()


def test_exact_first_cycle_then_breakdown_takes_no_step(oracle):
    """Closed form: a single cell with one zero-value face (A = 2/h^2 = 2 at
    h = 1) and a one-level hierarchy (the coarsest dense inverse, exact in
    binary) solves A x = 1 in one preconditioned iteration: x = 1/2 and r = 0
    exactly.  Forced further iterations then meet z = 0, where (p, A p) = 0
    and the plain step length would be 0/0; the restart takes no step, so x
    stays 1/2 exactly (a missing guard turns x into NaN)."""
    c = box((1, 1, 1), (1.0, 1.0, 1.0), dim=2, kinds=[C.OUTLET, C.WALL, C.WALL, C.WALL])
    mg = oracle.MG(c)
    b = np.ones((1, 1, 1))
    assert mg.apply(0, np.ones((1, 1, 1)))[0, 0, 0] == 2.0
    x, cyc, rel, st = mg.solve(b, forced=4)
    assert cyc == 4 and st == 0
    assert x[0, 0, 0] == 0.5 and rel == 0.0



def test_literal_jacobi_sweep_is_undamped_with_scalar_diagonal(oracle):
    """Algorithm 1 read literally (eq. jacobi_pc): one Jacobi sweep with the
    scalar D = 2 sum_d 1/h_d^2 (6/dx^2 at equal spacing) and no damping
    multiplies every eigenmode of A by exactly 1 - lambda/D, boundary cells
    included (a per-cell diagonal would not keep the sine modes)."""
    n = (8, 6, 5)
    h = (0.1, 0.13, 0.07)
    c = box(n, h, kinds=[C.OUTLET] * 6).copy(literal=1)
    mg = oracle.MG(c)
    Ds = sum(2 / hd ** 2 for hd in h)
    idx = np.meshgrid(np.arange(5), np.arange(6), np.arange(8), indexing="ij")
    for m in ((1, 1, 1), (3, 2, 4), (8, 6, 5)):
        v = np.ones((5, 6, 8))
        lam = 0.0
        for d, (ax, nd) in enumerate(((2, 8), (1, 6), (0, 5))):
            v = v * np.sin(math.pi * m[d] * (idx[ax] + 0.5) / nd)
            lam += 4 / h[d] ** 2 * math.sin(math.pi * m[d] / (2 * nd)) ** 2
        out = mg.smooth(0, v, np.zeros_like(v), 1)
        assert np.allclose(out, v * (1 - lam / Ds), rtol=0, atol=1e-12)
    # the highest mode grows in magnitude under the undamped sweep: |1 - lambda/D| > 1
    # is impossible here (lambda < 2 D), but it is barely damped: the smoothing
    # factor of undamped Jacobi is 1 on the checkerboard mode
    assert abs(1 - lam / Ds) > 0.9


def test_literal_plain_iteration_closed_form(oracle):
    """One level (the coarsest is the fine level, one sweep from zero): the
    literal cycle returns r / D, so the plain iteration x <- x + (b - A x)/D on
    an eigenmode b = v reaches x_k = (1 - (1 - lambda/D)^k) v / lambda."""
    n = (8, 6)
    h = (0.1, 0.13)
    c = box(n, h, dim=2, kinds=[C.OUTLET] * 4).copy(literal=1)
    mg = oracle.MG(c)
    Ds = sum(2 / hd ** 2 for hd in h)
    j, i = np.meshgrid(np.arange(6), np.arange(8), indexing="ij")
    v = (np.sin(math.pi * 2 * (i + 0.5) / 8) * np.sin(math.pi * (j + 0.5) / 6))[None]
    lam = 4 / h[0] ** 2 * math.sin(math.pi * 2 / 16) ** 2 + 4 / h[1] ** 2 * math.sin(math.pi / 12) ** 2
    e = mg.vcycle(np.zeros_like(v), v)
    assert np.allclose(e, v / Ds, rtol=0, atol=1e-15)
    for k in (1, 2, 7):
        x, cyc, rel, st = mg.solve(v, forced=k)
        want = (1 - (1 - lam / Ds) ** k) * v / lam
        assert cyc == k and np.allclose(x, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_literal_cycle_matches_algorithm_1_in_matrix_form(oracle):
    """Brute force: Algorithm 1 written out with assembled matrices (the level
    operators A_l column by column from the oracle's operator; RES the mean of
    the children, PROL nearest upsampling, D_l the scalar diagonal), its
    residual r = A p - b restricted to every level, one sweep per level on the
    way up with w <- PROL(w), p <- p - w and one fine sweep, gives the
    oracle's forced iterates."""
    n = (16, 8)
    h = (0.05, 0.07)
    pats = [C.Patch(0, (0, 0), (8, 1), kind=C.INLET), C.Patch(1, (2, 0), (6, 1), kind=C.OUTLET)]
    c = box(n, h, dim=2, patches=pats, n_levels=3).copy(literal=1)
    mg = oracle.MG(c)
    L = 3
    shapes = [mg.shape(l)[0] for l in range(L)]
    A = []
    for l in range(L):
        N = int(np.prod(shapes[l]))
        M = np.zeros((N, N))
        for q in range(N):
            e = np.zeros(N)
            e[q] = 1.0
            M[:, q] = mg.apply(l, e.reshape(shapes[l])).ravel()
        A.append(M)
    Ds = [sum(2 / (hd * 2 ** l) ** 2 for hd in h) for l in range(L)]

    def res(r, l):  # level l -> l + 1, mean of the 2 x 2 children
        f = r.reshape(shapes[l])[0]
        return (0.25 * (f[0::2, 0::2] + f[1::2, 0::2] + f[0::2, 1::2] + f[1::2, 1::2])).ravel()

    def prol(w, l):  # level l + 1 -> l, nearest
        cw = w.reshape(shapes[l + 1])[0]
        return np.repeat(np.repeat(cw, 2, axis=0), 2, axis=1).ravel()

    rng = np.random.default_rng(4)
    b = rng.standard_normal(shapes[0]).ravel()
    p = np.zeros_like(b)
    for it in range(1, 5):
        r = [A[0] @ p - b]
        for l in range(L - 1):
            r.append(res(r[-1], l))
        w = np.zeros_like(r[L - 1])
        for l in range(L - 1, 0, -1):
            w = w - (A[l] @ w) / Ds[l] + r[l] / Ds[l]
            w = prol(w, l - 1)
        p = p - w
        p = p - (A[0] @ p) / Ds[0] + b / Ds[0]
        x, cyc, rel, st = mg.solve(b.reshape(shapes[0]), forced=it)
        assert np.allclose(x.ravel(), p, rtol=0, atol=1e-12 * np.abs(p).max()), it


def test_coarse_sweep_count_schedule(oracle):
    """nu_coarse: the cycle written out from the level operators (damped
    Jacobi sweeps, mean-of-children restriction, interpolation, a dense
    solve on the coarsest level) with nu1 = 2 pre and nu2 = 1 post sweeps
    on the finest level and nu_coarse pre and post sweeps on every level
    below gives the oracle's cycle; nu_coarse = 0 keeps nu1, nu2 there."""
    for nuc in (0, 3):
        c = _vented_box(3).copy(nu1=2, nu2=1, nu_coarse=nuc)
        mg = oracle.MG(c)
        L = mg.L
        act = [mg.active(l).astype(bool) for l in range(L)]
        sh = mg.shape(L - 1)[0]
        ids = np.flatnonzero(act[L - 1])
        A = np.zeros((ids.size, ids.size))
        for q, i in enumerate(ids):
            e = np.zeros(act[L - 1].size)
            e[i] = 1.0
            A[:, q] = mg.apply(L - 1, e.reshape(sh)).ravel()[ids]

        def cycle(l, b):
            if l == L - 1:
                x = np.zeros(act[l].size)
                x[ids] = np.linalg.solve(A, b.ravel()[ids])
                return x.reshape(b.shape)
            pre, post = (2, 1) if l == 0 or nuc == 0 else (nuc, nuc)
            x = mg.smooth(l, np.zeros_like(b), b, pre)
            r = (b - mg.apply(l, x)) * act[l]
            x = mg.prolong_add(l, cycle(l + 1, mg.restrict(l, r)), x)
            return mg.smooth(l, x, b, post)

        b = np.random.default_rng(3).standard_normal(act[0].shape) * act[0]
        want = cycle(0, b)
        got = mg.vcycle(np.zeros_like(b), b)
        assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max()), nuc
    plain = oracle.MG(_vented_box(3).copy(nu1=2, nu2=1)).vcycle(np.zeros_like(b), b)
    assert not np.allclose(plain, got)


def test_coarse_sweeps_help_around_solid_blocks(oracle):
    """On a room with seeded solid blocks the rediscretised coarse operators
    approximate the fine one less well as the levels coarsen, and the
    preconditioned solve needs more iterations than on the empty room;
    more sweeps on the coarse levels (nu_coarse = 8) win most of them back,
    with the V shape of the cycle unchanged."""
    base = C.room3d(128, 64, 32, size=(10.0, 4.0, 3.0), seed=0, n_levels=6, precision=C.PREC_FP64)
    m = base.solid == 0
    # a smooth right-hand side (as the divergence of a developed flow is),
    # which leaves the most work to the coarse levels
    z, y, x = np.meshgrid(*(np.linspace(0, 1, k) for k in m.shape), indexing="ij")
    b = (np.sin(3.1 * x + 0.3) * np.cos(2.2 * y) + 0.5 * np.sin(5 * z) + 0.2) * m
    its = {}
    for nuc in (0, 8):
        xs, cyc, rel, st = oracle.MG(base.copy(nu_coarse=nuc)).solve(b, tol=1e-6, max_cycles=200)
        assert st == 0 and rel <= 1e-6
        its[nuc] = cyc
    print("iterations", its)
    assert its[8] <= 0.8 * its[0]
