"""Pins of the oracle's reverse mode of the pressure step (Sec. 2.4: the
Poisson right-hand side of eq. pc_residual, the solve of A phi = b and the
projection u = u* - dt grad(phi), p = p^n + phi).  The step is affine in u*,
so its Jacobian is exactly the difference of two forward evaluations; the
adjoint written as a scatter of each forward term must be its transpose:
checked against the Jacobian assembled column by column from the forward
functions (brute force on a small box with a solid block, an inlet and an
outlet), and by the dot-product identity <J v, y> = <v, J^T y> on a room
with seeded blocks."""
import numpy as np

from paper_2603_21869_amd import cases as C
from tests.boxcase import box


def _vented(n=(8, 6, 4), dim=3):
    solid = np.zeros((n[2], n[1], n[0]), dtype=np.uint8)
    solid[1:3, 2:4, 3:5] = 1
    pats = [C.Patch(0, (1, 0), (5, 3), kind=C.INLET, U=(0.7, 0.1, -0.2)),
            C.Patch(1, (2, 1), (6, 4), kind=C.OUTLET)]
    return box(n, (0.1, 0.12, 0.09), patches=pats, solid=solid, n_levels=2, dt=0.01)


def _forward(oracle, case, us, vs, ws, pn, Ainv):
    """(u, v, w, p) after the pressure step, the solve done exactly with the
    dense inverse of A on the active cells."""
    b = oracle.rhs_b(case, us, vs, ws)
    act = case.solid.ravel() == 0
    phi = np.zeros(b.size)
    phi[act] = Ainv @ b.ravel()[act]
    phi = phi.reshape(b.shape)
    p, u, v, w, _ = oracle.project(case, phi, us, vs, ws, pn)
    return u, v, w, p


def _dense_inverse(oracle, case):
    mg = oracle.MG(case)
    sh = mg.shape(0)[0]
    act = np.flatnonzero(case.solid.ravel() == 0)
    A = np.zeros((act.size, act.size))
    for q, i in enumerate(act):
        e = np.zeros(int(np.prod(sh)))
        e[i] = 1.0
        A[:, q] = mg.apply(0, e.reshape(sh)).ravel()[act]
    return np.linalg.inv(A)


def test_pressure_adjoint_is_transposed_jacobian(oracle):
    case = _vented()
    sh = (case.n[2], case.n[1], case.n[0])
    N = int(np.prod(sh))
    Ainv = _dense_inverse(oracle, case)
    z = np.zeros(sh)
    f0 = np.concatenate([a.ravel() for a in _forward(oracle, case, z, z, z, z, Ainv)])
    J = np.zeros((4 * N, 4 * N))
    for col in range(4 * N):
        e = np.zeros(4 * N)
        e[col] = 1.0
        ins = [e[m * N:(m + 1) * N].reshape(sh) for m in range(4)]
        J[:, col] = np.concatenate([a.ravel() for a in _forward(oracle, case, *ins, Ainv)]) - f0
    rng = np.random.default_rng(5)
    y = rng.standard_normal(4 * N)
    want = J.T @ y
    ub, vb, wb, pb = [y[m * N:(m + 1) * N].reshape(sh) for m in range(4)]
    usb, vsb, wsb, phib, lam, cyc, rel, st = oracle.pressure_adjoint(case, ub, vb, wb, pb,
                                                                     tol=1e-14, max_cycles=400)
    assert st == 0
    got = np.concatenate([usb.ravel(), vsb.ravel(), wsb.ravel(), pb.ravel()])
    assert np.allclose(got, want, rtol=0, atol=1e-9 * np.abs(want).max())
    # the adjoint of p^n is pbar: the step adds phi to it
    assert np.allclose(J[3 * N:, 3 * N:], np.eye(N))


def test_pressure_adjoint_dot_product_on_room(oracle):
    case = C.room3d(32, 16, 12, size=(10.0, 4.0, 3.0), seed=3, n_levels=3, precision=C.PREC_FP64)
    sh = (case.n[2], case.n[1], case.n[0])
    rng = np.random.default_rng(9)
    v = [rng.standard_normal(sh) for _ in range(4)]
    y = [rng.standard_normal(sh) for _ in range(4)]
    mg = oracle.MG(case)

    def fwd(us, vs, ws, pn):
        b = oracle.rhs_b(case, us, vs, ws)
        phi, cyc, rel, st = mg.solve(b, tol=1e-13, max_cycles=400)
        assert st == 0
        p, u, w_, ww, _ = oracle.project(case, phi, us, vs, ws, pn)
        return u, w_, ww, p

    z = np.zeros(sh)
    f0 = fwd(z, z, z, z)
    Jv = [a - b for a, b in zip(fwd(*v), f0)]
    usb, vsb, wsb, phib, lam, cyc, rel, st = oracle.pressure_adjoint(case, *y, tol=1e-13,
                                                                     max_cycles=400)
    assert st == 0
    lhs = sum(np.sum(a * b) for a, b in zip(Jv, y))
    rhs = sum(np.sum(a * b) for a, b in zip(v, (usb, vsb, wsb, y[3])))
    print("dot products", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-9 * max(abs(lhs), 1.0)
