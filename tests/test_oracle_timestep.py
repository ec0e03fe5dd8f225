"""Pins of the oracle's IMEX timesteppers and their adjoints (Supplementary, "Initial
value problems") on problems with closed-form solutions, and the inner-product test
<Y, Phi X> = <Phi^* Y, X> on a linear trajectory (Supplementary, "Verification")."""
import numpy as np
import pytest

from oracle import imex

GAMMA = 1.0 - 1.0 / np.sqrt(2.0)


class Linear:
    """M dX/dt + L X = C X with dense random blocks (F linear: F' = C)."""

    def __init__(self, M, L, C):
        self.M, self.L, self.C = M, L, C

    def F(self, X):
        return np.einsum("kij,kj->ki", self.C, X)

    def F_vjp(self, X, Yb):
        return np.einsum("kji,kj->ki", self.C.conj(), Yb)


def scalar(lam, a=0.0):
    one = np.ones((1, 1, 1), dtype=complex)
    return Linear(one, lam * one, a * one)


def test_rk222_implicit_amplification_closed_form():
    """For dX/dt = -lam X treated implicitly: X1 = X0/(1 + g z), X2 = (X0 - (1-g) z X1)/(1 + g z)."""
    lam, dt, n = 3.7, 0.05, 40
    P = scalar(lam)
    XN, _ = imex.rk_forward(P, np.ones((1, 1)), dt, n)
    z = dt * lam
    R = (1.0 - (1.0 - GAMMA) * z / (1.0 + GAMMA * z)) / (1.0 + GAMMA * z)
    assert abs(XN[0, 0] - R ** n) < 1e-14


def test_rk222_explicit_part_is_second_order_taylor():
    a, dt, n = 0.8, 0.1, 10
    XN, _ = imex.rk_forward(scalar(0.0, a), np.ones((1, 1)), dt, n)
    z = dt * a
    assert abs(XN[0, 0] - (1 + z + z * z / 2) ** n) < 1e-13


def test_ars443_third_order_conditions():
    """ARS(4,4,3) as a pair of tableaus with weights b = last row (stiffly accurate): row sums
    give the same abscissae c for both parts, and the order-3 conditions hold for each part
    (sum b = 1, b.c = 1/2, b.c^2 = 1/3, b.A.c = 1/6) and for the coupling (b_E.A_I.c and
    b_I.A_E.c = 1/6).  One more order (b.c^3 = 1/4 for both parts) does not hold."""
    A, H = imex.ars443_tableau()
    c = A.sum(axis=1)
    assert np.allclose(H.sum(axis=1), c, atol=1e-15)
    bE, bI = A[-1], H[-1]
    for b, M in ((bE, A), (bI, H)):
        assert abs(b.sum() - 1.0) < 1e-15
        assert abs(b @ c - 0.5) < 1e-15
        assert abs(b @ c ** 2 - 1.0 / 3.0) < 1e-15
        assert abs(b @ M @ c - 1.0 / 6.0) < 1e-15
    assert abs(bE @ H @ c - 1.0 / 6.0) < 1e-15 and abs(bI @ A @ c - 1.0 / 6.0) < 1e-15
    assert abs(bE @ c ** 3 - 0.25) > 1e-3 or abs(bI @ c ** 3 - 0.25) > 1e-3
    assert np.all(np.diag(H)[1:] == 0.5)


def test_ars443_third_order_convergence():
    lam, a, T = 2.0, 0.5, 1.0
    errs = []
    for n in (20, 40, 80):
        XN, _ = imex.rk_forward(scalar(lam, a), np.ones((1, 1)), T / n, n, tableau=imex.ars443_tableau())
        errs.append(abs(XN[0, 0] - np.exp((a - lam) * T)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 3.0) < 0.15), rates


@pytest.mark.parametrize("stepper", ["rk", "sbdf"])
def test_second_order_convergence_to_exponential(stepper):
    lam, a, T = 2.0, 0.5, 1.0
    errs = []
    for n in (40, 80, 160):
        dt = T / n
        P = scalar(lam, a)
        if stepper == "rk":
            XN, _ = imex.rk_forward(P, np.ones((1, 1)), dt, n)
        else:
            XN, _ = imex.sbdf_forward(P, np.ones((1, 1)), dt, n)
        errs.append(abs(XN[0, 0] - np.exp((a - lam) * T)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.1), rates


def test_sbdf2_matches_two_root_recurrence():
    """Implicit heat: SBDF1 step then (3/2 + z) X_n = 2 X_{n-1} - X_{n-2}/2."""
    lam, dt, n = 1.3, 0.1, 30
    XN, states = imex.sbdf_forward(scalar(lam), np.ones((1, 1)), dt, n)
    z = dt * lam
    x = [1.0, 1.0 / (1.0 + z)]
    # closed form of the linear recurrence from its characteristic roots
    r1, r2 = np.roots([1.5 + z, -2.0, 0.5])
    A = np.array([[1.0, 1.0], [r1, r2]])
    c1, c2 = np.linalg.solve(A, np.array(x, dtype=complex))
    ref = c1 * r1 ** n + c2 * r2 ** n
    assert abs(XN[0, 0] - ref) < 1e-14


def test_heat_adjoint_closed_form():
    """J = 1/2 |X_N|^2 with X_N = R^N X_0 gives dJ/dX_0 = R^(2N) X_0 (real R)."""
    lam, dt, n = 3.7, 0.05, 25
    X0 = np.array([[0.7 + 0.2j]])
    P = scalar(lam)
    XN, hist = imex.rk_forward(P, X0, dt, n)
    g = imex.rk_adjoint(P, XN, hist, dt)
    G = (XN[0, 0] / X0[0, 0]).real
    assert abs(G - ((1.0 - (1.0 - GAMMA) * dt * lam / (1.0 + GAMMA * dt * lam))
                    / (1.0 + GAMMA * dt * lam)) ** n) < 1e-15
    assert abs(g[0, 0] - G * G * X0[0, 0]) < 1e-15
    XN, states = imex.sbdf_forward(P, X0, dt, n)
    g = imex.sbdf_adjoint(P, XN, states, dt)
    G = (XN[0, 0] / X0[0, 0]).real
    assert abs(g[0, 0] - G * G * X0[0, 0]) < 1e-15


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_sbdf_order_conditions_and_ramp(k):
    """The steady row of SBDF-k is exact for polynomials in time of degree <= k: the backward
    difference sum_j a_j X(t_n - j dt) = dX/dt(t_n) (sum_j a_j (-j)^p dt^(p-1) = p 0^(p-1)) and
    the extrapolation sum_i c_i F(t_n - i dt) = F(t_n) for degree < k; the first k - 1 steps use
    the lower-order rows (the scheme reverts while the history is short)."""
    dt = 0.3
    a, b, c = imex.sbdf_coefficients(k, dt, order=k)
    j = np.arange(len(a))
    assert len(a) == k + 1 and len(c) == k + 1 and b[0] == 1.0 and np.all(b[1:] == 0.0)
    for p in range(k + 1):
        target = 1.0 if p == 1 else 0.0
        assert abs(np.sum(a * dt * (-j) ** p) - target) < 1e-13, (k, p)
    for p in range(k):
        target = 1.0 if p == 0 else 0.0
        assert abs(np.sum(c[1:] * (-j[1:]) ** p) - target) < 1e-13, (k, p)
    # one degree more is not exact (the order is k, not higher)
    assert abs(np.sum(a * dt * (-j) ** (k + 1))) > 1e-3
    for n in range(1, k):
        an, bn, cn = imex.sbdf_coefficients(n, dt, order=k)
        ar, br, cr = imex.sbdf_coefficients(n, dt, order=n)
        assert np.array_equal(an, ar) and np.array_equal(cn, cr) and len(an) == n + 1


@pytest.mark.parametrize("k", [3, 4])
def test_sbdf_principal_root_converges_at_order_k_plus_1(k):
    """For dX/dt = -lam X + mu X (lam implicit, mu explicit) the steady recurrence
    (a_0 + lam) r^k = sum_i (c_i mu - a_i) r^(k-i) has a principal root r(h) with
    |r(h) - exp((mu - lam) h)| = O(h^(k+1)) (local error of a k-th order scheme)."""
    lam, mu = 1.7, 0.6
    errs = []
    hs = [0.08, 0.04, 0.02]
    for h in hs:
        a, b, c = imex.sbdf_coefficients(k, h, order=k)
        poly = np.zeros(k + 1)
        poly[0] = a[0] + lam
        for i in range(1, k + 1):
            poly[i] = a[i] - c[i] * mu
        roots = np.roots(poly)
        ex = np.exp((mu - lam) * h)
        r = roots[np.argmin(np.abs(roots - ex))]
        errs.append(abs(r - ex))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - (k + 1)) < 0.15), rates


def steps(n, h, amp=0.4, seed=None):
    """A smoothly varying step sequence: h (1 + amp sin(2 pi i / n)), or i.i.d. factors in
    [1 - amp, 1 + amp] when seed is given."""
    if seed is None:
        return h * (1.0 + amp * np.sin(2.0 * np.pi * np.arange(n) / n))
    return h * (1.0 + amp * (2.0 * np.random.default_rng(seed).random(n) - 1.0))


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_variable_step_rows_reduce_to_the_constant_rows(k):
    h = np.full(8, 0.07)
    for n in range(1, 8):
        a, b, c = imex.sbdf_variable_coefficients(h, n, k)
        ar, br, cr = imex.sbdf_coefficients(n, 0.07, k)
        assert np.allclose(a, ar, rtol=1e-13, atol=1e-13 * np.abs(ar).max())
        assert np.allclose(c, cr, rtol=1e-13, atol=1e-13) and np.array_equal(b, br)


def test_variable_step_sbdf2_closed_form():
    """Variable-step SBDF2 with w = h_n / h_{n-1}: a_0 = (1 + 2w) / ((1 + w) h_n),
    a_1 = -(1 + w) / h_n, a_2 = w^2 / ((1 + w) h_n), c_1 = 1 + w, c_2 = -w."""
    h = steps(12, 0.05, seed=3)
    for n in range(2, 12):
        w = h[n - 1] / h[n - 2]
        hn = h[n - 1]
        a, b, c = imex.sbdf_variable_coefficients(h, n, 2)
        ref_a = np.array([(1 + 2 * w) / ((1 + w) * hn), -(1 + w) / hn, w * w / ((1 + w) * hn)])
        assert np.allclose(a, ref_a, rtol=1e-13)
        assert np.allclose(c, [0.0, 1 + w, -w], rtol=1e-13)


@pytest.mark.parametrize("k", [2, 3])
def test_variable_step_second_order_convergence(k):
    """dX/dt = -lam X + mu X over [0, 1] on steps that grow linearly by a factor 2: the error to
    the exponential falls at second order (SBDF3 is limited to second order by its SBDF1/SBDF2
    start).  Rows built for constant steps are inconsistent on such steps by -(w - 1)/2 X' with
    w the ratio of neighbouring steps, which on a monotone ramp does not average out: they
    converge at first order, so this pins the variable-step rows."""
    lam, mu, T = 2.0, 0.5, 1.0
    errs = []
    for n in (40, 80, 160):
        h = 1.0 + np.arange(n) / n
        h *= T / h.sum()
        XN, _ = imex.sbdf_forward(scalar(lam, mu), np.ones((1, 1)), h, n, order=k)
        errs.append(abs(XN[0, 0] - np.exp((mu - lam) * T)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.1), rates


@pytest.mark.parametrize("k", [2, 3, 4])
def test_variable_step_trajectory_inner_product(k):
    P = random_linear(8)
    rng = np.random.default_rng(9)
    X0 = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    Yb = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    n = 12
    h = steps(n, 0.05, seed=10)
    XN, states = imex.sbdf_forward(P, X0, h, n, order=k)
    Xb = imex.sbdf_adjoint(P, Yb, states, h, order=k)
    lhs = np.real(np.vdot(Yb, XN))
    rhs = np.real(np.vdot(Xb, X0))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def random_linear(seed, K=3, S=4):
    rng = np.random.default_rng(seed)
    c = lambda: rng.standard_normal((K, S, S)) + 1j * rng.standard_normal((K, S, S))
    M = c() + 4 * np.eye(S)[None]
    return Linear(M, 0.5 * c(), 0.3 * c())


@pytest.mark.parametrize("stepper", ["rk", "rk443", "sbdf", "sbdf3", "sbdf4"])
def test_linear_trajectory_inner_product(stepper):
    P = random_linear(5)
    rng = np.random.default_rng(6)
    X0 = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    Yb = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    dt, n = 0.05, 12
    if stepper in ("rk", "rk443"):
        tab = imex.ars443_tableau() if stepper == "rk443" else None
        XN, hist = imex.rk_forward(P, X0, dt, n, tableau=tab)
        Xb = imex.rk_adjoint(P, Yb, hist, dt, tableau=tab)
    else:
        order = {"sbdf": 2, "sbdf3": 3, "sbdf4": 4}[stepper]
        XN, states = imex.sbdf_forward(P, X0, dt, n, order=order)
        Xb = imex.sbdf_adjoint(P, Yb, states, dt, order=order)
    lhs = np.real(np.vdot(Yb, XN))
    rhs = np.real(np.vdot(Xb, X0))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_block_lu_adjoint_solve_inner_product():
    P = random_linear(7, K=2, S=9)
    lu = imex.BlockLU(P.M, P.L, 1.0, 0.3)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, 9)) + 1j * rng.standard_normal((2, 9))
    y = rng.standard_normal((2, 9)) + 1j * rng.standard_normal((2, 9))
    lhs = np.real(np.vdot(y, lu.solve(x)))
    rhs = np.real(np.vdot(lu.solve_adjoint(y), x))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
