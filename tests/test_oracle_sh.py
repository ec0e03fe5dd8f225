"""Pins of the Swift-Hohenberg oracle against facts that do not come from its own code:
explicit Fourier sums, the exact cube of a single mode, the PDE's closed-form linear rates,
Parseval, an exact (Richardson) difference of the cubic term, brute-force finite differences
of the whole discrete gradient on a tiny grid, and the Taylor-remainder rate 2."""
import numpy as np

from oracle import imex
from oracle.sh import SH


def explicit_grid(P, c, Ng, weighted=True):
    x = np.arange(Ng) * P.Lx / Ng
    X, Y = np.meshgrid(x, x)            # [y, x]
    u = np.zeros((Ng, Ng))
    for a in range(P.N):
        if a == P.N // 2:
            continue
        for b in range(P.N // 2):
            w = (1.0 if b == 0 else 2.0) if weighted else 1.0
            u += np.real(w * c[a, b] * np.exp(1j * (P.kx[b] * X + P.ky[a] * Y)))
    return u


def rand_c(P, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((P.N, P.N // 2)) + 1j * rng.standard_normal((P.N, P.N // 2))
    c[P.N // 2] = 0.0
    return c


def test_transforms_are_the_explicit_sums():
    P = SH(8, 0.3, L=10.0)
    c = rand_c(P, 0)
    for Ng in (8, 16):
        assert np.allclose(P.to_grid(c, Ng), explicit_grid(P, c, Ng), atol=1e-12, rtol=0)
        assert np.allclose(P.to_grid(c, Ng, weighted=False), explicit_grid(P, c, Ng, False), atol=1e-12, rtol=0)
    u = np.random.default_rng(1).standard_normal((16, 16))
    x = np.arange(16) * P.Lx / 16
    X, Y = np.meshgrid(x, x)
    cd = np.zeros_like(c)
    for a in range(P.N):
        for b in range(P.N // 2):
            if a != P.N // 2:
                cd[a, b] = np.sum(u * np.exp(-1j * (P.kx[b] * X + P.ky[a] * Y))) / 256.0
    assert np.allclose(P.from_grid(u, 16), cd, atol=1e-14, rtol=0)
    # round trip of the coefficients of a real field (their k_x = 0 column is Hermitian in
    # k_y) on any grid that holds the modes
    cf = P.from_grid(np.random.default_rng(2).standard_normal((8, 8)), 8)
    assert np.allclose(P.from_grid(P.to_grid(cf, 16), 16), cf, atol=1e-14, rtol=0)


def test_cube_of_a_single_mode():
    # u = A cos(k x) with coefficient A/2 at i_x = 1: u^3 = A^3 (3/4 cos(kx) + 1/4 cos(3kx))
    P = SH(16, 0.2)
    A = 0.7
    c = np.zeros((16, 8), complex)
    c[0, 1] = A / 2
    F = P.F(c.reshape(-1, 1)).reshape(16, 8)
    expect = np.zeros_like(c)
    expect[0, 1] = -0.75 * A ** 3 / 2
    expect[0, 3] = -0.25 * A ** 3 / 2
    assert np.allclose(F, expect, atol=1e-15, rtol=0)


def test_linear_rates_are_the_pde_closed_forms():
    # L = 16 pi: i_x = 8 is |k| = 1, where (1 + Laplacian) cos = 0 and u_t = r u;
    # (i_x, i_y) = (8, 8) has |k|^2 = 2: u_t = (r - 1) u.  One SBDF1 step of each mode alone
    # (amplitude small enough that u^3 is below rounding).
    P = SH(32, 0.35)
    dt = 0.02
    for (a, b, rate) in [(0, 8, 0.35), (8, 8, 0.35 - 1.0)]:
        c = np.zeros((32, 16), complex)
        c[a, b] = 1e-9
        X1, _ = imex.sbdf_forward(P, c.reshape(-1, 1), dt, 1)
        assert np.isclose(X1.reshape(32, 16)[a, b] / c[a, b], 1.0 / (1.0 - dt * rate), rtol=1e-12, atol=0)


def test_energy_is_parseval_of_a_single_mode():
    P = SH(16, 0.2)
    c = np.zeros((16, 8), complex)
    c[3, 2] = 0.4 - 0.3j
    # u = 2 Re(c e^{i k.x}) has mean square 2 |c|^2
    assert np.isclose(P.energy(c.reshape(-1, 1)), 0.5 * 2 * abs(c[3, 2]) ** 2, rtol=1e-13)
    X = 0.1 * rand_c(P, 2).reshape(-1, 1)
    d = rand_c(P, 3).reshape(-1, 1)
    eps = 1e-3
    fd = (P.energy(X + eps * d) - P.energy(X - eps * d)) / (2 * eps)     # exact: J is quadratic
    assert np.isclose(fd, np.real(np.vdot(P.energy_grad(X), d)), rtol=1e-10)


def test_F_vjp_inner_product_with_exact_difference():
    P = SH(12, 0.2, L=9.0)
    X = 0.5 * rand_c(P, 4).reshape(-1, 1)
    d = rand_c(P, 5).reshape(-1, 1)
    Yb = rand_c(P, 6).reshape(-1, 1)

    def D(e):
        return (P.F(X + e * d) - P.F(X - e * d)) / (2 * e)

    e = 1e-3
    Jd = (4 * D(e / 2) - D(e)) / 3      # exact for a cubic map (up to rounding)
    lhs = np.real(np.vdot(Yb, Jd))
    rhs = np.real(np.vdot(P.F_vjp(X, Yb), d))
    assert np.isclose(lhs, rhs, rtol=1e-9)


def gradient(P, u0, dt, n):
    X0 = P.initial_state(u0)
    XN, states = imex.sbdf_forward(P, X0, dt, n)
    g = imex.sbdf_adjoint(P, P.energy_grad(XN), states, dt)
    return P.energy(XN), P.initial_state_adjoint(g)


def test_gradient_brute_force_on_a_tiny_grid():
    P = SH(6, 0.4, L=7.0)
    dt, n = 0.05, 5
    u0 = np.random.default_rng(7).uniform(-0.5, 0.5, (6, 6))
    J0, g = gradient(P, u0, dt, n)
    eps = 1e-6
    fd = np.zeros_like(u0)
    for i in range(6):
        for j in range(6):
            e = np.zeros_like(u0)
            e[i, j] = eps
            fd[i, j] = (gradient(P, u0 + e, dt, n)[0] - gradient(P, u0 - e, dt, n)[0]) / (2 * eps)
    assert np.max(np.abs(fd - g)) < 1e-7 * np.max(np.abs(g))


def test_gradient_taylor_rate_two():
    P = SH(16, 0.3)
    dt, n = 0.02, 8
    rng = np.random.default_rng(8)
    u0 = rng.uniform(-0.1, 0.1, (16, 16))
    d = rng.standard_normal((16, 16))
    J0, g = gradient(P, u0, dt, n)
    gd = np.sum(g * d)
    es = [1e-2 / 2 ** i for i in range(4)]
    r = [abs(gradient(P, u0 + e * d, dt, n)[0] - J0 - e * gd) for e in es]
    rates = [np.log2(r[i] / r[i + 1]) for i in range(3)]
    assert all(abs(q - 2.0) < 0.05 for q in rates), rates
