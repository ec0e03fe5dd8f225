"""Pins of the Kolmogorov-flow oracle (with and without the closure): the laminar Kolmogorov
state is steady, the advection of a two-mode field equals its closed form, the advection
conserves enstrophy and energy, the F-VJP passes the inner-product test against exact
differences, and the rollout-loss gradients with respect to the initial vorticity and the
closure parameters match brute-force central differences and show the Taylor rate 2."""
import numpy as np
import pytest

from oracle import closure as cl
from oracle import imex
from oracle.kolmo import Kolmogorov, rollout_loss_and_gradients


def coeffs(P, fn):
    x = np.arange(P.N) * P.Lx / P.N
    X, Y = np.meshgrid(x, x)
    return P.T.from_grid(fn(X, Y), P.N)


@pytest.mark.parametrize("drag", [0.0, 0.1])
def test_laminar_kolmogorov_state_is_steady(drag):
    # nu Laplacian omega - drag omega = 4 cos 4y  ->  omega = -4 cos(4y) / (16 nu + drag)
    P = Kolmogorov(16, Re=40.0, drag=drag)
    lam = coeffs(P, lambda x, y: -4.0 * np.cos(4 * y) / (16.0 * P.nu + drag)).reshape(-1, 1)
    assert np.max(np.abs(P.F(lam) - P.f.reshape(-1, 1))) < 1e-12 * np.max(np.abs(lam))
    X1, _ = imex.sbdf_forward(P, lam, 0.05, 3)
    assert np.max(np.abs(X1 - lam)) < 1e-12 * np.max(np.abs(lam))


def test_advection_of_two_modes_closed_form():
    # omega = cos x + cos 2y: psi = cos x + cos(2y)/4, u.grad omega = -(3/2) sin x sin 2y
    P = Kolmogorov(16)
    c = coeffs(P, lambda x, y: np.cos(x) + np.cos(2 * y))
    ref = coeffs(P, lambda x, y: 1.5 * np.sin(x) * np.sin(2 * y))
    assert np.max(np.abs(P.advection(c) - ref)) < 1e-14


def test_advection_conserves_enstrophy_and_energy():
    P = Kolmogorov(16)
    rng = np.random.default_rng(0)
    c = P.T.from_grid(rng.standard_normal((16, 16)), 16)
    a = P.advection(c)
    x = np.arange(16) * P.Lx / 16
    om = P.T.to_grid(c, 16)
    ad = P.T.to_grid(a, 16)
    psi = P.T.to_grid(c * P.inv_k2, 16)
    assert abs(np.mean(om * ad)) < 1e-13 * np.mean(om * om)
    assert abs(np.mean(psi * ad)) < 1e-13 * np.sqrt(np.mean(psi * psi) * np.mean(ad * ad))


def test_F_vjp_inner_product_with_closure():
    P = Kolmogorov(12, params=cl.init_params(seed=1, C=3, scale=3.0), bf=False)
    P.params["w3"] *= 100.0
    rng = np.random.default_rng(2)
    X = P.T.from_grid(rng.standard_normal((12, 12)), 12).reshape(-1, 1)
    d = P.T.from_grid(rng.standard_normal((12, 12)), 12).reshape(-1, 1)
    Yb = P.T.from_grid(rng.standard_normal((12, 12)), 12).reshape(-1, 1)

    def D(e):
        return (P.F(X + e * d) - P.F(X - e * d)) / (2 * e)

    Jd = (4 * D(5e-4) - D(1e-3)) / 3
    lhs = np.real(np.vdot(Yb, Jd))
    rhs = np.real(np.vdot(P.F_vjp(X, Yb), d))
    assert np.isclose(lhs, rhs, rtol=1e-7)


def _setup_tiny():
    P = Kolmogorov(10, Re=50.0, params=cl.init_params(seed=3, C=2, scale=2.0), bf=False)
    P.params["w3"] *= 50.0
    rng = np.random.default_rng(4)
    X0 = P.T.from_grid(rng.standard_normal((10, 10)), 10).reshape(-1, 1)
    targets = [P.T.from_grid(rng.standard_normal((10, 10)), 10).reshape(-1, 1) for _ in range(4)]
    return P, X0, targets


def test_rollout_gradients_brute_force():
    P, X0, targets = _setup_tiny()
    dt, n = 0.05, 4
    J, g0, gp, _ = rollout_loss_and_gradients(P, X0, targets, dt, n)

    def Jof(X, params):
        Q = Kolmogorov(10, Re=50.0, params=params, bf=False)
        return rollout_loss_and_gradients(Q, X, targets, dt, n)[0]

    h = 1e-6
    # initial vorticity through its grid values
    u0 = P.T.to_grid(X0.reshape(10, 5), 10)
    gu = P.T.to_grid(g0.reshape(10, 5), 10, weighted=False) / 100.0
    for idx in [(0, 0), (3, 7), (9, 2)]:
        e = np.zeros_like(u0)
        e[idx] = h
        fd = (Jof(P.T.from_grid(u0 + e, 10).reshape(-1, 1), P.params)
              - Jof(P.T.from_grid(u0 - e, 10).reshape(-1, 1), P.params)) / (2 * h)
        assert np.isclose(fd, gu[idx], rtol=1e-6, atol=1e-12)
    theta = cl.flatten(P.params)
    for i in [0, 5, 17, 20, 40, theta.size - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (Jof(X0, cl.unflatten(tp, C=2)) - Jof(X0, cl.unflatten(tm, C=2))) / (2 * h)
        assert np.isclose(fd, gp[i], rtol=1e-6, atol=1e-12), i


def test_rollout_gradient_taylor_rate():
    P, X0, targets = _setup_tiny()
    dt, n = 0.05, 4
    J0, g0, gp, _ = rollout_loss_and_gradients(P, X0, targets, dt, n)
    theta = cl.flatten(P.params)
    d = np.random.default_rng(5).standard_normal(theta.size)
    gd = float(gp @ d)
    es = [1e-2 / 2 ** i for i in range(4)]
    r = []
    for e in es:
        Q = Kolmogorov(10, Re=50.0, params=cl.unflatten(theta + e * d, C=2), bf=False)
        r.append(abs(rollout_loss_and_gradients(Q, X0, targets, dt, n)[0] - J0 - e * gd))
    rates = [np.log2(r[i] / r[i + 1]) for i in range(3)]
    assert all(abs(q - 2.0) < 0.1 for q in rates), rates
