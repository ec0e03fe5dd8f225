"""Pins of the ultraspherical operators ("Sparse spectral methods") against library
evaluations of the Chebyshev and Gegenbauer polynomials at random points."""
import numpy as np
import numpy.polynomial.chebyshev as npc
import numpy.polynomial.legendre as npl
import scipy.special as ss
import pytest

from oracle import spectral as sp

RNG = np.random.default_rng(99)
N = 14
XS = RNG.uniform(-1, 1, 25)


def U_series(b, x):
    return sum(bn * ss.eval_chebyu(n, x) for n, bn in enumerate(b))


def C2_series(c, x):
    return sum(cn * ss.eval_gegenbauer(n, 2.0, x) for n, cn in enumerate(c))


def T_series(a, x):
    return npc.chebval(x, a)


def test_S0_converts_T_to_U():
    a = RNG.standard_normal(N)
    assert np.allclose(U_series(sp.S0(N) @ a, XS), T_series(a, XS), rtol=0, atol=1e-12)


def test_S1_converts_U_to_C2():
    b = RNG.standard_normal(N)
    assert np.allclose(C2_series(sp.S1(N) @ b, XS), U_series(b, XS), rtol=0, atol=1e-12)


def test_D0_differentiates_T_into_U():
    a = RNG.standard_normal(N)
    ref = npc.chebval(XS, npc.chebder(a))
    assert np.allclose(U_series(sp.D0(N) @ a, XS), ref, rtol=0, atol=1e-10)


def test_D1_differentiates_U_into_C2():
    b = RNG.standard_normal(N)
    ref = sum(bn * np.polyder(ss.chebyu(n))(XS) for n, bn in enumerate(b))
    assert np.allclose(C2_series(sp.D1(N) @ b, XS), ref, rtol=0, atol=1e-9)


def test_T_derivative_matches_chebder():
    a = RNG.standard_normal(N)
    d = sp.cheb_derivative_T(N) @ a
    ref = npc.chebder(a)
    assert np.allclose(d[:N - 1], ref, rtol=0, atol=1e-12) and d[N - 1] == 0.0


def test_boundary_and_integral_rows():
    a = RNG.standard_normal(N)
    assert abs(sp.boundary_row(N, -1) @ a - npc.chebval(-1.0, a)) < 1e-12
    assert abs(sp.boundary_row(N, +1) @ a - npc.chebval(1.0, a)) < 1e-12
    # int_0^1 of the series in z = (x + 1)/2
    ia = npc.chebint(a)
    ref = 0.5 * (npc.chebval(1.0, ia) - npc.chebval(-1.0, ia))
    assert abs(sp.integral_row(N, 0.0, 1.0) @ a - ref) < 1e-12


def test_gram_matches_quadrature():
    xq, wq = npl.leggauss(2 * N + 4)
    T = sp.chebyshev_T(N, xq)
    ref = 0.5 * (T.T * wq) @ T        # int_0^1 dz = 1/2 int_{-1}^{1} dx
    assert np.max(np.abs(sp.gram_T(N, 0.0, 1.0) - ref)) < 1e-14


@pytest.mark.parametrize("lam_lift", [1])
def test_lift_derivative_factor(lam_lift):
    """d/dz of U_{N-1}(2z - 1) equals 4 C2_{N-2}(2z - 1) (the lifted tau coefficient)."""
    z = (XS + 1) / 2
    h = 1e-6
    fd = (ss.eval_chebyu(N - 1, 2 * (z + h) - 1) - ss.eval_chebyu(N - 1, 2 * (z - h) - 1)) / (2 * h)
    assert np.allclose(fd, 4.0 * ss.eval_gegenbauer(N - 2, 2.0, XS), rtol=1e-6, atol=1e-5)
