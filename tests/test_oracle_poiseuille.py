"""Pins of the plane Poiseuille stability oracle (oracle/poiseuille.py) against values the
mathematics and the literature fix, not against itself:

* the Orr-Sommerfeld eigenvalue of Orszag (1971) at Re = 10^4, alpha = 1:
  c = 0.23752649 + 0.00373967 i (lambda = -i alpha c), to the 8 printed digits;
* the onset of instability, Re_c = 5772.22 at alpha_c = 1.02056 with phase speed
  c = 0.26400 (Orszag 1971): Newton on the growth rate with the adjoint sensitivity (the
  paper's neutral-curve procedure) lands there with a growth rate at rounding level;
* the eigenvalue sensitivities (equ:eigenvalue_sens) against central differences of the
  dense eigenvalue in Re and alpha;
* the left eigenvector solves the adjoint problem, and the exact base-flow products agree with
  a Chebyshev product evaluated pointwise.

A dropped base-flow term, a wrong sign of U' v or of the lifts, a transposed product or a
wrong derivative in the sensitivity moves one of these values far beyond its tolerance.
"""
import numpy as np
import pytest

from oracle.poiseuille import Poiseuille, mult_x


def test_orszag_eigenvalue():
    P = Poiseuille(80)
    lam, _, _ = P.eig(1.0, 1e4, 0.0037 - 0.2375j)
    c = 1j * lam / 1.0
    assert abs(c.real - 0.23752649) < 6e-9
    assert abs(c.imag - 0.00373967) < 6e-9


def test_onset_by_newton_with_the_adjoint_sensitivity():
    P = Poiseuille(80)
    Re, lam, solves, _ = P.neutral_Re(1.02056, 5000.0, -0.27j, tol=1e-12)
    assert abs(Re - 5772.22) < 0.01
    assert abs(lam.real) <= 1e-12
    assert abs((1j * lam / 1.02056).real - 0.26400) < 1e-5
    assert solves <= 6


def test_growth_rate_changes_sign_across_the_onset():
    P = Poiseuille(64)
    g_below = P.eig(1.02056, 5600.0, -0.27j)[0].real
    g_above = P.eig(1.02056, 6000.0, -0.27j)[0].real
    assert g_below < 0.0 < g_above


@pytest.mark.parametrize("alpha,Re", [(1.0, 6000.0), (0.8, 20000.0)])
def test_sensitivities_against_central_differences(alpha, Re):
    P = Poiseuille(64)
    lam, X, Y = P.eig(alpha, Re, -0.25j)
    dRe, dal = P.sensitivity(alpha, Re, X, Y)
    h = 1e-3 * Re
    fd_Re = (P.eig(alpha, Re + h, lam)[0] - P.eig(alpha, Re - h, lam)[0]) / (2 * h)
    h = 1e-5
    fd_al = (P.eig(alpha + h, Re, lam)[0] - P.eig(alpha - h, Re, lam)[0]) / (2 * h)
    assert abs(dRe - fd_Re) <= 1e-5 * abs(dRe)
    assert abs(dal - fd_al) <= 1e-6 * abs(dal)


def test_left_eigenvector_solves_the_adjoint_problem():
    P = Poiseuille(48)
    M, L = P.matrices(1.0, 8000.0)
    lam, X, Y = P.eig(1.0, 8000.0, -0.25j)
    r = (np.conj(lam) * M.conj().T + L.conj().T) @ Y
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(L) * np.linalg.norm(Y)
    assert np.linalg.norm((lam * M + L) @ X) <= 1e-10 * np.linalg.norm(L) * np.linalg.norm(X)


def test_base_flow_products_pointwise():
    """The C2 rows of U u and U' v are the exact products: converted back to values, the first
    N C2 coefficients of U u match (1 - x^2) u(x) up to the two dropped top modes, which vanish
    for a series of degree N - 3."""
    N = 12
    P = Poiseuille(N)
    rng = np.random.default_rng(4)
    a = np.zeros(N)
    a[:N - 2] = rng.standard_normal(N - 2)          # degree N - 3: the product has degree N - 1
    xs = np.linspace(-0.9, 0.9, 7)
    Tu = np.polynomial.chebyshev.chebval(xs, a)
    # C2 series from the T series of the exact product (via the T -> C2 conversion)
    def padN(c):
        return np.pad(c, (0, N))[:N]

    prod_T = padN(np.polynomial.chebyshev.chebmul(a, [0.5, 0.0, -0.5]))      # (1 - x^2) = T0/2 - T2/2
    np.testing.assert_allclose(P.SU @ a, P.S10 @ prod_T, atol=1e-14)
    np.testing.assert_allclose(np.polynomial.chebyshev.chebval(xs, prod_T), (1 - xs ** 2) * Tu, atol=1e-13)
    dprod_T = padN(np.polynomial.chebyshev.chebmul(a, [0.0, -2.0]))
    np.testing.assert_allclose(P.SdU @ a, P.S10 @ dprod_T, atol=1e-14)
    # multiplication by x against numpy's Chebyshev product
    np.testing.assert_allclose(mult_x(N) @ a, np.pad(np.polynomial.chebyshev.chebmulx(a), (0, N))[:N + 1], atol=1e-15)
