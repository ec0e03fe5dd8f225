"""GPU parity of the eigenvalue problem (Supplementary, "Eigenvalue problems") against the
oracle's dense generalized eigensolutions: the eigenvalue nearest the shift for every wavenumber
of the problem (inverse iteration through the blocked LU), the right and left eigenvectors (up
to a complex factor, compared by the alignment |<v_gpu, v_ref>| / (|v_gpu| |v_ref|) = 1), and the
sensitivities d lambda/dRa and d lambda/dk of equ:eigenvalue_sens; then Newton steps on the
GPU growth rate with the GPU sensitivity converge to the onset Ra = 1707.762 at k = 3.1163."""
import sys

import numpy as np
import pytest

from oracle.rbc import RBC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402

KC, RAC = 3.1163, 1707.762


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def build(Ra, nz=32, nx=8, lx=2.0 * np.pi / KC, Pr=1.0):
    P = RBC(Nx=nx, Nz=nz, Lx=lx, Ra=Ra, Pr=Pr)
    G = sps.Problem(sps.RBC2D, nx, nz, lx, Ra, Pr, 1.5, 1e-3, 1, 1)
    return P, G


def align(a, b):
    return abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))


@pytest.mark.parametrize("Ra,sigma", [(RAC, 0.0), (5000.0, 0.05)], ids=["onset", "unstable"])
def test_eigenpairs_and_sensitivities_vs_oracle(Ra, sigma):
    note(f"stability Ra = {Ra}, sigma = {sigma}")
    P, G = build(Ra)
    lam, X, Y, dl = G.stability(sigma, iters=60)
    G.sync()
    lam, X, Y, dl = lam.cpu().numpy(), X.cpu().numpy(), Y.cpu().numpy(), dl.cpu().numpy()
    for k in range(1, P.K):
        lr, Xr, Yr = P.stability_eig(k, sigma)
        dRa, dk = P.stability_sensitivity(k, lr, Xr, Yr)
        el = abs(lam[k] - lr) / max(abs(lr), 1e-3)
        ax, ay = align(X[k], Xr), align(Y[k], Yr)
        es = max(abs(dl[k, 0] - dRa) / abs(dRa), abs(dl[k, 1] - dk) / max(abs(dk), 1e-6))
        note(f"  k {k}: lambda {lam[k]:.10e} vs {lr:.10e} (rel {el:.1e}); align X {ax:.15f} Y {ay:.15f}; "
             f"sensitivities rel {es:.1e}")
        assert el < 1e-10
        assert abs(ax - 1.0) < 1e-10 and abs(ay - 1.0) < 1e-10
        assert es < 1e-8


def test_newton_on_gpu_growth_rate_finds_the_onset():
    note("Newton on the GPU growth rate")
    Ra = 1500.0
    for it in range(8):
        P, G = build(Ra)
        lam, X, Y, dl = G.stability(0.0, iters=40)
        G.sync()
        g, dg = lam[1].item(), dl[1, 0].item()
        note(f"  Ra {Ra:.9f}: growth {g.real:.3e}")
        Ra -= g.real / dg.real
    assert abs(Ra - RAC) < 2e-3 and abs(g.imag) < 1e-12


def test_stability_unsupported_for_other_problems():
    G = sps.Problem(sps.KS1D, 64, 0, 32.0 * np.pi, 0.0, 0.0, 1.5, 0.05, 1, 4)
    with pytest.raises(sps.SpsError) as e:
        G.stability(0.0, 5)
    assert e.value.code == -7
