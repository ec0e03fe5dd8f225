"""GPU parity of the eigenvalue problem (Supplementary, "Eigenvalue problems") against the
oracle's dense generalized eigensolutions: the eigenvalue nearest the shift for every wavenumber
of the problem (inverse iteration through the blocked LU), the right and left eigenvectors (up
to a complex factor, compared by the alignment |<v_gpu, v_ref>| / (|v_gpu| |v_ref|) = 1), and the
sensitivities d lambda/dRa and d lambda/dk of equ:eigenvalue_sens; then Newton steps on the
GPU growth rate with the GPU sensitivity converge to the onset Ra = 1707.762 at k = 3.1163.
The shift-invert Arnoldi from the same seeded start vectors as the oracle's: the Arnoldi
matrix column by column, the converged Ritz values against the oracle's and the dense
eigenvalues nearest the shift (same order), the Ritz vectors by alignment, at 32 modes and at
the 256x64 configuration (sampled wavenumbers)."""
import sys

import numpy as np
import pytest

from oracle.rbc import RBC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402
import workloads as wl  # noqa: E402

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


def dense_nearest(P, k, sigma, count):
    import scipy.linalg as sla
    w = sla.eig(P.stability_operator()[k], -P.M[k], right=False)
    w = w[np.isfinite(w)]
    return w[np.argsort(np.abs(w - sigma), kind="stable")][:count]


def arnoldi_case(P, G, sigma, m, nev, seed, ks, h_tol=1e-12, unconverged=()):
    """Tolerances: the Arnoldi matrix carries rounding of order ulp |nu_0| (nu_0 the dominant
    eigenvalue of the shift-inverted operator), so lambda_i = sigma - 1/nu_i differs between two
    correctly rounded runs by about ulp |nu_0| / |nu_i|^2 on top of 1e-10 relative; near an
    eigenvalue (|nu_0| large) the early columns of H differ by a similar amount (h_tol)."""
    S = P.M[1].shape[0]
    v0 = wl.random_state(seed, (P.K, S))
    lam, X, res, H = G.stability_arnoldi(sigma, m=m, nev=nev, v0=torch.from_numpy(v0).cuda(), want_H=True)
    G.sync()
    lam, X, res, H = lam.cpu().numpy(), X.cpu().numpy(), res.cpu().numpy(), H.cpu().numpy()
    for k in unconverged:
        # far from the shift nothing converges in m steps: the Arnoldi matrices still agree,
        # the first columns to rounding, later ones within the growth that the division by
        # h_{j+1,j} at every step allows
        Hr = P.stability_arnoldi(k, sigma, v0[k], m)[4]
        e = [np.linalg.norm(H[k][:, j] - Hr[:, j]) / np.linalg.norm(Hr) for j in range(m)]
        note(f"  k {k}: H columns 0..3 {max(e[:4]):.1e}, all {max(e):.1e}")
        assert max(e[:4]) < 1e-12 and max(e) < 1e-8
    for k in ks:
        lr, Xr, rr, _, Hr = P.stability_arnoldi(k, sigma, v0[k], m)
        nu_r = 1.0 / (sigma - lr[:nev])
        conv = rr[:nev] < 1e-10 * np.abs(nu_r)
        nconv = int(np.argmin(conv)) if not conv.all() else nev
        assert nconv >= 3, (k, nconv)
        # Arnoldi matrix: equal while the Krylov space has not converged to rounding level
        ecol = [np.linalg.norm(H[k][:, j] - Hr[:, j]) / np.linalg.norm(Hr) for j in range(m)]
        tol = 1e-10 * np.maximum(np.abs(lr[:nconv]), 1.0) + 1e-14 * np.abs(nu_r[0]) / np.abs(nu_r[:nconv]) ** 2
        el = np.max(np.abs(lam[k, :nconv] - lr[:nconv]) / tol)
        ed = np.max(np.abs(lam[k, :nconv] - dense_nearest(P, k, sigma, nconv)) / tol)
        al = min(abs(np.vdot(X[k, i], Xr[:, i])) for i in range(nconv))
        note(f"  k {k}: {nconv} converged, lambda err/tol {el:.1e} (dense {ed:.1e}), align {al:.15f}, "
             f"H col 0 {ecol[0]:.1e}, cols 0..3 {max(ecol[:4]):.1e}, all {max(ecol):.1e}")
        assert nconv >= 3
        assert max(ecol[:4]) < h_tol
        assert el < 1.0 and ed < 10.0
        assert abs(al - 1.0) < 1e-9
        assert np.all(res[k, :nconv] < 1e-8 * np.abs(nu_r[:nconv]))
    return lam, X, res


@pytest.mark.parametrize("Ra,k,sigma,m", [(5000.0, 3.0, 0.05, 30), (3000.0, 2.5, -0.3, 24)], ids=["unstable", "stable"])
def test_arnoldi_vs_oracle(Ra, k, sigma, m):
    note(f"arnoldi Ra {Ra}, k {k}, sigma {sigma}, m {m}")
    P, G = build(Ra, nz=24, lx=2.0 * np.pi / k)
    arnoldi_case(P, G, sigma, m, 6, seed=31, ks=range(1, P.K))


def test_arnoldi_large_m_global_work_arrays():
    """m = 56: the Hessenberg kernel's eigenvector work arrays no longer fit in LDS beside H and
    Z (m >= 50) and live in global memory; same checks as the smaller cases."""
    note("arnoldi m = 56")
    P, G = build(5000.0, nz=32, lx=2.0 * np.pi / 3.0)
    arnoldi_case(P, G, 0.05, 56, 6, seed=34, ks=range(1, P.K))


def test_arnoldi_onset_and_inverse_iteration():
    note("arnoldi at the onset")
    P, G = build(RAC)
    lam, X, res = arnoldi_case(P, G, 0.0, 24, 4, seed=32, ks=[1], h_tol=1e-7)
    assert abs(lam[1, 0]) < 1e-6 and abs(lam[1, 0].imag) < 1e-12
    li, Xi, _, _ = G.stability(0.0, iters=60)
    G.sync()
    assert abs(lam[1, 0] - li[1].item()) < 1e-12
    # default start vector
    lam2, _, _, _ = G.stability_arnoldi(0.0, m=24, nev=2, want_vectors=False)
    G.sync()
    assert abs(lam2[1, 0].item() - lam[1, 0]) < 1e-12


def test_arnoldi_full_size_sampled():
    note("arnoldi 256x64, sampled wavenumbers")
    P = RBC(Nx=256, Nz=64, Lx=4.0, Ra=1e6, Pr=1.0)
    G = sps.Problem(sps.RBC2D, 256, 64, 4.0, 1e6, 1.0, 1.5, 1e-3, 1, 1)
    arnoldi_case(P, G, 0.0, 32, 8, seed=33, ks=[1, 7, 16, 24], unconverged=[64, 127])


def test_arnoldi_arguments():
    P, G = build(RAC)
    for m, nev in ((1, 1), (65, 4), (10, 11), (10, 0)):
        with pytest.raises(sps.SpsError) as e:
            G.stability_arnoldi(0.0, m=m, nev=nev)
        assert e.value.code == -1
    Gk = sps.Problem(sps.KS1D, 64, 0, 32.0 * np.pi, 0.0, 0.0, 1.5, 0.05, 1, 4)
    with pytest.raises(sps.SpsError) as e:
        Gk.stability_arnoldi(0.0, m=8, nev=2)
    assert e.value.code == -7


@pytest.mark.parametrize("Ra,sigma", [(RAC, 0.0), (5000.0, 0.27)], ids=["onset", "unstable"])
def test_eigenvector_sensitivities_vs_oracle(Ra, sigma):
    """equ:eigenvector_sens on the GPU (sps_stability_vector_sens, 60 projected iterations
    through the factors of sigma M + L_s) against the oracle's direct solution of the singular
    system with the same eigenvector X (the GPU's, so both use one normalization), on every
    wavenumber whose contraction factor |lambda - sigma| / min_j |lambda_j - sigma| (dense
    eigenvalues) is below 1/2."""
    import scipy.linalg as sla
    note(f"eigenvector sensitivities Ra = {Ra}, sigma = {sigma}")
    P, G = build(Ra)
    lam, X, Y, dl = G.stability(sigma, iters=60)
    dX = G.stability_vector_sens(sigma, lam, X, Y, dl, iters=60)
    G.sync()
    lam, X, dX = lam.cpu().numpy(), X.cpu().numpy(), dX.cpu().numpy()
    checked = 0
    for k in range(1, P.K):
        w = sla.eig(P.stability_operator()[k], -P.M[k], right=False)
        w = np.sort_complex(w[np.isfinite(w)])
        i0 = np.argmin(np.abs(w - lam[k]))
        q = abs(lam[k] - sigma) / np.min(np.abs(np.delete(w, i0) - sigma))
        lr, _, Yr = P.stability_eig(k, sigma)
        Z = P.stability_vector_sensitivity(k, lr, X[k], Yr)
        e = [np.linalg.norm(dX[p, k] - Z[:, p]) / np.linalg.norm(Z[:, p]) for p in range(2)]
        note(f"  k {k}: contraction {q:.2e}, dX/dRa rel {e[0]:.1e}, dX/dk rel {e[1]:.1e}, "
             f"<X, dX> {abs(np.vdot(X[k], dX[0, k])):.1e}")
        if q < 0.5:
            assert max(e) < 1e-9
            checked += 1
    assert checked >= 1
