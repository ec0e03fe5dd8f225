"""torch.autograd bindings (Step / InitialState / Cost) on the GPU: the gradient of
J(b0) = cost(step(initial_state(b0))) through backward() equals the library's own gradient
call and the oracle's (1e-11), matches central finite differences of the GPU forward map,
and shows the Taylor-remainder rate 2 that the paper uses to validate its adjoints."""
import numpy as np
import pytest

from oracle import imex
from oracle.ks import KS
from oracle.rbc import RBC
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402
from paper_2506_14792_amd import autograd as sa  # noqa: E402

RBC_CFG = (24, 16, 3.0, 1e5, 0.7, 2e-3)   # nx, nz, lx, Ra, Pr, dt
NSTEPS = 6


def rbc_problem():
    nx, nz, lx, Ra, Pr, dt = RBC_CFG
    return sps.Problem(sps.RBC2D, nx, nz, lx, Ra, Pr, 1.5, dt, 4, NSTEPS)


def rbc_J(G, b0):
    return sa.cost(sa.step(sa.initial_state(b0, G), G, NSTEPS), G)


def test_rbc_backward_matches_library_and_oracle():
    print("autograd RBC backward", flush=True)
    nx, nz, lx, Ra, Pr, dt = RBC_CFG
    G = rbc_problem()
    b0_np = wl.rbc_b0(seed=21, Nx=nx, Nz=nz, amp=0.1)
    b0 = torch.from_numpy(b0_np.copy()).cuda().requires_grad_(True)
    J = rbc_J(G, b0)
    (gb,) = torch.autograd.grad(J, b0)
    # the library's gradient call
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.initial_state(b0.detach(), X0)
    gX = torch.zeros_like(X0)
    J2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.gradient(X0, NSTEPS, None, gX, J2)
    gb2 = torch.zeros_like(b0)
    G.initial_state_adjoint(gX, gb2)
    G.sync()
    assert torch.equal(gb, gb2) and J.item() == J2.item()
    # the oracle
    P = RBC(Nx=nx, Nz=nz, Lx=lx, Ra=Ra, Pr=Pr)
    X0r = P.initial_state(b0_np)
    XN, hist = imex.rk_forward(P, X0r, dt, NSTEPS)
    gref = P.initial_state_adjoint(imex.rk_adjoint(P, P.kinetic_energy_grad(XN), hist, dt))
    got = gb.cpu().numpy()
    assert np.max(np.abs(got - gref)) / np.max(np.abs(gref)) < 1e-11


def test_rbc_finite_differences_and_taylor_rate():
    print("autograd RBC finite differences / Taylor", flush=True)
    nx, nz = RBC_CFG[:2]
    G = rbc_problem()
    b0 = torch.from_numpy(wl.rbc_b0(seed=22, Nx=nx, Nz=nz, amp=0.1).copy()).cuda().requires_grad_(True)
    J0 = rbc_J(G, b0)
    (g,) = torch.autograd.grad(J0, b0)
    d = torch.from_numpy(np.random.default_rng(23).standard_normal((nx, nz))).cuda()
    gd = torch.sum(g * d).item()

    def J(eps):
        with torch.no_grad():
            return rbc_J(G, b0.detach() + eps * d).item()

    eps = 1e-4
    fd = (J(eps) - J(-eps)) / (2 * eps)
    assert abs(fd - gd) < 1e-6 * abs(gd)
    # Taylor remainder |J(b + e d) - J(b) - e <g, d>| = O(e^2)
    j0 = J0.item()
    es = [1e-2 / 2 ** i for i in range(5)]
    r = [abs(J(e) - j0 - e * gd) for e in es]
    rates = [np.log(r[i] / r[i + 1]) / np.log(2.0) for i in range(len(r) - 1)]
    print("Taylor remainders", r, "rates", rates, flush=True)
    assert all(abs(q - 2.0) < 0.1 for q in rates)


def test_ks_backward_finite_differences():
    print("autograd KS", flush=True)
    P = KS()
    nsteps, dt = 50, 0.05
    G = sps.Problem(sps.KS1D, 64, 0, P.Lx, 0.0, 0.0, 1.5, dt, 1, nsteps)
    c0 = wl.ks_c0(seed=24)[:, None]
    X0 = torch.from_numpy(np.ascontiguousarray(c0).view(np.float64).ravel().copy()).cuda().requires_grad_(True)
    J = sa.cost(sa.step(X0, G, nsteps), G)
    (g,) = torch.autograd.grad(J, X0)
    XN, states = imex.sbdf_forward(P, c0, dt, nsteps)
    gref = imex.sbdf_adjoint(P, P.energy_grad(XN), states, dt)
    got = g.cpu().numpy().view(np.complex128).reshape(gref.shape)
    assert np.max(np.abs(got - gref)) / np.max(np.abs(gref)) < 1e-11
    d = torch.from_numpy(np.random.default_rng(25).standard_normal(G.n) * 1e-2).cuda()

    def Jf(eps):
        with torch.no_grad():
            return sa.cost(sa.step(X0.detach() + eps * d, G, nsteps), G).item()

    eps = 1e-3
    fd = (Jf(eps) - Jf(-eps)) / (2 * eps)
    gd = torch.sum(g * d).item()
    assert abs(fd - gd) < 1e-6 * abs(gd)


def test_backward_of_a_stale_forward_raises():
    print("autograd stale tape", flush=True)
    G = rbc_problem()
    nx, nz = RBC_CFG[:2]
    b0 = torch.from_numpy(wl.rbc_b0(seed=26, Nx=nx, Nz=nz).copy()).cuda().requires_grad_(True)
    J1 = rbc_J(G, b0)
    rbc_J(G, b0.detach())          # a second forward run replaces the recorded one
    with pytest.raises(sps.SpsError):
        torch.autograd.grad(J1, b0)
