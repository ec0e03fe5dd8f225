"""GPU checks of step-size changes between runs (sps_set_dt; equ:imex, the implicit matrices
depend on the step): the 2D problem refactors M + dt gamma L of every wavenumber, and a run of
two segments with different steps, and the gradient through it by torch.autograd
(StepSegments: each segment reversed after sps_set_dt of its own step and a recomputation of
its forward sweep), match the oracle's chained RK222 sweeps and adjoints (1e-11) at 24x16 and
the full 256x64 configuration (Taylor remainder rate 2 there); returning to a step gives runs
bit-identical to a problem built with it, for the 2D problem and plane Couette; KS takes the new
step in its SBDF rows and RK stages; the batched Swift-Hohenberg and Kolmogorov problems in their
SBDF2 coefficients."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import imex
from oracle.ks import KS
from oracle.rbc import RBC
from parity import check_fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402
from paper_2506_14792_amd import autograd as sa  # noqa: E402

SMALL = (24, 16, 3.0, 1e5, 0.7, 2e-3)
TOL = 1e-11


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(X).view(np.float64).ravel().copy()).cuda()


def from_dev(t, shape):
    return t.detach().cpu().numpy().view(np.complex128).reshape(shape)


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def small(max_steps):
    nx, nz, lx, Ra, Pr, dt = SMALL
    P = RBC(Nx=nx, Nz=nz, Lx=lx, Ra=Ra, Pr=Pr)
    G = sps.Problem(sps.RBC2D, nx, nz, lx, Ra, Pr, 1.5, dt, 2, max_steps)
    X0 = P.initial_state(wl.rbc_b0(seed=6, Nx=nx, Nz=nz, amp=0.2))
    return P, G, X0


def test_two_segments_forward_and_gradient_vs_oracle():
    segs = [(2e-3, 5), (3.1e-3, 7), (1.3e-3, 4)]
    note(f"2D problem 24x16, segments {segs}")
    P, G, X0h = small(max_steps=8)
    X = X0h
    hists = []
    for dt, n in segs:
        X, h = imex.rk_forward(P, X, dt, n)
        hists.append((dt, h))
    XN_ref = X
    g_ref = P.kinetic_energy_grad(XN_ref)
    J_ref = P.kinetic_energy(XN_ref)
    for dt, h in reversed(hists):
        g_ref = imex.rk_adjoint(P, g_ref, h, dt)
    X0 = to_dev(X0h).requires_grad_(True)
    XN = sa.step_segments(X0, G, segs)
    J = sa.cost(XN, G)
    (g,) = torch.autograd.grad(J, X0)
    G.sync()
    base = P.lbvp_solve(np.zeros((P.K, P.S), complex))
    ex = check_fields(from_dev(XN, XN_ref.shape), XN_ref, P.Nz, TOL, base=base, what="X_N")
    eg = check_fields(from_dev(g, g_ref.shape), g_ref, P.Nz, TOL, what="dJ/dX0")
    note(f"  XN rel {ex:.1e}, J rel {abs(J.item() - J_ref) / J_ref:.1e}, dJ/dX0 rel {eg:.1e}")
    assert abs(J.item() - J_ref) < TOL * J_ref
    # the recorded run was dropped by the change of step
    G.set_dt(2e-3)
    with pytest.raises(sps.SpsError) as e:
        G.adjoint_step(torch.zeros(G.n, dtype=torch.float64, device="cuda"), 4)
    assert e.value.code == -6
    # sps_solve applies the matrix of the new step
    G.set_dt(3.1e-3)
    R = wl.random_state(3, X0h.shape)
    out = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.solve(to_dev(R), out)
    G.sync()
    lu = imex.BlockLU(P.M, P.L, 1.0, 3.1e-3 * (1.0 - 1.0 / np.sqrt(2.0)))
    check_fields(from_dev(out, R.shape), lu.solve(R), P.Nz, TOL, what="solve after set_dt")


def test_return_to_a_step_is_bit_identical_to_a_fresh_problem():
    note("set_dt round trip, 2D problem and Couette")
    P, G, X0h = small(max_steps=6)
    nx, nz, lx, Ra, Pr, dt = SMALL
    Gf = sps.Problem(sps.RBC2D, nx, nz, lx, Ra, Pr, 1.5, 2.5e-3, 2, 6)
    G.set_dt(4e-3)
    G.set_dt(2.5e-3)
    outs = []
    for H in (G, Gf):
        XN = torch.zeros(H.n, dtype=torch.float64, device="cuda")
        g = torch.zeros_like(XN)
        J = torch.zeros(1, dtype=torch.float64, device="cuda")
        H.gradient(to_dev(X0h), 6, XN, g, J)
        H.sync()
        outs.append((XN, g, J))
    assert all(torch.equal(a, b) for a, b in zip(*outs))
    Gc = sps.Couette(8, 12, 8, Re=400.0, dt=0.01, checkpoint_every=2, max_steps=5)
    Gc2 = sps.Couette(8, 12, 8, Re=400.0, dt=0.015, checkpoint_every=2, max_steps=5)
    uvw = wl.couette_perturbation(seed=3, Nx=8, Ny=12, Nz=8, energy=1e-3)
    X0 = Gc.state_from_velocity(uvw)
    Gc.set_dt(0.015)
    res = []
    for H in (Gc, Gc2):
        XN = torch.zeros_like(X0)
        g = torch.zeros_like(X0)
        J = torch.zeros(1, dtype=torch.float64, device="cuda")
        H.gradient(X0, 5, XN, g, J)
        H.sync()
        res.append((XN, g, J))
    assert all(torch.equal(a, b) for a, b in zip(*res))


def test_full_size_segments_taylor():
    """256x64, three segments of 100, 150 and 50 steps at dt = 1e-3, 1.5e-3, 0.7e-3 (checkpoints
    every 50), differentiated with respect to the initial buoyancy grid: the Taylor remainder
    |J(b0 + e d) - J - e <g, d>| of the autograd gradient falls at rate 2, with J from GPU runs."""
    note("256x64 segments, Taylor test")
    G = sps.Problem(sps.RBC2D, 256, 64, 4.0, 1e6, 1.0, 1.5, 1e-3, 50, 150)
    segs = [(1e-3, 100), (1.5e-3, 150), (0.7e-3, 50)]

    def J_of(b):
        return sa.cost(sa.step_segments(sa.initial_state(b, G), G, segs), G)

    b0 = torch.from_numpy(wl.rbc_b0(seed=0, Nx=256, Nz=64).copy()).cuda().requires_grad_(True)
    J = J_of(b0)
    (g,) = torch.autograd.grad(J, b0)
    G.sync()
    d = torch.from_numpy(np.random.default_rng(24).standard_normal((256, 64))).cuda()
    gd = torch.sum(g * d).item()
    J0 = J.item()
    rem = []
    for e in (1e-2, 5e-3, 2.5e-3, 1.25e-3):
        with torch.no_grad():
            rem.append(abs(J_of(b0.detach() + e * d).item() - J0 - e * gd))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    note(f"  J {J0:.6e}, <g, d> {gd:.6e}, remainders {rem}, rates {rates}")
    assert np.all(np.abs(rates - 2.0) < 0.1)


@pytest.mark.parametrize("scheme", ["sbdf2", "rk443"])
def test_ks_set_dt(scheme):
    note(f"KS {scheme} set_dt")
    P = KS()
    code = {"sbdf2": sps.SBDF2, "rk443": sps.RK443}[scheme]
    G = sps.Problem(sps.KS1D, 64, 0, P.Lx, 0.0, 0.0, 1.5, 0.05, 1, 100, scheme=code)
    G.set_dt(0.03)
    X0 = wl.ks_c0(seed=22, amp=0.5)[:, None]
    XN = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    g = torch.zeros_like(XN)
    G.gradient(to_dev(X0), 100, XN, g, None)
    G.sync()
    if scheme == "sbdf2":
        XN_ref, states = imex.sbdf_forward(P, X0, 0.03, 100)
        g_ref = imex.sbdf_adjoint(P, P.energy_grad(XN_ref), states, 0.03)
    else:
        tab = imex.ars443_tableau()
        XN_ref, hist = imex.rk_forward(P, X0, 0.03, 100, tableau=tab)
        g_ref = imex.rk_adjoint(P, P.energy_grad(XN_ref), hist, 0.03, tableau=tab)
    assert rel(from_dev(XN, XN_ref.shape), XN_ref) < TOL and rel(from_dev(g, g_ref.shape), g_ref) < TOL


def test_set_dt_arguments():
    P, G, _ = small(max_steps=2)
    for bad in (0.0, -1e-3, float("nan"), float("inf")):
        with pytest.raises(sps.SpsError) as e:
            G.set_dt(bad)
        assert e.value.code == -1


def test_batched_problems_set_dt():
    """The batched Swift-Hohenberg and Kolmogorov problems after sps_set_dt match problems built
    with the new step: SH gradients within 1e-12 (the two builds may tune different tiles),
    Kolmogorov forward runs and reverse sweeps bit-identical."""
    note("set_dt on the batched problems")
    sizes, rs, u0 = wl.sh_batch(seed=0, batch=3, sizes=(64, 96))
    grid = torch.from_numpy(np.concatenate([u.ravel() for u in u0])).cuda()
    outs = []
    for dt0 in (0.02, 0.01):
        B = sps.ShBatch(sizes, rs, 16.0 * np.pi, dt0, max_steps=20)
        if dt0 != 0.01:
            B.set_dt(0.01)
        X0 = torch.zeros(B.n, dtype=torch.float64, device="cuda")
        B.initial_state(grid, X0)
        g = torch.zeros_like(X0)
        XN = torch.zeros_like(X0)
        J = torch.zeros(len(sizes), dtype=torch.float64, device="cuda")
        B.gradient(X0, 20, XN, g, J)
        B.sync()
        outs.append((XN, g, J))
    for a, b in zip(*outs):
        assert (a - b).abs().max().item() <= 1e-12 * b.abs().max().item()
    c0 = wl.kolmo_vorticity(seed=1, N=16, batch=2)
    Yb = wl.kolmo_vorticity(seed=5, N=16, batch=2)
    res = []
    for dt0 in (0.02, 0.005):
        G = sps.Kolmogorov(2, 16, Re=1000.0, dt=dt0, max_steps=8, closure=False, keep_history=True)
        if dt0 != 0.005:
            G.set_dt(0.005)
        # device layout X[b][m][iy] from the coefficient arrays c[iy, m]
        X = torch.from_numpy(np.concatenate([np.ascontiguousarray(c.T).view(np.float64).ravel() for c in c0])).cuda()
        G.step(X, 8)
        Xb = torch.from_numpy(np.concatenate([np.ascontiguousarray(c.T).view(np.float64).ravel() for c in Yb])).cuda()
        G.adjoint_step(Xb, 8)
        G.sync()
        res.append((X, Xb))
    assert all(torch.equal(a, b) for a, b in zip(*res))


def test_ks_step_segments_autograd():
    """KS with RK443 in two segments of different steps (0.05 x 40, then 0.03 x 60) through
    torch.autograd (StepSegments, Cost) against the oracle's chained RK443 sweeps and adjoints."""
    note("KS rk443 step segments through autograd")
    P = KS()
    tab = imex.ars443_tableau()
    G = sps.Problem(sps.KS1D, 64, 0, P.Lx, 0.0, 0.0, 1.5, 0.05, 1, 60, scheme=sps.RK443)
    segs = [(0.05, 40), (0.03, 60)]
    X0h = wl.ks_c0(seed=24, amp=0.5)[:, None]
    X, hists = X0h, []
    for dt, n in segs:
        X, h = imex.rk_forward(P, X, dt, n, tableau=tab)
        hists.append((dt, h))
    g_ref = P.energy_grad(X)
    J_ref = P.energy(X)
    for dt, h in reversed(hists):
        g_ref = imex.rk_adjoint(P, g_ref, h, dt, tableau=tab)
    X0 = to_dev(X0h).requires_grad_(True)
    J = sa.cost(sa.step_segments(X0, G, segs), G)
    (g,) = torch.autograd.grad(J, X0)
    G.sync()
    eg = rel(from_dev(g, g_ref.shape), g_ref)
    note(f"  J rel {abs(J.item() - J_ref) / J_ref:.1e}, dJ/dX0 rel {eg:.1e}")
    assert abs(J.item() - J_ref) < TOL * J_ref and eg < TOL
