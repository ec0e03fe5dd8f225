"""The 2D problem under the third-order ARS(4,4,3) IMEX scheme (four implicit stages, implicit
diagonal 1/2) against the FP64 oracle's rk_forward / rk_adjoint with the same tableau, called
through the C ABI: the forward run, J, dJ/dX0 and the gradient on the b0 grid (ragged checkpoint
segments, three and more segments, the 128 x 32 and 256 x 64 grid-row kernels), the parameter
gradient dJ/dRa, dJ/dPr, the implicit matrix M + dt/2 L of sps_solve, a step change by
sps_set_dt, the binomial and two-level schedules (the same bits as the uniform one), graph
replay, and a batch of Rayleigh numbers.  Bounds: tests/parity.py, 1e-11 of each field group."""
import sys

import numpy as np
import pytest

from oracle import imex
from oracle.imex import BlockLU
from oracle.rbc import RBC
import workloads as wl
from parity import check_fields

pytestmark = pytest.mark.gpu

TOL = 1e-11

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402

SMALL = (24, 16, 3.0, 1e5, 0.7, 2e-3)
MID = (128, 32, 4.0, 1e6, 1.0, 1e-3)
FULL = (256, 64, 4.0, 1e6, 1.0, 1e-3)
TAB = imex.ars443_tableau()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(X).view(np.float64).ravel().copy()).cuda()


def from_dev(t, shape):
    return t.cpu().numpy().view(np.complex128).reshape(shape)


def build(cfg, ce=1, max_steps=1):
    nx, nz, lx, Ra, Pr, dt = cfg
    P = RBC(Nx=nx, Nz=nz, Lx=lx, Ra=Ra, Pr=Pr)
    G = sps.Problem(sps.RBC2D, nx, nz, lx, Ra, Pr, 1.5, dt, ce, max_steps, scheme=sps.RK443)
    return P, G


def conduction(P):
    return P.lbvp_solve(np.zeros((P.K, P.S), complex))


def test_scheme_accepted_and_implicit_matrix():
    """sps_solve's matrix under RK443 is M + dt/2 L (forward and transposed solves)."""
    note("RK443 implicit matrix")
    cfg = SMALL
    P, G = build(cfg)
    rng = np.random.default_rng(3)
    R = rng.standard_normal((P.K, P.S)) + 1j * rng.standard_normal((P.K, P.S))
    lu = BlockLU(P.M, P.L, 1.0, 0.5 * cfg[5])
    X = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.solve(to_dev(R), X, adjoint=False)
    G.sync()
    ref = lu.solve(R)
    assert np.max(np.abs(from_dev(X, R.shape) - ref)) <= TOL * np.max(np.abs(ref))
    G.solve(to_dev(R), X, adjoint=True)
    G.sync()
    ref = lu.solve_adjoint(R)
    assert np.max(np.abs(from_dev(X, R.shape) - ref)) <= TOL * np.max(np.abs(ref))


@pytest.mark.parametrize("cfg,nsteps", [(SMALL, 6), (FULL, 3)], ids=["small", "full"])
def test_forward_steps(cfg, nsteps):
    note(f"RK443 forward {cfg} x {nsteps}")
    P, G = build(cfg, ce=2, max_steps=nsteps)
    X0 = P.initial_state(wl.rbc_b0(seed=21, Nx=cfg[0], Nz=cfg[1], amp=0.1))
    X = to_dev(X0)
    G.step(X, nsteps)
    G.sync()
    XN, _ = imex.rk_forward(P, X0, cfg[5], nsteps, tableau=TAB)
    check_fields(from_dev(X, X0.shape), XN, P.Nz, TOL, base=conduction(P), what="X_N")


@pytest.mark.parametrize("cfg,nsteps,ce", [(SMALL, 7, 3), (MID, 5, 2), (FULL, 5, 2)], ids=["small", "mid", "full"])
def test_gradient(cfg, nsteps, ce):
    note(f"RK443 gradient {cfg} x {nsteps} ce={ce}")
    P, G = build(cfg, ce=ce, max_steps=nsteps)
    b0 = wl.rbc_b0(seed=22, Nx=cfg[0], Nz=cfg[1], amp=0.1)
    X0 = P.initial_state(b0)
    XN_ref, hist = imex.rk_forward(P, X0, cfg[5], nsteps, tableau=TAB)
    J_ref = P.kinetic_energy(XN_ref)
    g_ref = imex.rk_adjoint(P, P.kinetic_energy_grad(XN_ref), hist, cfg[5], tableau=TAB)
    XN = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    g = torch.zeros_like(XN)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.gradient(to_dev(X0), nsteps, XN, g, J)
    G.sync()
    check_fields(from_dev(XN, X0.shape), XN_ref, P.Nz, TOL, base=conduction(P), what="X_N")
    eJ = abs(J.item() - J_ref) / abs(J_ref)
    note(f"  J rel {eJ:.1e}")
    assert eJ <= TOL
    check_fields(from_dev(g, X0.shape), g_ref, P.Nz, TOL, what="dJ/dX0")
    gb = torch.zeros(b0.size, dtype=torch.float64, device="cuda")
    G.initial_state_adjoint(g, gb)
    G.sync()
    ref = P.initial_state_adjoint(g_ref)
    assert np.max(np.abs(gb.cpu().numpy().reshape(b0.shape) - ref)) <= TOL * np.max(np.abs(ref))


def test_parameter_gradient_and_schedules():
    """dJ/dRa, dJ/dPr under RK443 (three checkpoint segments) against the oracle's; the binomial
    and two-level schedules and graph replay give the uniform schedule's dJ/dX0 bit for bit."""
    cfg, nsteps, ce = SMALL, 7, 3
    note(f"RK443 parameter gradient and schedules {cfg} x {nsteps} ce={ce}")
    P, G = build(cfg, ce=ce, max_steps=nsteps)
    X0 = P.initial_state(wl.rbc_b0(seed=23, Nx=cfg[0], Nz=cfg[1], amp=0.1))
    XN_ref, hist = imex.rk_forward(P, X0, cfg[5], nsteps, tableau=TAB)
    g_ref, th_ref = imex.rk_adjoint(P, P.kinetic_energy_grad(XN_ref), hist, cfg[5], tableau=TAB,
                                    dLs=P.param_dL(), XN=XN_ref)
    x0 = to_dev(X0)
    g = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    th = torch.zeros(2, dtype=torch.float64, device="cuda")
    G.gradient(x0, nsteps, None, g, None, dJdtheta=th)
    G.sync()
    check_fields(from_dev(g, X0.shape), g_ref, P.Nz, TOL, what="dJ/dX0")
    t = th.cpu().numpy()
    e = np.abs(t - th_ref) / np.abs(th_ref)
    note(f"  dJ/dRa {t[0]:.15e} vs {th_ref[0]:.15e} ({e[0]:.1e}); dJ/dPr {t[1]:.15e} vs {th_ref[1]:.15e} ({e[1]:.1e})")
    assert np.all(e <= TOL)
    G.set_graph(True)
    for _ in range(2):
        g2 = torch.zeros_like(g)
        G.gradient(x0, nsteps, None, g2, None)
        G.sync()
        assert torch.equal(g2, g)
    G.set_graph(False)
    for scheme, slots in ((sps.CKPT_BINOMIAL, 2), (sps.CKPT_TWO_LEVEL, 2)):
        G.set_checkpointing(scheme, slots)
        g2 = torch.zeros_like(g)
        G.gradient(x0, nsteps, None, g2, None)
        G.sync()
        note(f"  schedule {scheme} with {slots} slots: bit-identical {torch.equal(g2, g)}")
        assert torch.equal(g2, g)
    G.set_checkpointing(sps.CKPT_UNIFORM)


def test_step_change():
    """A run of 3 steps at dt then 2 at dt/2 (sps_set_dt between two segments), reversed segment
    by segment with the cotangent handed over, against the oracle run of the same steps."""
    cfg = SMALL
    dt = cfg[5]
    note("RK443 step change")
    P, G = build(cfg, ce=2, max_steps=3)
    X0 = P.initial_state(wl.rbc_b0(seed=24, Nx=cfg[0], Nz=cfg[1], amp=0.1))
    X1r, h1 = imex.rk_forward(P, X0, dt, 3, tableau=TAB)
    X2r, h2 = imex.rk_forward(P, X1r, 0.5 * dt, 2, tableau=TAB)
    y = imex.rk_adjoint(P, P.kinetic_energy_grad(X2r), h2, 0.5 * dt, tableau=TAB)
    g_ref = imex.rk_adjoint(P, y, h1, dt, tableau=TAB)
    X = to_dev(X0)
    G.step(X, 3)
    X1 = X.clone()
    G.set_dt(0.5 * dt)          # drops the recorded run of the first segment
    G.step(X, 2)
    seed = torch.zeros_like(X)
    G.cost(X, None, seed)
    G.adjoint_step(seed, 2)     # cotangent of X_3
    G.set_dt(dt)
    Xr = to_dev(X0)
    G.step(Xr, 3)               # the first segment's forward run again
    G.adjoint_step(seed, 3)
    G.sync()
    check_fields(from_dev(X1, X0.shape), X1r, P.Nz, TOL, base=conduction(P), what="X_3")
    check_fields(from_dev(seed, X0.shape), g_ref, P.Nz, TOL, what="dJ/dX0")


def test_batch():
    """Two instances (Rayleigh numbers 1e5 and 3e4) of a batch under RK443, each against the
    oracle."""
    nx, nz, lx, _, Pr, dt = SMALL
    ras, nsteps = (1e5, 3e4), 5
    note("RK443 batch")
    G = sps.RbcBatch(list(ras), nx, nz, lx, Pr, dt=dt, checkpoint_every=2, max_steps=nsteps, scheme=sps.RK443)
    Ps = [RBC(Nx=nx, Nz=nz, Lx=lx, Ra=r, Pr=Pr) for r in ras]
    Xs = [P.initial_state(wl.rbc_b0(seed=25 + b, Nx=nx, Nz=nz, amp=0.1)) for b, P in enumerate(Ps)]
    X0 = torch.from_numpy(np.concatenate([X.view(np.float64).ravel() for X in Xs])).cuda()
    g = torch.zeros_like(X0)
    J = torch.zeros(2, dtype=torch.float64, device="cuda")
    G.gradient(X0, nsteps, None, g, J)
    G.sync()
    gh = g.cpu().numpy().view(np.complex128).reshape((2,) + Xs[0].shape)
    for b, P in enumerate(Ps):
        XN, hist = imex.rk_forward(P, Xs[b], dt, nsteps, tableau=TAB)
        g_ref = imex.rk_adjoint(P, P.kinetic_energy_grad(XN), hist, dt, tableau=TAB)
        assert abs(J[b].item() - P.kinetic_energy(XN)) <= TOL * P.kinetic_energy(XN)
        check_fields(gh[b], g_ref, nz, TOL, what=f"instance {b} dJ/dX0")
