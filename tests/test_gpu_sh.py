"""GPU parity of the batched Swift-Hohenberg path (one persistent launch per sweep) against
the FP64 oracle, through the C ABI: the initial transform and its adjoint, F and its VJP, the
diagonal solve, the cost, forward runs and the discrete-adjoint gradient, on a mixed-size
batch; at the full configuration (128 instances of 64^2..192^2, dt = 0.02, 500 steps) the
launch bench.py times is checked on sampled instances against the oracle, and every
instance's result is checked to be independent of the batch it runs in (bit for bit).
Tolerance: 1e-11 in max|gpu - oracle| / max|oracle| per array."""
import numpy as np
import pytest

from oracle import imex
from oracle.sh import SH
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-11
L = 16.0 * np.pi

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402

SMALL_N = [8, 12, 24, 16, 8, 18]
SMALL_R = [0.3, 0.15, 0.45, 0.25, 0.5, 0.2]


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def split_states(t, sizes):
    """GPU state (instances of [N/2][N] complex) -> list of oracle states c[iy, ix]."""
    v = t.cpu().numpy().view(np.complex128)
    out, o = [], 0
    for N in sizes:
        k = N * (N // 2)
        out.append(v[o:o + k].reshape(N // 2, N).T.copy())
        o += k
    return out


def join_states(cs):
    return torch.from_numpy(np.concatenate([c.T.ravel() for c in cs]).view(np.float64).copy()).cuda()


def split_grids(t, sizes):
    v = t.cpu().numpy()
    out, o = [], 0
    for N in sizes:
        out.append(v[o:o + N * N].reshape(N, N))
        o += N * N
    return out


def join_grids(us):
    return torch.from_numpy(np.concatenate([u.ravel() for u in us]).copy()).cuda()


def oracles(sizes, rs):
    return [SH(N, r, L=L) for N, r in zip(sizes, rs)]


def test_sh_pieces_mixed_batch():
    print("SH pieces", flush=True)
    sizes, rs, dt = SMALL_N, SMALL_R, 0.02
    G = sps.ShBatch(sizes, rs, L, dt, max_steps=2)
    Ps = oracles(sizes, rs)
    rng = np.random.default_rng(41)
    u0 = [rng.uniform(-0.5, 0.5, (N, N)) for N in sizes]
    X = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.initial_state(join_grids(u0), X)
    G.sync()
    Xs = split_states(X, sizes)
    for P, u, c in zip(Ps, u0, Xs):
        assert rel(c, P.initial_state(u).reshape(P.N, P.N // 2)) < TOL
    # F and its VJP at O(1) states (the cubic term matters)
    cs = [P.from_grid(rng.uniform(-1, 1, (P.N, P.N)), P.N) for P in Ps]
    gs = [P.from_grid(rng.uniform(-1, 1, (P.N, P.N)), P.N) for P in Ps]
    out = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.eval_F(join_states(cs), out)
    G.sync()
    for P, c, f in zip(Ps, cs, split_states(out, sizes)):
        assert rel(f, P.F(c.reshape(-1, 1)).reshape(P.N, P.N // 2)) < TOL
    G.eval_F_vjp(join_states(cs), join_states(gs), out)
    G.sync()
    for P, c, g, v in zip(Ps, cs, gs, split_states(out, sizes)):
        assert rel(v, P.F_vjp(c.reshape(-1, 1), g.reshape(-1, 1)).reshape(P.N, P.N // 2)) < TOL
    # diagonal solve (SBDF2 matrix)
    G.solve(join_states(gs), out)
    G.sync()
    for P, g, v in zip(Ps, gs, split_states(out, sizes)):
        lu = imex.BlockLU(P.M, P.L, 1.5 / dt, 1.0)
        assert rel(v, lu.solve(g.reshape(-1, 1)).reshape(P.N, P.N // 2)) < TOL
    # cost and initial-transform adjoint
    J = torch.zeros(len(sizes), dtype=torch.float64, device="cuda")
    G.cost(join_states(cs), J, out)
    G.sync()
    for P, c, j, dj in zip(Ps, cs, J.cpu().numpy(), split_states(out, sizes)):
        assert abs(j - P.energy(c.reshape(-1, 1))) < TOL * P.energy(c.reshape(-1, 1))
        assert rel(dj, P.energy_grad(c.reshape(-1, 1)).reshape(P.N, P.N // 2)) < TOL
    gb = torch.zeros(G.grid_size, dtype=torch.float64, device="cuda")
    G.initial_state_adjoint(join_states(gs), gb)
    G.sync()
    for P, g, v in zip(Ps, gs, split_grids(gb, sizes)):
        assert rel(v, P.initial_state_adjoint(g.reshape(-1, 1))) < TOL


def sh_reference(P, u0, dt, n):
    X0 = P.initial_state(u0)
    XN, states = imex.sbdf_forward(P, X0, dt, n)
    g = imex.sbdf_adjoint(P, P.energy_grad(XN), states, dt)
    return XN.reshape(P.N, P.N // 2), P.energy(XN), g.reshape(P.N, P.N // 2)


@pytest.mark.parametrize("nsteps", [1, 2, 7])
def test_sh_gradient_mixed_batch(nsteps):
    print(f"SH gradient x {nsteps}", flush=True)
    sizes, rs, dt = SMALL_N, SMALL_R, 0.05
    G = sps.ShBatch(sizes, rs, L, dt, max_steps=nsteps)
    Ps = oracles(sizes, rs)
    rng = np.random.default_rng(42)
    u0 = [rng.uniform(-0.8, 0.8, (N, N)) for N in sizes]
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.initial_state(join_grids(u0), X0)
    XN = torch.zeros_like(X0)
    g = torch.zeros_like(X0)
    J = torch.zeros(len(sizes), dtype=torch.float64, device="cuda")
    G.gradient(X0, nsteps, XN, g, J)
    G.sync()
    for i, (P, u) in enumerate(zip(Ps, u0)):
        xr, jr, gr = sh_reference(P, u, dt, nsteps)
        assert rel(split_states(XN, sizes)[i], xr) < TOL
        assert abs(J[i].item() - jr) < TOL * jr
        assert rel(split_states(g, sizes)[i], gr) < TOL
    # step + adjoint_step reproduce the gradient bit for bit
    X = X0.clone()
    G.step(X, nsteps)
    dJ = torch.zeros_like(X)
    G.cost(X, J, dJ)
    G.adjoint_step(dJ, nsteps)
    G.sync()
    assert torch.equal(X, XN) and torch.equal(dJ, g)


def test_sh_full_batch_sampled_and_batch_independent():
    """The configuration bench.py times: 128 instances, sizes from {64, 96, 128, 192}, dt = 0.02,
    500 steps.  Two sampled instances against the oracle over all 500 steps, and every instance
    equal (bitwise) to the same instance run alone."""
    print("SH full batch", flush=True)
    sizes, rs, u0 = wl.sh_batch(seed=0)
    nsteps, dt = 500, 0.02
    G = sps.ShBatch(sizes, rs, L, dt, max_steps=nsteps)
    print("tuning", G.tuning(), flush=True)
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.initial_state(join_grids(u0), X0)
    g = torch.zeros_like(X0)
    J = torch.zeros(len(sizes), dtype=torch.float64, device="cuda")
    G.gradient(X0, nsteps, None, g, J)
    gb = torch.zeros(G.grid_size, dtype=torch.float64, device="cuda")
    G.initial_state_adjoint(g, gb)
    G.sync()
    gs, grids = split_states(g, sizes), split_grids(gb, sizes)
    for N in (64, 192):
        i = sizes.index(N)
        P = SH(N, rs[i], L=L)
        xr, jr, gr = sh_reference(P, u0[i], dt, nsteps)
        print(f"instance {i} N={N}: J {J[i].item():.6e} vs {jr:.6e}", flush=True)
        assert abs(J[i].item() - jr) < TOL * jr
        assert rel(gs[i], gr) < TOL
        assert rel(grids[i], P.initial_state_adjoint(gr.reshape(-1, 1))) < TOL
    # batch independence on a few instances of every size (different tiles, same bits)
    for N in (64, 96, 128, 192):
        i = sizes.index(N)
        G1 = sps.ShBatch([N], [rs[i]], L, dt, max_steps=nsteps)
        x1 = torch.zeros(G1.n, dtype=torch.float64, device="cuda")
        G1.initial_state(join_grids([u0[i]]), x1)
        g1 = torch.zeros_like(x1)
        J1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        G1.gradient(x1, nsteps, None, g1, J1)
        G1.sync()
        assert np.array_equal(split_states(g1, [N])[0], gs[i]) and J1.item() == J[i].item()
