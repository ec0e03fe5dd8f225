"""The benchmarked gradient itself against the oracle: 2D Rayleigh-Benard 256x64, Ra = 1e6,
Pr = 1, RK222 dt = 1e-3, 1000 steps, checkpoints every 50, initial buoyancy of seed 0 with
noise amplitude 1e-3, the gradient recorded and replayed as a HIP graph exactly as the
benchmark launches it.

The oracle needs minutes for this run, so its result comes from tests/golden/
rbc_bench_256x64.txt, written by tests/golden/make_rbc_bench_golden.py (oracle/ only): J,
sampled entries of the final state (conduction state subtracted) and of dJ/dX_0 per field
group (u, w, b, p and the taus, the k = 0 row and the rows k >= 1 apart, with each group's
largest magnitude), and sampled entries of the gradient on the b_0 grid.  The bounds are those
of tests/parity.py: every sampled field entry within 1e-11 of its group's largest magnitude
(plus, for b and p, the rounding of the conduction background, 1e-13 of its size), taus within
1e-9 of their wavenumbers' whole state, groups that are zero in exact arithmetic within 1e-13 of
the array's largest entry.  The file also records the oracle's own rounding floor at this
horizon (the same run on a grid shifted by one point), which every bound must clear."""
import os
import sys

import numpy as np
import pytest

import workloads as wl
from parity import ABS_FLOOR, BACKGROUND, TAU_TOL, ZERO_GROUP

pytestmark = pytest.mark.gpu

TOL = 1e-11
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "rbc_bench_256x64.txt")

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_14792_amd as sps  # noqa: E402

NX, NZ, LX, RA, PR, DT, NSTEPS, CE, SEED, AMP = 256, 64, 4.0, 1e6, 1.0, 1e-3, 1000, 50, 0, 1e-3


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def read_golden():
    with open(GOLDEN) as f:
        lines = [l.split() for l in f if l.strip() and not l.startswith("#")]
    out = {"groups": {}, "grid": None}
    i = 0
    while i < len(lines):
        t = lines[i]
        if t[0] == "J":
            out["J"], out["J_floor"] = float(t[1]), float(t[3])
            i += 1
        elif t[0] == "group":
            label, name, scale, floor, n = t[1], t[2], float(t[4]), float(t[6]), int(t[8])
            pts = [(int(a[0]), int(a[1]), complex(float(a[2]), float(a[3]))) for a in lines[i + 1:i + 1 + n]]
            out["groups"][(label, name)] = (scale, floor, pts)
            i += 1 + n
        elif t[0] == "grid":
            scale, floor, n = float(t[3]), float(t[5]), int(t[7])
            pts = [(int(a[0]), int(a[1]), float(a[2])) for a in lines[i + 1:i + 1 + n]]
            out["grid"] = (scale, floor, pts)
            i += 1 + n
        else:
            raise ValueError(f"bad golden line {t}")
    return out


def conduction_state(K, N):
    """b = 1 - z and the hydrostatic pressure z - z^2/2 - 1/3 (zero mean) as T_n(2z - 1)
    coefficients at k = 0, no flow: the base state subtracted from X_N in the golden file."""
    S = 4 * N + 7
    X = np.zeros((K, S), complex)
    X[0, 2 * N:2 * N + 2] = [0.5, -0.5]
    X[0, 3 * N:3 * N + 3] = [-1.0 / 48.0, 0.25, -1.0 / 16.0]
    return X


def check_groups(got, gold, label, what, background=None):
    """background: largest magnitude of the subtracted base per field (u, w, b, p), or None."""
    groups = {k[1]: v for k, v in gold["groups"].items() if k[0] == label}
    overall = max(v[0] for v in groups.values())
    bg = dict(zip(("u", "w", "b", "p"), background or (0.0, 0.0, 0.0, 0.0)))
    worst = 0.0
    for name, (scale, floor, pts) in groups.items():
        field, rows = name.split("[")
        rowmax = max(v[0] for n, v in groups.items() if n.endswith("[" + rows))
        if field == "tau":
            # relative to the whole state of the row (background included)
            bound = TAU_TOL * max(rowmax, max(bg.values()) if rows.startswith("k=0") else 0.0)
            kind = "tau"
        elif scale <= ZERO_GROUP * overall:
            bound, kind = ABS_FLOOR * overall, "abs"
        else:
            bound, kind = TOL * scale + BACKGROUND * bg[field], "rel"
        assert floor * scale <= bound, f"{what} {name}: oracle floor {floor:.1e} does not clear the bound"
        err = max(abs(got[k, s] - v) for k, s, v in pts)
        note(f"  {what} {name}: |d| {err:.2e} <= {bound:.2e} ({kind}; {err / scale if scale else 0:.1e} of the "
             f"group, oracle floor {floor:.1e})")
        assert err <= bound, f"{what} {name}: {err:.2e} > {bound:.2e}"
        if kind == "rel":
            worst = max(worst, err / scale)
    return worst


def test_benchmarked_gradient_against_oracle():
    note("benchmark configuration 256x64 x 1000 steps, ce = 50, graph mode")
    gold = read_golden()
    G = sps.Problem(sps.RBC2D, NX, NZ, LX, RA, PR, 1.5, DT, CE, NSTEPS)
    K, S = NX // 2, 4 * NZ + 7
    b0 = torch.from_numpy(wl.rbc_b0(seed=SEED, Nx=NX, Nz=NZ, amp=AMP).ravel().copy()).cuda()
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    gX = torch.zeros_like(X0)
    gb = torch.zeros_like(b0)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.initial_state(b0, X0)
    G.set_graph(True)
    G.gradient(X0, NSTEPS, None, gX, J)        # records the graph and launches it
    G.initial_state_adjoint(gX, gb)
    G.sync()
    g_first, J_first = gX.clone(), J.item()
    G.gradient(X0, NSTEPS, None, gX, J)        # replays it
    G.initial_state_adjoint(gX, gb)
    G.sync()
    G.set_graph(False)
    assert torch.equal(gX, g_first) and J.item() == J_first
    eJ = abs(J.item() - gold["J"]) / abs(gold["J"])
    note(f"  J {J.item():.15e} vs {gold['J']:.15e}: rel {eJ:.2e} (oracle floor {gold['J_floor']:.1e})")
    assert eJ <= TOL
    g = gX.cpu().numpy().view(np.complex128).reshape(K, S)
    eg = check_groups(g, gold, "G", "dJ/dX0")
    # the final state, from the forward sweep alone (same kernels, eager launches)
    XN = X0.clone()
    G.step(XN, NSTEPS)
    G.sync()
    xn = XN.cpu().numpy().view(np.complex128).reshape(K, S) - conduction_state(K, NZ)
    ex = check_groups(xn, gold, "XN", "X_N", background=(0.0, 0.0, 0.5, 0.25))
    scale, floor, pts = gold["grid"]
    gbh = gb.cpu().numpy().reshape(NX, NZ)
    egb = max(abs(gbh[i, j] - v) for i, j, v in pts) / scale
    note(f"  dJ/db0 grid: {egb:.2e} (oracle floor {floor:.1e}); worst field: X_N {ex:.2e}, dJ/dX0 {eg:.2e}")
    assert egb <= TOL
