"""Write tests/golden/rbc_bench_256x64.txt: the oracle's result for the benchmarked 2D
Rayleigh-Benard gradient (256x64, Ra = 1e6, Pr = 1, RK222 dt = 1e-3, 1000 steps, initial
buoyancy of seed 0 with noise amplitude 1e-3), and the oracle's own rounding floor at that
horizon.

Calls only oracle/ and the seeded input generator.  Run from the repository root:

    python tests/golden/make_rbc_bench_golden.py

(about five minutes on 8 cores: two full oracle gradients.)

Contents: J; for the final state X_N (conduction state subtracted) and for dJ/dX_0, per
group (the u, w, b, p blocks and the taus, the k = 0 row and the rows k >= 1 apart) the
group's largest magnitude, the oracle's self-floor and sampled entries; for dJ/db_0 on the
256x64 grid its largest magnitude, self-floor and sampled entries.

Self-floor: the same run with the initial grid rolled by one point in x.  The discrete model
is equivariant under that shift (coefficient k picks up the phase exp(i k_x dx), the grid
gradient rolls with the grid), so the two runs agree in exact arithmetic and differ only by
rounding; their difference, relative to each group's largest entry, is the floor below which
no two correct FP64 implementations can be told apart at this horizon.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import imex  # noqa: E402
from oracle.rbc import RBC  # noqa: E402

NX, NZ, LX, RA, PR, DT, NSTEPS, SEED, AMP = 256, 64, 4.0, 1e6, 1.0, 1e-3, 1000, 0, 1e-3
NSAMP = 40
OUT = os.path.join(ROOT, "tests", "golden", "rbc_bench_256x64.txt")
FIELDS = ("u", "w", "b", "p")


def groups(N, S):
    out = []
    for r0, r1, tag in ((0, 1, "k=0"), (1, None, "k>0")):
        for f, name in enumerate(FIELDS):
            out.append((f"{name}[{tag}]", r0, r1, f * N, (f + 1) * N))
        out.append((f"tau[{tag}]", r0, r1, 4 * N, S))
    return out


def run(P, b0):
    X0 = P.initial_state(b0)
    XN, hist = imex.rk_forward(P, X0, DT, NSTEPS)
    J = P.kinetic_energy(XN)
    g = imex.rk_adjoint(P, P.kinetic_energy_grad(XN), hist, DT)
    return X0, XN, J, g, P.initial_state_adjoint(g)


def main():
    t0 = time.time()
    P = RBC(Nx=NX, Nz=NZ, Lx=LX, Ra=RA, Pr=PR)
    base = P.lbvp_solve(np.zeros((P.K, P.S), complex))
    b0 = wl.rbc_b0(seed=SEED, Nx=NX, Nz=NZ, amp=AMP)
    X0, XN, J, g, gb = run(P, b0)
    print(f"run 1: J = {J:.17e} ({time.time() - t0:.0f} s)", flush=True)
    X0s, XNs, Js, gs, gbs = run(P, np.roll(b0, -1, axis=0))
    print(f"run 2 (rolled): J = {Js:.17e} ({time.time() - t0:.0f} s)", flush=True)
    # the phase of the shift, checked on the initial states
    ph = np.exp(1j * P.kx * (LX / NX))[:, None]
    assert np.max(np.abs(X0s - ph * X0)) <= 1e-15 * np.max(np.abs(X0)), "shift phase"
    rng = np.random.default_rng(12345)
    lines = ["# Oracle result of the benchmarked 2D Rayleigh-Benard gradient and the oracle's self-floor.",
             "# Written by tests/golden/make_rbc_bench_golden.py (oracle/ only); see that script.",
             f"# config nx {NX} nz {NZ} lx {LX} Ra {RA} Pr {PR} dt {DT} nsteps {NSTEPS} seed {SEED} amp {AMP}",
             f"J {J:.17e} floor {abs(Js - J) / abs(J):.3e}"]
    for label, A, As in (("XN", XN - base, XNs - base), ("G", g, gs)):
        for name, r0, r1, s0, s1 in groups(P.N, P.S):
            blk = A[r0:r1, s0:s1]
            # the rolled run maps back by the conjugate phase (the conduction state sits at k = 0,
            # where the phase is 1)
            blks = (np.conj(ph) * (As + base) - base)[r0:r1, s0:s1] if label == "XN" else (np.conj(ph) * As)[r0:r1, s0:s1]
            scale = float(np.max(np.abs(blk)))
            floor = float(np.max(np.abs(blks - blk)) / scale) if scale > 0 else 0.0
            flat = np.argmax(np.abs(blk))
            picks = [int(flat)] + [int(v) for v in rng.choice(blk.size, size=min(NSAMP, blk.size), replace=False)]
            lines.append(f"group {label} {name} scale {scale:.17e} floor {floor:.3e} n {len(picks)}")
            for q in picks:
                i, j = divmod(q, blk.shape[1])
                k, s = r0 + i, s0 + j
                v = blk[i, j]
                lines.append(f"{k} {s} {v.real:.17e} {v.imag:.17e}")
    scale = float(np.max(np.abs(gb)))
    floor = float(np.max(np.abs(np.roll(gbs, 1, axis=0) - gb)) / scale)
    picks = [int(np.argmax(np.abs(gb)))] + [int(v) for v in rng.choice(gb.size, size=256, replace=False)]
    lines.append(f"grid gb scale {scale:.17e} floor {floor:.3e} n {len(picks)}")
    for q in picks:
        i, j = divmod(q, NZ)
        lines.append(f"{i} {j} {gb[i, j]:.17e}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
