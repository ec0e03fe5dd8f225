"""Benchmark: forward+adjoint timesteps/s and gradients/s of the 2D Rayleigh-Benard
problem (Fourier x Chebyshev 256 x 64, FP64, RK222 dt = 1e-3, 1000 steps, checkpoint
every 50) on one MI355X.

One benchmark step is one full gradient: initial transform of b0, 1000 forward steps
with checkpoints, cost seed, reverse sweep with segment recompute, and the gradient on
the b0 grid.  Inputs are resident in HBM before the timed region starts.  The steps are
timed twice: with eager launches (which also feed the per-kernel timer behind the
roofline figure) and with each gradient's launch sequence replayed as a HIP graph (the
headline value); both are printed.

Prints one JSON line.  Extra modes: --copy-calibration (a plain device copy of known
size, used to scale rocprof FETCH_SIZE / WRITE_SIZE counters) and --no-cpu.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "forward+adjoint timesteps/s and gradients/s, 2D Fourier×Chebyshev 256×64, FP64"
CFG = dict(nx=256, nz=64, lx=4.0, Ra=1e6, Pr=1.0, dt=1e-3, nsteps=1000, checkpoint_every=50, seed=0)
HBM_PEAK_GBS = 8000.0
# sources of the stage kernel: counters taken on other sources are not reported
KERNEL_SOURCES = ("paper_2506_14792_amd/csrc/rbc.hip", "paper_2506_14792_amd/csrc/band_lu.h",
                  "paper_2506_14792_amd/csrc/sps_device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rbc_kfwd_256x64.json")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per stage-kernel launch from the rocprof FETCH_SIZE + WRITE_SIZE passes
    (scaled by the copy-kernel calibration), or None when the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def stage_kernel_bytes(nx, nz, K=None):
    """Algorithmic HBM bytes of one launch of the per-wavenumber forward stage kernel
    (average of the two RK222 stages): each operand streamed once.
    Per wavenumber: LU factors (n*kl multipliers + n*(kl+ku+1) U entries + n pivots),
    state in/out, nonlinear terms in, stage-0 F out/in, six z-grid fields out."""
    K, N = (nx // 2 if K is None else K), nz
    S = 4 * N + 7
    Ngz = 3 * N // 2
    kl, ku = 7, 20
    factors = S * (kl + kl + ku + 1) * 8 + S * 4
    state = S * 16
    nl = 3 * Ngz * 16
    f0 = 3 * N * 16
    zg = 6 * Ngz * 16
    tables = 2 * N * Ngz * 8 / K          # Chebyshev matrices, shared by all wavenumbers
    stage1 = factors + state + state + nl + f0 + zg + tables
    stage2 = factors + 2 * state + state + nl + f0 + zg + tables
    return K * 0.5 * (stage1 + stage2)


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and its logical CPU count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(nsteps=60, nsteps_single=10):
    """The oracle (numpy/scipy FP64) on a bounded sample: nsteps forward + nsteps adjoint
    steps of the same 256 x 64 problem from the same b0, with the BLAS thread pool at its
    default size (all host cores) and, for nsteps_single + nsteps_single steps, on one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import imex
    from oracle.rbc import RBC
    import workloads as wl
    P = RBC(Nx=CFG["nx"], Nz=CFG["nz"], Lx=CFG["lx"], Ra=CFG["Ra"], Pr=CFG["Pr"])
    X0 = P.initial_state(wl.rbc_b0(seed=CFG["seed"], Nx=CFG["nx"], Nz=CFG["nz"]))

    def run(n):
        t0 = time.perf_counter()
        XN, hist = imex.rk_forward(P, X0, CFG["dt"], n)
        imex.rk_adjoint(P, P.kinetic_energy_grad(XN), hist, CFG["dt"])
        return time.perf_counter() - t0

    t = run(nsteps)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        t1 = run(nsteps_single)
    model, ncpu = host_cpu_model()
    return {"value": 2 * nsteps / t, "unit": "timesteps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{nsteps} forward + {nsteps} adjoint RK222 steps at 256x64 (dense LU, matrix transforms), "
                      f"{t:.1f} s on {threads} BLAS threads; host: {ncpu} logical CPUs, {model}",
            "single_thread": {"value": 2 * nsteps_single / t1, "unit": "timesteps/s", "cores": 1,
                              "sample": f"{nsteps_single} forward + {nsteps_single} adjoint steps, {t1:.1f} s"},
            "host_cpu_model": model, "host_logical_cpus": ncpu}


KS_CFG = dict(nx=64, L=32.0 * np.pi, dt=0.05, nsteps=200, seed=0)


def ks_timing(reps=20):
    """The 1D Kuramoto-Sivashinsky workload (64 modes, SBDF2 dt = 0.05, 200 steps,
    gradient of 1/2 ||u(T)||^2 w.r.t. the initial coefficients): GPU gradient time and the
    oracle's CPU seconds for the same gradient."""
    import torch
    import paper_2506_14792_amd as sps
    import workloads as wl
    from oracle import imex
    from oracle.ks import KS
    c = KS_CFG
    G = sps.Problem(sps.KS1D, c["nx"], 0, c["L"], 0.0, 0.0, 1.5, c["dt"], 1, c["nsteps"])
    c0 = wl.ks_c0(seed=c["seed"], Nx=c["nx"])[:, None]
    X0 = torch.from_numpy(np.ascontiguousarray(c0).view(np.float64).ravel().copy()).cuda()
    g = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.gradient(X0, c["nsteps"], None, g, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.gradient(X0, c["nsteps"], None, g, None)
    torch.cuda.synchronize()
    gpu_s = (time.perf_counter() - t0) / reps
    G.sync()
    P = KS(Nx=c["nx"], L=c["L"])
    t0 = time.perf_counter()
    XN, states = imex.sbdf_forward(P, c0, c["dt"], c["nsteps"])
    imex.sbdf_adjoint(P, P.energy_grad(XN), states, c["dt"])
    cpu_s = time.perf_counter() - t0
    # the same gradient with the higher-order multistep schemes and the IMEX RK schemes
    higher = {}
    for name, scheme in (("sbdf3", sps.SBDF3), ("sbdf4", sps.SBDF4), ("rk222", sps.RK222), ("rk443", sps.RK443)):
        Gh = sps.Problem(sps.KS1D, c["nx"], 0, c["L"], 0.0, 0.0, 1.5, c["dt"], 1, c["nsteps"], scheme=scheme)
        gh = torch.zeros(Gh.n, dtype=torch.float64, device="cuda")
        Gh.gradient(X0, c["nsteps"], None, gh, None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            Gh.gradient(X0, c["nsteps"], None, gh, None)
        torch.cuda.synchronize()
        hs = (time.perf_counter() - t0) / reps
        Gh.sync()
        higher[name] = {"gpu_gradient_s": hs, "gpu_timesteps_per_s": 2 * c["nsteps"] / hs}
    # SBDF2 on variable steps (a linear ramp of the step size from 0.67 dt to 1.33 dt)
    G.set_timesteps(c["dt"] * (0.67 + 0.67 * np.arange(c["nsteps"]) / c["nsteps"]))
    G.gradient(X0, c["nsteps"], None, g, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.gradient(X0, c["nsteps"], None, g, None)
    torch.cuda.synchronize()
    higher["sbdf2_variable_steps"] = {"gpu_gradient_s": (time.perf_counter() - t0) / reps}
    G.set_timesteps(None)
    G.sync()
    return {"workload": "Kuramoto-Sivashinsky 1D, 64 Fourier modes, L = 32 pi, SBDF2 dt = 0.05, 200 steps, "
                        "gradient of 1/2 ||u(T)||^2", "gpu_gradient_s": gpu_s, "oracle_cpu_gradient_s": cpu_s,
            "gpu_timesteps_per_s": 2 * c["nsteps"] / gpu_s, "higher_order": higher}


SH_CFG = dict(nsteps=500, dt=0.02, L=16.0 * np.pi, seed=0)


def sh_state_complex(sizes):
    return sum(n * (n // 2) for n in sizes)


def sh_timing(reps=2):
    """Batched Swift-Hohenberg configuration: 128 instances, sizes drawn from {64, 96, 128, 192}^2,
    r in [0.1, 0.5], SBDF2 dt = 0.02, 500 steps; one gradient of the summed energies = one
    persistent launch (forward sweep, cost seed, reverse sweep).  Reported beside the same
    instances solved one problem at a time (plain launches, one instance of each size timed and
    weighted by the batch's size counts) and the oracle on one instance of each size for 10
    steps, extrapolated.  Algorithmic bytes per instance state of S complex modes: forward step
    13 S x 16 B (column phase: products' x-spectra, two previous states, two F, the new state and
    F, the new state's y-transform; row phase: 4 S in and out), reverse step 17 S x 16 B."""
    import torch
    import paper_2506_14792_amd as sps
    import workloads as wl
    from oracle import imex
    from oracle.sh import SH
    c = SH_CFG
    sizes, rs, u0 = wl.sh_batch(seed=c["seed"])
    G = sps.ShBatch(sizes, rs, c["L"], c["dt"], max_steps=c["nsteps"])
    grid = torch.from_numpy(np.concatenate([u.ravel() for u in u0])).cuda()
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    g = torch.zeros_like(X0)
    gb = torch.zeros_like(grid)
    J = torch.zeros(len(sizes), dtype=torch.float64, device="cuda")

    def one():
        G.initial_state(grid, X0)
        G.gradient(X0, c["nsteps"], None, g, J)
        G.initial_state_adjoint(g, gb)

    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one()
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / reps
    G.sync()
    S = sh_state_complex(sizes)
    bytes_grad = c["nsteps"] * (13 + 17) * S * 16.0
    # plain launches: each size alone
    plain = 0.0
    counts = {n: sizes.count(n) for n in set(sizes)}
    for n in sorted(counts):
        i = sizes.index(n)
        G1 = sps.ShBatch([n], [rs[i]], c["L"], c["dt"], max_steps=c["nsteps"])
        x1 = torch.zeros(G1.n, dtype=torch.float64, device="cuda")
        G1.initial_state(torch.from_numpy(u0[i].ravel().copy()).cuda(), x1)
        g1 = torch.zeros_like(x1)
        G1.gradient(x1, c["nsteps"], None, g1, None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        G1.gradient(x1, c["nsteps"], None, g1, None)
        torch.cuda.synchronize()
        plain += counts[n] * (time.perf_counter() - t1)
        G1.sync()
        G1.close()
    tuning = G.tuning()
    # every library handle is closed before the function returns, so nothing of the library is
    # left for interpreter teardown
    G.close()
    # oracle sample
    ocpu = 0.0
    for n in sorted(counts):
        i = sizes.index(n)
        P = SH(n, rs[i], L=c["L"])
        t1 = time.perf_counter()
        XN, states = imex.sbdf_forward(P, P.initial_state(u0[i]), c["dt"], 10)
        imex.sbdf_adjoint(P, P.energy_grad(XN), states, c["dt"])
        ocpu += counts[n] * (time.perf_counter() - t1) * c["nsteps"] / 10
    return {"workload": "batched Swift-Hohenberg: 128 instances, sizes {64,96,128,192}^2 (seeded), r in [0.1, 0.5], "
                        "L = 16 pi, 2x padding, SBDF2 dt = 0.02, 500 steps, gradient of the summed energies",
            "gpu_gradient_s": batch_s, "gpu_instance_timesteps_per_s": 2 * c["nsteps"] * len(sizes) / batch_s,
            "hbm_achieved_GBps": bytes_grad / batch_s / 1e9, "hbm_frac": bytes_grad / batch_s / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_gradient": bytes_grad, "tuning": tuning,
            "plain_launch_gradient_s": plain, "batched_speedup_vs_plain": plain / batch_s,
            "oracle_cpu_gradient_s_extrapolated": ocpu}


def lbvp_timing(reps=200):
    """Boundary value problem of the headline operator (256 x 64, Lx = 4, Ra = 1e6, Pr = 1):
    L X = M f + c with L factored once, the solve and the adjoint (L^H Y = Xbar through the same
    factors, then M^H Y) per call, and the LBVP-then-IVP gradient: the seeded smooth forcing's
    gradient of the kinetic energy after the 1000-step RK222 run (sps_lbvp_solve, sps_gradient,
    sps_lbvp_adjoint) against the IVP gradient alone.  Algorithmic bytes of a solve: the LU
    factors once (as counted for the stage kernel) plus the input, the right-hand side (out and
    in) and the output, 4 S x 16 B per wavenumber."""
    import torch
    import workloads as wl
    import paper_2506_14792_amd as sps
    from oracle.rbc import RBC
    c = CFG
    n = c["nsteps"]
    G = sps.Problem(sps.RBC2D, c["nx"], c["nz"], c["lx"], c["Ra"], c["Pr"], 1.5, c["dt"], c["checkpoint_every"], n)
    fh = wl.rbc_forcing(seed=c["seed"], Nx=c["nx"], Nz=c["nz"])
    f = torch.from_numpy(fh.view(np.float64).ravel().copy()).cuda()
    X = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    fb = torch.zeros_like(X)
    G.factor()
    G.lbvp_solve(f, X)            # factors L on the first call
    G.lbvp_adjoint(X, fb)
    torch.cuda.synchronize()

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    solve_s = timed(lambda: G.lbvp_solve(f, X), reps)
    adj_s = timed(lambda: G.lbvp_adjoint(X, fb), reps)
    K, S = c["nx"] // 2, 4 * c["nz"] + 7
    kl, ku = 7, 20
    bytes_solve = K * (S * (kl + kl + ku + 1) * 8 + S * 4 + 4 * S * 16)
    g = torch.zeros_like(X)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.lbvp_solve(f, X)
    X0 = X.clone()
    G.gradient(X0, n, None, g, J)

    def chain():
        G.lbvp_solve(f, X)
        G.gradient(X, n, None, g, J)
        G.lbvp_adjoint(g, fb)

    ivp_s = timed(lambda: G.gradient(X0, n, None, g, J), 3)
    chain_s = timed(chain, 3)
    G.sync()
    P = RBC(Nx=c["nx"], Nz=c["nz"], Lx=c["lx"], Ra=c["Ra"], Pr=c["Pr"])
    t0 = time.perf_counter()
    P.lbvp_adjoint(P.lbvp_solve(fh))
    ocpu = time.perf_counter() - t0
    return {"workload": "boundary value problem L X = M f + c of the Rayleigh-Benard operator, 256x64, Ra=1e6, "
                        "Pr=1 (steady Stokes-Boussinesq with the IVP's walls), seeded smooth forcing; its solution "
                        "starts the 1000-step RK222 run whose kinetic energy is differentiated w.r.t. the forcing",
            "solve_ms": solve_s * 1e3, "adjoint_ms": adj_s * 1e3,
            "bytes_per_solve": bytes_solve, "solve_hbm_GBps": bytes_solve / solve_s / 1e9,
            "solve_hbm_frac": bytes_solve / solve_s / 1e9 / HBM_PEAK_GBS,
            "ivp_gradient_s": ivp_s, "lbvp_ivp_gradient_s": chain_s, "J": J.item(),
            "oracle_cpu_solve_plus_adjoint_s": ocpu,
            "speedup_vs_oracle": ocpu / (solve_s + adj_s)}


def dtchange_timing(reps=3):
    """Step-size changes on the headline configuration (256 x 64): the cost of sps_set_dt (the
    RK222 matrices M + dt gamma L of all 128 wavenumbers refactored), and the gradient of a
    1000-step run in four segments of 250 steps at dt = 1.0, 1.2, 0.9, 1.1 x 1e-3 through
    torch.autograd (StepSegments: forward with a refactorization per segment; backward sets each
    segment's step again, recomputes its forward sweep and reverses it) beside the gradient of
    1000 steps at one step."""
    import torch
    import workloads as wl
    import paper_2506_14792_amd as sps
    from paper_2506_14792_amd import autograd as sa
    c = CFG
    G = sps.Problem(sps.RBC2D, c["nx"], c["nz"], c["lx"], c["Ra"], c["Pr"], 1.5, c["dt"], c["checkpoint_every"], 250)
    b0 = torch.from_numpy(wl.rbc_b0(seed=c["seed"], Nx=c["nx"], Nz=c["nz"]).ravel().copy()).cuda()
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.initial_state(b0, X0)
    G.set_dt(1.1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(20):
        G.set_dt(1e-3 if i % 2 == 0 else 1.2e-3)
    torch.cuda.synchronize()
    set_dt_s = (time.perf_counter() - t0) / 20
    segs = [(1.0e-3, 250), (1.2e-3, 250), (0.9e-3, 250), (1.1e-3, 250)]

    def seg_grad():
        X = X0.clone().requires_grad_(True)
        J = sa.cost(sa.step_segments(X, G, segs), G)
        return torch.autograd.grad(J, X)[0]

    seg_grad()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        seg_grad()
    torch.cuda.synchronize()
    seg_s = (time.perf_counter() - t0) / reps
    G.sync()
    G1 = sps.Problem(sps.RBC2D, c["nx"], c["nz"], c["lx"], c["Ra"], c["Pr"], 1.5, c["dt"], c["checkpoint_every"], 1000)
    g = torch.zeros_like(X0)
    G1.gradient(X0, 1000, None, g, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G1.gradient(X0, 1000, None, g, None)
    torch.cuda.synchronize()
    one_s = (time.perf_counter() - t0) / reps
    G1.sync()
    return {"workload": "256x64 RK222, step changes: sps_set_dt (refactor of 128 wavenumbers' M + dt gamma L); "
                        "gradient of 1000 steps in 4 segments of different dt through autograd",
            "set_dt_ms": set_dt_s * 1e3, "segmented_gradient_s": seg_s, "single_step_gradient_s": one_s,
            "segmented_over_single": seg_s / one_s}


def ckpt_timing(slot_counts=(5, 10, 20, 50)):
    """Checkpoint schedules on the headline configuration (256 x 64, 1000 RK222 steps; two levels
    with the outer level in host memory or in a file): the
    eager gradient with the default schedule (a stored state every 50 steps, one segment's stage
    fields recorded, segments recomputed on a second stream) against binomial checkpointing with
    a few slot counts (all launches on one stream; the fewest recomputed steps for the storage).
    Reports seconds per gradient, forward steps per gradient (schedule count: forward sweep,
    recomputation and the recorded turns) and the device memory of the stored data."""
    import torch
    import workloads as wl
    import paper_2506_14792_amd as sps
    c = CFG
    n = c["nsteps"]
    G = sps.Problem(sps.RBC2D, c["nx"], c["nz"], c["lx"], c["Ra"], c["Pr"], 1.5, c["dt"], c["checkpoint_every"], n)
    b0 = torch.from_numpy(wl.rbc_b0(seed=c["seed"], Nx=c["nx"], Nz=c["nz"]).ravel().copy()).cuda()
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    G.initial_state(b0, X0)
    g = torch.zeros_like(X0)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")

    def timed(k=2):
        G.gradient(X0, n, None, g, J)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            G.gradient(X0, n, None, g, J)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    K, S, Ngz = c["nx"] // 2, 4 * c["nz"] + 7, 3 * c["nz"] // 2
    state_mb = K * S * 16 / 1e6
    stage_mb = 6 * Ngz * K * 16 / 1e6            # z-grid fields of one stage
    ce = c["checkpoint_every"]   # the last segment is recorded by the forward sweep, not recomputed
    out = {"workload": "Rayleigh-Benard 256x64, 1000 RK222 steps, gradient of the final kinetic energy",
           "uniform": {"gradient_s": timed(), "forward_steps": 2 * n - ce,
                       "stored_MB": (n // ce) * state_mb + 2 * ce * 2 * stage_mb}}
    for slots in slot_counts:
        G.set_checkpointing(sps.CKPT_BINOMIAL, slots)
        fwd, rev = sps.checkpoint_schedule(n, slots)
        steps = sum(b - a for op, a, b in fwd + rev if op == 1) + sum(1 for op, _, _ in rev if op == 4)
        out[f"binomial_{slots}"] = {"gradient_s": timed(), "forward_steps": steps,
                                    "stored_MB": slots * state_mb + 2 * stage_mb}
    # two levels: segment starts (every 50 steps) in pinned host memory, binomial inside
    for slots in (3, 8):
        G.set_checkpointing(sps.CKPT_TWO_LEVEL, slots)
        fs, rs = sps.checkpoint_schedule(ce, slots)
        last = max(i for i, a in enumerate(fs) if a[0] == 2)
        seg_steps = (sum(b - a for op, a, b in fs[:last + 1] if op == 1)
                     + sum(b - a for op, a, b in rs if op == 1) + sum(1 for op, _, _ in rs if op == 4))
        out[f"two_level_{slots}"] = {"gradient_s": timed(), "forward_steps": n + (n // ce) * seg_steps,
                                     "stored_MB": slots * state_mb + 2 * stage_mb,
                                     "host_stored_MB": (n // ce) * state_mb}
    # nested: 4 outer (host) states for the 20 segment starts, 8 device slots
    G.set_checkpointing(sps.CKPT_TWO_LEVEL, 8)
    G.set_outer_slots(4)
    out["nested_4_outer_8_device"] = {"gradient_s": timed(), "host_stored_MB": 4 * state_mb,
                                      "stored_MB": 8 * state_mb + 2 * stage_mb}
    G.set_outer_slots(0)
    # the disk level: the same segment starts in a file instead of host memory (8 slots)
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        G.set_checkpointing(sps.CKPT_TWO_LEVEL, 8)
        G.set_checkpoint_file(os.path.join(tmp, "segment_starts.bin"))
        out["two_level_8_disk"] = {"gradient_s": timed(), "file_MB": (n // ce) * state_mb,
                                   "stored_MB": 8 * state_mb + 2 * stage_mb + 2 * state_mb}
        # nested on the file with 4 outer states: the binomial placement of the segment starts
        # against the least-cost placement for outer writes and reads priced at the time of a
        # state's write and read through a file on this host, in forward steps
        buf = np.zeros(K * S * 2)
        path = os.path.join(tmp, "probe.bin")
        t0 = time.perf_counter()
        for _ in range(5):
            buf.tofile(path)
            np.fromfile(path)
        io_steps = (time.perf_counter() - t0) / 10 / (out["uniform"]["gradient_s"] / (out["uniform"]["forward_steps"] + n))
        G.set_outer_slots(4)
        nseg = n // ce

        def outer_counts(f, r):
            return {"recomputed_segments": sum(b - a for op, a, b in r if op == 1),
                    "outer_writes": sum(1 for op, _, _ in f + r if op == 2),
                    "outer_reads": sum(1 for op, _, _ in r if op == 3)}
        nb = {"gradient_s": timed(), **outer_counts(*sps.checkpoint_schedule(nseg, 4))}
        G.set_outer_costs(io_steps, io_steps)
        fc, rc, _ = sps.checkpoint_schedule_costs(nseg, 4, float(ce), io_steps, io_steps)
        nc = {"gradient_s": timed(), **outer_counts(fc, rc)}
        G.set_outer_costs(-1.0, -1.0)
        G.set_outer_slots(0)
        out["nested_4_outer_8_device_file"] = {"io_cost_forward_steps": io_steps, "binomial_placement": nb,
                                               "least_cost_placement": nc}
        G.set_checkpoint_file(None)
    G.set_checkpointing(sps.CKPT_UNIFORM)
    G.sync()
    return out


def stability_timing(iters=30):
    """Eigenvalue problem of the conduction state's perturbations: (a) all 128 wavenumbers of the
    headline operator (256 x 64, Ra = 1e6, Pr = 1) in one sps_stability call (one LU of
    sigma M + L_s per wavenumber, `iters` inverse iterations for the right and the left
    eigenvector, the sensitivities), against the oracle's dense generalized eigensolve (left
    and right vectors, no sensitivities) of a sample of wavenumbers scaled to all 128; (b) the onset at k = 3.1163 (nz = 32) by Newton
    steps on the growth rate with the adjoint sensitivity d lambda/dRa, from Ra = 1500; the
    eigenvector sensitivities dX/dRa and dX/dk of all 128 wavenumbers (20 iterations); (c) the
    shift-invert Arnoldi on the same 128 wavenumbers (m = 32 steps, the 8 eigenvalues nearest 0
    with Ritz vectors and residuals), against the oracle's Arnoldi on a sample scaled to all
    128, with the count of converged pairs (residual below 1e-10 |nu|)."""
    import torch
    import paper_2506_14792_amd as sps
    from oracle.rbc import RBC
    c = CFG
    G = sps.Problem(sps.RBC2D, c["nx"], c["nz"], c["lx"], c["Ra"], c["Pr"], 1.5, c["dt"], 1, 1)
    G.stability(0.0, iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        lam, X, Y, dl = G.stability(0.0, iters)
    torch.cuda.synchronize()
    call_s = (time.perf_counter() - t0) / reps
    G.sync()
    P = RBC(Nx=c["nx"], Nz=c["nz"], Lx=c["lx"], Ra=c["Ra"], Pr=c["Pr"])
    t0 = time.perf_counter()
    sample = (1, 32, 64, 127)
    for k in sample:
        P.stability_eig(k, 0.0)   # dense generalized eigensolve with left and right vectors
    ocpu = (time.perf_counter() - t0) * (c["nx"] // 2) / len(sample)
    kc, Ra = 3.1163, 1500.0
    t0 = time.perf_counter()
    for it in range(5):
        Gn = sps.Problem(sps.RBC2D, 8, 32, 2.0 * np.pi / kc, Ra, 1.0, 1.5, 1e-3, 1, 1)
        lam_n, _, _, dl_n = Gn.stability(0.0, 40)
        g, dg = lam_n[1].item(), dl_n[1, 0].item()
        Ra -= g.real / dg.real
    newton_s = time.perf_counter() - t0
    # eigenvector sensitivities of all 128 wavenumbers (20 projected iterations per parameter)
    G.stability_vector_sens(0.0, lam, X, Y, dl, iters=20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.stability_vector_sens(0.0, lam, X, Y, dl, iters=20)
    torch.cuda.synchronize()
    vsens_s = (time.perf_counter() - t0) / reps
    G.sync()
    # (c) Arnoldi, several eigenvalues per shift
    m, nev = 32, 8
    G.stability_arnoldi(0.0, m=m, nev=nev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        la, Xa, ra, _ = G.stability_arnoldi(0.0, m=m, nev=nev)
    torch.cuda.synchronize()
    arn_s = (time.perf_counter() - t0) / reps
    G.sync()
    nu = 1.0 / (0.0 - la.cpu().numpy())
    nconv = int((ra.cpu().numpy() < 1e-10 * np.abs(nu)).sum())
    import workloads as wl
    v0 = wl.random_state(0, (P.K, P.M[1].shape[0]))
    t0 = time.perf_counter()
    for k in sample:
        P.stability_arnoldi(k, 0.0, v0[k], m)
    arn_cpu = (time.perf_counter() - t0) * (c["nx"] // 2) / len(sample)
    arnoldi = {"m": m, "nev": nev, "gpu_call_s": arn_s, "converged_pairs_of_1024": nconv,
               "oracle_cpu_s_all_wavenumbers_extrapolated": arn_cpu, "speedup_vs_oracle": arn_cpu / arn_s}
    return {"workload": "linear stability of the conduction state (eigenvalue nearest 0, right and adjoint "
                        "eigenvectors, d lambda/dRa and d lambda/dk): 256x64 Ra=1e6 all 128 wavenumbers; onset by "
                        "Newton at k=3.1163, nz=32",
            "iterations": iters, "gpu_call_s": call_s, "gpu_us_per_wavenumber": call_s / (c["nx"] // 2) * 1e6,
            "oracle_cpu_eig_s_all_wavenumbers_extrapolated": ocpu, "speedup_vs_oracle": ocpu / call_s,
            "newton_onset_Ra": Ra, "newton_final_growth": g.real, "newton_5_solves_s": newton_s,
            "eigenvector_sensitivities_s": vsens_s, "arnoldi": arnoldi}


COU_CFG = dict(nx=128, ny=64, nz=64, Lx=4.0 * np.pi, Lz=2.0 * np.pi, Re=400.0, dt=0.01, nsteps=2000,
               checkpoint_every=100, seed=0, energy=1e-6)


def couette_timing():
    """Differentiation configuration: 3D plane Couette flow 128 x 64 x 64 (Fourier x Chebyshev x
    Fourier, Lx = 4 pi, Lz = 2 pi, walls y = -1, 1 moving -1, 1), Re = 400, RK222 dt = 0.01 to T = 20
    (2000 steps), checkpoints every 100; the gradient of the energy gain E(T)/E(0) of a seeded
    divergence-free perturbation of energy 1e-6 through the torch.autograd Functions (Step with
    checkpoint-and-recompute, Cost).  Reports the gradient time and the per-mode stage kernel
    (4096 systems of 263 unknowns: the banded solves in the HBM regime) against the roofline:
    algorithmic bytes per launch as for the 2D kernel, times 4096 systems."""
    import torch
    import workloads as wl
    import paper_2506_14792_amd as sps
    from paper_2506_14792_amd import autograd as sa
    c = COU_CFG
    n = c["nsteps"]
    G = sps.Couette(c["nx"], c["ny"], c["nz"], c["Lx"], c["Lz"], Re=c["Re"], dt=c["dt"],
                    checkpoint_every=c["checkpoint_every"], max_steps=n)
    uvw = wl.couette_perturbation(seed=c["seed"], Nx=c["nx"], Ny=c["ny"], Nz=c["nz"], Lx=c["Lx"], Lz=c["Lz"],
                                  energy=c["energy"])
    x0 = G.state_from_velocity(uvw)

    def one():
        x = x0.clone().requires_grad_(True)
        J = sa.cost(sa.step(x, G, n), G) / sa.cost(x, G)
        (g,) = torch.autograd.grad(J, x)
        return J, g

    G.factor()
    one()
    G.sync()
    G.timer_enable(0, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, g = one()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    G.sync()
    launches, kern_ms = G.timer_read()
    G.timer_enable(0, False)
    K = (c["nx"] // 2) * c["nz"]
    bytes_launch = stage_kernel_bytes(0, c["ny"], K=K)
    avg = kern_ms / max(launches, 1)
    achieved = bytes_launch / (avg * 1e-3) / 1e9
    return {"workload": "plane Couette 3D 128x64x64 (Fourier x Chebyshev x Fourier), Re=400, RK222 dt=0.01, "
                        "2000 steps, checkpoint every 100, energy-gain gradient through torch.autograd",
            "gpu_gradient_s": t, "timesteps_per_s": 3 * n / t, "forward_adjoint_timesteps_per_s": 2 * n / t,
            "energy_gain": float(J.item()), "gradient_norm": float(g.norm().item()),
            "stage_kernel": {"kernel": "rbc_kfwd on 4096 Couette modes (transforms in y, RHS, banded LU solve)",
                             "bytes_per_launch": bytes_launch, "avg_launch_ms": avg, "launches_timed": launches,
                             "achieved_GBps": achieved, "frac": achieved / HBM_PEAK_GBS}}


KOL_CFG = dict(n_fine=512, factor=8, Re=1000.0, drag=0.1, dt=0.002, rollout=200, ntrain=4, ntest=2,
               spinup=16000, nsnap=600, batch=16, iters=40, lr=1e-3, seed=100)


def kolmo_timing():
    """Learned-closure configuration: 2D Kolmogorov flow on [0, 2 pi)^2, Re = 1000, forcing
    sin(4y), linear drag 0.1.  Fine runs of the unclosed solver (512^2 modes, 768^2 padded grid,
    step dt/8) from seeded k^-3 vorticity give the truth, truncated to 64^2 modes every 8 steps;
    the coarse solver (64^2, step dt = 0.002) carries the closure network (3x3 convolutions
    1 -> 32 -> 32 -> 1, GELU, bf16 weights and activations, FP32 accumulation on MFMA), trained
    with the rollout loss of 200-step coarse runs through the adjoint and Adam.  Reports the fine
    solver's throughput (HBM bytes of the design: 21 S x 16 B per instance step, S = N^2/2
    modes), the coarse step with and without the closure, one training iteration, and the
    rollout error against the truncated fine run without and with the trained closure on
    held-out runs."""
    import torch
    import workloads as wl
    import paper_2506_14792_amd as sps
    from paper_2506_14792_amd import closure_train as ct
    c = KOL_CFG
    nf, fac, nc = c["n_fine"], c["factor"], c["n_fine"] // c["factor"]
    nb = c["ntrain"] + c["ntest"]
    v = wl.kolmo_vorticity(seed=c["seed"], N=nf, batch=nb)
    X0 = torch.from_numpy(np.ascontiguousarray(np.transpose(v, (0, 2, 1))).view(np.float64).ravel().copy()).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = ct.fine_snapshots(X0, nf, fac, c["Re"], c["drag"], c["dt"], c["spinup"], c["nsnap"])
    t_fine = time.perf_counter() - t0
    fine_steps = c["spinup"] + c["nsnap"] * fac
    fine_bytes = 21 * (nf * nf // 2) * 16.0 * nb * fine_steps
    Str, Ste = S[:, : c["ntrain"]].contiguous(), S[:, c["ntrain"]:].contiguous()
    n, B = c["rollout"], c["batch"]
    # coarse steps with and without the closure (forward runs of B windows, no history)
    picks = [(s, b % c["ntrain"]) for b, s in enumerate(range(0, B * 10, 10))]
    Xc, _ = ct.gather_windows(Str, picks, n)
    theta0 = torch.from_numpy(wl.closure_theta(seed=0, C=32, scale=1.0)).cuda()
    step_ms = {}
    for name, clo in (("plain", False), ("closure", True)):
        G = sps.Kolmogorov(B, nc, Re=c["Re"], dt=c["dt"], max_steps=1, closure=clo, keep_history=False,
                           drag=c["drag"])
        if clo:
            G.set_params(theta0)
        XN = torch.empty_like(Xc)
        G.forward(Xc, n, XN=XN)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        G.forward(Xc, n, XN=XN)
        torch.cuda.synchronize()
        step_ms[name] = (time.perf_counter() - t1) / n * 1e3
        G.close()
    held = [(s, b) for s in range(0, c["nsnap"] - n + 1, 100) for b in range(c["ntest"])]
    J_plain = ct.rollout_losses(Ste, held, n, nc, c["Re"], c["drag"], c["dt"], None)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    theta, losses = ct.train(Str, theta0, n, nc, c["Re"], c["drag"], c["dt"], B, c["iters"], c["lr"],
                             list(range(0, c["nsnap"] - n + 1, 10)), seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    J_closed = ct.rollout_losses(Ste, held, n, nc, c["Re"], c["drag"], c["dt"], theta)
    twox = kolmo_twice_resolution(X0, S, Str, Ste, held, picks, c, J_plain, step_ms["closure"])
    return {"workload": "Kolmogorov flow 2D, Re=1000, forcing sin(4y), drag 0.1: coarse 64^2 (dt 0.002) with the "
                        "closure network, trained on 8x spectrally truncated 512^2 fine runs (dt 0.00025) from "
                        "seeded k^-3 vorticity, loss on 200-step coarse rollouts through the adjoint",
            "fine_instances": nb, "fine_steps": fine_steps, "fine_s": t_fine,
            "fine_instance_steps_per_s": nb * fine_steps / t_fine,
            "fine_hbm_GBps": fine_bytes / t_fine / 1e9, "fine_hbm_frac": fine_bytes / t_fine / 1e9 / HBM_PEAK_GBS,
            "coarse_batch": B, "coarse_plain_step_ms": step_ms["plain"], "coarse_closure_step_ms": step_ms["closure"],
            "closure_step_cost_vs_plain": step_ms["closure"] / step_ms["plain"],
            "train_iterations": c["iters"], "train_s_per_iteration": t_train / c["iters"],
            "train_loss_first_last": [losses[0], losses[-1]],
            "heldout_windows": len(held), "heldout_error_no_closure": float(J_plain.mean()),
            "heldout_error_trained_closure": float(J_closed.mean()),
            "error_ratio_no_closure_over_closure": float(J_plain.mean() / J_closed.mean()),
            "cost_matched_baseline": twox}


def kolmo_rollout_error(H, T, N):
    """The coarse rollout loss's metric (per window: the mean over the N x N grid of the squared
    difference, averaged over the steps) of states H against targets T, both [steps][windows][N/2
    x N complex modes] as the library stores them (kx >= 0 half plane: the kx = 0 row counted
    once after taking its Hermitian part, the others twice; the ky Nyquist column dropped)."""
    import torch
    n, B = H.shape[0], H.shape[1]
    D = torch.view_as_complex((H - T).reshape(n, B, N // 2, N, 2))
    iy = torch.arange(N, device=D.device)
    D0 = 0.5 * (D[:, :, 0, :] + torch.conj(D[:, :, 0, (N - iy) % N]))
    w = (D0.abs() ** 2)[:, :, iy != N // 2].sum(-1) + 2.0 * (D[:, :, 1:, :].abs() ** 2)[:, :, :, iy != N // 2].sum((-1, -2))
    return (w.sum(0) / n).cpu().numpy()


def kolmo_twice_resolution(X0, S, Str, Ste, held, picks, c, J_plain, closure_step_ms):
    """Cost-matched baseline of the closure: the unclosed solver at twice the coarse resolution
    (128^2 modes, step dt/2) started from the same fine runs truncated to 128^2 modes, its state
    every second step truncated to 64^2 modes and scored against the same held-out targets with the
    rollout loss's metric, and its cost per coarse time step (two of its steps) beside a closed
    64^2 step.  The metric is checked against the library's own loss on the unclosed 64^2 runs."""
    import torch
    import paper_2506_14792_amd as sps
    from paper_2506_14792_amd import closure_train as ct
    nf, fac = c["n_fine"], c["factor"]
    nc, n2 = nf // fac, 2 * (nf // fac)
    n, B = c["rollout"], c["batch"]
    S2 = ct.fine_snapshots(X0, nf, fac // 2, c["Re"], c["drag"], c["dt"] / 2, c["spinup"], 2 * c["nsnap"])
    ntr = c["ntrain"]
    # the unclosed 64^2 runs' states through the forward run's snapshots: the metric against J_plain
    X64, T = ct.gather_windows(Ste, held, n)
    T = T.view(n, len(held), nc * nc)
    G = sps.Kolmogorov(len(held), nc, Re=c["Re"], dt=c["dt"], max_steps=1, closure=False, keep_history=False,
                       drag=c["drag"])
    H = torch.empty(n * len(held) * nc * nc, dtype=torch.float64, device=X0.device)
    G.forward(X64, n, snap=H, every=1, nc=nc)
    torch.cuda.synchronize()
    G.close()
    e_plain = kolmo_rollout_error(H.view(n, len(held), nc * nc), T, nc)
    # the 128^2 runs
    idx = torch.as_tensor([2 * s for s, _ in held], device=X0.device)
    inst = torch.as_tensor([ntr + b for _, b in held], device=X0.device)
    X128 = S2[idx, inst].reshape(-1).contiguous()
    G = sps.Kolmogorov(len(held), n2, Re=c["Re"], dt=c["dt"] / 2, max_steps=1, closure=False, keep_history=False,
                       drag=c["drag"])
    H2 = torch.empty(n * len(held) * nc * nc, dtype=torch.float64, device=X0.device)
    G.forward(X128, 2 * n, snap=H2, every=2, nc=nc)
    torch.cuda.synchronize()
    G.close()
    e_2x = kolmo_rollout_error(H2.view(n, len(held), nc * nc), T, nc)
    # cost: B windows, as for the coarse step times
    idt = torch.as_tensor([2 * s for s, _ in picks], device=X0.device)
    itr = torch.as_tensor([b for _, b in picks], device=X0.device)
    Xt = S2[idt, itr].reshape(-1).contiguous()
    G = sps.Kolmogorov(B, n2, Re=c["Re"], dt=c["dt"] / 2, max_steps=1, closure=False, keep_history=False,
                       drag=c["drag"])
    XN = torch.empty_like(Xt)
    G.forward(Xt, 2 * n, XN=XN)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    G.forward(Xt, 2 * n, XN=XN)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) / n * 1e3
    G.close()
    del S2
    return {"solver": "unclosed, 128^2 modes, dt 0.001 (two steps per coarse step), from the fine runs truncated "
                      "to 128^2, scored on its states truncated to 64^2",
            "heldout_error": float(e_2x.mean()),
            "metric_check_max_rel_diff_vs_library_loss": float(np.max(np.abs(e_plain - J_plain) / J_plain)),
            "ms_per_coarse_time_step": ms,
            "cost_vs_closed_64_step": ms / closure_step_ms}


def copy_calibration(nbytes=1 << 28, reps=5):
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_dispatch": nbytes, "reps": reps}))


RBC_BATCH_CFG = dict(batch=64, nx=256, nz=64, lx=4.0, Pr=1.0, ra_min=5e5, ra_max=2e6, dt=1e-3, nsteps=100,
                     checkpoint_every=50, seed=100)


def rbc_batch_timing(reps=2):
    """A batch of 64 instances of the 256 x 64 problem with Rayleigh numbers drawn uniformly from
    [5e5, 2e6] (seeded; each instance has its own factors, 9.6 MB of banded LU factors, i.e.
    615 MB for the batch), RK222 dt = 1e-3, a 100-step gradient with checkpoints every 50: every
    stage launch covers all instances (8192 per-wavenumber systems, 6144 grid rows).  Reports
    instance timesteps per second and, per stage kernel, the algorithmic bytes of a launch (64
    times the single problem's, the factors counted per instance), the live average launch time
    (HIP events on the launch stream, eager gradients) and the fraction of 8 TB/s."""
    import torch
    import paper_2506_14792_amd as sps
    import workloads as wl
    c = RBC_BATCH_CFG
    B, n = c["batch"], c["nsteps"]
    ras = list(np.random.default_rng(c["seed"]).uniform(c["ra_min"], c["ra_max"], size=B))
    G = sps.RbcBatch(ras, c["nx"], c["nz"], c["lx"], c["Pr"], dt=c["dt"], checkpoint_every=c["checkpoint_every"],
                     max_steps=n)
    grid = torch.from_numpy(np.concatenate([wl.rbc_b0(seed=c["seed"] + b, Nx=c["nx"], Nz=c["nz"]).ravel()
                                            for b in range(B)])).cuda()
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    g = torch.zeros_like(X0)
    J = torch.zeros(B, dtype=torch.float64, device="cuda")
    G.initial_state(grid, X0)
    G.gradient(X0, n, None, g, J)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.gradient(X0, n, None, g, J)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    kb = kernel_bytes(c["nx"], c["nz"])
    per = {}
    for kind, name in ((0, "rbc_kfwd"), (1, "rbc_kadj"), (2, "rbc_xfwd"), (3, "rbc_xadj")):
        G.timer_enable(kind, True)
        G.gradient(X0, n, None, g, J)
        torch.cuda.synchronize()
        nk, ms = G.timer_read()
        G.timer_enable(kind, False)
        avg = ms / max(nk, 1)
        byt = B * kb[name]
        per[name] = {"bytes_per_launch": byt, "avg_launch_ms": avg, "launches_timed": nk,
                     "achieved_GBps": byt / (avg * 1e-3) / 1e9, "frac": byt / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS}
    G.sync()
    finite = bool(torch.isfinite(g).all().item())
    G.close()
    return {"workload": "batch of 64 Rayleigh-Benard 256x64 instances, Ra uniform in [5e5, 2e6] (seeded), Pr=1, "
                        "RK222 dt=1e-3, 100-step gradient, checkpoints every 50, one launch per stage for all instances",
            "batch": B, "gpu_gradient_s": sec, "instance_timesteps_per_s": 2 * n * B / sec,
            "gradients_per_s_per_instance": B / sec, "per_kernel": per, "finite": finite}


def poiseuille_timing():
    """Plane Poiseuille stability (the neutral-curve example), nz = 128 (S = 389): (a) the onset at
    alpha = 1.02056 by Newton in Re from Re = 5000 in one launch (factorization, 20 inverse
    iterations for each of the right and left eigenvectors and the sensitivities per Newton step),
    against the oracle's dense eigensolves with left vectors for the same Newton steps; (b) a batch
    of 128 neutral points in one launch: Newton in Re from Re = 5000 at 128 wavenumbers from 0.9
    to 1.09 (both branches near the onset); (c) 20 continuation steps along the curve from the
    onset, one launch each."""
    import torch
    import paper_2506_14792_amd as sps
    from oracle.poiseuille import Poiseuille
    nz = 128
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    G = sps.PoiseuilleStability(nz, 128)
    lam, dl, info = z(2), z(4), z(3)
    G.solve([(1.02056, 5000.0, -0.27j)], lam, dl, info, iters=20, mode=G.NEWTON_RE, tol=1e-12, maxit=12)
    G.sync()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        G.solve([(1.02056, 5000.0, -0.27j)], lam, dl, info, iters=20, mode=G.NEWTON_RE, tol=1e-12, maxit=12)
    G.sync()
    onset_s = (time.perf_counter() - t0) / reps
    a0, Re0, solves0 = info.cpu().numpy()
    P = Poiseuille(nz)
    t0 = time.perf_counter()
    Re_o, _, solves_o, _ = P.neutral_Re(1.02056, 5000.0, -0.27j, tol=1e-12)
    onset_cpu = time.perf_counter() - t0
    alphas = np.linspace(0.9, 1.09, 128)
    pars = [(al, 5000.0, -0.264j * al) for al in alphas]
    lb, db, ib = z(2 * 128), z(4 * 128), z(3 * 128)
    G.solve(pars, lb, db, ib, iters=20, mode=G.NEWTON_RE, tol=1e-12, maxit=15)
    G.sync()
    t0 = time.perf_counter()
    G.solve(pars, lb, db, ib, iters=20, mode=G.NEWTON_RE, tol=1e-12, maxit=15)
    G.sync()
    batch_s = time.perf_counter() - t0
    grow = np.abs(lb.cpu().numpy()[0::2])
    inf = ib.cpu().numpy().reshape(128, 3)
    a, Re, sg = float(a0), float(Re0), complex(*lam.cpu().numpy())
    t0 = time.perf_counter()
    steps = []
    for _ in range(20):
        G.solve([(a, Re, sg, 0.1)], lam, dl, info, iters=20, mode=G.CONTINUE, tol=1e-12, maxit=12)
        G.sync()
        a, Re, nsol = info.cpu().numpy()
        sg = complex(*lam.cpu().numpy())
        steps.append(int(nsol))
    cont_s = time.perf_counter() - t0
    G.close()
    return {"workload": "plane Poiseuille stability, nz=128 (389 unknowns, complex band kl=11, ku=19)",
            "onset": {"Re_c": float(Re0), "alpha_c": 1.02056, "eigenvalue_solves": int(solves0), "gpu_s": onset_s,
                      "oracle_Re_c": Re_o, "oracle_solves": solves_o, "oracle_cpu_s": onset_cpu},
            "batch_neutral_points": {"points": 128, "gpu_s": batch_s, "max_abs_growth": float(grow.max()),
                                     "mean_solves": float(inf[:, 2].mean()),
                                     "Re_range": [float(inf[:, 1].min()), float(inf[:, 1].max())]},
            "continuation": {"steps": 20, "ds": 0.1, "gpu_s": cont_s, "mean_solves": float(np.mean(steps)),
                             "end": [float(a), float(Re)]}}


def kernel_bytes(nx, nz):
    """Algorithmic HBM bytes per launch of each stage kernel of the 2D problem (each operand
    streamed once; factors in banded form): the per-wavenumber forward kernel (average of the
    two RK222 stages, stage_kernel_bytes), the per-wavenumber adjoint kernel (factors, the six
    z-grid cotangent columns, two state-size vectors in, one out, the nonlinear-term cotangents
    out), and the grid-row kernels (forward: 6 spectra in, 3 out per row; adjoint: 6 primal
    spectra and 3 cotangents in, 6 cotangents out per row)."""
    K, N = nx // 2, nz
    S, Ngz = 4 * N + 7, 3 * N // 2
    kl, ku = 7, 20
    factors = S * (kl + kl + ku + 1) * 8 + S * 4
    kadj = K * (factors + 6 * Ngz * 16 + 2 * S * 16 + S * 16 + 3 * Ngz * 16)
    return {"rbc_kfwd": stage_kernel_bytes(nx, nz), "rbc_kadj": kadj,
            "rbc_xfwd": Ngz * 9 * K * 16, "rbc_xadj": Ngz * 15 * K * 16}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nsteps", type=int, default=CFG["nsteps"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--skip-extra", action="store_true",
                    help="only the headline configuration (for counter and trace runs)")
    ap.add_argument("--only", choices=["ks", "sh", "closure", "couette", "lbvp", "ckpt", "stability", "dtchange",
                                       "rbcbatch", "poiseuille"],
                    default=None,
                    help="run one secondary configuration alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "sharding is a design note only", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only:
        import torch
        torch.cuda.set_device(0)
        fn = {"ks": ks_timing, "sh": sh_timing, "closure": kolmo_timing, "couette": couette_timing,
              "lbvp": lbvp_timing, "ckpt": ckpt_timing, "stability": stability_timing,
              "dtchange": dtchange_timing, "rbcbatch": rbc_batch_timing, "poiseuille": poiseuille_timing}[args.only]
        print(json.dumps({args.only: fn()}))
        return

    import torch
    import paper_2506_14792_amd as sps
    import workloads as wl

    torch.cuda.set_device(0)
    c = CFG
    n = args.nsteps
    G = sps.Problem(sps.RBC2D, c["nx"], c["nz"], c["lx"], c["Ra"], c["Pr"], 1.5, c["dt"], c["checkpoint_every"], n)
    b0 = torch.from_numpy(wl.rbc_b0(seed=c["seed"], Nx=c["nx"], Nz=c["nz"]).ravel().copy()).cuda()
    X0 = torch.zeros(G.n, dtype=torch.float64, device="cuda")
    gX = torch.zeros_like(X0)
    gb = torch.zeros_like(b0)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")

    def one_gradient():
        G.initial_state(b0, X0)
        G.gradient(X0, n, None, gX, J)
        G.initial_state_adjoint(gX, gb)

    G.factor()
    for _ in range(args.warmup):
        one_gradient()
    G.sync()
    G.timer_enable(0, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_gradient()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    G.sync()
    launches, kern_ms = G.timer_read()
    G.timer_enable(0, False)
    # the two halves of a gradient on their own (outside the timed region): forward sweep with
    # checkpoints, then the reverse sweep (segment recompute overlapped with the adjoint)
    Xf = X0.clone()
    G.initial_state(b0, Xf)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    G.step(Xf, n)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    Xb = torch.zeros_like(Xf)
    G.cost(Xf, J, Xb)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    G.adjoint_step(Xb, n)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    G.sync()
    # the other stage kernels, one eager gradient each with the timer on that kernel class
    per_kernel = {}
    kb = kernel_bytes(c["nx"], c["nz"])
    for kind, name in ((1, "rbc_kadj"), (2, "rbc_xfwd"), (3, "rbc_xadj")):
        G.timer_enable(kind, True)
        one_gradient()
        torch.cuda.synchronize()
        nk, msk = G.timer_read()
        G.timer_enable(kind, False)
        avg = msk / max(nk, 1)
        per_kernel[name] = {"bytes_per_launch": kb[name], "avg_launch_ms": avg, "launches_timed": nk,
                            "achieved_GBps": kb[name] / (avg * 1e-3) / 1e9,
                            "frac": kb[name] / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS}
    sec = (t1 - t0) / args.steps
    grads_per_s = 1.0 / sec
    bytes_launch = stage_kernel_bytes(c["nx"], c["nz"])
    avg_ms = kern_ms / max(launches, 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    per_kernel = dict({"rbc_kfwd": {"bytes_per_launch": bytes_launch, "avg_launch_ms": avg_ms,
                                    "launches_timed": launches, "achieved_GBps": achieved,
                                    "frac": achieved / HBM_PEAK_GBS}}, **per_kernel)
    # the same gradients with the launch sequence recorded once as a HIP graph and replayed
    G.set_graph(True)
    one_gradient()
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    for _ in range(args.steps):
        one_gradient()
    torch.cuda.synchronize()
    t7 = time.perf_counter()
    G.set_graph(False)
    G.sync()
    graph_sec = (t7 - t6) / args.steps
    traffic = measured_traffic()
    ks = sh = kol = cou = lbvp = ckpt = stab = dtc = rbatch = pois = None
    if not args.skip_extra:
        rbatch = rbc_batch_timing()
        lbvp = lbvp_timing()
        ckpt = ckpt_timing()
        dtc = dtchange_timing()
        stab = stability_timing()
        pois = poiseuille_timing()
        ks = ks_timing()
        sh = sh_timing()
        kol = kolmo_timing()
        cou = couette_timing()
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_steps)
    out = {
        "metric": METRIC,
        "value": 2 * n / graph_sec,
        "unit": "timesteps/s",
        "gradients_per_s": 1.0 / graph_sec,
        "launch": "graph (each gradient's launch sequence recorded once and replayed)",
        "eager_variant": {"value": 2 * n * grads_per_s, "ms_per_step": sec * 1e3, "gradients_per_s": grads_per_s},
        "forward_steps_per_s": n / (t3 - t2),
        "adjoint_steps_per_s": n / (t5 - t4),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": graph_sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Rayleigh-Benard 2D, Fourier(x, Lx=4) x Chebyshev(z, [0,1]) 256x64, Ra=1e6, Pr=1, "
                               "RK222 dt=1e-3, 1000 steps, checkpoint every 50, gradient of final kinetic energy "
                               "w.r.t. initial buoyancy",
                   "nx": c["nx"], "nz": c["nz"], "nsteps": n, "checkpoint_every": c["checkpoint_every"],
                   "seed": c["seed"], "step": "one full gradient (forward + recompute + adjoint)"},
        "roofline": {"bound": "hbm", "kernel": "rbc_kfwd (RK222 stage: z-transforms, RHS, banded LU solve)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": bytes_launch, "avg_launch_ms": avg_ms,
                     "launches_timed": launches, "per_kernel": per_kernel},
        "cpu_baseline": cpu,
        "rbc_batched_config": rbatch,
        "ks_config": ks,
        "sh_batched_config": sh,
        "closure_config": kol,
        "couette_autograd_config": cou,
        "lbvp_config": lbvp,
        "checkpointing_config": ckpt,
        "step_change_config": dtc,
        "stability_config": stab,
        "poiseuille_config": pois,
        "J": J.item(),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
