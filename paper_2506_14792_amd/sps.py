"""ctypes binding of the C ABI declared in include/sps.h (argument marshalling only)."""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsps.so")

RBC2D, KS1D, SH2D = 1, 2, 3
RK222, SBDF2, SBDF3, SBDF4, RK443 = 1, 2, 3, 4, 5
CKPT_UNIFORM, CKPT_BINOMIAL, CKPT_TWO_LEVEL = 0, 1, 2

_STATUS = {0: "SPS_OK", -1: "SPS_E_ARG", -2: "SPS_E_NOMEM", -3: "SPS_E_HIP", -4: "SPS_E_SINGULAR",
           -5: "SPS_E_NONFINITE", -6: "SPS_E_STATE", -7: "SPS_E_UNSUPPORTED", -8: "SPS_E_NOCONV",
           -9: "SPS_E_IO"}


class SpsDesc(ctypes.Structure):
    _fields_ = [("equation", ctypes.c_int), ("scheme", ctypes.c_int), ("nx", ctypes.c_int),
                ("nz", ctypes.c_int), ("lx", ctypes.c_double), ("param0", ctypes.c_double),
                ("param1", ctypes.c_double), ("dealias", ctypes.c_double), ("dt", ctypes.c_double),
                ("checkpoint_every", ctypes.c_int), ("max_steps", ctypes.c_int)]


class SpsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None
_P = ctypes.c_void_p
_D = ctypes.c_void_p  # device double*
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_alloc_refs = None   # the callbacks handed to the library (kept alive while installed)


def lib():
    """Load libsps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with paper_2506_14792_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "sps_set_allocator": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
        "sps_build_problem": (ctypes.c_int, [ctypes.POINTER(SpsDesc), _P, ctypes.POINTER(_P)]),
        "sps_build_rbc_batch": (ctypes.c_int, [ctypes.POINTER(SpsDesc), ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                               _P, ctypes.POINTER(_P)]),
        "sps_state_size": (ctypes.c_longlong, [_P]),
        "sps_factor": (ctypes.c_int, [_P]),
        "sps_step": (ctypes.c_int, [_P, _D, ctypes.c_int]),
        "sps_adjoint_step": (ctypes.c_int, [_P, _D, ctypes.c_int]),
        "sps_cost": (ctypes.c_int, [_P, _D, _D, _D]),
        "sps_gradient": (ctypes.c_int, [_P, _D, ctypes.c_int, _D, _D, _D, _D, _D]),
        "sps_initial_state": (ctypes.c_int, [_P, _D, _D]),
        "sps_initial_state_adjoint": (ctypes.c_int, [_P, _D, _D]),
        "sps_eval_F": (ctypes.c_int, [_P, _D, _D]),
        "sps_eval_F_vjp": (ctypes.c_int, [_P, _D, _D, _D]),
        "sps_eval_F_noalloc": (ctypes.c_int, [_P, _D, _D]),
        "sps_couette_frame": (ctypes.c_int, [_P, _D, _D, ctypes.c_int, ctypes.c_int]),
        "sps_solve": (ctypes.c_int, [_P, _D, _D, ctypes.c_int]),
        "sps_set_dt": (ctypes.c_int, [_P, ctypes.c_double]),
        "sps_set_checkpoint_file": (ctypes.c_int, [_P, ctypes.c_char_p]),
        "sps_set_outer_slots": (ctypes.c_int, [_P, ctypes.c_int]),
        "sps_set_outer_costs": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double]),
        "sps_checkpoint_schedule_costs": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                         ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                         ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                         ctypes.POINTER(ctypes.c_double)]),
        "sps_stability": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int, _D, _D, _D, _D]),
        "sps_stability_vector_sens": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int, _D, _D, _D, _D, _D]),
        "sps_stability_arnoldi": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D,
                                                 _D]),
        "sps_set_timesteps": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
        "sps_set_checkpointing": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
        "sps_checkpoint_schedule": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_int)]),
        "sps_lbvp_solve": (ctypes.c_int, [_P, _D, _D]),
        "sps_lbvp_adjoint": (ctypes.c_int, [_P, _D, _D]),
        "sps_timer_enable": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
        "sps_timer_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]),
        "sps_set_graph": (ctypes.c_int, [_P, ctypes.c_int]),
        "sps_build_sh_batch": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, ctypes.POINTER(_P)]),
        "sps_sh_tuning": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_double)]),
        "sps_build_couette": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _P,
                                             ctypes.POINTER(_P)]),
        "sps_build_kolmo": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, _P, ctypes.POINTER(_P)]),
        "sps_kolmo_set_params": (ctypes.c_int, [_P, _D]),
        "sps_kolmo_forward": (ctypes.c_int, [_P, _D, ctypes.c_int, _D, _D, ctypes.c_int, ctypes.c_int]),
        "sps_kolmo_rollout": (ctypes.c_int, [_P, _D, _D, ctypes.c_int, _D, _D, _D, _D]),
        "sps_kolmo_param_vjp": (ctypes.c_int, [_P, _D, _D, _D]),
        "sps_kolmo_adam": (ctypes.c_int, [_P, _D, _D, _D, _D, ctypes.c_double, ctypes.c_int]),
        "sps_cnn_build": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, ctypes.POINTER(_P)]),
        "sps_cnn_nparam": (ctypes.c_int, []),
        "sps_cnn_set_params": (ctypes.c_int, [_P, _D]),
        "sps_cnn_forward": (ctypes.c_int, [_P, _D, _D]),
        "sps_cnn_vjp": (ctypes.c_int, [_P, _D, _D, _D, _D]),
        "sps_cnn_destroy": (None, [_P]),
        "sps_sync": (ctypes.c_int, [_P]),
        "sps_last_error": (ctypes.c_char_p, []),
        "sps_destroy": (None, [_P]),
        "sps_rbc_host_bands": (ctypes.c_int, [ctypes.POINTER(SpsDesc), ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int), _P, _P, _P, _P, _P, _P, _P]),
        "sps_build_poiseuille": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, ctypes.POINTER(_P)]),
        "sps_poiseuille_solve": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                ctypes.c_int, _D, _D, _D, _D, _D]),
        "sps_poiseuille_host_band": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                                    _P, _P, _P, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def use_torch_allocator(on=True):
    """Device memory of the problems built from now on comes from torch's caching allocator
    (sps_set_allocator with callbacks into torch.cuda.caching_allocator_alloc / _delete);
    on=False returns to hipMalloc."""
    global _alloc_refs
    if not on:
        _check(lib().sps_set_allocator(None, None, None))
        _alloc_refs = None
        return
    import torch
    dev = torch.cuda.current_device()

    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev)
        except Exception:   # out of memory: the library reports SPS_E_NOMEM
            return None

    def free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    refs = (_ALLOC_T(alloc), _FREE_T(free))
    _check(lib().sps_set_allocator(ctypes.cast(refs[0], ctypes.c_void_p), ctypes.cast(refs[1], ctypes.c_void_p), None))
    _alloc_refs = refs


def _check(rc):
    if rc != 0:
        raise SpsError(rc, lib().sps_last_error().decode())


def _ptr(t, n=None):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 tensor on the GPU")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} doubles, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def make_desc(equation, nx, nz=0, lx=1.0, param0=0.0, param1=0.0, dealias=1.5, dt=1e-3,
              checkpoint_every=1, max_steps=1, scheme=None):
    if scheme is None:
        scheme = RK222 if equation == RBC2D else SBDF2
    return SpsDesc(equation, scheme, nx, nz, lx, param0, param1, dealias, dt, checkpoint_every, max_steps)


def checkpoint_schedule(nsteps, slots):
    """The binomial checkpointing schedule as two lists of (op, a, b) actions, forward sweep and
    reverse sweep (op 1 advance a -> b, 2 store step b in slot a, 3 load slot a (step b),
    4 record step a and run its adjoint).  Host-only: no device is used."""
    out = []
    for phase in (0, 1):
        count = ctypes.c_int(0)
        rc = lib().sps_checkpoint_schedule(nsteps, slots, phase, None, 0, ctypes.byref(count))
        if rc not in (0, -1) or count.value == 0:
            _check(rc)
        buf = (ctypes.c_int * (3 * count.value))()
        _check(lib().sps_checkpoint_schedule(nsteps, slots, phase, buf, count.value, ctypes.byref(count)))
        out.append([tuple(buf[3 * i:3 * i + 3]) for i in range(count.value)])
    return out[0], out[1]


def checkpoint_schedule_costs(nsteps, slots, adv, wr, rd):
    """The checkpointing schedule of least cost (adv per forward step of the reverse sweep, wr per
    stored state, rd per loaded state) in the format of checkpoint_schedule, and its cost."""
    out = []
    cost = ctypes.c_double(0.0)
    for phase in (0, 1):
        count = ctypes.c_int(0)
        rc = lib().sps_checkpoint_schedule_costs(nsteps, slots, adv, wr, rd, phase, None, 0, ctypes.byref(count), None)
        if rc not in (0, -1) or count.value == 0:
            _check(rc)
        buf = (ctypes.c_int * (3 * count.value))()
        _check(lib().sps_checkpoint_schedule_costs(nsteps, slots, adv, wr, rd, phase, buf, count.value,
                                                   ctypes.byref(count), ctypes.byref(cost)))
        out.append([tuple(buf[3 * i:3 * i + 3]) for i in range(count.value)])
    return out[0], out[1], cost.value


class Problem:
    """A built problem on the current HIP stream (torch.cuda.current_stream())."""

    nparam_grad = 0   # length of dJdtheta (0: the problem has no parameter gradient)

    def __init__(self, equation, nx, nz=0, lx=1.0, param0=0.0, param1=0.0, dealias=1.5, dt=1e-3,
                 checkpoint_every=1, max_steps=1, scheme=None, stream=None):
        import torch
        self.desc = make_desc(equation, nx, nz, lx, param0, param1, dealias, dt, checkpoint_every, max_steps, scheme)
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = _P()
        _check(lib().sps_build_problem(ctypes.byref(self.desc), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n = int(lib().sps_state_size(h))
        self.tape_id = 0   # advanced by every forward sweep; a reverse sweep needs the latest one
        # the 2D problem's parameter gradient: (dJ/dRa, dJ/dPr)
        self.nparam_grad = 2 if equation == RBC2D else 0

    def close(self):
        if getattr(self, "_h", None):
            lib().sps_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- ABI calls
    def factor(self):
        _check(lib().sps_factor(self._h))

    def step(self, X, nsteps):
        _check(lib().sps_step(self._h, _ptr(X, self.n), nsteps))
        self.tape_id += 1

    def adjoint_step(self, Xbar, nsteps):
        _check(lib().sps_adjoint_step(self._h, _ptr(Xbar, self.n), nsteps))

    def cost(self, X, J, dJdX):
        _check(lib().sps_cost(self._h, _ptr(X, self.n), _ptr(J, 1), _ptr(dJdX, self.n)))

    def gradient(self, X0, nsteps, XN, dJdX0, J, dJdXN=None, dJdtheta=None):
        self.tape_id += 1
        _check(lib().sps_gradient(self._h, _ptr(X0, self.n), nsteps, _ptr(dJdXN, self.n), _ptr(XN, self.n),
                                  _ptr(dJdX0, self.n), _ptr(dJdtheta, self.nparam_grad or None), _ptr(J, 1)))

    def initial_state(self, grid, X):
        _check(lib().sps_initial_state(self._h, _ptr(grid), _ptr(X, self.n)))

    def initial_state_adjoint(self, Xbar, grid_bar):
        _check(lib().sps_initial_state_adjoint(self._h, _ptr(Xbar, self.n), _ptr(grid_bar)))

    def eval_F(self, X, F):
        _check(lib().sps_eval_F(self._h, _ptr(X, self.n), _ptr(F, self.n)))

    def frame(self, X, out, to_library=True, cotangent=False):
        """Physical (u, v, w, p, taus) <-> library (u_par, v, u_perp, p, scaled taus) layout of a
        state or of a cotangent (sps_couette_frame), device tensors of n doubles."""
        _check(lib().sps_couette_frame(self._h, _ptr(X, self.n), _ptr(out, self.n), int(bool(to_library)),
                                       int(bool(cotangent))))

    def eval_F_noalloc(self, X, F):
        _check(lib().sps_eval_F_noalloc(self._h, _ptr(X, self.n), _ptr(F, self.n)))

    def eval_F_vjp(self, X, Fbar, Xbar):
        _check(lib().sps_eval_F_vjp(self._h, _ptr(X, self.n), _ptr(Fbar, self.n), _ptr(Xbar, self.n)))

    def solve(self, R, X, adjoint=False):
        _check(lib().sps_solve(self._h, _ptr(R, self.n), _ptr(X, self.n), int(bool(adjoint))))

    def stability(self, sigma=0.0, iters=30):
        """Growth rate nearest sigma of every wavenumber's perturbation of the conduction state,
        right and left eigenvectors and (d lambda/dRa, d lambda/dk): complex CUDA tensors
        lam [K], X [K, S], Y [K, S], dlam [K, 2] (2D problem)."""
        import torch
        K = self.n // (2 * (4 * self.desc.nz + 7))
        S = 4 * self.desc.nz + 7
        lam = torch.zeros(2 * K, dtype=torch.float64, device="cuda")
        X = torch.zeros(self.n, dtype=torch.float64, device="cuda")
        Y = torch.zeros_like(X)
        dlam = torch.zeros(4 * K, dtype=torch.float64, device="cuda")
        _check(lib().sps_stability(self._h, float(sigma), int(iters), _ptr(lam), _ptr(X, self.n), _ptr(Y, self.n),
                                   _ptr(dlam)))
        c = lambda t, *shape: torch.view_as_complex(t.view(*shape, 2))
        return c(lam, K), c(X, K, S), c(Y, K, S), c(dlam, K, 2)

    def stability_vector_sens(self, sigma, lam, X, Y, dlam, iters=20):
        """Eigenvector sensitivities dX/dRa and dX/dk (<X, dX> = 0) from the outputs of
        stability(sigma): complex CUDA tensor [2, K, S]."""
        import torch
        S = 4 * self.desc.nz + 7
        K = self.n // (2 * S)
        dX = torch.zeros(2 * self.n, dtype=torch.float64, device="cuda")
        args = [torch.view_as_real(t.to(torch.complex128).contiguous()).reshape(-1) for t in (lam, X, Y, dlam)]
        _check(lib().sps_stability_vector_sens(self._h, float(sigma), int(iters), *[_ptr(a) for a in args],
                                               _ptr(dX)))
        return torch.view_as_complex(dX.view(2, K, S, 2))

    def stability_arnoldi(self, sigma=0.0, m=24, nev=4, v0=None, want_vectors=True, want_H=False):
        """The nev eigenvalues nearest sigma of every wavenumber by shift-invert Arnoldi with m
        steps: complex CUDA tensors lam [K, nev], X [K, nev, S] (or None), residuals res
        [K, nev] (float64) and the Arnoldi matrices H [K, m+1, m] (or None).  v0: complex
        [K, S] start vectors (CUDA), None for the fixed start (2D problem)."""
        import torch
        S = 4 * self.desc.nz + 7
        K = self.n // (2 * S)
        lam = torch.zeros(2 * K * nev, dtype=torch.float64, device="cuda")
        res = torch.zeros(K * nev, dtype=torch.float64, device="cuda")
        X = torch.zeros(2 * K * nev * S, dtype=torch.float64, device="cuda") if want_vectors else None
        H = torch.zeros(2 * K * (m + 1) * m, dtype=torch.float64, device="cuda") if want_H else None
        v = None
        if v0 is not None:
            v = torch.view_as_real(v0.to(torch.complex128).contiguous()).reshape(-1)
            assert v.numel() == self.n and v.is_cuda
        _check(lib().sps_stability_arnoldi(self._h, float(sigma), int(m), int(nev), _ptr(v), _ptr(lam), _ptr(X),
                                           _ptr(res), _ptr(H)))
        c = lambda t, *shape: None if t is None else torch.view_as_complex(t.view(*shape, 2))
        return c(lam, K, nev), c(X, K, nev, S), res.view(K, nev), c(H, K, m + 1, m)

    def set_outer_slots(self, slots):
        """Outer-level states of CKPT_TWO_LEVEL (0: one per segment; fewer: nested binomial)."""
        _check(lib().sps_set_outer_slots(self._h, int(slots)))
        self.tape_id += 1

    def set_outer_costs(self, write_cost, read_cost):
        """Write and read costs of one outer state in forward steps (both >= 0: the nested
        schedule of least cost; both negative: the binomial placement)."""
        _check(lib().sps_set_outer_costs(self._h, float(write_cost), float(read_cost)))
        self.tape_id += 1

    def set_checkpoint_file(self, path):
        """Disk level of CKPT_TWO_LEVEL: segment starts in this file (created, removed with the
        problem); None returns to pinned host memory."""
        _check(lib().sps_set_checkpoint_file(self._h, None if path is None else str(path).encode()))
        self.tape_id += 1

    def set_dt(self, dt):
        """A new constant step for the following runs (refactors the implicit matrices; drops the
        recorded run)."""
        _check(lib().sps_set_dt(self._h, float(dt)))
        self.tape_id += 1

    def set_timesteps(self, dts=None):
        """Variable step sizes (a host sequence) for the following runs; None: the constant dt."""
        if dts is None:
            _check(lib().sps_set_timesteps(self._h, None, 0))
        else:
            import numpy as np
            h = np.ascontiguousarray(dts, dtype=np.float64)
            _check(lib().sps_set_timesteps(self._h, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(h.size)))
        self.tape_id += 1

    def set_checkpointing(self, scheme, slots=0):
        """CKPT_UNIFORM (checkpoints every checkpoint_every steps), CKPT_BINOMIAL with `slots`
        stored states, or CKPT_TWO_LEVEL (segment starts in host memory, binomial inside a segment
        on `slots` device states); drops the recorded forward run."""
        _check(lib().sps_set_checkpointing(self._h, int(scheme), int(slots)))
        self.tape_id += 1

    def lbvp_solve(self, f, X):
        """X = L^-1 (M f + c): the boundary value problem of the operator (2D problem only)."""
        _check(lib().sps_lbvp_solve(self._h, _ptr(f, self.n), _ptr(X, self.n)))

    def lbvp_adjoint(self, Xbar, fbar):
        """fbar = M^H L^-H Xbar: the cotangent of the forcing of lbvp_solve."""
        _check(lib().sps_lbvp_adjoint(self._h, _ptr(Xbar, self.n), _ptr(fbar, self.n)))

    def timer_enable(self, kind=0, on=True):
        _check(lib().sps_timer_enable(self._h, kind, int(bool(on))))

    def timer_read(self):
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        _check(lib().sps_timer_read(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def set_graph(self, on=True):
        _check(lib().sps_set_graph(self._h, int(bool(on))))

    def sync(self):
        _check(lib().sps_sync(self._h))


class RbcBatch(Problem):
    """A batch of 2D problems (nx x nz, Lx, Pr, dt, checkpoints and max_steps shared) with one
    Rayleigh number per instance; states, grids and J hold the instances in order."""

    def __init__(self, ra, nx, nz, lx, Pr, dt=1e-3, checkpoint_every=1, max_steps=1, scheme=RK222, stream=None):
        import torch
        self.batch = len(ra)
        self.desc = make_desc(RBC2D, nx, nz, lx, float(ra[0]), Pr, 1.5, dt, checkpoint_every, max_steps, scheme)
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        arr = (ctypes.c_double * self.batch)(*[float(v) for v in ra])
        h = _P()
        _check(lib().sps_build_rbc_batch(ctypes.byref(self.desc), self.batch, arr, ctypes.c_void_p(stream.cuda_stream),
                                         ctypes.byref(h)))
        self._h = h
        self.n = int(lib().sps_state_size(h))
        self.tape_id = 0
        self.grid_size = self.batch * nx * nz

    def cost(self, X, J, dJdX):
        _check(lib().sps_cost(self._h, _ptr(X, self.n), _ptr(J, self.batch), _ptr(dJdX, self.n)))

    def gradient(self, X0, nsteps, XN, dJdX0, J, dJdXN=None):
        self.tape_id += 1
        _check(lib().sps_gradient(self._h, _ptr(X0, self.n), nsteps, _ptr(dJdXN, self.n), _ptr(XN, self.n),
                                  _ptr(dJdX0, self.n), None, _ptr(J, self.batch)))

    def initial_state(self, grid, X):
        _check(lib().sps_initial_state(self._h, _ptr(grid, self.grid_size), _ptr(X, self.n)))

    def initial_state_adjoint(self, Xbar, grid_bar):
        _check(lib().sps_initial_state_adjoint(self._h, _ptr(Xbar, self.n), _ptr(grid_bar, self.grid_size)))


class ShBatch(Problem):
    """A batch of independent 2D Swift-Hohenberg problems (sizes n[i] x n[i], parameters r[i])
    in one problem handle; states and grids of the instances are concatenated."""

    def __init__(self, n, r, lx=16.0 * np.pi, dt=0.02, max_steps=1, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        self.sizes = [int(v) for v in n]
        self.batch = len(self.sizes)
        na = (ctypes.c_int * self.batch)(*self.sizes)
        ra = (ctypes.c_double * self.batch)(*[float(v) for v in r])
        h = _P()
        _check(lib().sps_build_sh_batch(self.batch, na, ra, float(lx), float(dt), int(max_steps),
                                        ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n = int(lib().sps_state_size(h))
        self.tape_id = 0
        self.grid_size = sum(v * v for v in self.sizes)

    def cost(self, X, J, dJdX):
        _check(lib().sps_cost(self._h, _ptr(X, self.n), _ptr(J, self.batch), _ptr(dJdX, self.n)))

    def gradient(self, X0, nsteps, XN, dJdX0, J, dJdXN=None):
        self.tape_id += 1
        _check(lib().sps_gradient(self._h, _ptr(X0, self.n), nsteps, _ptr(dJdXN, self.n), _ptr(XN, self.n),
                                  _ptr(dJdX0, self.n), None, _ptr(J, self.batch)))

    def initial_state(self, grid, X):
        _check(lib().sps_initial_state(self._h, _ptr(grid, self.grid_size), _ptr(X, self.n)))

    def initial_state_adjoint(self, Xbar, grid_bar):
        _check(lib().sps_initial_state_adjoint(self._h, _ptr(Xbar, self.n), _ptr(grid_bar, self.grid_size)))

    def tuning(self):
        ct = (ctypes.c_int * 4)()
        rt = (ctypes.c_int * 4)()
        b = ctypes.c_int()
        t = ctypes.c_int()
        ms = ctypes.c_double()
        _check(lib().sps_sh_tuning(self._h, ct, rt, ctypes.byref(b), ctypes.byref(t), ctypes.byref(ms)))
        return {"col_tile": list(ct), "row_pairs": list(rt), "blocks": b.value, "threads": t.value,
                "step_ms": ms.value}


class Couette(Problem):
    """3D plane Couette flow (nx x ny x nz: Fourier x Chebyshev x Fourier, periods lx, lz, walls
    y = -1, 1 moving with -1, 1, Reynolds number Re), RK222 step dt with checkpoints; states per
    mode k = m nz + n in the layout (u_par, v, u_perp, p, taus) of the library's header."""

    def __init__(self, nx, ny, nz, lx=4.0 * np.pi, lz=2.0 * np.pi, Re=400.0, dt=0.01, checkpoint_every=100,
                 max_steps=1, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.K = (self.nx // 2) * self.nz
        h = _P()
        _check(lib().sps_build_couette(self.nx, self.ny, self.nz, float(lx), float(lz), float(Re), float(dt),
                                       int(checkpoint_every), int(max_steps), ctypes.c_void_p(stream.cuda_stream),
                                       ctypes.byref(h)))
        self._h = h
        self.n = int(lib().sps_state_size(h))
        self.tape_id = 0
        self.lx, self.lz = float(lx), float(lz)

    def state_from_velocity(self, c, cotangent=False):
        """(K, 3, ny) complex Chebyshev coefficients of (u, v, w) per mode (host) -> a device state
        in the library layout (p and taus zero): the coefficients are placed into the physical
        layout on the host and rotated into the library's frame by sps_couette_frame."""
        import torch
        K, N = self.K, self.ny
        X = np.zeros((K, 4 * N + 7), complex)
        X[:, :3 * N] = np.asarray(c).reshape(K, 3 * N)
        phys = torch.from_numpy(np.ascontiguousarray(X).view(np.float64).ravel().copy()).cuda()
        out = torch.empty_like(phys)
        self.frame(phys, out, True, cotangent)
        return out


class Kolmogorov(Problem):
    """A batch of 2D Kolmogorov flows (N x N modes on [0, 2 pi)^2, Re, linear drag, SBDF2 step dt), with the
    closure network in the explicit term when closure is set.  States of the instances are
    concatenated; keep_history keeps every state of the last forward run for the gradients."""

    def __init__(self, batch, N, Re=1000.0, dt=0.01, max_steps=1, closure=False, keep_history=True, drag=0.0,
                 stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        self.batch, self.N = int(batch), int(N)
        h = _P()
        _check(lib().sps_build_kolmo(self.batch, self.N, float(Re), float(drag), float(dt), int(max_steps),
                                     int(bool(closure)),
                                     int(bool(keep_history)), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n = int(lib().sps_state_size(h))
        self.nparam = int(lib().sps_cnn_nparam())
        self.tape_id = 0

    def set_params(self, theta):
        _check(lib().sps_kolmo_set_params(self._h, _ptr(theta, self.nparam)))

    def forward(self, X0, nsteps, XN=None, snap=None, every=1, nc=0):
        self.tape_id += 1
        ns = None if snap is None else (nsteps // every) * self.batch * nc * nc
        _check(lib().sps_kolmo_forward(self._h, _ptr(X0, self.n), int(nsteps), _ptr(XN, self.n), _ptr(snap, ns),
                                       int(every), int(nc)))

    def rollout(self, X0, targets, nsteps, XN=None, J=None, dJdX0=None, dJdtheta=None):
        self.tape_id += 1
        _check(lib().sps_kolmo_rollout(self._h, _ptr(X0, self.n), _ptr(targets, nsteps * self.n), int(nsteps),
                                       _ptr(XN, self.n), _ptr(J, self.batch), _ptr(dJdX0, self.n),
                                       _ptr(dJdtheta, self.nparam)))

    def param_vjp(self, X, Fbar, theta_bar):
        _check(lib().sps_kolmo_param_vjp(self._h, _ptr(X, self.n), _ptr(Fbar, self.n), _ptr(theta_bar, self.nparam)))

    def adam(self, theta, grad, m1, m2, lr, t):
        _check(lib().sps_kolmo_adam(self._h, _ptr(theta, self.nparam), _ptr(grad, self.nparam), _ptr(m1, self.nparam),
                                    _ptr(m2, self.nparam), float(lr), int(t)))


class ClosureNet:
    """The closure network alone (batch images of H x W on the GPU)."""

    def __init__(self, batch, H, W, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.batch, self.H, self.W = batch, H, W
        h = _P()
        _check(lib().sps_cnn_build(batch, H, W, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.nparam = int(lib().sps_cnn_nparam())
        self.npix = batch * H * W

    def close(self):
        if getattr(self, "_h", None):
            lib().sps_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        _check(lib().sps_cnn_set_params(self._h, _ptr(theta, self.nparam)))

    def forward(self, x, y):
        _check(lib().sps_cnn_forward(self._h, _ptr(x, self.npix), _ptr(y, self.npix)))

    def vjp(self, x, ybar, xbar, theta_bar=None):
        _check(lib().sps_cnn_vjp(self._h, _ptr(x, self.npix), _ptr(ybar, self.npix), _ptr(xbar, self.npix),
                                 _ptr(theta_bar, self.nparam)))


class PoiseuilleStability(Problem):
    """Linear stability of plane Poiseuille flow (the neutral-curve example): nsys systems of
    (alpha, Re, shift) solved at once, one thread block each, by sps_poiseuille_solve.  States are
    S = 3 nz + 5 complex slots (u, v, p Chebyshev coefficients and five taus)."""

    EIGENPAIR, NEWTON_RE, NEWTON_ALPHA, CONTINUE = 0, 1, 2, 3

    def __init__(self, nz, max_systems=1, stream=None):
        import torch
        self.nz = nz
        self.max_systems = max_systems
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = _P()
        _check(lib().sps_build_poiseuille(int(nz), int(max_systems), ctypes.c_void_p(stream.cuda_stream),
                                          ctypes.byref(h)))
        self._h = h
        self.S = int(lib().sps_state_size(h)) // 2
        self.n = 2 * self.S

    def solve(self, params, lam, dlam, info, iters=20, mode=0, tol=1e-12, maxit=1, X=None, Y=None):
        """params: sequence of (alpha, Re, sigma) or (alpha, Re, sigma, ds) with sigma complex;
        lam (2 nsys doubles), dlam (4 nsys), info (3 nsys), X, Y (2 S nsys, optional): device
        float64 tensors."""
        ns = len(params)
        rows = [tuple(p) + (0.0,) * (4 - len(p)) for p in params]
        arr = (ctypes.c_double * (5 * ns))(*[float(v) for a, r, sg, ds in rows
                                              for v in (a, r, complex(sg).real, complex(sg).imag, ds)])
        _check(lib().sps_poiseuille_solve(self._h, ns, ctypes.cast(arr, ctypes.c_void_p), int(iters), int(mode),
                                          float(tol), int(maxit), _ptr(lam, 2 * ns), _ptr(dlam, 4 * ns),
                                          _ptr(info, 3 * ns), _ptr(X, self.n * ns), _ptr(Y, self.n * ns)))


def poiseuille_host_band(nz, alpha, Re, sigma):
    """Host-assembled complex band of sigma M + L of the Poiseuille stability problem (no GPU)."""
    S, kl, ku = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    sg = complex(sigma)
    _check(lib().sps_poiseuille_host_band(int(nz), float(alpha), float(Re), sg.real, sg.imag, ctypes.byref(S),
                                          ctypes.byref(kl), ctypes.byref(ku), None, None, None, None))
    n, bw = S.value, kl.value + ku.value + 1
    band = np.zeros((n, bw), complex)
    rowmap = np.zeros(n, np.int32); colmap = np.zeros(n, np.int32); rho = np.zeros(n)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().sps_poiseuille_host_band(int(nz), float(alpha), float(Re), sg.real, sg.imag, ctypes.byref(S),
                                          ctypes.byref(kl), ctypes.byref(ku), p(band), p(rowmap), p(colmap), p(rho)))
    return dict(S=n, kl=kl.value, ku=ku.value, band=band, rowmap=rowmap, colmap=colmap, rho=rho)


def rbc_host_bands(nx, nz, lx, Ra, Pr, dt=1e-3):
    """Host-assembled real banded systems of the RBC problem (no GPU needed)."""
    d = make_desc(RBC2D, nx, nz, lx, Ra, Pr, 1.5, dt, 1, 1)
    kl, ku = ctypes.c_int(), ctypes.c_int()
    _check(lib().sps_rbc_host_bands(ctypes.byref(d), ctypes.byref(kl), ctypes.byref(ku),
                                    None, None, None, None, None, None, None))
    K, S = nx // 2, 4 * nz + 7
    bw = kl.value + ku.value + 1
    BM = np.zeros((K, S, bw)); BL = np.zeros((K, S, bw))
    rowmap = np.zeros(S, np.int32); colmap = np.zeros(S, np.int32)
    rowph = np.zeros(S, np.int8); colph = np.zeros(S, np.int8); rho = np.zeros(S)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().sps_rbc_host_bands(ctypes.byref(d), ctypes.byref(kl), ctypes.byref(ku), p(BM), p(BL),
                                    p(rowmap), p(colmap), p(rowph), p(colph), p(rho)))
    return dict(kl=kl.value, ku=ku.value, BM=BM, BL=BL, rowmap=rowmap, colmap=colmap, rowph=rowph,
                colph=colph, rho=rho)
