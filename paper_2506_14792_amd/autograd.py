"""torch.autograd bindings of the library: the forward sweep and its discrete adjoint
(equ:adjoint; the reverse sweep with checkpoint-and-recompute of the Supplementary's IVP
adjoint), the initial transform of a grid field, the boundary value problem of the operator
and the built-in cost.

States are float64 CUDA tensors in the library's state layout (complex coefficients as
(re, im) pairs); cotangents use the real inner product of that layout, which is the
convention of the library's adjoint calls.  Each call runs on the problem's HIP stream and
only marshals arguments: every step of the computation is a library kernel.

A Problem records one forward run at a time; `Step.backward` checks that the run it reverses
is still the recorded one and raises otherwise (run backward before the next forward).
"""
import torch

from .sps import SpsError


class Step(torch.autograd.Function):
    """X_N = step(X_0) over nsteps steps; backward is sps_adjoint_step through the checkpoints."""

    @staticmethod
    def forward(ctx, X0, problem, nsteps):
        X = X0.detach().contiguous().clone()
        problem.step(X, nsteps)
        ctx.problem, ctx.nsteps, ctx.tape = problem, nsteps, problem.tape_id
        return X

    @staticmethod
    def backward(ctx, gX):
        P = ctx.problem
        if P.tape_id != ctx.tape:
            raise SpsError(-6, "the forward run of this Step is no longer the recorded one")
        g = gX.detach().contiguous().clone()
        P.adjoint_step(g, ctx.nsteps)
        return g, None, None


class StepSegments(torch.autograd.Function):
    """X_N over segments of constant step: for each (dt, nsteps) in turn, sps_set_dt(dt) (the
    implicit matrices refactored) and nsteps steps.  Backward reverses the segments from the
    last: each is set to its own step again, its forward sweep recomputed from the segment's
    stored initial state and reversed by sps_adjoint_step.  The problem is left at the first
    segment's step after backward and at the last one's after forward."""

    @staticmethod
    def forward(ctx, X0, problem, segments):
        X = X0.detach().contiguous().clone()
        starts = []
        for dt, n in segments:
            starts.append(X.clone())
            problem.set_dt(dt)
            problem.step(X, n)
        ctx.problem, ctx.segments, ctx.starts = problem, list(segments), starts
        return X

    @staticmethod
    def backward(ctx, gX):
        P = ctx.problem
        g = gX.detach().contiguous().clone()
        for (dt, n), X in zip(reversed(ctx.segments), reversed(ctx.starts)):
            P.set_dt(dt)
            P.step(X.clone(), n)
            P.adjoint_step(g, n)
        return g, None, None


class InitialState(torch.autograd.Function):
    """X_0 = T(grid): the scale-1 grid field into the state (e.g. the initial buoyancy)."""

    @staticmethod
    def forward(ctx, grid, problem):
        X = torch.zeros(problem.n, dtype=torch.float64, device=grid.device)
        problem.initial_state(grid.detach().contiguous(), X)
        ctx.problem, ctx.shape = problem, grid.shape
        return X

    @staticmethod
    def backward(ctx, gX):
        g = torch.zeros(ctx.shape, dtype=torch.float64, device=gX.device)
        ctx.problem.initial_state_adjoint(gX.detach().contiguous(), g)
        return g, None


class Cost(torch.autograd.Function):
    """The problem's built-in objective J(X) (kinetic energy for RBC, 1/2 ||u||^2 for KS)."""

    @staticmethod
    def forward(ctx, X, problem):
        J = torch.zeros(1, dtype=torch.float64, device=X.device)
        dJ = torch.zeros(problem.n, dtype=torch.float64, device=X.device)
        problem.cost(X.detach().contiguous(), J, dJ)
        ctx.save_for_backward(dJ)
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        (dJ,) = ctx.saved_tensors
        return dJ * gJ, None


class Lbvp(torch.autograd.Function):
    """X = L^-1 (M f + c), the boundary value problem of the operator (Supplementary, "Linear
    boundary value problems"); backward is its adjoint, M^H L^-H through the same factors."""

    @staticmethod
    def forward(ctx, f, problem):
        X = torch.zeros(problem.n, dtype=torch.float64, device=f.device)
        problem.lbvp_solve(f.detach().contiguous(), X)
        ctx.problem = problem
        return X

    @staticmethod
    def backward(ctx, gX):
        g = torch.zeros_like(gX)
        ctx.problem.lbvp_adjoint(gX.detach().contiguous(), g)
        return g, None


def lbvp(f, problem):
    return Lbvp.apply(f, problem)


def step(X0, problem, nsteps):
    return Step.apply(X0, problem, nsteps)


def step_segments(X0, problem, segments):
    return StepSegments.apply(X0, problem, segments)


def initial_state(grid, problem):
    return InitialState.apply(grid, problem)


def cost(X, problem):
    return Cost.apply(X, problem)
