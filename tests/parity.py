"""Field-by-field parity of states in the per-wavenumber layout X[k][s] (S = 4N + 7 slots:
four blocks of N Chebyshev coefficients, then seven tau slots), shared by the GPU parity tests
of the 2D Rayleigh-Benard problem, its boundary value problem and plane Couette flow.

A whole-array error max|gpu - ref| / max|ref| lets a field far smaller than the array's
largest entry go almost unchecked (at 256x64 the buoyancy is about 0.5 while the velocities
are about 1e-5).  Here every field is held to the tolerance of its own size: the u, w, b, p
blocks, each split into the k = 0 row (the horizontal means: conduction profile, hydrostatic
pressure) and the rows k >= 1, each group relative to its own largest reference entry.

Two allowances follow from what FP64 can resolve, not from the GPU:

* Background.  An optional base state (the conduction state, b = 1 - z and its hydrostatic
  pressure) is subtracted from both sides, so that a group measures the perturbation of the
  field.  Both implementations compute the whole field, background included; the rounding of
  the background's sums (a transform sums up to Ng = 384 grid values, so N_g eps ~ 4e-14 of the
  background's size, twice) cannot be subtracted away.  A group with a base therefore allows
  BACKGROUND times the largest entry of that field's base, on top of the relative tolerance.
* Taus.  The tau slots are auxiliary unknowns of each wavenumber's linear solve, often far
  smaller than the fields (at the plane Couette mean mode 5e-5 of them).  Their columns in the
  stage matrix M + dt gamma L carry dt gamma 4 nu or dt gamma 4 kappa (1.2e-6 at Ra = 1e6,
  dt = 1e-3), so an FP64 solve - any FP64 solve - resolves them only to about eps / 1.2e-6
  ~ 1e-10 of their wavenumbers' solution vector, while their effect on the fields (the tau
  times that coefficient) stays at rounding level.  The tau groups are therefore held relative
  to the largest entry of the state rows they belong to (k = 0, or k >= 1), at TAU_TOL = 1e-9
  (that floor with a margin of 10); every field is held at the test's own tolerance.

A group whose reference is below ZERO_GROUP times the whole array's largest entry is zero in
exact arithmetic (w and its taus at k = 0 by continuity and the walls, tau_p at k != 0, the
pressure and tau cotangents of an initial state) and holds only rounding noise; it is checked
absolutely, at ABS_FLOOR times the array's largest entry.
"""
import numpy as np

ZERO_GROUP = 1e-9
ABS_FLOOR = 1e-13
BACKGROUND = 1e-13
TAU_TOL = 1e-9

FIELD_NAMES = ("u", "w", "b", "p")


def groups(N, S):
    """(name, field index or None for the taus, slot slice, rows) of the groups of a [K][S] state."""
    out = []
    for rows, tag in ((slice(0, 1), "k=0"), (slice(1, None), "k>0")):
        for f, name in enumerate(FIELD_NAMES):
            out.append((f"{name}[{tag}]", f, slice(f * N, (f + 1) * N), rows))
        out.append((f"tau[{tag}]", None, slice(4 * N, S), rows))
    return out


def field_errors(got, ref, N, base=None, names=FIELD_NAMES):
    """Per-group results {name: (error, kind, raw)}: kind 'rel' (error beyond the background
    allowance over the group's scale, compared with the tolerance), 'tau' (the same for a tau
    group, compared with TAU_TOL) or 'abs' (zero group, over the whole array's largest entry,
    compared with ABS_FLOOR); raw is the error over the scale without the allowance."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    bg = np.zeros(len(FIELD_NAMES))
    full = ref   # the whole state (background included): the scale of the solve's rounding
    if base is not None:
        base = np.asarray(base)
        for f in range(len(FIELD_NAMES)):
            bg[f] = np.max(np.abs(base[:, f * N:(f + 1) * N])) if base.shape[1] > f * N else 0.0
        got = got - base
        ref = ref - base
    scale = np.max(np.abs(ref))
    res = {}
    for name, fi, sl, rows in groups(N, ref.shape[1]):
        label = name if fi is None else names[fi] + name[len(FIELD_NAMES[fi]):]
        r = ref[rows, sl]
        g = got[rows, sl]
        if r.size == 0:
            continue
        d = np.max(np.abs(g - r))
        m = np.max(np.abs(r))
        if fi is None:   # taus: relative to the whole state of their wavenumbers
            m = max(m, np.max(np.abs(full[rows, :])))
        if scale == 0.0:
            res[label] = (d, "abs", d)
        elif m > ZERO_GROUP * scale:
            # the relative tolerance on the group, widened by the background's rounding
            allow = BACKGROUND * bg[fi] if fi is not None else 0.0
            res[label] = (max(d - allow, 0.0) / m, "rel" if fi is not None else "tau", d / m)
        else:
            res[label] = (d / scale, "abs", d / scale)
    return res


def check_fields(got, ref, N, tol, base=None, what="", names=FIELD_NAMES):
    """Assert every group within tol (relative groups) or ABS_FLOOR (zero groups); returns
    the largest relative-group error."""
    errs = field_errors(got, ref, N, base, names)
    bound = {"rel": tol, "tau": max(tol, TAU_TOL), "abs": ABS_FLOOR}
    bad = {k: v for k, v in errs.items() if not v[0] <= bound[v[1]]}

    def fmt(k, v):
        tag = {"rel": "", "tau": " (tau)", "abs": " abs"}[v[1]]
        extra = f" [raw {v[2]:.1e}]" if v[1] == "rel" and v[2] > v[0] else ""
        return f"{k} {v[0]:.2e}{tag}{extra}"

    print(f"{what}: " + ", ".join(fmt(k, v) for k, v in errs.items()), flush=True)
    assert not bad, f"{what}: fields over the bound: {bad}"
    rel = [v[0] for v in errs.values() if v[1] == "rel"]
    return max(rel) if rel else 0.0
