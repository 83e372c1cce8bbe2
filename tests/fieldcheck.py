"""Field comparison used by the GPU parity tests (not a test module).

The criterion is the relative L-inf error per field, max_x |a - b| / max_x |b|
with b the reference (the oracle, or a reference GPU run where a test says
so), for n and eps.  The flow u = (U^x, U^y) is compared as a vector:
max_x |u_a - u_b| / max(max_x |u_b|, U_REST), with |.| the Euclidean norm of
the two components.  A component that vanishes by symmetry (U^y of a tube)
is then judged against the size of the flow, not against its own
rounding-level maximum.  A fluid at rest has no flow scale of its own (its u
is rounding noise, ~1e-16 in FP64), so flows slower than U_REST = 1e-3 (in
units of c) are judged against that speed; every moving workload of the
tests is faster.
"""
import sys

import numpy as np

FLOOR = 1e-300
U_REST = 1e-3


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def rel_linf(a, b):
    den = np.abs(b).max()
    if den < FLOOR:
        return float(np.abs(a - b).max())
    return float(np.abs(a - b).max() / den)


def flow_error(ux, uy, rux, ruy):
    """max |u - u_ref| / max(max |u_ref|, U_REST) over the grid, u as a 2-vector."""
    du = np.hypot(np.asarray(ux) - rux, np.asarray(uy) - ruy).max()
    umax = np.hypot(rux, ruy).max()
    return float(du / max(umax, U_REST))


def field_errors(got, exp):
    """(n, eps, u) errors of got = (n, eps, ux, uy) against exp."""
    return (rel_linf(got[0], exp[0]), rel_linf(got[1], exp[1]),
            flow_error(got[2], got[3], exp[2], exp[3]))


def check_fields(got, exp, tol, label):
    """Assert every field of got within tol of exp; returns the errors."""
    errs = field_errors(got, exp)
    say("%s n=%.3e eps=%.3e u=%.3e (tol %.0e)" % ((label,) + errs + (tol,)))
    for name, e in zip(("n", "eps", "u"), errs):
        assert e <= tol, (label, name, e, tol)
    return errs


def site_errors(got, ref, uscale):
    """Errors at one site: n and eps relative to the reference site value,
    the flow vector relative to max(uscale, U_REST), uscale being the largest
    reference |u| among the sampled sites (so that a site at rest is judged
    against the flow's size)."""
    n, eps, ux, uy = got
    rn, reps, rux, ruy = ref
    e_u = np.hypot(ux - rux, uy - ruy)
    return abs(n - rn) / abs(rn), abs(eps - reps) / abs(reps), e_u / max(uscale, U_REST)
