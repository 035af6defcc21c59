"""Parity bars of the GPU tests against the FP64 oracle.

TEST INFRASTRUCTURE ONLY: used by the tests and the smoke check.

The oracle and the FP64 kernels evaluate the same method in independent
operation orders (the oracle: per-edge transverse splits, the update formula
as written, plain quotients, Gaussian elimination in the source stages; the
kernels: their own fused order), so they round differently.

TOL.  Every conserved field within 1e-11 of the oracle, relative to the
field's largest magnitude.

Deep water.  Depths of kilometres take the auxiliary fields (and, less, the
momenta) below what FP64 resolves.  The depth h is stored in FP64, so at
4000 m it carries an absolute rounding of up to 4.5e-13 m; the hydrostatic
term g h^ (d eta) passes that error to the acoustic waves and their
c^2-weighted components (c^2 = 9 g H = 3.5e5 m^2/s^2) into hp and h p_b.
The step map itself amplifies a one-ulp change of h into relative changes of
about 2e-10 in hp within one step, and the FP64 oracle is about 1e-10 away
from the extended-precision build of the same source on such cases (pinned
by tests/test_oracle_conditioning.py).  No two FP64 evaluations can agree to
1e-11 there.  The bar of a field is then the larger of TOL and SPREAD times the
oracle's own spread: the largest relative change of that field when the
oracle runs the case again from depths moved by one unit in the last place
(up or down, seeded, per wet cell).  The depth field itself keeps TOL,
because its spread is about 1e-15.
"""
import copy
import dataclasses

import numpy as np

TOL = 1e-11
SPREAD = 10.0
TWIN_SEEDS = (1, 2)


def field_errors(got, exp):
    """per field: max |got - exp| over max |exp| (absolute where exp is 0)"""
    scale = np.abs(exp).max(axis=(1, 2))
    err = np.abs(got - exp).max(axis=(1, 2))
    return np.where(scale > 0, err / np.where(scale > 0, scale, 1.0), err)


def perturb_depths(q, seed):
    """q with the depth of every wet cell moved one ulp up or down"""
    q = np.array(q, dtype=np.float64, copy=True)
    s = np.random.default_rng(seed).integers(0, 2, q[0].shape)
    moved = np.where(s > 0, np.nextafter(q[0], np.inf), np.nextafter(q[0], -np.inf))
    q[0] = np.where(q[0] > 0, moved, q[0])
    return q


def twin(w, seed):
    """a copy of a workload (single grid or patch set) whose initial depths
    are perturbed by one ulp"""
    w2 = copy.copy(w)
    if hasattr(w, "patches"):
        w2.patches = [dataclasses.replace(p, q=perturb_depths(p.q, seed + 7919 * k))
                      for k, p in enumerate(w.patches)]
    else:
        w2.q = perturb_depths(w.q, seed)
    return w2


def bars(exp, twins):
    """per-field bars for one state: max(TOL, SPREAD x spread of the twins)"""
    spread = np.zeros(exp.shape[0])
    for t in twins:
        spread = np.maximum(spread, field_errors(t, exp))
    return np.maximum(TOL, SPREAD * spread)


def oracle_bars(run, w, seeds=TWIN_SEEDS):
    """run(w) -> list of oracle states (7, ny, nx); returns (states, bars)
    with bars[k] the per-field bar of states[k]"""
    exp = run(w)
    runs = [run(twin(w, s)) for s in seeds]
    for r in runs:
        assert len(r) == len(exp) and all(a.shape == b.shape for a, b in zip(r, exp)), \
            "a twin run took another path (patch list or shapes differ)"
    return exp, [bars(e, [r[k] for r in runs]) for k, e in enumerate(exp)]


def assert_within(got, exp, bar, what=""):
    e = field_errors(got, exp)
    assert np.all(e <= bar), "%s field errors %s bars %s" % (
        what, np.array2string(e, precision=2), np.array2string(bar, precision=2))
    return e
