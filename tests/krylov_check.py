"""Shared parity check of a GPU (F)GMRES result against the oracle.

The oracle runs the same restarted iteration three times: with modified
Gram-Schmidt (the reference run), with classical Gram-Schmidt applied twice,
and with modified Gram-Schmidt from a right-hand side moved by a random
1e-15 relative perturbation.  The three are correct FP64 evaluations of one
iteration, so their spread measures how far rounding-level differences grow
over it on this input; the GPU result must stay inside that envelope:

* residual histories: 1e-8 relative above an absolute floor (relative to
  ||f||) of max(1e-11, 10 D), D the largest difference between the reference
  history and the two others, up to the step where those oracle histories
  part by more than 1e-8 relative; within a factor 10 after it;
* iteration counts: equal, except that a stop decided inside the rounding
  floor may move by the oracle runs' own spread (or a few steps once the
  floor reaches 1e-3 of the tolerance);
* solutions, relative L2 distance to the nearest of the three oracle runs:
  tier 1 = 1e-10; tier 2 = ten times the largest distance between any two
  oracle runs.  Nothing looser is accepted.  The tier that passed is
  printed.
"""

from __future__ import annotations

import numpy as np

from oracle import krylov as K

HIST_FLOOR = 1e-11     # absolute rounding floor of a relative-residual history
SOLUTION_BAR = 1e-10   # tier 1 of the solution check


def say(*a):
    print(*a, flush=True)


def perturbed(f, seed=99):
    """f moved by a random 1e-15 relative perturbation."""
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(len(f)) + 1j * rng.standard_normal(len(f))
    return f + 1e-15 * np.linalg.norm(f) / np.linalg.norm(p) * p


def compare_hist(got, want, tol=1e-8, stop=None, floor=HIST_FLOOR):
    """Element-wise: |got - want| <= tol |want| + floor over the common
    prefix (cut after the first entry above `stop`)."""
    m = min(len(got), len(want))
    if stop is not None:
        above = np.nonzero(np.asarray(want[:m]) > stop)[0]
        if len(above):
            m = min(m, above[0] + 1)
    g, w = np.asarray(got[:m]), np.asarray(want[:m])
    excess = np.abs(g - w) - (tol * np.abs(w) + floor)
    assert excess.max() <= 0, (float(np.abs(g - w)[excess.argmax()]), int(excess.argmax()), m)
    return m


def drift(h1, h2):
    m = min(len(h1), len(h2))
    return float(np.abs(np.asarray(h1[:m]) - np.asarray(h2[:m])).max())


def diverge_index(h1, h2, floor=HIST_FLOOR):
    """First step where two correct FP64 runs part beyond 1e-8 relative."""
    m = min(len(h1), len(h2))
    h1, h2 = np.asarray(h1[:m]), np.asarray(h2[:m])
    bad = np.nonzero(np.abs(h1 - h2) > 1e-8 * np.abs(h1) + floor)[0]
    return int(bad[0]) if len(bad) else m


def within_factor(got, want, m, factor=10.0, floor=HIST_FLOOR):
    g, w = np.asarray(got[m:]), np.asarray(want[m:])
    k = min(len(g), len(w))
    assert np.all(g[:k] <= factor * w[:k] + floor) and np.all(w[:k] <= factor * g[:k] + floor), m


def solution_tier(got_x, x, others, label=""):
    """Tier 1 (1e-10) or tier 2 (ten times the oracle runs' own spread);
    fails otherwise.  Returns the tier.  x is the reference run, others the
    other correct FP64 runs of the same iteration: the distance is taken to
    the nearest of them (the GPU orthogonalises like one of the variants, not
    necessarily like the reference), the spread is the largest distance
    between any two of them."""
    runs = [x] + list(others)
    nx = np.linalg.norm(x)
    err = min(np.linalg.norm(got_x - r) for r in runs) / nx
    spread = max(np.linalg.norm(a - b) for i, a in enumerate(runs) for b in runs[i + 1:]) / nx
    if err < SOLUTION_BAR:
        tier = 1
    else:
        assert err <= 10 * spread, ("solution outside the oracle's rounding envelope", label, err, spread)
        tier = 2
    say("parity tier %d %s: solution error %.3e, oracle spread %.3e" % (tier, label, err, spread))
    return tier


def check_krylov(got_x, got_hist, got_its, A, M, f, rtol, maxit, restart=20, flexible=False, label=""):
    """GPU GMRES / FGMRES result against the oracle under the bars of the
    module docstring.  Returns the oracle's iteration count."""
    x, hist, it, st = K.gmres(A, M, f, rtol=rtol, restart=restart, maxit=maxit, flexible=flexible)
    x2, hist2, it2, _ = K.gmres(A, M, f, rtol=rtol, restart=restart, maxit=maxit, flexible=flexible,
                                ortho="cgs2")
    x3, hist3, it3, _ = K.gmres(A, M, perturbed(f), rtol=rtol, restart=restart, maxit=maxit, flexible=flexible)
    assert st == "converged"
    floor = max(HIST_FLOOR, 10 * max(drift(hist, hist2), drift(hist, hist3)))
    slack = 0 if floor < 1e-3 * rtol else max(3, it // 100)
    assert abs(got_its - it) <= max(slack, abs(it2 - it), abs(it3 - it)), (got_its, it, it2, it3)
    mdiv = min(diverge_index(hist, hist2), diverge_index(hist, hist3))
    compare_hist(got_hist[:mdiv], hist[:mdiv], 1e-8, floor=floor)
    within_factor(got_hist, hist, mdiv)
    solution_tier(got_x, x, (x2, x3), label)
    return it
