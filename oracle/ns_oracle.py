"""Static parallel nested sampling: a plain, slow FP64 reference.

TEST INFRASTRUCTURE ONLY. Only tests/, the package's smoke check and bench.py's CPU leg may
import this module; the library never does.

It follows the paper's section 3 ("Parallel Nested Sampling": prior sampling, evidence
estimation, posterior samples, parallel prior sampling) and its algorithm "Static Parallel Nested
Sampling", step by step, with a priority-free list of live points:

  * K live points in the unit cube, each with its log-likelihood;
  * each iteration: L_min is the smallest live log-likelihood; a batch of candidates (supplied by
    the caller, so that random numbers are inputs) is evaluated; candidates with L >= L_min are
    accepted; then, for each accepted candidate, the live point with the smallest L becomes dead
    and the candidate takes its place;
  * the prior volume of each dead point's contour and the Riemann sum of the evidence (Eq. of the
    evidence integral, sum over dX_i L_i);
  * a stopping test after each iteration; at the end the remaining live points are added in
    ascending order;
  * the posterior importance weights p_i = L_i dX_i / Z.

Readings taken where the paper is silent or loose (each one also has a test):
  N1  Order of replacement. The paper replaces "for i = 1 to n'" without fixing the order of the
      accepted candidates. They are used in ascending order of L. Then every dead point has a
      likelihood no lower than the one before it (the contour sequence stays monotone) and no
      accepted candidate is wasted.
  N2  Prior volume with several replacements per iteration. The paper gives ln X_i = -i/K, which
      is exact in expectation for one replacement per iteration. With n' accepted candidates drawn
      inside the contour of the current worst live point, the first dead point of the iteration
      shrinks the volume by the largest of K uniform draws (E ln t = -1/K) and the j-th (j >= 2)
      by the largest of K + n' - j + 1 (E ln t = -1/(K + n' - j + 1)). This reduces to the
      paper's -1/K per dead point when n' = 1. `volume="paper"` keeps -1/K for every dead point.
  N3  Stopping. The change in ln Z from one iteration to the next is tiny from the first
      iterations on when K is large, so the test uses the largest change the remaining volume
      can still make: ln(Z + L_max X) - ln Z <= eps, checked after each iteration that replaced
      at least one live point.
  N4  Final live points. The remaining K live points each get an equal share X_last / K of the
      remaining volume (the expected shares when they are removed one by one, smallest L first,
      as the paper's closing loop does).

Parity status: pinned (tests/test_ns_oracle.py: closed-form contour volumes of a radial
likelihood, a constant likelihood, the serial special case, a hand-worked tiny run, invariants).
"""
from __future__ import annotations

import math

import numpy as np


def _logaddexp(a: float, b: float) -> float:
    if a == -math.inf:
        return b
    if b == -math.inf:
        return a
    m = max(a, b)
    return m + math.log(math.exp(a - m) + math.exp(b - m))


def _log_one_minus_exp(x: float) -> float:
    """ln(1 - e^{-x}) for x > 0."""
    return math.log(-math.expm1(-x))


def run(loglike, live_u, propose, eps=0.1, max_iter=100000, volume="order"):
    """Run static parallel nested sampling.

    loglike(u[n, d]) -> ln L[n] (the caller folds in the prior transform).
    live_u[K, d]: the initial live points, drawn from the prior by the caller.
    propose(it, live_u, live_logl) -> u[n, d] candidates in the unit cube, or None to stop.

    Returns a dict with the dead points in order (u, ln L, ln dX, ln X), ln Z, the log posterior
    weights, the iteration count and the number of accepted candidates per iteration.
    """
    if volume not in ("order", "paper"):
        raise ValueError("volume is 'order' or 'paper'")
    live_u = np.array(live_u, dtype=np.float64)
    K = live_u.shape[0]
    live_l = np.asarray(loglike(live_u), dtype=np.float64).copy()
    dead_u, dead_l, dead_ldx, dead_lx = [], [], [], []
    ln_x = 0.0          # ln X of the last dead point's contour (starts at the whole prior)
    ln_z = -math.inf
    n_acc = []
    it = 0
    ncall = K
    while it < max_iter:
        l_min = float(np.min(live_l))
        cand = propose(it, live_u.copy(), live_l.copy())
        if cand is None:
            break
        cand = np.asarray(cand, dtype=np.float64)
        cl = np.asarray(loglike(cand), dtype=np.float64)
        ncall += len(cand)
        it += 1
        ok = np.where(cl >= l_min)[0]
        ok = ok[np.argsort(cl[ok], kind="stable")]           # reading N1: ascending order
        nacc = len(ok)
        n_acc.append(nacc)
        for j, c in enumerate(ok, start=1):
            k = int(np.argmin(live_l))                        # the live point with L_min
            if volume == "paper" or j == 1:
                d = 1.0 / K
            else:
                d = 1.0 / (K + nacc - j + 1)                  # reading N2
            ln_dx = ln_x + _log_one_minus_exp(d)              # X_{i-1} - X_i
            ln_x = ln_x - d
            dead_u.append(live_u[k].copy())
            dead_l.append(live_l[k])
            dead_ldx.append(ln_dx)
            dead_lx.append(ln_x)
            ln_z = _logaddexp(ln_z, live_l[k] + ln_dx)
            live_u[k] = cand[c]
            live_l[k] = cl[c]
        if nacc > 0:                                          # reading N3
            bound = _logaddexp(ln_z, float(np.max(live_l)) + ln_x)
            if bound - ln_z <= eps:
                break
    # reading N4: remaining live points, smallest L first, equal shares of X_last
    order = np.argsort(live_l, kind="stable")
    ln_share = ln_x - math.log(K)
    for m, k in enumerate(order, start=1):
        dead_u.append(live_u[k].copy())
        dead_l.append(live_l[k])
        dead_ldx.append(ln_share)
        dead_lx.append(ln_x + math.log((K - m) / K) if m < K else -math.inf)
        ln_z = _logaddexp(ln_z, live_l[k] + ln_share)
    dead_l = np.array(dead_l)
    dead_ldx = np.array(dead_ldx)
    return {
        "u": np.array(dead_u), "logl": dead_l, "log_dx": dead_ldx, "log_x": np.array(dead_lx),
        "logz": ln_z, "log_w": dead_l + dead_ldx - ln_z, "niter": it, "n_accepted": np.array(n_acc),
        "ncall": ncall, "nlive": K,
    }


def information(res) -> float:
    """Kullback-Leibler information H = sum_i p_i ln(L_i / Z) of the run (nats)."""
    w = np.exp(res["log_w"])
    return float(np.sum(w * (res["logl"] - res["logz"])))
