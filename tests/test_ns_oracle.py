"""Pins of the nested-sampling oracle against closed forms, special cases and invariants.

The test likelihood is radial about the centre of the unit cube, ln L = -r^2 / (2 s^2). Its
contour at radius r encloses the prior volume of a d-ball, V_d r^d, while r <= 1/2, and its
evidence is a product of error functions. Constrained prior draws are exact: uniform in the ball
of the current worst live point, clipped to the cube.
"""
import math

import numpy as np
import pytest

from oracle import ns_oracle as ns


def ball_volume(d, r):
    return math.pi ** (d / 2) / math.gamma(d / 2 + 1) * r ** d


def radial(s):
    def loglike(u):
        u = np.atleast_2d(u)
        return -np.sum((u - 0.5) ** 2, axis=1) / (2 * s * s)
    return loglike


def ball_proposer(d, n, s, seed, accept_all=True):
    """Candidates uniform inside the contour of the current worst live point (exact constrained
    prior draws), by ball sampling when the ball fits in the cube, by rejection otherwise."""
    rng = np.random.default_rng(seed)

    def propose(it, live_u, live_l):
        r = math.sqrt(-2 * s * s * float(np.min(live_l)))
        out = []
        while len(out) < n:
            if r <= 0.5:
                z = rng.standard_normal((n, d))
                z /= np.linalg.norm(z, axis=1, keepdims=True)
                c = 0.5 + r * z * rng.random((n, 1)) ** (1.0 / d)
            else:
                c = rng.random((4 * n, d))
                c = c[np.sum((c - 0.5) ** 2, axis=1) <= r * r]
            out.extend(c[: n - len(out)])
        return np.array(out)
    return propose


def prior_proposer(d, n, seed):
    rng = np.random.default_rng(seed)
    return lambda it, live_u, live_l: rng.random((n, d))


def test_serial_case_volume_is_minus_i_over_k():
    """One accepted candidate per iteration: ln X_i = -i/K exactly (the paper's estimate)."""
    d, K, s = 2, 50, 0.1
    res = ns.run(radial(s), np.random.default_rng(1).random((K, d)), ball_proposer(d, 1, s, 2), eps=0.5)
    assert np.all(res["n_accepted"] == 1)
    n_dead = res["niter"]
    np.testing.assert_allclose(res["log_x"][:n_dead], -np.arange(1, n_dead + 1) / K, rtol=0, atol=1e-12)


def test_tiny_run_by_hand():
    """K = 3 in one dimension, two iterations of scripted candidates, checked step by step."""
    loglike = lambda u: -np.abs(np.atleast_2d(u)[:, 0] - 0.5) * 10.0
    live = np.array([[0.1], [0.45], [0.8]])           # ln L = -4, -0.5, -3
    script = [np.array([[0.05], [0.3], [0.6], [0.7]]),  # ln L = -4.5 (no), -2, -1, -2
              np.array([[0.52]])]                      # ln L = -0.2
    res = ns.run(loglike, live, lambda it, lu, ll: script[it] if it < 2 else None, eps=-1.0)
    # iteration 1: L_min = -4; accepted -2, -2, -1 ascending (ties keep draw order)
    #   dead -4 (0.1); -3 (0.8) ; then the live set is {-0.5, -2(0.3), -2(0.7)} -> dead -2 (0.3)
    # iteration 2: L_min = -2; accepted -0.2 -> dead -2 (0.7)
    assert res["niter"] == 2
    np.testing.assert_allclose(res["logl"][:4], [-4.0, -3.0, -2.0, -2.0])
    np.testing.assert_allclose(res["u"][:4, 0], [0.1, 0.8, 0.3, 0.7])
    # volumes: iteration 1 has n' = 3: 1/3, then 1/(3+3-2+1) = 1/5, then 1/4; iteration 2: 1/3
    np.testing.assert_allclose(res["log_x"][:4], -np.cumsum([1 / 3, 1 / 5, 1 / 4, 1 / 3]))
    # final live points ascending: -1 (0.6), -0.5 (0.45), -0.2 (0.52), equal shares
    np.testing.assert_allclose(res["logl"][4:], [-1.0, -0.5, -0.2])
    lx = -(1 / 3 + 1 / 5 + 1 / 4 + 1 / 3)
    np.testing.assert_allclose(res["log_dx"][4:], lx - math.log(3))
    x = np.exp(np.concatenate([[0.0], res["log_x"][:4]]))
    z = np.sum(np.exp(res["logl"][:4]) * (x[:-1] - x[1:])) + np.exp(lx) / 3 * np.sum(np.exp([-1.0, -0.5, -0.2]))
    assert res["logz"] == pytest.approx(math.log(z), abs=1e-12)


def test_constant_likelihood_gives_its_value():
    """All candidates tie with L_min and are accepted; the volumes telescope to 1, so ln Z = c."""
    K, d = 20, 3
    res = ns.run(lambda u: np.full(len(np.atleast_2d(u)), -7.25), np.random.default_rng(3).random((K, d)),
                 prior_proposer(d, 7, 4), eps=1e-3, max_iter=30)
    assert res["logz"] == pytest.approx(-7.25, abs=1e-12)
    assert np.exp(res["log_w"]).sum() == pytest.approx(1.0, abs=1e-12)
    assert np.all(res["n_accepted"] == 7)   # the constraint is L >= L_min: a plateau is accepted


@pytest.mark.parametrize("n", [1, 16, 400])
def test_contour_volumes_match_the_ball(n):
    """Estimated ln X_i against the exact ln V_d r_i^d for dead points inside the half-unit ball,
    in units of the estimate's own standard deviation sqrt(sum of 1/m^2)."""
    d, K, s = 3, 100, 0.05
    res = ns.run(radial(s), np.random.default_rng(5).random((K, d)), ball_proposer(d, n, s, 6), eps=0.01)
    nd = len(res["logl"]) - K
    r = np.sqrt(-2 * s * s * res["logl"][:nd])
    inside = r <= 0.5
    true = np.log(ball_volume(d, r[inside]))
    est = res["log_x"][:nd][inside]
    # variance of each estimate: sum of the squared decrements up to it (E ln t = -1/m, Var = 1/m^2)
    dec = -np.diff(np.concatenate([[0.0], res["log_x"][:nd]]))
    sd = np.sqrt(np.cumsum(dec ** 2))[inside]
    z = (est - true) / sd
    assert np.abs(z).max() < 5.0, np.abs(z).max()


def test_paper_volume_is_biased_when_many_replace_at_once():
    """With n' >> K accepted per iteration, -1/K per dead point overshoots the true shrinkage."""
    d, K, s = 3, 20, 0.05
    kw = dict(eps=0.01)
    order = ns.run(radial(s), np.random.default_rng(7).random((K, d)), ball_proposer(d, 400, s, 8), **kw)
    paper = ns.run(radial(s), np.random.default_rng(7).random((K, d)), ball_proposer(d, 400, s, 8),
                   volume="paper", **kw)
    z_true = 3 * math.log(math.sqrt(2 * math.pi) * s * math.erf(0.5 / (s * math.sqrt(2))))
    h = ns.information(order)
    assert abs(order["logz"] - z_true) < 4 * math.sqrt(h / K) + 0.05
    assert paper["logz"] - z_true < -20.0


def test_gaussian_evidence_and_posterior_moments():
    d, K, s = 2, 400, 0.08
    res = ns.run(radial(s), np.random.default_rng(9).random((K, d)), ball_proposer(d, 64, s, 10), eps=0.01)
    z_true = d * math.log(math.sqrt(2 * math.pi) * s * math.erf(0.5 / (s * math.sqrt(2))))
    h = ns.information(res)
    assert abs(res["logz"] - z_true) < 4 * math.sqrt(h / K)
    w = np.exp(res["log_w"])
    mean = np.sum(w[:, None] * res["u"], axis=0)
    var = np.sum(w[:, None] * (res["u"] - mean) ** 2, axis=0)
    ess = 1.0 / np.sum(w ** 2)
    assert np.all(np.abs(mean - 0.5) < 5 * s / math.sqrt(ess))
    np.testing.assert_allclose(var, s * s, rtol=0.25)


def test_invariants_with_prior_draws():
    """Plain prior draws (the paper's own proposal): monotone contours, decreasing volumes,
    normalised weights, and the stop test's bound met at exit."""
    d, K, s = 2, 40, 0.15
    res = ns.run(radial(s), np.random.default_rng(11).random((K, d)), prior_proposer(d, 256, 12), eps=0.1)
    nd = len(res["logl"]) - K
    assert np.all(np.diff(res["logl"][:nd]) >= 0)
    assert np.all(np.diff(res["log_x"][:nd]) < 0)
    assert np.exp(res["log_w"]).sum() == pytest.approx(1.0, abs=1e-12)
    assert res["n_accepted"].sum() == nd
    assert res["ncall"] == K + 256 * res["niter"]
    # the stop test: the remaining-volume bound ln(Z + L_max X) - ln Z first falls to eps at the
    # last iteration (live points at the end of each iteration rebuilt from the dead sequence)
    ends = np.cumsum(res["n_accepted"])
    lz = np.logaddexp.accumulate(res["logl"][:nd] + res["log_dx"][:nd])
    final_live_max = res["logl"][nd:].max()
    for i, e in enumerate(ends):
        if res["n_accepted"][i] == 0:
            continue
        # the largest live L after iteration i is the largest L seen so far among dead points after
        # e and the final live points, since live points only leave by dying
        lmax_i = max(final_live_max, res["logl"][e:nd].max() if e < nd else -np.inf)
        bound = np.logaddexp(lz[e - 1], lmax_i + res["log_x"][e - 1]) - lz[e - 1]
        if i == len(ends) - 1:
            assert bound <= 0.1
        else:
            assert bound > 0.1
