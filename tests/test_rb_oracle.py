"""Pins of the relative-binning oracle: partition of unity, exactness when every bin is an edge,
second-order convergence in the edge spacing, and the edge rule itself."""
import math

import numpy as np
import pytest
import torch

from oracle import gw_oracle as o
from oracle import rb_oracle as rb
from tests.helpers import event_inputs


@pytest.fixture(scope="module")
def small():
    # c1's detectors, PSD and noise on 20-300 Hz (2241 bins), injection at theta0
    spec, f, psd, data, dets = event_inputs(1, f_hi=300.0)
    return spec, f, psd, data, dets


def near(theta0, k, seed=0, scale=1.0):
    """k points around theta0 (small offsets in every parameter)."""
    rng = np.random.default_rng(seed)
    step = scale * np.array([0.05, 0.01, 0.02, 0.02, 10.0, 0.01, 0.01, 0.02, 0.02, 0.05, 1e-4])
    return theta0 + step * rng.standard_normal((k, 11))


def test_edges_follow_the_phase_bound(small):
    spec, f, psd, data, dets = small
    eps = 0.3
    idx = rb.edges(f, eps)
    assert idx[0] == 0 and idx[-1] == len(f) - 1
    assert np.all(np.diff(idx) > 0)
    dpsi = rb.phase_bound(f, f[0], f[-1])
    assert np.all(np.diff(dpsi) > 0)                       # the bound increases with f
    for a, b in zip(idx[:-1], idx[1:]):                    # every bin between edges in one eps cell
        assert dpsi[b - 1] - dpsi[a] < eps
    assert len(idx) < len(f) / 5                           # a real compression on this grid


def test_hats_partition_unity(small):
    f = small[1]
    idx = rb.edges(f, 0.3)
    w = rb.hat_weights(f, idx)
    np.testing.assert_allclose(w.sum(axis=0), 1.0, atol=1e-13)
    np.testing.assert_allclose(w[:, idx], np.eye(len(idx)), atol=1e-13)


def test_exact_at_the_fiducial(small):
    """r = 1 at theta_fid, so the summary data reproduce <d|h0> exactly."""
    spec, f, psd, data, dets = small
    summ = rb.summary(data, psd, dets, f, spec.df, spec.theta0, 0.3)
    a = rb.logl(spec.theta0[None], summ, psd, dets, f, spec.df)
    b = o.logl(spec.theta0[None], data, psd, dets, f, spec.df)
    assert float(a[0]) == pytest.approx(float(b[0]), abs=1e-9 * abs(float(b[0])) + 1e-9)


def test_exact_when_every_bin_is_an_edge(small):
    spec, f, psd, data, dets = small
    summ = rb.summary(data, psd, dets, f, spec.df, spec.theta0, 1e-12)
    assert len(summ["idx"]) == len(f)
    th = near(spec.theta0, 3, seed=1, scale=20.0)
    np.testing.assert_allclose(rb.logl(th, summ, psd, dets, f, spec.df).numpy(),
                               o.logl(th, data, psd, dets, f, spec.df).numpy(), rtol=1e-10, atol=1e-8)


def test_second_order_convergence(small):
    """Linear interpolation of r: halving the edge spacing cuts the error about fourfold."""
    spec, f, psd, data, dets = small
    th = near(spec.theta0, 4, seed=2, scale=3.0)
    full = o.logl(th, data, psd, dets, f, spec.df).numpy()
    errs = []
    for eps in (0.4, 0.2, 0.1):
        summ = rb.summary(data, psd, dets, f, spec.df, spec.theta0, eps)
        errs.append(np.abs(rb.logl(th, summ, psd, dets, f, spec.df).numpy() - full).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 2.5 < r1 < 6.5 and 2.5 < r2 < 6.5, errs


def test_gradient_matches_central_differences(small):
    spec, f, psd, data, dets = small
    summ = rb.summary(data, psd, dets, f, spec.df, spec.theta0, 0.3)
    th = near(spec.theta0, 1, seed=3)[0]
    _, g = rb.logl_grad(th[None], summ, psd, dets, f, spec.df)
    for i in (0, 4, 10):
        h = 1e-6 * max(abs(th[i]), 1.0)
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (rb.logl(tp[None], summ, psd, dets, f, spec.df) - rb.logl(tm[None], summ, psd, dets, f, spec.df)) / (2 * h)
        assert float(g[0, i]) == pytest.approx(float(fd[0]), rel=1e-5, abs=1e-6)


def _cal_cols(k, nnode, ndet, seed, scale=0.05):
    return np.random.default_rng(seed).normal(0.0, scale, (k, 2 * nnode * ndet))


def test_calibrated_rb_reduces_to_plain_rb_at_zero_calibration(small):
    spec, f, psd, data, dets = small
    summ = rb.summary(data, psd, dets, f, spec.df, spec.theta0, 0.3)
    th = near(spec.theta0, 3, seed=4)
    cal = np.concatenate([th, np.zeros((3, 2 * 6 * 3))], axis=1)
    np.testing.assert_allclose(rb.logl(cal, summ, psd, dets, f, spec.df, nnode=6).numpy(),
                               rb.logl(th, summ, psd, dets, f, spec.df).numpy(), rtol=1e-13, atol=1e-10)


def test_calibrated_rb_is_exact_when_every_bin_is_an_edge(small):
    """Every bin an edge: the binned, calibrated likelihood is the calibration oracle's."""
    from oracle import cal_oracle as co
    spec, f, psd, data, dets = small
    summ = rb.summary(data, psd, dets, f, spec.df, spec.theta0, 1e-12)
    th = np.concatenate([near(spec.theta0, 3, seed=5, scale=5.0), _cal_cols(3, 5, 3, seed=6)], axis=1)
    np.testing.assert_allclose(rb.logl(th, summ, psd, dets, f, spec.df, nnode=5).numpy(),
                               co.logl(th, data, psd, dets, f, spec.df, 5).numpy(), rtol=1e-10, atol=1e-8)
