"""Pins of the calibration-model oracle: the spline interpolates its nodes and reproduces linear
functions of ln f; a constant amplitude or phase offset has a closed-form logL; zero calibration
reduces to the uncalibrated oracle; the gradient matches central differences."""
import math

import numpy as np
import pytest
import torch

from oracle import cal_oracle as cal
from oracle import gw_oracle as o
from tests.helpers import event_inputs

N = 10


@pytest.fixture(scope="module")
def ev():
    spec, f, psd, data, dets = event_inputs(1, f_hi=300.0)
    return spec, f, psd, data, dets


def full_theta(theta11, nd, amp=None, phase=None):
    cal_part = np.zeros(2 * N * nd)
    for d in range(nd):
        if amp is not None:
            cal_part[2 * N * d:2 * N * d + N] = amp[d]
        if phase is not None:
            cal_part[2 * N * d + N:2 * N * (d + 1)] = phase[d]
    return np.concatenate([theta11, cal_part])


def test_spline_interpolates_and_reproduces_lines(ev):
    f = ev[1]
    nodes = cal.node_frequencies(f[0], f[-1], N)
    vals = torch.tensor(np.random.default_rng(1).normal(size=N))
    np.testing.assert_allclose(cal.spline(nodes, vals, f[0], f[-1]).numpy(), vals.numpy(), atol=1e-12)
    a, b = 0.3, -0.07
    line = torch.tensor(a + b * np.log(nodes))
    np.testing.assert_allclose(cal.spline(f, line, f[0], f[-1]).numpy(), a + b * np.log(f), atol=1e-12)


def test_spline_is_local(ev):
    """Moving one node changes the spline only within two node intervals of it."""
    f = ev[1]
    nodes = cal.node_frequencies(f[0], f[-1], N)
    base = torch.zeros(N)
    bump = torch.zeros(N)
    bump[5] = 1.0
    d = cal.spline(f, bump, f[0], f[-1]).numpy() - cal.spline(f, base, f[0], f[-1]).numpy()
    outside = (f < nodes[3]) | (f > nodes[7])
    assert np.all(d[outside] == 0.0)


def test_zero_calibration_is_the_plain_model(ev):
    spec, f, psd, data, dets = ev
    th = full_theta(spec.theta0, len(dets))
    a = cal.logl(th[None], data, psd, dets, f, spec.df, N)
    b = o.logl(spec.theta0[None], data, psd, dets, f, spec.df)
    assert float(a[0]) == pytest.approx(float(b[0]), rel=1e-13, abs=1e-10)


def test_constant_amplitude_offset_closed_form(ev):
    """dA = a on every node: h scales by (1 + a), logL = (1 + a) <d|h> - (1 + a)^2 <h|h> / 2."""
    spec, f, psd, data, dets = ev
    nd = len(dets)
    a = 0.07
    th = full_theta(spec.theta0, nd, amp=[a] * nd)
    got = float(cal.logl(th[None], data, psd, dets, f, spec.df, N)[0])
    dh = hh = 0.0
    for i in range(nd):
        h = o.detector_strain(torch.tensor(f), torch.tensor(spec.theta0), tuple(dets[i]))
        dh += float(o.inner(torch.tensor(data[i]), h, torch.tensor(psd[i]), spec.df))
        hh += float(o.inner(h, h, torch.tensor(psd[i]), spec.df))
    assert got == pytest.approx((1 + a) * dh - 0.5 * (1 + a) ** 2 * hh, rel=1e-12)


def test_constant_phase_offset_closed_form(ev):
    """dphi = b on every node of one detector: logL = Re(e^{ib} <d|h>_c) - <h|h>/2 with the complex
    inner product 4 df sum conj(d) h / S for that detector."""
    spec, f, psd, data, dets = ev
    nd = len(dets)
    b = 0.3
    th = full_theta(spec.theta0, nd, phase=[b, 0.0, 0.0])
    got = float(cal.logl(th[None], data, psd, dets, f, spec.df, N)[0])
    ref = 0.0
    for i in range(nd):
        h = o.detector_strain(torch.tensor(f), torch.tensor(spec.theta0), tuple(dets[i])).numpy()
        c = 4 * spec.df * np.sum(np.conj(data[i]) * h / psd[i])
        rot = np.exp(1j * b) if i == 0 else 1.0
        ref += float(np.real(rot * c)) - 0.5 * 4 * spec.df * float(np.sum(np.abs(h) ** 2 / psd[i]))
    assert got == pytest.approx(ref, rel=1e-12)


def test_gradient_matches_central_differences(ev):
    spec, f, psd, data, dets = ev
    nd = len(dets)
    rng = np.random.default_rng(5)
    th = full_theta(spec.theta0, nd, amp=rng.normal(0, 0.05, (nd, N)), phase=rng.normal(0, 0.05, (nd, N)))
    _, g = cal.logl_grad(th[None], data, psd, dets, f, spec.df, N)
    for i in (0, 10, 11 + 3, 11 + N + 4, 11 + 2 * N + 7):
        h = 1e-6 * max(abs(th[i]), 1.0)
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (cal.logl(tp[None], data, psd, dets, f, spec.df, N) - cal.logl(tm[None], data, psd, dets, f, spec.df, N)) / (2 * h)
        assert float(g[0, i]) == pytest.approx(float(fd[0]), rel=1e-5, abs=1e-5)
