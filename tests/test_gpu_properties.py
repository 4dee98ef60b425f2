"""Properties of logL that hold at any size, checked on the full c1 launch (3 detectors,
16,225 bins, 65,536 prior draws) through the C ABI, in both precisions.

- Detector additivity: the three-detector logL is the sum of the one-detector logLs.
- Distance: logL = a/D - b/D^2 in the luminosity distance D, so three distances fix the fourth.
- Coalescence phase: logL = C + A cos(phi_c) + B sin(phi_c), so three phases fix the fourth.
- Polarisation angle: psi -> psi + pi leaves the antenna patterns, hence logL, unchanged.
- Cauchy-Schwarz: logL <= <d|d>/2 for every parameter point.
"""
import numpy as np
import pytest
import torch

from paper_1909_11873_amd import gwlike as gw
from paper_1909_11873_amd import synth
from tests.helpers import event_inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {"fp64": 1e-7, "mixed": 2e-3}


@pytest.fixture(scope="module")
def c1():
    spec, f, psd, data, dets = event_inputs(1)
    t = lambda x: torch.tensor(x, device=DEV)
    full = gw.Event(t(data), t(psd), dets, t(f), spec.df)
    singles = [gw.Event(t(data[i:i + 1]), t(psd[i:i + 1]), dets[i:i + 1], t(f), spec.df) for i in range(3)]
    th = synth.theta_batch(spec)
    th[0] = spec.theta0
    return spec, f, psd, data, full, singles, th


def scale_tol(prec, ref):
    return TOL[prec] * np.maximum(1.0, np.abs(ref) / 1e3)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_detector_additivity(c1, prec):
    spec, f, psd, data, full, singles, th = c1
    t = torch.tensor(th, device=DEV)
    whole = gw.logl(t, full, prec).cpu().numpy()
    parts = sum(gw.logl(t, ev, prec).cpu().numpy() for ev in singles)
    err = np.abs(whole - parts)
    print(f"additivity {prec}: max {err.max():.3e} over {len(th)} points")
    assert np.all(err <= 2 * scale_tol(prec, whole))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_distance_law(c1, prec):
    spec, f, psd, data, full, singles, th = c1
    th = th[:8192]
    ds = [300.0, 700.0, 1500.0, 1100.0]
    vals = []
    for d in ds:
        x = th.copy()
        x[:, 4] = d
        vals.append(gw.logl(torch.tensor(x, device=DEV), full, prec).cpu().numpy())
    # a/D - b/D^2 from the first two, checked at the other two
    m = np.array([[1 / ds[0], -1 / ds[0] ** 2], [1 / ds[1], -1 / ds[1] ** 2]])
    ab = np.linalg.solve(m, np.stack([vals[0], vals[1]]))
    for d, v in zip(ds[2:], vals[2:]):
        pred = ab[0] / d - ab[1] / d ** 2
        assert np.all(np.abs(pred - v) <= 3 * scale_tol(prec, v) + 1e-9 * np.abs(ab).max(axis=0))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_phase_law(c1, prec):
    spec, f, psd, data, full, singles, th = c1
    th = th[:8192]
    phis = [0.3, 1.9, 4.0, 5.5]
    vals = []
    for p in phis:
        x = th.copy()
        x[:, 9] = p
        vals.append(gw.logl(torch.tensor(x, device=DEV), full, prec).cpu().numpy())
    m = np.array([[1.0, np.cos(p), np.sin(p)] for p in phis[:3]])
    coef = np.linalg.solve(m, np.stack(vals[:3]))
    pred = coef[0] + coef[1] * np.cos(phis[3]) + coef[2] * np.sin(phis[3])
    assert np.all(np.abs(pred - vals[3]) <= 4 * scale_tol(prec, vals[3]))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_polarisation_period(c1, prec):
    spec, f, psd, data, full, singles, th = c1
    x = th.copy()
    x[:, 8] = x[:, 8] + np.pi
    a = gw.logl(torch.tensor(th, device=DEV), full, prec).cpu().numpy()
    b = gw.logl(torch.tensor(x, device=DEV), full, prec).cpu().numpy()
    assert np.all(np.abs(a - b) <= 2 * scale_tol(prec, a))


def test_cauchy_schwarz_bound(c1):
    spec, f, psd, data, full, singles, th = c1
    dd = 4 * spec.df * np.sum(np.abs(data) ** 2 / psd)
    for prec in ("fp64", "mixed"):
        v = gw.logl(torch.tensor(th, device=DEV), full, prec).cpu().numpy()
        assert np.all(v <= 0.5 * dd + 1e-3)
