"""The sidereal angle (GMST) on the GPU: every path against the FP64 oracle at a non-zero angle.

The detectors' antenna patterns and delays depend on the source's right ascension through
ra - gmst (the multi-detector sum of Eq. 2 at a fixed Earth orientation); the oracle pins that
reading on the CPU (zenith delay at ra = gmst + longitude, logL(ra, gmst) = logL(ra - gmst, 0)).
These tests run the single-event, relative-binning and multi-event paths at gmst = 1.3 rad in
both precisions, with data injected at the same angle.
"""
import numpy as np
import pytest
import torch

from oracle import gw_oracle as o
from oracle import rb_oracle as rb
from paper_1909_11873_amd import gwlike as gw
from paper_1909_11873_amd import synth
from tests.helpers import event_inputs, scaled_grad_error
from tests.test_rb_oracle import near

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GMST = 1.3
TOL = {"mixed": 1e-3, "fp64": 1e-6}


def t(x):
    return torch.tensor(x, device=DEV)


@pytest.fixture(scope="module")
def c1_gmst():
    spec, f, psd, data, dets = event_inputs(1, gmst=GMST)
    ev = gw.Event(t(data), t(psd), dets, t(f), spec.df, gmst=GMST)
    th = synth.theta_batch(spec, 8192)
    th[0] = spec.theta0
    loud = np.argsort(th[:, 0] ** (5 / 3) / th[:, 4] ** 2)[-4:]
    sample = np.unique(np.concatenate([[0, 1, 2, 63, 64, 8191], loud]))
    return spec, f, psd, data, dets, ev, th, sample


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_event_at_gmst(c1_gmst, prec):
    """c1 shapes (3 detectors, 16,225 bins), 8,192 points: values on sampled points and the
    gradient on four, against the oracle at the same angle."""
    spec, f, psd, data, dets, ev, th, sample = c1_gmst
    ref = o.logl(th[sample], data, psd, dets, f, spec.df, gmst=GMST).numpy()
    got = gw.logl(t(th), ev, prec).cpu().numpy()
    err = np.abs(got[sample] - ref)
    print(f"gmst {GMST} c1 {prec}: max |dlogL| {err.max():.3e}, logL(theta0) {ref[0]:.3f}")
    assert err.max() <= TOL[prec]
    # the angle matters: the same data read at gmst = 0 give a different likelihood at theta0
    assert abs(ref[0] - float(o.logl(th[:1], data, psd, dets, f, spec.df, gmst=0.0)[0])) > 1.0
    g_idx = sample[:4]
    vref, gref = o.logl_grad(th[g_idx], data, psd, dets, f, spec.df, gmst=GMST)
    v, g = gw.logl_grad(t(th[g_idx]), ev, prec)
    assert np.abs(v.cpu().numpy() - vref.numpy()).max() <= TOL[prec]
    e = scaled_grad_error(g.cpu().numpy(), gref.numpy())
    print(f"gmst {GMST} c1 {prec}: gradient max scaled error {e.max():.3e}")
    assert e.max() <= 1e-4


def test_relative_binning_at_gmst():
    spec, f, psd, data, dets = event_inputs(1, gmst=GMST)
    ev = gw.Event(t(data), t(psd), dets, t(f), spec.df, gmst=GMST, fiducial=spec.theta0, rb_eps=0.1)
    summ = rb.summary(data, psd, dets, f, spec.df, spec.theta0, 0.1, gmst=GMST)
    th = near(spec.theta0, 8, seed=4, scale=0.3)
    th[0] = spec.theta0
    ref = rb.logl(th, summ, psd, dets, f, spec.df, gmst=GMST).numpy()
    for prec in ("fp64", "mixed"):
        got = gw.logl(t(th), ev, prec).cpu().numpy()
        err = np.abs(got - ref)
        print(f"gmst {GMST} RB {prec}: max |dlogL| vs RB oracle {err.max():.3e}")
        assert err.max() <= (1e-9 * max(1.0, np.abs(ref).max()) if prec == "fp64" else 1e-3)
    _, gref = rb.logl_grad(th[:3], summ, psd, dets, f, spec.df, gmst=GMST)
    _, g = gw.logl_grad(t(th[:3]), ev, "mixed")
    assert scaled_grad_error(g.cpu().numpy(), gref.numpy()).max() <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multi_event_plan_at_several_angles(prec):
    """Three events at different sidereal angles (one of them relative-binning) in one plan."""
    angles = [0.4, GMST, 2.9]
    events, thetas, refs = [], [], []
    for i, g in enumerate(angles):
        spec = synth.event_spec(4, i)
        df = 0.25
        f = synth.freq_grid(20.0, 400.0, df)
        s = synth.psd_fit(f)
        psd = np.stack([s] * 3)
        nz = np.stack([synth.noise(spec.seed_base + d, s, df) for d in range(3)])
        dets = np.array([synth.detector_rad(n) for n in spec.det_names])
        data = nz + o.strain_all(spec.theta0, dets, f, g).numpy()
        if i == 1:
            ev = gw.Event(t(data), t(psd), dets, t(f), df, gmst=g, fiducial=spec.theta0, rb_eps=0.2)
            th = near(spec.theta0, 40, seed=9, scale=0.3)
            summ = rb.summary(data, psd, dets, f, df, spec.theta0, 0.2, gmst=g)
            refs.append(rb.logl_grad(th[:3], summ, psd, dets, f, df, gmst=g))
        else:
            ev = gw.Event(t(data), t(psd), dets, t(f), df, gmst=g)
            th = synth.prior_draw(np.random.default_rng(spec.seed_base + 10), 100)
            th[0] = spec.theta0
            refs.append(o.logl_grad(th[:3], data, psd, dets, f, df, gmst=g))
        events.append(ev)
        thetas.append(t(th))
    plan = gw.MultiPlan(events, [len(x) for x in thetas], prec, with_grad=True)
    logls, grads, _ = plan.launch(thetas)
    for i, (l, gr, (vref, gref)) in enumerate(zip(logls, grads, refs)):
        err = np.abs(l.cpu().numpy()[:3] - vref.numpy())
        ge = scaled_grad_error(gr.cpu().numpy()[:3], gref.numpy())
        print(f"gmst {angles[i]} multi {prec}: max |dlogL| {err.max():.3e}, gradient {ge.max():.3e}")
        assert err.max() <= TOL[prec]
        assert ge.max() <= 1e-4
    plan.close()
    for ev in events:
        ev.close()
