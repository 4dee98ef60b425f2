"""The calibrated likelihood on the GPU (gwl_event_create_cal) against the calibration oracle."""
import numpy as np
import pytest
import torch

from oracle import cal_oracle as cal
from oracle import gw_oracle as o
from paper_1909_11873_amd import gwlike as gw
from paper_1909_11873_amd import synth
from tests.helpers import WIDTHS, event_inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def cal_theta(theta11, nd, n, rng, sigma):
    k = theta11.shape[0]
    c = rng.normal(0.0, sigma, (k, 2 * n * nd))
    return np.concatenate([theta11, c], axis=1)


def make(cfg, n, f_hi=None, ndet=None):
    spec, f, psd, data, dets = event_inputs(cfg, f_hi=f_hi, ndet=ndet)
    t = lambda x: torch.tensor(x, device=DEV)
    ev = gw.Event(t(data), t(psd), dets, t(f), spec.df, calibration_nodes=n)
    return spec, f, psd, data, dets, ev


@pytest.mark.parametrize("n", [4, 10, 16])
def test_zero_calibration_is_the_plain_model(n):
    spec, f, psd, data, dets, ev = make(1, n, f_hi=400.0)
    t = lambda x: torch.tensor(x, device=DEV)
    plain = gw.Event(t(data), t(psd), dets, t(f), spec.df)
    th = synth.theta_batch(spec, 150)
    thc = np.concatenate([th, np.zeros((150, 2 * n * 3))], axis=1)
    for prec, tol in (("fp64", 1e-9), ("mixed", 2e-4)):
        a = gw.logl(t(thc), ev, prec).cpu().numpy()
        b = gw.logl(t(th), plain, prec).cpu().numpy()
        assert np.all(np.abs(a - b) <= tol * np.maximum(1.0, np.abs(b)))


@pytest.mark.parametrize("ndet,n", [(3, 10), (1, 4), (2, 16)])
def test_calibrated_logl_matches_the_oracle(ndet, n):
    spec, f, psd, data, dets, ev = make(1, n, f_hi=20.0 + 0.125 * 3000, ndet=ndet)   # 3001 bins
    rng = np.random.default_rng(ndet * 100 + n)
    th = cal_theta(synth.theta_batch(spec, 70), ndet, n, rng, 0.05)
    th[0, :11] = spec.theta0
    ref = cal.logl(th[:12], data, psd, dets, f, spec.df, n).numpy()
    for prec, tol in (("fp64", 1e-9), ("mixed", 1e-3)):
        got = gw.logl(torch.tensor(th, device=DEV), ev, prec).cpu().numpy()[:12]
        err = np.abs(got - ref)
        print(f"calibrated ndet {ndet} n {n} {prec}: max |dlogL| {err.max():.3e}")
        assert np.all(err <= tol * (np.maximum(1.0, np.abs(ref)) if prec == "fp64" else 1.0))


def test_calibrated_full_size_sampled():
    """c1 (16,225 bins, 3 detectors, 10 nodes each), the full 65,536-point launch, sampled."""
    n = 10
    spec, f, psd, data, dets, ev = make(1, n)
    rng = np.random.default_rng(3)
    th = cal_theta(synth.theta_batch(spec), 3, n, rng, 0.05)
    th[0, :11] = spec.theta0
    sample = np.array([0, 1, 2, 4096, 40000, 65535])
    ref = cal.logl(th[sample], data, psd, dets, f, spec.df, n).numpy()
    got = gw.logl(torch.tensor(th, device=DEV), ev, "mixed").cpu().numpy()[sample]
    err = np.abs(got - ref)
    print(f"calibrated c1 full size mixed: max |dlogL| {err.max():.3e}, logL(theta0) {ref[0]:.2f}")
    assert err.max() <= 1e-3


def test_calibrated_gradient_matches_the_oracle():
    n, nd = 10, 3
    spec, f, psd, data, dets, ev = make(1, n, f_hi=400.0)
    rng = np.random.default_rng(9)
    th = cal_theta(np.stack([spec.theta0, synth.theta_batch(spec, 2)[1]]), nd, n, rng, 0.05)
    _, gref = cal.logl_grad(th, data, psd, dets, f, spec.df, n)
    widths = np.concatenate([WIDTHS, np.full(2 * n * nd, 0.1)])
    for prec, tol in (("fp64", 1e-8), ("mixed", 1e-4)):
        _, g = gw.logl_grad(torch.tensor(th, device=DEV), ev, prec)
        gs, rs = g.cpu().numpy() * widths, gref.numpy() * widths
        scale = np.maximum(np.abs(rs), 1e-3 * np.abs(rs).max(axis=1, keepdims=True))
        err = np.abs(gs - rs) / scale
        print(f"calibrated gradient {prec}: max scaled error {err.max():.3e} (signal {err[:, :11].max():.3e}, "
              f"calibration {err[:, 11:].max():.3e})")
        assert err.max() <= tol


def test_tiny_grid_with_empty_node_intervals():
    """Fewer bins than node intervals: empty chunks are harmless."""
    n = 10
    spec, f, psd, data, dets, ev = make(1, n, f_hi=20.0 + 0.125 * 6)   # 7 bins
    rng = np.random.default_rng(2)
    th = cal_theta(synth.theta_batch(spec, 5), 3, n, rng, 0.05)
    ref = cal.logl(th, data, psd, dets, f, spec.df, n).numpy()
    got = gw.logl(torch.tensor(th, device=DEV), ev, "fp64").cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_calibrated_events_in_multi_plans(prec):
    """A plan mixing calibrated events (their own kernels after the persistent launch, theta of
    11 + 2 n ndet columns), a calibrated relative-binning event and plain events: every event's
    values and gradients equal its single-event calls (bit for bit on the calibrated ones, which run
    the same kernels); a calibrated event's values against the oracle."""
    from tests.test_rb_oracle import near
    n = 6
    spec, f, psd, data, dets = event_inputs(1, f_hi=300.0)
    t = lambda x: torch.tensor(x, device=DEV)
    evs = [gw.Event(t(data), t(psd), dets, t(f), spec.df, calibration_nodes=n),
           gw.Event(t(data), t(psd), dets, t(f), spec.df),
           gw.Event(t(data), t(psd), dets, t(f), spec.df, fiducial=spec.theta0, rb_eps=0.2, calibration_nodes=n),
           gw.Event(t(data), t(psd), dets, t(f), spec.df, calibration_nodes=n)]
    rng = np.random.default_rng(31)
    batches = [70, 129, 40, 0]
    thetas = [cal_theta(synth.theta_batch(spec, 70), 3, n, rng, 0.05), synth.theta_batch(spec, 129),
              cal_theta(near(spec.theta0, 40, seed=3, scale=0.3), 3, n, rng, 0.05), np.zeros((0, 11 + 6 * n))]
    tt = [t(x) for x in thetas]
    plan = gw.MultiPlan(evs, batches, prec, with_grad=True)
    logls, grads, lat = plan.launch(tt, latency=True)
    for ev, x, l, g, b in zip(evs, tt, logls, grads, batches):
        assert l.shape == (b,) and g.shape == x.shape
        if b == 0:
            continue
        sv, sg = gw.logl_grad(x, ev, prec)
        if ev.ncal:                         # the same kernels as a single call: the same bits
            assert torch.equal(l, sv) and torch.equal(g, sg)
        else:                               # the persistent kernel sums in another order
            assert np.abs(l.cpu().numpy() - sv.cpu().numpy()).max() <= (1e-8 if prec == "fp64" else 2e-4)
            tol = 1e-8 if prec == "fp64" else 2e-4
            assert np.abs(g.cpu().numpy() - sg.cpu().numpy()).max() <= tol * max(1.0, float(sg.abs().max()))
    ref = cal.logl(thetas[0][:4], data, psd, dets, f, spec.df, n).numpy()
    assert np.abs(logls[0].cpu().numpy()[:4] - ref).max() <= (1e-6 if prec == "fp64" else 1e-3)
    assert all(x > 0 for x, b in zip(lat, batches) if b > 0) and lat[3] == 0.0
    plan.close()


def test_calibrated_relative_binning_matches_the_composed_oracle():
    """Relative binning with the calibration model (gwl_event_create_rb_cal) against the oracle's
    composition of the two: the calibration factor at the edges multiplies h / h0, and
    <h_cal|h_cal> over every bin. Values in both precisions (both run the float64 edge loop) and
    the gradient over all 11 + 2 n ndet parameters."""
    from oracle import rb_oracle as rb
    from tests.test_rb_oracle import near
    n, nd, eps = 8, 3, 0.1
    spec, f, psd, data, dets = event_inputs(1, f_hi=600.0)
    t = lambda x: torch.tensor(x, device=DEV)
    ev = gw.Event(t(data), t(psd), dets, t(f), spec.df, fiducial=spec.theta0, rb_eps=eps, calibration_nodes=n)
    ne, nb = ev.rb_info()
    summ = rb.summary(data, psd, dets, f, spec.df, spec.theta0, eps)
    assert (ne, nb) == (len(summ["idx"]), len(f)) and ne < len(f) / 10
    rng = np.random.default_rng(13)
    th = cal_theta(near(spec.theta0, 8, seed=12, scale=0.3), nd, n, rng, 0.05)
    th[0, :11] = spec.theta0
    ref = rb.logl(th, summ, psd, dets, f, spec.df, nnode=n).numpy()
    for prec in ("fp64", "mixed"):
        got = gw.logl(t(th), ev, prec).cpu().numpy()
        err = np.abs(got - ref)
        tol = 1e-9 * np.maximum(1.0, np.abs(ref)) if prec == "fp64" else 1e-3
        print(f"calibrated RB ({ne} edges of {nb} bins) {prec}: max |dlogL| vs composed oracle {err.max():.3e}")
        assert np.all(err <= tol)
    _, gref = rb.logl_grad(th[:3], summ, psd, dets, f, spec.df, nnode=n)
    widths = np.concatenate([WIDTHS, np.full(2 * n * nd, 0.1)])
    for prec in ("fp64", "mixed"):
        _, g = gw.logl_grad(t(th[:3]), ev, prec)
        gs, rs = g.cpu().numpy() * widths, gref.numpy() * widths
        scale = np.maximum(np.abs(rs), 1e-3 * np.abs(rs).max(axis=1, keepdims=True))
        err = np.abs(gs - rs) / scale
        print(f"calibrated RB gradient {prec}: max scaled error {err.max():.3e}")
        assert err.max() <= 1e-8


def test_many_calibrated_events_share_the_plans_side_streams():
    """Seven calibrated events of different batch sizes (more events than the plan's side
    streams, so streams run several events in turn, in workspaces sized for their largest): every
    event's values and gradients equal its single calls bit for bit, on two launches in a row with
    different parameter points."""
    n = 4
    spec, f, psd, data, dets = event_inputs(1, f_hi=200.0)
    t = lambda x: torch.tensor(x, device=DEV)
    evs = [gw.Event(t(data), t(psd), dets, t(f), spec.df, calibration_nodes=n) for _ in range(7)]
    batches = [300, 7, 64, 129, 1, 250, 65]
    rng = np.random.default_rng(77)
    plan = gw.MultiPlan(evs, batches, "mixed", with_grad=True)
    try:
        base = synth.theta_batch(spec, 1000)
        for _ in range(2):
            tt = [t(cal_theta(base[rng.permutation(len(base))[:b]], 3, n, rng, 0.05)) for b in batches]
            logls, grads, _ = plan.launch(tt)
            for ev, x, l, g in zip(evs, tt, logls, grads):
                sv, sg = gw.logl_grad(x, ev, "mixed")
                assert torch.equal(l, sv) and torch.equal(g, sg)
    finally:
        plan.close()
        for ev in evs:
            ev.close()


@pytest.mark.parametrize("ndet", [1, 2, 4])
def test_calibrated_gradient_other_detector_counts(ndet):
    """The calibrated adjoint at 1, 2 and 4 detectors (the mixed kernel keeps its window moments'
    float64 totals in LDS, 8 ndet per lane) against the oracle's gradient over all
    11 + 2 n ndet parameters, on a batch spanning several point groups."""
    n = 6
    spec, f, psd, data, dets, ev = make(1, n, f_hi=300.0, ndet=ndet)
    rng = np.random.default_rng(60 + ndet)
    th = cal_theta(synth.theta_batch(spec, 150), ndet, n, rng, 0.05)
    th[0, :11] = spec.theta0
    idx = np.array([0, 1, 77, 149])
    _, gref = cal.logl_grad(th[idx], data, psd, dets, f, spec.df, n)
    widths = np.concatenate([WIDTHS, np.full(2 * n * ndet, 0.1)])
    for prec, tol in (("fp64", 1e-8), ("mixed", 1e-4)):
        _, g = gw.logl_grad(torch.tensor(th, device=DEV), ev, prec)
        gs, rs = g.cpu().numpy()[idx] * widths, gref.numpy() * widths
        scale = np.maximum(np.abs(rs), 1e-3 * np.abs(rs).max(axis=1, keepdims=True))
        err = np.abs(gs - rs) / scale
        print(f"calibrated gradient, {ndet} detectors, {prec}: max scaled error {err.max():.3e}")
        assert err.max() <= tol
    ev.close()


def test_calibrated_plan_launched_on_a_side_stream():
    """A plan with five calibrated events (more than one per side stream for some) launched from a
    torch stream other than the default: the results, read on that stream straight after the
    launch, equal the default-stream launch's bit for bit (the side streams fork from and join
    back into the caller's stream)."""
    n = 4
    spec, f, psd, data, dets = event_inputs(1, f_hi=200.0)
    t = lambda x: torch.tensor(x, device=DEV)
    evs = [gw.Event(t(data), t(psd), dets, t(f), spec.df, calibration_nodes=n) for _ in range(5)]
    batches = [200, 64, 3, 130, 90]
    rng = np.random.default_rng(91)
    base = synth.theta_batch(spec, 1000)
    tt = [t(cal_theta(base[rng.permutation(len(base))[:b]], 3, n, rng, 0.05)) for b in batches]
    plan = gw.MultiPlan(evs, batches, "mixed", with_grad=True)
    try:
        ref_v, ref_g, _ = plan.launch(tt)
        torch.cuda.synchronize()
        ref_v, ref_g = [x.clone() for x in ref_v], [x.clone() for x in ref_g]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            v, g, _ = plan.launch(tt)
            vc = [x * 1.0 for x in v]       # consumed on the side stream without a host wait
            gc = [x * 1.0 for x in g]
        torch.cuda.synchronize()
        for a, b in zip(vc + gc, ref_v + ref_g):
            assert torch.equal(a, b)
    finally:
        plan.close()
        for ev in evs:
            ev.close()
