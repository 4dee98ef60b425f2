"""Multi-event persistent launch (HIP graph) against single-event calls and the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import gw_oracle as o
from paper_1909_11873_amd import gwlike as gw
from paper_1909_11873_amd import synth
from tests.helpers import WIDTHS, scaled_grad_error

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

# five events of the uneven-batching workload's kind, band-limited to keep the oracle quick;
# one event has an empty batch and one a single point
DURATIONS = [4.0, 16.0, 8.0, 4.0, 32.0]
BATCHES = [70, 300, 0, 1, 129]


def build_events(f_hi=300.0):
    out = []
    for i, (dur, b) in enumerate(zip(DURATIONS, BATCHES)):
        spec = synth.event_spec(4, i)
        df = 1.0 / dur
        f = synth.freq_grid(20.0, f_hi, df)
        s = synth.psd_fit(f)
        psd = np.stack([s] * 3)
        nz = np.stack([synth.noise(spec.seed_base + d, s, df) for d in range(3)])
        dets = np.array([synth.detector_rad(n) for n in spec.det_names])
        data = nz + o.strain_all(spec.theta0, dets, f).numpy()
        th = synth.prior_draw(np.random.default_rng(spec.seed_base + 10), b)
        ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                      torch.tensor(f, device=DEV), df)
        out.append(dict(ev=ev, th=th, f=f, psd=psd, data=data, dets=dets, df=df))
    return out


@pytest.fixture(scope="module")
def events():
    return build_events()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multi_forward_matches_single_calls_and_oracle(events, prec):
    plan = gw.MultiPlan([e["ev"] for e in events], BATCHES, prec, with_grad=False)
    thetas = [torch.tensor(e["th"], device=DEV).reshape(-1, 11) for e in events]
    logls, grads, lat = plan.launch(thetas, latency=True)
    assert grads is None
    for e, t, l in zip(events, thetas, logls):
        if t.shape[0] == 0:
            assert l.shape == (0,)
            continue
        single = gw.logl(t, e["ev"], prec).cpu().numpy()
        got = l.cpu().numpy()
        assert np.abs(got - single).max() <= (1e-8 if prec == "fp64" else 2e-4)
        n = min(4, t.shape[0])
        ref = o.logl(e["th"][:n], e["data"], e["psd"], e["dets"], e["f"], e["df"]).numpy()
        assert np.abs(got[:n] - ref).max() <= (1e-6 if prec == "fp64" else 1e-3)
    assert len(lat) == len(events)
    assert all(x > 0 for x, b in zip(lat, BATCHES) if b > 0)
    assert lat[BATCHES.index(0)] == 0.0
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multi_gradient_matches_oracle(events, prec):
    plan = gw.MultiPlan([e["ev"] for e in events], BATCHES, prec, with_grad=True)
    thetas = [torch.tensor(e["th"], device=DEV).reshape(-1, 11) for e in events]
    logls, grads, _ = plan.launch(thetas)
    for e, t, l, g in zip(events, thetas, logls, grads):
        if t.shape[0] == 0:
            continue
        n = min(2, t.shape[0])
        v, gr = o.logl_grad(e["th"][:n], e["data"], e["psd"], e["dets"], e["f"], e["df"])
        assert np.abs(l.cpu().numpy()[:n] - v.numpy()).max() <= (1e-6 if prec == "fp64" else 1e-3)
        assert scaled_grad_error(g.cpu().numpy()[:n], gr.numpy()).max() <= 1e-4
    plan.close()


def test_multi_graph_replays_are_identical(events):
    """Replays of the captured graph, with eager work in between, reproduce the first result bitwise."""
    plan = gw.MultiPlan([e["ev"] for e in events], BATCHES, "mixed", with_grad=True)
    thetas = [torch.tensor(e["th"], device=DEV).reshape(-1, 11) for e in events]
    first, gfirst, _ = plan.launch(thetas)
    first = [x.cpu().numpy() for x in first]
    gfirst = [x.cpu().numpy() for x in gfirst]
    for rep in range(4):
        torch.cuda.synchronize()
        _ = gw.logl(thetas[1], events[1]["ev"], "mixed")   # eager work between replays
        again, g, _ = plan.launch(thetas)
        for a, b in zip(first, again):
            assert np.array_equal(a, b.cpu().numpy())
        for a, b in zip(gfirst, g):
            assert np.array_equal(a, b.cpu().numpy())
    # new inputs through the same plan
    th2 = [t.flip(0).contiguous() for t in thetas]
    l2, _, _ = plan.launch(th2)
    for e, t, l in zip(events, th2, l2):
        if t.shape[0]:
            assert np.abs(l.cpu().numpy() - gw.logl(t, e["ev"], "mixed").cpu().numpy()).max() <= 2e-4
    plan.close()


def test_queue_order_does_not_change_results(events):
    """Plans queued by ascending and by descending work give the same values and gradients bit
    for bit (each item writes its own partial sums, added in a fixed order)."""
    thetas = [torch.tensor(e["th"], device=DEV).reshape(-1, 11) for e in events]
    out = {}
    for order in ("ascending", "descending", "tuned"):
        plan = gw.MultiPlan([e["ev"] for e in events], BATCHES, "mixed", with_grad=True, order=order)
        l, g, lat = plan.launch(thetas, latency=True)
        out[order] = ([x.cpu().numpy() for x in l], [x.cpu().numpy() for x in g])
        assert plan.info()[1] == (order == "descending") or order == "tuned"
        plan.close()
    for order in ("descending", "tuned"):
        for a, b in zip(out["ascending"][0] + out["ascending"][1], out[order][0] + out[order][1]):
            assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        gw.MultiPlan([e["ev"] for e in events], BATCHES, "mixed", order="random")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multi_autotune_roundtrip(events, prec, tmp_path):
    """The tuner times plan shapes, records the fastest, and a new plan for the same workload
    takes it; its results match the heuristic plan's."""
    evs = [e["ev"] for e in events]
    thetas = [torch.tensor(e["th"], device=DEV).reshape(-1, 11) for e in events]
    base = gw.MultiPlan(evs, BATCHES, prec, with_grad=True)
    l0, g0, _ = base.launch(thetas)
    path = str(tmp_path / "tune.json")
    gw.multi_autotune(evs, BATCHES, prec, with_grad=True, cache_path=path)
    text = open(path).read()
    assert '"multi": 1' in text
    import json
    entry = [x for x in json.loads(text)["entries"] if x.get("multi") == 1 and x["mixed"] == (prec == "mixed")][0]
    plan = gw.MultiPlan(evs, BATCHES, prec, with_grad=True)
    chunk, desc, items = plan.info()
    assert (chunk, int(desc)) == (entry["chunk"], entry["descending"])
    assert items > 0
    l1, g1, _ = plan.launch(thetas)
    tol = 1e-9 if prec == "fp64" else 2e-4
    for a, b, ga, gb, t in zip(l0, l1, g0, g1, thetas):
        if t.shape[0]:
            assert np.abs(a.cpu().numpy() - b.cpu().numpy()).max() <= tol
            scale = np.abs(ga.cpu().numpy()).max()
            assert np.abs(ga.cpu().numpy() - gb.cpu().numpy()).max() <= 1e-6 * scale
    gw.autotune_load(path)   # the file parses back
    plan.close()
    base.close()


def test_multi_plan_argument_errors(events):
    with pytest.raises(ValueError):
        gw.MultiPlan([events[0]["ev"]], [1, 2])
    plan = gw.MultiPlan([events[0]["ev"]], [70], "mixed")
    with pytest.raises(ValueError):
        plan.launch([torch.zeros(3, 11, dtype=torch.float64, device=DEV)])
    plan.close()
    # events of one plan share their detector count
    e = events[0]
    one = gw.Event(torch.tensor(e["data"][:1], device=DEV), torch.tensor(e["psd"][:1], device=DEV), e["dets"][:1],
                   torch.tensor(e["f"], device=DEV), e["df"])
    with pytest.raises(gw.GWLError, match="detector count"):
        gw.MultiPlan([e["ev"], one], [70, 5], "mixed")
    one.close()


def test_c4_full_workload_sampled():
    """All 64 uneven events at full size in one mixed-precision launch with gradients (the launch the
    benchmark times); four or five points of every event (the injection, the loudest prior draw and
    three more), values and gradients, against the FP64 oracle; then the float64 plan's gradient on
    the same points to 1e-4 per width-scaled component."""
    from tests.helpers import event_inputs

    evs, ths, inputs = [], [], []
    for e in range(64):
        spec, f, psd, data, dets = event_inputs(4, e)
        evs.append(gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                            torch.tensor(f, device=DEV), spec.df))
        th = synth.theta_batch(spec)
        th[0] = spec.theta0
        ths.append(th)
        inputs.append((f, psd, data, dets, spec.df))
    batches = [len(t) for t in ths]
    # the committed plan shape, loaded as the benchmark loads it
    import json
    import os
    cache = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "paper_1909_11873_amd", "tuning_gfx950.json")
    gw.autotune_load(cache)
    tuned = [(e["chunk"], bool(e["descending"])) for e in json.load(open(cache))["entries"]
             if e.get("multi") and e["events"] == 64 and e["mixed"] == 1 and e["grad"] == 1]
    plan = gw.MultiPlan(evs, batches, "mixed", with_grad=True)
    assert len(tuned) == 1 and plan.info()[:2] == tuned[0]
    logls, grads, lat = plan.launch([torch.tensor(t, device=DEV) for t in ths], latency=True)
    worst, worst_g, worst_v = 0.0, 0.0, 0.0
    fp64_checks = []
    for e, (th, l, g, inp) in enumerate(zip(ths, logls, grads, inputs)):
        f, psd, data, dets, df = inp
        b = len(th)
        # the injection, the loudest prior draw of the event and three more points
        loud = int(np.argmax(th[1:, 0] ** (5 / 3) / th[1:, 4] ** 2)) + 1
        sample = np.unique([0, 1, loud, b // 2, b - 1])
        ref, gr = o.logl_grad(th[sample], data, psd, dets, f, df)
        err = np.abs(l.cpu().numpy()[sample] - ref.numpy())
        worst = max(worst, float(err.max()))
        assert err.max() <= 1e-3, (e, len(f), err)
        ge = scaled_grad_error(g.cpu().numpy()[sample], gr.numpy())
        gs, rs = g.cpu().numpy()[sample] * WIDTHS, gr.numpy() * WIDTHS
        vec = np.linalg.norm(gs - rs, axis=1) / np.linalg.norm(rs, axis=1)
        worst_g = max(worst_g, float(ge.max()))
        worst_v = max(worst_v, float(vec.max()))
        # the mixed adjoint carries the phasor in float32: per component it is held to 1e-3 of
        # max(|g_i|, 1e-3 |g|_inf) and as a vector to 1e-5 (components a thousand times below their
        # natural size need the float64 adjoint for 1e-4; see the float64 plan below)
        assert ge.max() <= 1e-3 and vec.max() <= 1e-5, (e, len(f), ge.max(), vec.max())
        fp64_checks.append((e, sample, gr.numpy()))
    print(f"c4: {sum(batches)} points, max |dlogL| {worst:.3e}, max scaled grad error {worst_g:.3e} (vector form "
          f"{worst_v:.3e}), latency p50 {np.percentile(lat, 50):.0f} us p99 {np.percentile(lat, 99):.0f} us")
    assert all(x > 0 for x in lat)
    plan.close()
    # the float64 plan on the same workload meets 1e-4 per width-scaled component on every point
    plan64 = gw.MultiPlan(evs, batches, "fp64", with_grad=True)
    _, grads64, _ = plan64.launch([torch.tensor(t, device=DEV) for t in ths])
    worst64 = 0.0
    for e, sample, gref in fp64_checks:
        ge = scaled_grad_error(grads64[e].cpu().numpy()[sample], gref)
        worst64 = max(worst64, float(ge.max()))
    print(f"c4 float64 plan: max scaled grad error {worst64:.3e}")
    assert worst64 <= 1e-4
    plan64.close()
    for ev in evs:
        ev.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multi_with_relative_binning_events(events, prec):
    """A plan may mix relative-binning events (rows on the edges, the fiducial's phase subtracted
    at set-up) with full-grid events: each event's results equal its single-event calls."""
    mixed_events = []
    for i, e in enumerate(events):
        if i % 2 == 0:
            fid = synth.event_spec(4, i).theta0
            ev = gw.Event(torch.tensor(e["data"], device=DEV), torch.tensor(e["psd"], device=DEV), e["dets"],
                          torch.tensor(e["f"], device=DEV), e["df"], fiducial=fid, rb_eps=0.2)
            assert 0 < ev.rb_edges < len(e["f"])
            mixed_events.append(ev)
        else:
            mixed_events.append(e["ev"])
    # points near each event's fiducial, where relative binning is meant to be used
    rng = np.random.default_rng(5)
    step = np.array([0.05, 0.01, 0.02, 0.02, 10.0, 0.01, 0.01, 0.02, 0.02, 0.05, 1e-4]) * 0.3
    thetas = [torch.tensor(synth.event_spec(4, i).theta0 + step * rng.standard_normal((b, 11)), device=DEV)
              for i, b in enumerate(BATCHES)]
    for grad in (False, True):
        plan = gw.MultiPlan(mixed_events, BATCHES, prec, with_grad=grad)
        logls, grads, _ = plan.launch(thetas)
        for ev, t, l, g in zip(mixed_events, thetas, logls, grads if grad else [None] * len(thetas)):
            if t.shape[0] == 0:
                continue
            if grad:
                sv, sg = gw.logl_grad(t, ev, prec)
                tol = 1e-8 if prec == "fp64" else 2e-4
                assert np.abs(g.cpu().numpy() - sg.cpu().numpy()).max() <= tol * max(1.0, float(sg.abs().max()))
            else:
                sv = gw.logl(t, ev, prec)
            assert np.abs(l.cpu().numpy() - sv.cpu().numpy()).max() <= (1e-8 if prec == "fp64" else 2e-4)
        plan.close()
    for i, ev in enumerate(mixed_events):
        if i % 2 == 0:
            ev.close()


@pytest.mark.parametrize("grad", [False, True])
def test_many_small_events_in_one_plan(events, grad):
    """300 events of 0 to 3 points each, drawn from the five events above (the same event may
    appear many times in one plan): every value and gradient against that event's single call,
    with the latency of every non-empty event positive."""
    rng = np.random.default_rng(17)
    pick = rng.integers(0, len(events), 300)
    batches = [int(b) for b in rng.integers(0, 4, 300)]
    evs = [events[i]["ev"] for i in pick]
    thetas = []
    for b in batches:
        th = synth.prior_draw(np.random.default_rng(int(rng.integers(1 << 30))), b)
        thetas.append(torch.tensor(th, device=DEV).reshape(-1, 11))
    plan = gw.MultiPlan(evs, batches, "mixed", with_grad=grad)
    try:
        logls, grads, lat = plan.launch(thetas, latency=True)
        for k, (ev, t, l) in enumerate(zip(evs, thetas, logls)):
            if t.shape[0] == 0:
                assert l.shape == (0,) and lat[k] == 0.0
                continue
            assert lat[k] > 0
            if grad:
                sv, sg = gw.logl_grad(t, ev, "mixed")
                g = grads[k]
                assert np.abs(g.cpu().numpy() - sg.cpu().numpy()).max() <= 2e-4 * max(1.0, float(sg.abs().max()))
            else:
                sv = gw.logl(t, ev, "mixed")
            assert np.abs(l.cpu().numpy() - sv.cpu().numpy()).max() <= 2e-4
    finally:
        plan.close()
