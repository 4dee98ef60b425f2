"""Launch layouts give the same results: the per-point set-up inside the evaluation kernel (its
intrinsic and extrinsic halves on two wavefronts, or both on one when the workgroup has a single
wavefront) against the separate set-up kernel, for the same bin chunks. The chunks and their
order are the same, so values and gradients must agree bit for bit; against the oracle the
usual tolerances hold.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import gw_oracle as o
from paper_1909_11873_amd import gwlike as gw
from paper_1909_11873_amd import synth
from tests.helpers import event_inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1909_11873_amd",
                     "tuning_gfx950.json")


def load_layout(path, nd, M, prec, grad, batch, waves, groups, setup, sepepi=0):
    """Make (waves, groups, setup) the layout of calls with this shape (the tuner's cache format);
    sepepi: the value's reduction over the groups by the separate epilogue kernel."""
    npg = (batch + 63) // 64
    bucket = 1
    while bucket < npg:
        bucket *= 2
    entry = {"ndet": nd, "mixed": int(prec == "mixed"), "grad": int(grad), "M": M, "npg_bucket": bucket,
             "waves": waves, "groups": groups, "setup": setup, "sepepi": sepepi, "ms": 1.0}
    with open(path, "w") as fh:
        fh.write('{"arch": "gfx950", "entries": [\n  ' + json.dumps(entry) + "\n]}\n")
    gw.autotune_load(path)


@pytest.fixture(scope="module")
def events():
    out = {}
    for cfg, f_hi, batch in ((0, None, 1000), (1, 300.0, 700)):
        spec, f, psd, data, dets = event_inputs(cfg) if f_hi is None else event_inputs(cfg, f_hi=f_hi)
        ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                      torch.tensor(f, device=DEV), spec.df)
        th = synth.theta_batch(spec, batch)
        th[0] = spec.theta0
        out[cfg] = (spec, f, psd, data, dets, ev, th)
    yield out
    for v in out.values():
        v[5].close()
    gw.autotune_load(CACHE)


@pytest.mark.parametrize("cfg", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("grad", [False, True])
def test_setup_in_kernel_matches_setup_kernel(events, cfg, prec, grad, tmp_path):
    spec, f, psd, data, dets, ev, th = events[cfg]
    t = torch.tensor(th, device=DEV)
    path = str(tmp_path / "layout.json")
    try:
        for waves, groups in ((16, 8), (4, 2), (1, 4)):
            got = []
            for setup in (1, 0):
                load_layout(path, len(dets), len(f), prec, grad, len(th), waves, groups, setup)
                assert gw.launch_layout(ev, len(th), prec, grad) == (waves, groups, bool(setup))
                if grad:
                    v, g = gw.logl_grad(t, ev, prec)
                    got.append((v.cpu().numpy(), g.cpu().numpy()))
                else:
                    got.append((gw.logl(t, ev, prec).cpu().numpy(), None))
            (v1, g1), (v0, g0) = got
            print(f"c{cfg} {prec} grad={grad} W{waves} G{groups}: max |in-kernel - separate| "
                  f"{np.abs(v1 - v0).max():.3e}")
            assert np.array_equal(v1, v0)
            if grad:
                assert np.array_equal(g1, g0)
        # the values against the oracle on a few points, at the last layout
        idx = np.array([0, 1, 63, 64, len(th) - 1])
        ref = o.logl(th[idx], data, psd, dets, f, spec.df).numpy()
        assert np.abs(v1[idx] - ref).max() <= (1e-3 if prec == "mixed" else 1e-6)
    finally:
        gw.autotune_load(CACHE)


def test_out_of_range_point_is_nan_with_the_split_setup(events, tmp_path):
    """A point whose phase could exceed the supported range (t_c far outside the segment) gets NaN
    from the in-kernel set-up as from the set-up kernel; its neighbours are unaffected."""
    spec, f, psd, data, dets, ev, th = events[0]
    th = th.copy()
    th[5, 10] = 1e9          # t_c: 1e9 s, far beyond the phase range at 1 kHz
    t = torch.tensor(th, device=DEV)
    path = str(tmp_path / "layout.json")
    try:
        for setup, sepepi in ((1, 0), (1, 1), (0, 0), (0, 1)):
            for grad in (False, True):
                load_layout(path, 1, len(f), "fp64", grad, len(th), 16, 8, setup, sepepi if not grad else 0)
                if grad:
                    v, g = gw.logl_grad(t, ev, "fp64")
                    g = g.cpu().numpy()
                    assert np.isnan(g[5]).any() and np.isfinite(g[[4, 6]]).all()
                else:
                    v = gw.logl(t, ev, "fp64")
                v = v.cpu().numpy()
                assert np.isnan(v[5]) and np.isfinite(v[[4, 6]]).all()
    finally:
        gw.autotune_load(CACHE)


@pytest.mark.parametrize("cfg", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_separate_value_epilogue_matches_the_last_workgroup(events, cfg, prec, tmp_path):
    """The value's reduction over G workgroups by the separate epilogue kernel gives the bits of
    the last-arriving workgroup's reduction (same order, same epilogue arithmetic), with the
    set-up in its own kernel or in the evaluation kernel (whose first workgroup per point group
    then leaves the epilogue's rows), also for the first rows of a live-length call."""
    spec, f, psd, data, dets, ev, th = events[cfg]
    t = torch.tensor(th, device=DEV)
    path = str(tmp_path / "layout.json")
    try:
        for waves, groups in ((16, 8), (4, 3), (1, 16)):
            got = []
            for setup in (0, 1):
                for sepepi in (0, 1):
                    load_layout(path, len(dets), len(f), prec, False, len(th), waves, groups, setup, sepepi)
                    got.append(gw.logl(t, ev, prec).cpu().numpy())
            for other in got[1:]:
                assert np.array_equal(got[0], other), (waves, groups)
        live = torch.tensor([len(th) // 3], dtype=torch.int64, device=DEV)
        out = torch.full((len(th),), 7.0, dtype=torch.float64, device=DEV)
        gw.logl_live(t, live, ev, prec, out=out)
        v = out.cpu().numpy()
        n = len(th) // 3
        assert np.all(v[n:] == 7.0) and np.all(np.isfinite(v[:n]))
        ref = gw.logl(t, ev, prec).cpu().numpy()[:n]
        assert np.abs(v[:n] - ref).max() <= (1e-4 if prec == "mixed" else 1e-9)
    finally:
        gw.autotune_load(CACHE)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_separate_value_epilogue_with_the_isco_cutoff(prec, tmp_path):
    """With the ISCO cut-off the separate epilogue takes each point's kept share of K_det as the
    fused one does: bitwise equal values, with the set-up in either kernel."""
    spec, f, psd, data, dets = event_inputs(1, f_hi=600.0)
    ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                  torch.tensor(f, device=DEV), spec.df, isco_cutoff=True)
    th = synth.theta_batch(spec, 500)
    th[:, 0] = np.linspace(20.0, 60.0, len(th))     # cut-offs across the band
    t = torch.tensor(th, device=DEV)
    path = str(tmp_path / "layout.json")
    try:
        got = []
        for setup in (0, 1):
            for sepepi in (0, 1):
                load_layout(path, len(dets), len(f), prec, False, len(th), 8, 4, setup, sepepi)
                got.append(gw.logl(t, ev, prec).cpu().numpy())
        assert np.all(np.isfinite(got[0])) and all(np.array_equal(got[0], x) for x in got[1:])
    finally:
        ev.close()
        gw.autotune_load(CACHE)
