"""gwl_logl_batch_live (a batch whose length the device decides): the first *live points come out
bit for bit as in the same call with every point live, and within rounding of gwl_logl_batch
(whose launch may split the bins differently); the rest of the output is left as it was; both
precisions, at tuned and heuristic shapes, and under graph capture with the length changed
between replays."""
import numpy as np
import pytest
import torch

from paper_1909_11873_amd import gwlike as gw
from paper_1909_11873_amd import synth
from tests.helpers import event_inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TUNE = "paper_1909_11873_amd/tuning_gfx950.json"


def _event(cfg, f_hi=None):
    spec, f, psd, data, dets = event_inputs(cfg, f_hi=f_hi)
    t = lambda x: torch.tensor(x, device=DEV)
    return spec, gw.Event(t(data), t(psd), dets, t(f), spec.df)


@pytest.mark.parametrize("cfg,B,f_hi", [(1, 8192, None), (0, 1000, None), (1, 193, 300.0)])
def test_live_rows_equal_a_full_call(cfg, B, f_hi):
    gw.autotune_load(TUNE)
    spec, ev = _event(cfg, f_hi)
    th = torch.tensor(synth.theta_batch(spec, B), device=DEV)
    for prec in ("fp64", "mixed"):
        ref = gw.logl(th, ev, prec)
        full = gw.logl_live(th, torch.tensor(B, dtype=torch.int64, device=DEV), ev, prec)
        tol = 1e-9 * ref.abs().clamp(min=1.0) if prec == "fp64" else 2e-4
        assert bool(((full - ref).abs() <= tol).all()), prec
        for n in (0, 1, 63, 64, 65, B // 3, B - 1, B, B + 100):
            live = torch.tensor(n, dtype=torch.int64, device=DEV)
            out = torch.full((B,), 123.5, dtype=torch.float64, device=DEV)
            gw.logl_live(th, live, ev, prec, out=out)
            k = min(n, B)
            assert torch.equal(out[:k], full[:k]), (prec, n)
            assert bool((out[k:] == 123.5).all()), (prec, n)
    ev.close()


def test_live_length_changes_between_graph_replays():
    spec, ev = _event(1)
    B = 2048
    th = torch.tensor(synth.theta_batch(spec, B), device=DEV)
    live = torch.tensor(B, dtype=torch.int64, device=DEV)
    full = gw.logl_live(th, live, ev, "mixed")
    out = torch.zeros(B, dtype=torch.float64, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gw.logl_live(th, live, ev, "mixed", out=out)           # reserves the workspace on s
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gw.logl_live(th, live, ev, "mixed", out=out)
    for n in (B, 700, 0, 1, 1999):
        out.fill_(-7.0)
        live.fill_(n)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[:n], full[:n]) and bool((out[n:] == -7.0).all()), n
    ev.close()


def test_live_rejections():
    spec, ev = _event(0)
    th = torch.tensor(synth.theta_batch(spec, 10), device=DEV)
    with pytest.raises(ValueError):
        gw.logl_live(th, torch.tensor(3, dtype=torch.int32, device=DEV), ev)   # not int64
    L = gw.lib()
    import ctypes
    out = torch.empty(10, dtype=torch.float64, device=DEV)
    st = L.gwl_logl_batch_live(ev.handle, ctypes.c_void_p(th.data_ptr()), 10, None, gw.GWL_MIXED,
                               ctypes.c_void_p(out.data_ptr()), None)
    assert st == -1                                                         # live is required
    ev.close()
    cspec, f, psd, data, dets = event_inputs(0)
    t = lambda x: torch.tensor(x, device=DEV)
    cev = gw.Event(t(data), t(psd), dets, t(f), cspec.df, calibration_nodes=4)
    thc = torch.zeros(10, 11 + 8, dtype=torch.float64, device=DEV)
    with pytest.raises(gw.GWLError):
        gw.logl_live(thc, torch.tensor(3, dtype=torch.int64, device=DEV), cev)
    cev.close()
