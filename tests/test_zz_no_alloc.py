"""gwl_logl_batch_noalloc (the forward call whose workspace is a fixed device array) against
gwl_logl_batch, called through the C ABI: two calls in a row, the second with a smaller batch,
in both precisions, on a full-size three-detector event; and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1909_11873_amd import gwlike as gw
from paper_1909_11873_amd import synth
from tests.helpers import event_inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
SCRATCH_BYTES = 64 << 20


def noalloc(ev, theta, prec):
    out = torch.full((theta.shape[0],), float("nan"), dtype=torch.float64, device=DEV)
    st = gw.lib().gwl_logl_batch_noalloc(ev.handle, ctypes.c_void_p(theta.data_ptr()), theta.shape[0], gw._prec(prec),
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    return st, out


def test_noalloc_matches_logl_batch_twice_then_smaller():
    spec, f, psd, data, dets = event_inputs(1)
    ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets, torch.tensor(f, device=DEV),
                  spec.df)
    th = synth.theta_batch(spec, 20000)
    th[0] = spec.theta0
    big = torch.tensor(th, device=DEV)
    small = torch.tensor(th[5:1234][::-1].copy(), device=DEV)      # a different, smaller batch
    for prec in ("fp64", "mixed"):
        for theta in (big, small):
            ref = gw.logl(theta, ev, prec).cpu().numpy()
            st, got = noalloc(ev, theta, prec)
            assert st == 0, gw.lib().gwl_last_error().decode()
            got = got.cpu().numpy()
            assert np.all(np.isfinite(got))
            err = np.abs(got - ref)
            tol = 1e-9 * np.maximum(1.0, np.abs(ref)) if prec == "fp64" else 1e-3
            print(f"noalloc {prec} B={theta.shape[0]}: max |diff| vs gwl_logl_batch {err.max():.2e}")
            assert np.all(err <= tol)
    ev.close()


def test_noalloc_adapts_its_shape_to_the_scratch_and_rejects_bad_sizes():
    """A batch whose tuned launch would need more workspace than the fixed arrays hold (the set-up
    rows of 300,032 points alone are 72 MB) still runs, with a shape that fits, and agrees with
    gwl_logl_batch; sizes outside [0, 2^30] are refused before anything is launched."""
    spec, f, psd, data, dets = event_inputs(1, f_hi=60.0)
    ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets, torch.tensor(f, device=DEV),
                  spec.df)
    n = 300032
    th = torch.tensor(synth.prior_draw(np.random.default_rng(8), n), device=DEV)
    assert 30 * 8 * n > SCRATCH_BYTES
    for prec in ("mixed", "fp64"):
        st, out = noalloc(ev, th, prec)
        assert st == 0, gw.lib().gwl_last_error().decode()
        ref = gw.logl(th, ev, prec)
        tol = 1e-3 if prec == "mixed" else 1e-9 * max(1.0, float(ref.abs().max()))
        assert float((out - ref).abs().max()) <= tol
    small = th[:10]
    st = gw.lib().gwl_logl_batch_noalloc(ev.handle, ctypes.c_void_p(small.data_ptr()), (1 << 30) + 1, 1,
                                         ctypes.c_void_p(small.data_ptr()), None)
    assert st == -2 and "outside" in gw.lib().gwl_last_error().decode()
    st = gw.lib().gwl_logl_batch_noalloc(ev.handle, ctypes.c_void_p(small.data_ptr()), -1, 1,
                                         ctypes.c_void_p(small.data_ptr()), None)
    assert st == -2
    ev.close()
