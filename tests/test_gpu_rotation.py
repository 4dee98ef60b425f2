"""The float64 loop on uniform grids against the per-detector table phasor.

On a uniform grid the float64 kernels take every detector after the first from detector 0's
phasor: the forward by a Horner recurrence in the ratio exp(2 pi i df (T_det - T_0)) closed with
the exact phasor at each block's last bin, the adjoint by rotated phasors restarted every 32
bins. The same event with one frequency moved by 1e-11 Hz is not uniform, so it keeps the table
lookup per detector. Moving that one bin changes logL by about 4e-11; the two loops differ
by rounding only, which is far tighter than the oracle tolerance (1e-6) and so checks the
recurrence's algebra and block handling on their own: different detector counts, chunk layouts
whose chunks are not multiples of the block length, and the multi-event kernel.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1909_11873_amd import gwlike as gw
from paper_1909_11873_amd import synth
from tests.helpers import event_inputs, scaled_grad_error

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1909_11873_amd",
                     "tuning_gfx950.json")
BATCH = 700


def _event(f, psd, data, dets, df):
    return gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                    torch.tensor(f, device=DEV), df)


@pytest.fixture(scope="module", params=[2, 3, 4])
def pair(request):
    nd = request.param
    spec, f, psd, data, dets = event_inputs(1, f_hi=300.0, ndet=nd)
    moved = f.copy()
    moved[len(f) // 2] += 1e-11
    evu = _event(f, psd, data, dets, spec.df)
    evn = _event(moved, psd, data, dets, spec.df)
    th = synth.theta_batch(spec, BATCH)
    th[0] = spec.theta0
    yield nd, len(f), evu, evn, torch.tensor(th, device=DEV)
    evu.close()
    evn.close()
    gw.autotune_load(CACHE)


def _load_layout(path, nd, M, grad, waves, groups):
    npg = (BATCH + 63) // 64
    bucket = 1 << (npg - 1).bit_length()
    entry = {"ndet": nd, "mixed": 0, "grad": int(grad), "M": M, "npg_bucket": bucket,
             "waves": waves, "groups": groups, "setup": 0, "ms": 1.0}
    with open(path, "w") as fh:
        fh.write('{"arch": "gfx950", "entries": [\n  ' + json.dumps(entry) + "\n]}\n")
    gw.autotune_load(path)


@pytest.mark.parametrize("layout", [(16, 8), (4, 2), (1, 3)])
def test_uniform_grid_loop_matches_the_table_lookup(pair, layout, tmp_path):
    nd, M, evu, evn, t = pair
    path = str(tmp_path / "layout.json")
    try:
        for grad in (False, True):
            _load_layout(path, nd, M, grad, *layout)
            assert gw.launch_layout(evu, BATCH, "fp64", grad) == (layout[0], layout[1], False)
            if grad:
                (vu, gu), (vn, gn) = gw.logl_grad(t, evu, "fp64"), gw.logl_grad(t, evn, "fp64")
                err = scaled_grad_error(gu.cpu().numpy(), gn.cpu().numpy()).max()
                print(f"{nd} detectors, W{layout[0]} G{layout[1]}: adjoint max scaled gradient difference {err:.2e}")
                assert err <= 2e-9
            else:
                vu, vn = gw.logl(t, evu, "fp64"), gw.logl(t, evn, "fp64")
            vu, vn = vu.cpu().numpy(), vn.cpu().numpy()
            d = np.abs(vu - vn)
            print(f"{nd} detectors, W{layout[0]} G{layout[1]}, grad={grad}: max |dlogL| {d.max():.2e}")
            assert np.all(np.isfinite(vu)) and d.max() <= 1e-9 + 1e-13 * np.abs(vn).max()
    finally:
        gw.autotune_load(CACHE)


def test_multi_event_float64_loop_matches_the_table_lookup(pair):
    nd, M, evu, evn, t = pair
    out = []
    for ev in (evu, evn):
        plan = gw.MultiPlan([ev], [BATCH], "fp64", with_grad=True)
        v, g, _ = plan.launch([t])
        out.append((v[0].cpu().numpy(), g[0].cpu().numpy()))
        plan.close()
    (vu, gu), (vn, gn) = out
    assert np.abs(vu - vn).max() <= 1e-9 + 1e-13 * np.abs(vn).max()
    assert scaled_grad_error(gu, gn).max() <= 2e-9
