"""Shared test inputs: synthetic events with injections made by the FP64 oracle."""
from __future__ import annotations

import functools
import math

import numpy as np

from oracle import gw_oracle as o
from paper_1909_11873_amd import synth

# prior widths used to scale gradient components (relative step and error scale)
WIDTHS = np.array([50.0, 0.8, 1.8, 1.8, 1900.0, 2 * math.pi, math.pi, math.pi, math.pi, 2 * math.pi, 0.2])


@functools.lru_cache(maxsize=8)
def event_inputs(cfg: int, event: int = 0, f_hi: float | None = None, ndet: int | None = None, gmst: float = 0.0):
    """(spec, fgrid, psd, data, dets) of a workload; data = noise + oracle injection at theta0
    (seen at sidereal angle gmst)."""
    spec = synth.event_spec(cfg, event)
    f, psd, nz, dets = synth.event_arrays(spec)
    if f_hi is not None:
        m = int(round((f_hi - spec.f_lo) / spec.df)) + 1
        f, psd, nz = f[:m], psd[:, :m], nz[:, :m]
    if ndet is not None:
        names = (["D1", "D2", "D3", "D1"] * 2)[:ndet]
        dets = np.array([synth.detector_rad(n) for n in names])
        if ndet == 4:  # a fourth site so that no two detectors coincide
            dets[3] = np.radians([-31.4, 115.7, 0.0, 90.0])
        psd = np.stack([psd[0]] * ndet)
        nz = np.stack([synth.noise(spec.seed_base + 50 + i, psd[0], spec.df) for i in range(ndet)])
    data = nz + o.strain_all(spec.theta0, dets, f, gmst).numpy()
    return spec, f, psd, data, dets


def scaled_grad_error(g, gref):
    """Per-component error of theta-width-scaled gradients, relative to max(|g_i|, 1e-3 ||g||_inf)."""
    gs = np.asarray(g) * WIDTHS
    rs = np.asarray(gref) * WIDTHS
    scale = np.maximum(np.abs(rs), 1e-3 * np.max(np.abs(rs), axis=-1, keepdims=True))
    return np.abs(gs - rs) / scale
