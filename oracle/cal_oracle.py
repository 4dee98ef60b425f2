"""Detector calibration model: a plain FP64 reference.

TEST INFRASTRUCTURE ONLY. Only tests/, the package's smoke check and bench.py's CPU leg may
import this module; the library never does.

The paper's section 2 ("Models and parameter spaces") and its GW150914 set-up model the
uncertainty of each detector's calibration by amplitudes and phases at a set of frequency nodes,
typically ten per detector (20 parameters per detector), interpolated in frequency. It gives no
formulas; the readings taken here (each one pinned in tests/test_cal_oracle.py):

  C1  Nodes: n frequencies spaced uniformly in ln f from the grid's first to its last bin.
  C2  Interpolation: a cubic Catmull-Rom spline in ln f through the node values (it passes
      through every node, is continuous with its first derivative, and each bin depends on the
      four nearest nodes only). Beyond the end nodes the missing neighbour is the linear
      extrapolation of the last two, so linear functions of ln f are reproduced exactly.
  C3  The calibrated model is h_cal(f) = h(f) (1 + dA(f)) exp(i dphi(f)), dA and dphi the splines
      of the amplitude and phase node values of that detector.
  C4  Parameters: theta[11 + 2 n ndet] = the 11 signal parameters, then per detector its n
      amplitude node values followed by its n phase node values (radians).

logL = sum_det [ <d|h_cal> - 1/2 <h_cal|h_cal> ], all bins, as in the uncalibrated oracle.

Parity status: pinned (interpolation through the nodes, linear reproduction, closed forms for a
constant amplitude and a constant phase offset, reduction to the uncalibrated oracle at zero).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle import gw_oracle as o


def node_frequencies(f_lo, f_hi, n):
    """C1: n nodes uniform in ln f on [f_lo, f_hi]."""
    return np.exp(np.linspace(math.log(f_lo), math.log(f_hi), n))


def spline(fgrid, values, f_lo, f_hi):
    """C2: Catmull-Rom spline in ln f through `values` (torch [n]) at the nodes, on fgrid."""
    values = torch.as_tensor(values, dtype=o.DT)
    n = values.shape[0]
    x = torch.log(torch.as_tensor(fgrid, dtype=o.DT))
    x0, x1 = math.log(f_lo), math.log(f_hi)
    h = (x1 - x0) / (n - 1)
    s = ((x - x0) / h).clamp(0.0, n - 1)
    j = torch.clamp(torch.floor(s).long(), 0, n - 2)
    t = s - j
    # node values with one linearly extrapolated ghost node at each end
    ext = torch.cat([(2 * values[0] - values[1])[None], values, (2 * values[-1] - values[-2])[None]])
    pm, p0, p1, p2 = ext[j], ext[j + 1], ext[j + 2], ext[j + 3]
    return 0.5 * (2 * p0 + (p1 - pm) * t + (2 * pm - 5 * p0 + 4 * p1 - p2) * t ** 2
                  + (3 * p0 - pm - 3 * p1 + p2) * t ** 3)


def factor(fgrid, amp_nodes, phase_nodes):
    """C3: (1 + dA(f)) exp(i dphi(f)) on the grid."""
    f = torch.as_tensor(fgrid, dtype=o.DT)
    f_lo, f_hi = float(f[0]), float(f[-1])
    da = spline(f, amp_nodes, f_lo, f_hi)
    dp = spline(f, phase_nodes, f_lo, f_hi)
    return (1.0 + da).to(o.CDT) * torch.exp(1j * dp.to(o.CDT))


def logl_point(theta, data, psd, dets, fgrid, df, nnode, gmst=0.0):
    """logL of the calibrated model for one point; theta [11 + 2 nnode ndet] (C4)."""
    data = torch.as_tensor(data).to(o.CDT)
    psd = torch.as_tensor(psd).to(o.DT)
    fgrid = torch.as_tensor(fgrid).to(o.DT)
    total = torch.zeros((), dtype=o.DT)
    for i in range(len(dets)):
        base = 11 + 2 * nnode * i
        cal = factor(fgrid, theta[base:base + nnode], theta[base + nnode:base + 2 * nnode])
        h = o.detector_strain(fgrid, theta[:11], tuple(float(v) for v in dets[i]), gmst) * cal
        total = total + o.inner(data[i], h, psd[i], df) - 0.5 * o.inner(h, h, psd[i], df)
    return total


def logl(theta, data, psd, dets, fgrid, df, nnode, gmst=0.0):
    th = torch.as_tensor(theta, dtype=o.DT)
    th = th.reshape(th.shape[0], -1) if th.dim() > 1 else th.reshape(1, -1)
    out = torch.empty(th.shape[0], dtype=o.DT)
    with torch.no_grad():
        for b in range(th.shape[0]):
            out[b] = logl_point(th[b], data, psd, dets, fgrid, df, nnode, gmst)
    return out


def logl_grad(theta, data, psd, dets, fgrid, df, nnode, gmst=0.0):
    th = torch.as_tensor(theta, dtype=o.DT)
    th = th.reshape(th.shape[0], -1) if th.dim() > 1 else th.reshape(1, -1)
    val = torch.empty(th.shape[0], dtype=o.DT)
    grad = torch.empty_like(th)
    for b in range(th.shape[0]):
        tb = th[b].clone().requires_grad_(True)
        lb = logl_point(tb, data, psd, dets, fgrid, df, nnode, gmst)
        (g,) = torch.autograd.grad(lb, tb)
        val[b] = lb.detach()
        grad[b] = g
    return val, grad
