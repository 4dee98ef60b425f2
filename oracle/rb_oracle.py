"""Relative binning of <d|h>: a plain FP64 reference.

TEST INFRASTRUCTURE ONLY. Only tests/, the package's smoke check and bench.py's CPU leg may
import this module; the library never does.

The paper's section 5 names relative binning as the next multiplier: the data are compressed
into summary data against a fiducial waveform h0, and a waveform h close to h0 is then needed
only on a sparse set of frequencies, because the ratio h/h0 varies slowly. The paper gives no
formulas; the readings taken here (each one pinned in tests/test_rb_oracle.py):

  RB1  Edges. With the power laws of the post-Newtonian phase, gamma in {-5/3, -2/3, 1, 5/3, 7/3},
       the largest phase difference a waveform in the prior can have from h0 grows like
       dpsi(f) = 2 pi sum_gamma sign(gamma) (f / f_gamma)^gamma, f_gamma = f_hi for gamma > 0 and
       f_lo for gamma < 0 (dpsi increases with f). The edges are the grid frequencies at which
       floor(dpsi / eps) changes, plus both ends of the grid.
  RB2  Between two adjacent edges the ratio r(f) = h(f) / h0(f) is replaced by its linear
       interpolant, i.e. r(f) = sum_e r(f_e) hat_e(f) with hat_e the piecewise-linear "hat"
       function of edge e (1 at f_e, 0 at the neighbouring edges).
  RB3  Summary data per detector and edge: V_e = 4 df sum_k conj(d_k) h0_k hat_e(f_k) / S_k, so
       that <d|h>_RB = Re sum_e V_e r(f_e).
  RB4  <h|h> is not binned: it is evaluated over every bin, as in the full likelihood. (For the
       Newtonian-amplitude model it is a per-point constant times a fixed spectral sum, so
       binning it would only add error.)

logL_RB(theta) = sum_det [ <d|h>_RB - 1/2 <h|h> ].

Parity status: pinned (partition of unity at the fiducial, exactness when every bin is an edge,
second-order convergence in the edge spacing, the edge rule itself). With the calibration model:
pinned by reduction to the plain binned likelihood at zero calibration and to the calibrated
full likelihood when every bin is an edge.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle import cal_oracle as co
from oracle import gw_oracle as o

GAMMAS = (-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0)


def phase_bound(f, f_lo, f_hi):
    """RB1's dpsi(f) (radians)."""
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    for g in GAMMAS:
        fg = f_hi if g > 0 else f_lo
        out += math.copysign(1.0, g) * (f / fg) ** g
    return 2.0 * math.pi * out


def edges(fgrid, eps):
    """Indices into fgrid of the edges (RB1), increasing, first and last bin included."""
    f = np.asarray(fgrid, dtype=np.float64)
    cell = np.floor(phase_bound(f, f[0], f[-1]) / eps)
    idx = [0]
    for k in range(1, len(f)):
        if cell[k] != cell[k - 1]:
            idx.append(k)
    if idx[-1] != len(f) - 1:
        idx.append(len(f) - 1)
    return np.array(idx, dtype=np.int64)


def hat_weights(fgrid, idx):
    """hat[e, k]: the piecewise-linear hat functions of the edges evaluated on the grid (RB2)."""
    f = np.asarray(fgrid, dtype=np.float64)
    fe = f[idx]
    w = np.zeros((len(idx), len(f)))
    for e in range(len(idx)):
        if e > 0:                                    # rising flank over (f_{e-1}, f_e]
            m = (f > fe[e - 1]) & (f <= fe[e])
            w[e, m] = (f[m] - fe[e - 1]) / (fe[e] - fe[e - 1])
        if e < len(idx) - 1:                         # falling flank over [f_e, f_{e+1})
            m = (f >= fe[e]) & (f < fe[e + 1])
            w[e, m] = (fe[e + 1] - f[m]) / (fe[e + 1] - fe[e])
        else:
            w[e, f >= fe[e]] = 1.0
    return w


def summary(data, psd, dets, fgrid, df, theta_fid, eps, gmst=0.0):
    """Edges, their frequencies, h0 at the edges and the summary data V[det, e] (RB3)."""
    f = np.asarray(fgrid, dtype=np.float64)
    idx = edges(f, eps)
    hat = hat_weights(f, idx)
    h0 = o.strain_all(theta_fid, dets, f, gmst).numpy()
    data = np.asarray(data)
    psd = np.asarray(psd)
    c = 4.0 * df * np.conj(data) * h0 / psd                 # [det, M]
    V = c @ hat.T                                           # [det, E]
    return {"idx": idx, "fe": f[idx], "h0e": h0[:, idx], "V": V, "eps": eps}


def logl_point(theta, summ, psd, dets, fgrid, df, gmst=0.0, nnode=0):
    """logL_RB for one point (torch, differentiable in theta). With nnode > 0 the model carries
    the calibration factor of cal_oracle (theta [11 + 2 nnode ndet], columns as there): the
    ratio at the edges becomes h_cal / h0 (the factor is smooth in f, so its product with h / h0
    is interpolated like h / h0 itself), and <h_cal|h_cal> is taken over every bin."""
    fe = torch.as_tensor(summ["fe"], dtype=o.DT)
    fgrid = torch.as_tensor(fgrid, dtype=o.DT)
    psd = torch.as_tensor(psd, dtype=o.DT)
    V = torch.as_tensor(summ["V"], dtype=o.CDT)
    h0e = torch.as_tensor(summ["h0e"], dtype=o.CDT)
    total = torch.zeros((), dtype=o.DT)
    for i in range(len(dets)):
        det = tuple(float(v) for v in dets[i])
        he = o.detector_strain(fe, theta[:11], det, gmst)
        h = o.detector_strain(fgrid, theta[:11], det, gmst)
        if nnode:
            base = 11 + 2 * nnode * i
            amp, ph = theta[base:base + nnode], theta[base + nnode:base + 2 * nnode]
            he = he * co.factor(fe, amp, ph)
            h = h * co.factor(fgrid, amp, ph)
        r = he / h0e[i]
        dh = torch.sum(torch.real(V[i] * r))
        total = total + dh - 0.5 * o.inner(h, h, psd[i], df)
    return total


def _rows(theta, nnode, ndet):
    return torch.as_tensor(theta, dtype=o.DT).reshape(-1, 11 + 2 * nnode * ndet)


def logl(theta, summ, psd, dets, fgrid, df, gmst=0.0, nnode=0):
    """logL_RB for every row of theta[B, 11 + 2 nnode ndet]; float64 tensor [B]."""
    th = _rows(theta, nnode, len(dets))
    out = torch.empty(th.shape[0], dtype=o.DT)
    with torch.no_grad():
        for b in range(th.shape[0]):
            out[b] = logl_point(th[b], summ, psd, dets, fgrid, df, gmst, nnode)
    return out


def logl_grad(theta, summ, psd, dets, fgrid, df, gmst=0.0, nnode=0):
    """(logL_RB[B], its gradient [B, 11 + 2 nnode ndet]) by reverse-mode autograd."""
    th = _rows(theta, nnode, len(dets))
    val = torch.empty(th.shape[0], dtype=o.DT)
    grad = torch.empty_like(th)
    for b in range(th.shape[0]):
        tb = th[b].clone().requires_grad_(True)
        lb = logl_point(tb, summ, psd, dets, fgrid, df, gmst, nnode)
        (g,) = torch.autograd.grad(lb, tb)
        val[b] = lb.detach()
        grad[b] = g
    return val, grad
