"""FP64 CPU oracle for the frequency-domain compact-binary log-likelihood ratio.

TEST INFRASTRUCTURE ONLY. This module is the slow, plain reference that the
HIP library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and it
shares no code, constants or tables with the library.

What it computes (paper section 2, Eq. 2): the Gaussian-noise likelihood over
detectors i and frequency bins j. Eq. 2 is read as a product over bins of
independent complex Gaussians whose exponent is -(2/T)|d-h|^2/S. With df=1/T
that exponent is -(1/2) 4 df |d-h|^2 / S, so the log-likelihood ratio against
the no-signal hypothesis is

    logL(theta) = sum_i [ <d|h>_i - 1/2 <h|h>_i ],   <a|b> = 4 df Re sum_j conj(a_j) b_j / S_j.

The signal model is the one the synthetic workloads name (the paper names
none that is available here): a TaylorF2 inspiral with 3.5PN non-spinning
phase, aligned-spin terms at 1.5PN (beta) and 2PN (sigma), and Newtonian
amplitude, projected onto L-shaped detectors on a spherical Earth. The oracle
builds h_+ and h_x on every bin from the full phase formula, projects them,
and forms both inner products directly; it never uses the factored form the
GPU kernels use. The gradient is reverse-mode autograd through this same code.

Parameter order of theta[11]: chirp mass (Msun, detector frame), q = m2/m1 in
(0, 1], chi1, chi2 (aligned), luminosity distance (Mpc), right ascension,
declination, inclination, polarisation angle, coalescence phase (rad),
coalescence time (s, geocentre).

Parity status of each part (what pins it, in the tests):
  * Eq. 2 reading and 4df normalisation: pinned against Eq. 2's own exponent.
  * amplitude constant and f^(-7/6): pinned by the stationary-phase amplitude
    of the Newtonian quadrupole chirp and by the Hurwitz-zeta closed form of
    <h|h> under a flat PSD.
  * Newtonian, 1PN, 1.5PN (with beta) and 2PN (with sigma) phase terms: pinned
    by the published 2PN time-frequency relation t(f) through dPsi/df = 2 pi t(f).
  * every non-spinning phase coefficient, 2.5PN, 3PN and 3.5PN included: pinned
    by the stationary-phase integral of the PN energy balance (binding energy to
    3PN, gravitational-wave flux to 3.5PN with its logarithm), which gives the
    same series by an independent route. The spin terms beyond 2PN are absent.
  * antenna patterns: pinned by the detector-frame closed form of F+^2 + Fx^2,
    the polarisation-rotation law and the 4/25 sky/orientation average.
  * time delays: pinned by zenith, nadir and horizon special cases; the sign of
    the delay factor exp(-2 pi i f dt) by the time-shift theorem (the detector
    strain equals the geocentre strain of a source with t_c + dt).
  * the sidereal angle: pinned by the zenith delay at right ascension
    gmst + longitude and by logL(ra, gmst) = logL(ra - gmst, 0).
  * the sum over bins: pinned by its convergence to the continuous inner
    product (composite Gauss-Legendre quadrature) at first, then, with the
    Euler-Maclaurin end term, second order in df; the float64 rounding by a
    50-digit evaluation of the per-bin definition (agreement to ~1e-15).
  * the optional ISCO cut-off: its frequency pinned by Kepler's law at r = 6GM/c^2
    (twice the orbital frequency), the cut by evaluating on the grid truncated
    there.
  * the sign of i in h_x and of the phase exponent are conventions of this
    build (FT with exp(-2 pi i f t)); they are checked for internal consistency
    by the time-shift and phase invariances only.
"""
from __future__ import annotations

import math
from typing import Sequence

import torch

DT = torch.float64
CDT = torch.complex128

# Physical constants (SI), frozen for this library's conventions.
C_SI = 299792458.0                 # speed of light, m/s
T_SUN = 4.925490947641267e-6       # G Msun / c^3, s
MPC_SI = 3.0856775814913673e22     # megaparsec, m
R_EARTH = 6.371e6                  # spherical Earth radius, m
GAMMA_E = 0.5772156649015329       # Euler-Mascheroni constant


def _t(x):
    """Float64 tensor view of a number or tensor (keeps autograd history)."""
    return x.to(DT) if torch.is_tensor(x) else torch.tensor(x, dtype=DT)


# ----------------------------------------------------------------------------------------------
# Masses and the TaylorF2 phase
# ----------------------------------------------------------------------------------------------
def masses(mc, q):
    """Symmetric mass ratio, total mass and component masses (Msun) from chirp mass and q."""
    eta = q / (1.0 + q) ** 2
    mtot = mc * eta ** (-0.6)
    m1 = mtot / (1.0 + q)
    m2 = q * mtot / (1.0 + q)
    return eta, mtot, m1, m2


def pn_coefficients(mc, q, chi1, chi2, v):
    """phi_k of the TaylorF2 series, k = 0..7 (phi_5 and phi_6 carry their ln v dependence)."""
    eta, mtot, m1, m2 = masses(mc, q)
    pi = math.pi
    # spin-orbit (1.5PN) and spin-spin (2PN) combinations for spins along L
    beta = (113.0 / 12.0 * (m1 / mtot) ** 2 + 25.0 / 4.0 * eta) * chi1 + \
           (113.0 / 12.0 * (m2 / mtot) ** 2 + 25.0 / 4.0 * eta) * chi2
    sigma = (eta / 48.0) * (-247.0 * chi1 * chi2 + 721.0 * chi1 * chi2)
    phi0 = torch.ones_like(v)
    phi2 = 3715.0 / 756.0 + 55.0 * eta / 9.0
    phi3 = -16.0 * pi + 4.0 * beta
    phi4 = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta ** 2 / 72.0 - 10.0 * sigma
    phi5 = pi * (38645.0 / 756.0 - 65.0 * eta / 9.0) * (1.0 + 3.0 * torch.log(v))
    phi6 = (11583231236531.0 / 4694215680.0 - 640.0 * pi ** 2 / 3.0 - 6848.0 * GAMMA_E / 21.0
            - 6848.0 / 21.0 * torch.log(4.0 * v)
            + (-15737765635.0 / 3048192.0 + 2255.0 * pi ** 2 / 12.0) * eta
            + 76055.0 * eta ** 2 / 1728.0 - 127825.0 * eta ** 3 / 1296.0)
    phi7 = pi * (77096675.0 / 254016.0 + 378515.0 * eta / 1512.0 - 74045.0 * eta ** 2 / 756.0)
    return eta, mtot, (phi0, phi2, phi3, phi4, phi5, phi6, phi7)


def phase(f, theta):
    """Psi(f) in radians: 2 pi f tc - phic - pi/4 + 3/(128 eta v^5) sum_k phi_k v^k."""
    mc, q, chi1, chi2 = theta[0], theta[1], theta[2], theta[3]
    phic, tc = theta[9], theta[10]
    _, mtot, _, _ = masses(mc, q)
    v = (math.pi * T_SUN * mtot * f) ** (1.0 / 3.0)
    eta, _, (p0, p2, p3, p4, p5, p6, p7) = pn_coefficients(mc, q, chi1, chi2, v)
    series = p0 + p2 * v ** 2 + p3 * v ** 3 + p4 * v ** 4 + p5 * v ** 5 + p6 * v ** 6 + p7 * v ** 7
    return 2.0 * math.pi * f * tc - phic - math.pi / 4.0 + 3.0 / (128.0 * eta * v ** 5) * series


def amplitude(theta):
    """Newtonian Fourier amplitude prefactor A, |h~| = A f^(-7/6) for a face-on source (s^(-1/6) units)."""
    mc_s = T_SUN * theta[0]
    return math.sqrt(5.0 / 24.0) * math.pi ** (-2.0 / 3.0) * mc_s ** (5.0 / 6.0) * C_SI / (theta[4] * MPC_SI)


def polarizations(f, theta):
    """(h_+, h_x) complex128 on the grid f; h_+ = A f^-7/6 (1+cos^2 i)/2 e^{-i Psi}, h_x = -i A f^-7/6 cos i e^{-i Psi}."""
    amp = amplitude(theta) * f ** (-7.0 / 6.0)
    ci = torch.cos(theta[7])
    carrier = torch.exp(-1j * phase(f, theta))
    hp = (amp * 0.5 * (1.0 + ci ** 2)).to(CDT) * carrier
    hc = -1j * (amp * ci).to(CDT) * carrier
    return hp, hc


# ----------------------------------------------------------------------------------------------
# Detector geometry
# ----------------------------------------------------------------------------------------------
def detector_geometry(lat, lon, az_x, az_y):
    """Vertex position (m) and detector tensor D = (x x - y y)/2 of an L-shaped detector."""
    lat, lon, az_x, az_y = (_t(v) for v in (lat, lon, az_x, az_y))
    e_north = torch.stack([-torch.sin(lat) * torch.cos(lon), -torch.sin(lat) * torch.sin(lon), torch.cos(lat)])
    e_east = torch.stack([-torch.sin(lon), torch.cos(lon), torch.zeros((), dtype=DT)])
    r = R_EARTH * torch.stack([torch.cos(lat) * torch.cos(lon), torch.cos(lat) * torch.sin(lon), torch.sin(lat)])
    xa = torch.cos(az_x) * e_north + torch.sin(az_x) * e_east
    ya = torch.cos(az_y) * e_north + torch.sin(az_y) * e_east
    d = 0.5 * (torch.outer(xa, xa) - torch.outer(ya, ya))
    return r, d


def source_frame(ra, dec, psi, gmst=0.0):
    """Direction to the source k and the polarisation axes X, Y (X x Y = -k, the propagation direction)."""
    ra, dec, psi = _t(ra), _t(dec), _t(psi)
    h = ra - gmst
    k = torch.stack([torch.cos(dec) * torch.cos(h), torch.cos(dec) * torch.sin(h), torch.sin(dec)])
    u = torch.stack([-torch.sin(dec) * torch.cos(h), -torch.sin(dec) * torch.sin(h), torch.cos(dec)])
    v = torch.stack([-torch.sin(h), torch.cos(h), torch.zeros((), dtype=DT)])
    x = torch.cos(psi) * u + torch.sin(psi) * v
    y = -torch.sin(psi) * u + torch.cos(psi) * v
    return k, x, y


def antenna(det_tensor, ra, dec, psi, gmst=0.0):
    """(F_+, F_x) = (D : e_+, D : e_x) with e_+ = XX - YY, e_x = XY + YX."""
    _, x, y = source_frame(ra, dec, psi, gmst)
    e_plus = torch.outer(x, x) - torch.outer(y, y)
    e_cross = torch.outer(x, y) + torch.outer(y, x)
    return (det_tensor * e_plus).sum(), (det_tensor * e_cross).sum()


def time_delay(r_det, ra, dec, gmst=0.0):
    """Arrival time at the detector minus arrival time at the geocentre: -(r . k) / c."""
    k, _, _ = source_frame(ra, dec, 0.0, gmst)
    return -(r_det * k).sum() / C_SI


def detector_strain(f, theta, det, gmst=0.0):
    """h~ seen by one detector: (F_+ h_+ + F_x h_x) exp(-2 pi i f dt)."""
    r, d = detector_geometry(*det)
    fp, fx = antenna(d, theta[5], theta[6], theta[8], gmst)
    dt = time_delay(r, theta[5], theta[6], gmst)
    hp, hc = polarizations(f, theta)
    return (fp * hp + fx * hc) * torch.exp(-2j * math.pi * f * dt)


# ----------------------------------------------------------------------------------------------
# Inner products and the likelihood ratio
# ----------------------------------------------------------------------------------------------
def inner(a, b, psd, df):
    """<a|b> = 4 df Re sum conj(a) b / S."""
    return 4.0 * df * torch.sum(torch.real(torch.conj(a) * b) / psd)


def isco_frequency(theta):
    """Gravitational-wave frequency at the innermost stable circular orbit of a Schwarzschild
    black hole of the binary's total mass: twice the orbital frequency at r = 6 G M / c^2,
    f = c^3 / (6^(3/2) pi G M)."""
    _, mtot, _, _ = masses(theta[0], theta[1])
    return 1.0 / (6.0 ** 1.5 * math.pi * T_SUN * mtot)


def logl_point(theta, data, psd, dets, fgrid, df, gmst=0.0, isco=False):
    """logL for one parameter point; data[ndet, M] complex128, psd[ndet, M], dets[ndet] x 4.
    With isco the model is zero above the ISCO frequency (both inner products lose those bins)."""
    total = torch.zeros((), dtype=DT)
    keep = fgrid <= isco_frequency(theta) if isco else None
    for i in range(len(dets)):
        h = detector_strain(fgrid, theta, tuple(float(v) for v in dets[i]), gmst)
        if keep is not None:
            h = torch.where(keep, h, torch.zeros_like(h))
        total = total + inner(data[i], h, psd[i], df) - 0.5 * inner(h, h, psd[i], df)
    return total


def _as_inputs(data, psd, fgrid):
    data = torch.as_tensor(data).to(CDT)
    psd = torch.as_tensor(psd).to(DT)
    fgrid = torch.as_tensor(fgrid).to(DT)
    return data, psd, fgrid


def logl(theta, data, psd, dets, fgrid, df, gmst=0.0, isco=False):
    """logL for every row of theta[B, 11] (float64 numpy or tensor); returns float64 tensor [B]."""
    data, psd, fgrid = _as_inputs(data, psd, fgrid)
    th = torch.as_tensor(theta, dtype=DT).reshape(-1, 11)
    out = torch.empty(th.shape[0], dtype=DT)
    with torch.no_grad():
        for b in range(th.shape[0]):
            out[b] = logl_point(th[b], data, psd, dets, fgrid, df, gmst, isco)
    return out


def logl_grad(theta, data, psd, dets, fgrid, df, gmst=0.0, isco=False):
    """(logL[B], dlogL/dtheta[B, 11]) by reverse-mode autograd through logl_point (with isco the
    cut is a step in theta: its derivative is that of the model on the bins kept)."""
    data, psd, fgrid = _as_inputs(data, psd, fgrid)
    th = torch.as_tensor(theta, dtype=DT).reshape(-1, 11)
    val = torch.empty(th.shape[0], dtype=DT)
    grad = torch.empty(th.shape[0], 11, dtype=DT)
    for b in range(th.shape[0]):
        tb = th[b].clone().requires_grad_(True)
        lb = logl_point(tb, data, psd, dets, fgrid, df, gmst, isco)
        (g,) = torch.autograd.grad(lb, tb)
        val[b] = lb.detach()
        grad[b] = g
    return val, grad


def strain_all(theta, dets: Sequence, fgrid, gmst=0.0):
    """h~ for one point on every detector: complex128 [ndet, M] (used to build injections)."""
    fgrid = torch.as_tensor(fgrid).to(DT)
    th = torch.as_tensor(theta, dtype=DT)
    with torch.no_grad():
        return torch.stack([detector_strain(fgrid, th, tuple(float(v) for v in d), gmst) for d in dets])
