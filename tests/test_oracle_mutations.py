"""Planted mistakes in the oracle must be caught by its pins.

Each case patches one oracle function with a plausible error (a dropped or
mistyped term, a wrong sign, a wrong exponent or factor) and checks that at
least one pin in test_oracle_pins fails. The mistakes live only in this CPU
test; nothing here touches the GPU.
"""
import math

import pytest
import torch

from oracle import gw_oracle as o
from tests import test_oracle_pins as pins


def _wrap_pn(index, fn):
    orig = o.pn_coefficients

    def bad(mc, q, chi1, chi2, v):
        eta, mt, phis = orig(mc, q, chi1, chi2, v)
        phis = list(phis)
        phis[index] = fn(phis[index], eta, chi1, chi2)
        return eta, mt, tuple(phis)
    return bad


def _phase_tc_sign():
    orig = o.phase

    def bad(f, theta):
        return orig(f, theta) - 4.0 * math.pi * f * theta[10]
    return bad


def _amp_power():
    def bad(theta):
        mc_s = o.T_SUN * theta[0]
        return math.sqrt(5.0 / 24.0) * math.pi ** (-2.0 / 3.0) * mc_s ** (5.0 / 3.0) * o.C_SI / (theta[4] * o.MPC_SI)
    return bad


def _pol(kind):
    def bad(f, theta):
        amp = o.amplitude(theta) * f ** (-7.0 / 6.0 if kind != "fexp" else -7.0 / 3.0)
        ci = torch.cos(theta[7])
        carrier = torch.exp(-1j * o.phase(f, theta))
        fplus = 0.5 * (1.0 + ci ** 2) if kind != "plusfactor" else (1.0 + ci ** 2)
        fcross = ci if kind != "nocos" else torch.ones_like(ci)
        return (amp * fplus).to(o.CDT) * carrier, -1j * (amp * fcross).to(o.CDT) * carrier
    return bad


def _antenna_cross_antisym():
    def bad(det_tensor, ra, dec, psi, gmst=0.0):
        _, x, y = o.source_frame(ra, dec, psi, gmst)
        e_plus = torch.outer(x, x) - torch.outer(y, y)
        e_cross = torch.outer(x, y) - torch.outer(y, x)
        return (det_tensor * e_plus).sum(), (det_tensor * e_cross).sum()
    return bad


def _delay_sign():
    orig = o.time_delay
    return lambda r, ra, dec, gmst=0.0: -orig(r, ra, dec, gmst)


def _inner_factor():
    return lambda a, b, psd, df: 2.0 * df * torch.sum(torch.real(torch.conj(a) * b) / psd)


def _logl_half():
    def bad(theta, data, psd, dets, fgrid, df, gmst=0.0):
        total = torch.zeros((), dtype=o.DT)
        for i in range(len(dets)):
            h = o.detector_strain(fgrid, theta, tuple(float(v) for v in dets[i]), gmst)
            total = total + o.inner(data[i], h, psd[i], df) - o.inner(h, h, psd[i], df)
        return total
    return bad


def _strain_delay_exponent_sign():
    def bad(f, theta, det, gmst=0.0):
        r, d = o.detector_geometry(*det)
        fp, fx = o.antenna(d, theta[5], theta[6], theta[8], gmst)
        dt = o.time_delay(r, theta[5], theta[6], gmst)
        hp, hc = o.polarizations(f, theta)
        return (fp * hp + fx * hc) * torch.exp(2j * math.pi * f * dt)
    return bad


def _strain_delay_ignores_gmst():
    def bad(f, theta, det, gmst=0.0):
        r, d = o.detector_geometry(*det)
        fp, fx = o.antenna(d, theta[5], theta[6], theta[8], gmst)
        dt = o.time_delay(r, theta[5], theta[6])
        hp, hc = o.polarizations(f, theta)
        return (fp * hp + fx * hc) * torch.exp(-2j * math.pi * f * dt)
    return bad


def _gmst_sign():
    orig = o.source_frame
    return lambda ra, dec, psi, gmst=0.0: orig(ra, dec, psi, -gmst)


def _inner_drops_last_bin():
    return lambda a, b, psd, df: 4.0 * df * torch.sum((torch.real(torch.conj(a) * b) / psd)[..., :-1])


def _isco_orbital_not_gw():
    orig = o.isco_frequency
    return lambda theta: 0.5 * orig(theta)


MUTATIONS = [
    ("phi2 mistyped", "pn_coefficients", lambda: _wrap_pn(1, lambda p, e, a, b: p + 0.01),
     [lambda: pins.test_phase_derivative_matches_2pn_time_frequency_relation(0.0, 0.0)]),
    ("phi3 beta sign", "pn_coefficients", lambda: _wrap_pn(2, lambda p, e, a, b: -p - 32.0 * math.pi),
     [lambda: pins.test_phase_derivative_matches_2pn_time_frequency_relation(0.7, -0.4)]),
    ("phi4 sigma sign", "pn_coefficients",
     lambda: _wrap_pn(3, lambda p, e, a, b: p + 20.0 * (e / 48.0) * 474.0 * a * b),
     [lambda: pins.test_phase_derivative_matches_2pn_time_frequency_relation(-0.85, 0.9)]),
    ("phi4 dropped", "pn_coefficients", lambda: _wrap_pn(3, lambda p, e, a, b: 0.0 * p),
     [lambda: pins.test_phase_derivative_matches_2pn_time_frequency_relation(0.0, 0.0)]),
    ("phi5 eta term mistyped", "pn_coefficients",
     lambda: _wrap_pn(4, lambda p, e, a, b: p * (38645.0 / 756.0 - 56.0 * e / 9.0) / (38645.0 / 756.0 - 65.0 * e / 9.0)),
     [lambda: pins.test_phase_coefficients_follow_from_pn_energy_and_flux(0.5)]),
    ("phi6 gamma_E term dropped", "pn_coefficients",
     lambda: _wrap_pn(5, lambda p, e, a, b: p + 6848.0 * 0.5772156649015329 / 21.0),
     [lambda: pins.test_phase_coefficients_follow_from_pn_energy_and_flux(1.0)]),
    ("phi6 eta^3 sign", "pn_coefficients",
     lambda: _wrap_pn(5, lambda p, e, a, b: p + 2.0 * 127825.0 * e ** 3 / 1296.0),
     [lambda: pins.test_phase_coefficients_follow_from_pn_energy_and_flux(1.0)]),
    ("phi7 eta^2 sign", "pn_coefficients",
     lambda: _wrap_pn(6, lambda p, e, a, b: p + 2.0 * math.pi * 74045.0 * e ** 2 / 756.0),
     [lambda: pins.test_phase_coefficients_follow_from_pn_energy_and_flux(0.2)]),
    ("tc sign", "phase", _phase_tc_sign, [pins.test_phase_constant_terms]),
    ("amplitude mass power", "amplitude", _amp_power, [pins.test_amplitude_matches_spa_of_quadrupole_chirp]),
    ("amplitude f exponent", "polarizations", lambda: _pol("fexp"), [pins.test_flat_psd_hurwitz_zeta_closed_form]),
    ("plus factor 1/2 dropped", "polarizations", lambda: _pol("plusfactor"),
     [pins.test_amplitude_matches_spa_of_quadrupole_chirp]),
    ("cross cos(iota) dropped", "polarizations", lambda: _pol("nocos"),
     [pins.test_sky_and_orientation_average_is_4_over_25, pins.test_quadrupole_radiation_pattern_edge_on]),
    ("cross polarisation tensor antisymmetric", "antenna", _antenna_cross_antisym,
     [pins.test_antenna_detector_frame_closed_form_and_bound]),
    ("time delay sign", "time_delay", _delay_sign, [pins.test_time_delay_special_cases]),
    ("inner product factor", "inner", _inner_factor, [pins.test_eq2_exponent_ratio]),
    ("missing 1/2 on <h|h>", "logl_point", _logl_half, [pins.test_eq2_exponent_ratio]),
    ("detector delay exponent sign", "detector_strain", _strain_delay_exponent_sign,
     [pins.test_detector_delay_is_a_time_shift_of_the_geocentre_signal]),
    ("detector delay at GMST 0", "detector_strain", _strain_delay_ignores_gmst,
     [pins.test_sidereal_angle_turns_the_sky_with_the_earth]),
    ("GMST sign", "source_frame", _gmst_sign, [pins.test_sidereal_angle_turns_the_sky_with_the_earth]),
    ("inner product drops the last bin", "inner", _inner_drops_last_bin,
     [pins.test_discrete_likelihood_converges_to_the_frequency_integral]),
    ("ISCO at the orbital frequency", "isco_frequency", _isco_orbital_not_gw,
     [pins.test_isco_frequency_is_twice_the_kepler_frequency_at_6m]),
]


@pytest.mark.parametrize("name,attr,make,catchers", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, attr, make, catchers):
    monkeypatch.setattr(o, attr, make())
    caught = False
    for c in catchers:
        try:
            c()
        except AssertionError:
            caught = True
            break
    assert caught, f"planted mistake '{name}' passed every pin"
