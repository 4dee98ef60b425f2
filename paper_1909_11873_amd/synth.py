"""Seeded synthetic inputs for the batched GW log-likelihood workloads.

This module draws inputs only: frequency grids, the analytic PSD fit, coloured
Gaussian noise, detector sites and parameter batches from the prior. It holds
none of the likelihood's arithmetic (no waveform, projection or inner
product), so the FP64 oracle and the HIP path can both consume what it makes
without sharing any of the computation under test. Signal injections are added
by the caller: the tests inject with the oracle's waveform, the benchmark with
the library's own waveform entry point.

Workloads (paper section 2, Eq. 2 and section 4.1 give the structure: a few
detectors, seconds-long segments, 20 Hz to ~2 kHz, Gaussian stationary noise
coloured by a PSD; the numbers below fix the synthetic stand-ins):

  c0  1 detector,   4 s, df=1/4 Hz,   20-1024 Hz  (4017 bins),   B=1000, no spins
  c1  3 detectors,  8 s, df=1/8 Hz,   20-2048 Hz  (16225 bins),  B=65536
  c2  3 detectors, 128 s, df=1/128 Hz, 20-2048 Hz (259585 bins), B=4096, Mc in [1, 1.5]
  c3  c1 shapes, B=16384 (gradient workload)
  c4  64 events, durations log-uniform in [4, 128] s (integer), B_e uniform in [256, 8192]
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

NPARAM = 11
PARAM_NAMES = ("mc", "q", "chi1", "chi2", "dl", "ra", "dec", "iota", "psi", "phic", "tc")

# Synthetic L-shaped detectors: (latitude, longitude, x-arm azimuth, y-arm azimuth) in degrees,
# azimuths clockwise from local North. Placed near the Hanford, Livingston and Virgo sites with
# made-up arm orientations; each is right-handed (x cross y points up).
DETECTORS_DEG = {
    "D1": (46.5, -119.4, 126.0, 36.0),
    "D2": (30.6, -90.8, 198.0, 108.0),
    "D3": (43.6, 10.5, 71.0, 341.0),
}


def detector_rad(name: str) -> Tuple[float, float, float, float]:
    return tuple(math.radians(v) for v in DETECTORS_DEG[name])


def psd_fit(f: np.ndarray) -> np.ndarray:
    """Analytic one-sided noise PSD fit S(f) in 1/Hz, x = f / 215 Hz."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    return 1e-49 * (x ** -4.14 - 5.0 * x ** -2 + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))


def freq_grid(f_lo: float, f_hi: float, df: float) -> np.ndarray:
    """f_k = f_lo + k df, both band edges included."""
    m = int(round((f_hi - f_lo) / df)) + 1
    return f_lo + df * np.arange(m, dtype=np.float64)


def prior_draw(rng: np.random.Generator, n: int, mc_range=(10.0, 60.0), spins=True,
               dl_range=(100.0, 2000.0), tc_half=0.1) -> np.ndarray:
    """n x 11 prior draws by inverse CDF from one block of uniforms (columns in PARAM_NAMES order)."""
    u = rng.random((n, NPARAM))
    th = np.empty((n, NPARAM), dtype=np.float64)
    th[:, 0] = mc_range[0] + (mc_range[1] - mc_range[0]) * u[:, 0]
    th[:, 1] = 0.2 + 0.8 * u[:, 1]
    if spins:
        th[:, 2] = -0.9 + 1.8 * u[:, 2]
        th[:, 3] = -0.9 + 1.8 * u[:, 3]
    else:
        th[:, 2] = 0.0
        th[:, 3] = 0.0
    lo3, hi3 = dl_range[0] ** 3, dl_range[1] ** 3
    th[:, 4] = np.cbrt(lo3 + u[:, 4] * (hi3 - lo3))
    th[:, 5] = 2.0 * math.pi * u[:, 5]
    th[:, 6] = np.arcsin(2.0 * u[:, 6] - 1.0)
    th[:, 7] = np.arccos(2.0 * u[:, 7] - 1.0)
    th[:, 8] = math.pi * u[:, 8]
    th[:, 9] = 2.0 * math.pi * u[:, 9]
    th[:, 10] = -tc_half + 2.0 * tc_half * u[:, 10]
    return th


def noise(seed: int, psd: np.ndarray, df: float) -> np.ndarray:
    """Complex Gaussian noise with Re, Im ~ N(0, S/(4 df)) independently per bin."""
    rng = np.random.default_rng(seed)
    sig = np.sqrt(psd / (4.0 * df))
    re = rng.standard_normal(psd.shape[0])
    im = rng.standard_normal(psd.shape[0])
    return sig * (re + 1j * im)


THETA0_BBH = np.array([30.0, 0.8, 0.0, 0.0, 400.0, 2.0, -0.5, 0.6, 1.0, 0.7, 0.0])
THETA0_BNS = np.array([1.2, 0.8, 0.0, 0.0, 100.0, 2.0, -0.5, 0.6, 1.0, 0.7, 0.0])


@dataclasses.dataclass
class EventSpec:
    """One event: detectors, grid, PSD, noise and a batch of parameter points."""
    name: str
    det_names: List[str]
    f_lo: float
    f_hi: float
    duration: float
    batch: int
    mc_range: Tuple[float, float]
    spins: bool
    theta0: np.ndarray
    seed_base: int

    @property
    def df(self) -> float:
        return 1.0 / self.duration

    @property
    def ndet(self) -> int:
        return len(self.det_names)

    @property
    def nbins(self) -> int:
        return int(round((self.f_hi - self.f_lo) * self.duration)) + 1


def event_spec(cfg: int, event: int = 0, batch: int | None = None) -> EventSpec:
    """Specification of configuration cfg (0..4); for cfg 4, of event `event` (0..63)."""
    d3 = ["D1", "D2", "D3"]
    if cfg == 0:
        s = EventSpec("c0", ["D1"], 20.0, 1024.0, 4.0, 1000, (10.0, 60.0), False, THETA0_BBH.copy(), 0)
    elif cfg == 1:
        s = EventSpec("c1", d3, 20.0, 2048.0, 8.0, 65536, (10.0, 60.0), True, THETA0_BBH.copy(), 1000)
    elif cfg == 2:
        s = EventSpec("c2", d3, 20.0, 2048.0, 128.0, 4096, (1.0, 1.5), True, THETA0_BNS.copy(), 2000)
    elif cfg == 3:
        s = EventSpec("c3", d3, 20.0, 2048.0, 8.0, 16384, (10.0, 60.0), True, THETA0_BBH.copy(), 3000)
    elif cfg == 4:
        if not 0 <= event < 64:
            raise ValueError("config 4 has events 0..63")
        seed_base = 40000 + 100 * event
        rng = np.random.default_rng(seed_base + 30)
        dur = float(round(math.exp(rng.uniform(math.log(4.0), math.log(128.0)))))
        b_e = int(rng.integers(256, 8193))
        th0 = prior_draw(np.random.default_rng(seed_base + 20), 1)[0]
        s = EventSpec(f"c4e{event}", d3, 20.0, 2048.0, dur, b_e, (10.0, 60.0), True, th0, seed_base)
    else:
        raise ValueError("configurations are 0..4")
    if batch is not None:
        s.batch = int(batch)
    return s


def event_arrays(spec: EventSpec):
    """Return (fgrid[M], psd[ndet, M], noise[ndet, M] complex128, dets[ndet, 4] rad)."""
    f = freq_grid(spec.f_lo, spec.f_hi, spec.df)
    assert f.shape[0] == spec.nbins
    s = psd_fit(f)
    psd = np.stack([s] * spec.ndet)
    nz = np.stack([noise(spec.seed_base + i, s, spec.df) for i in range(spec.ndet)])
    dets = np.array([detector_rad(n) for n in spec.det_names], dtype=np.float64)
    return f, psd, nz, dets


def theta_batch(spec: EventSpec, n: int | None = None) -> np.ndarray:
    """The event's batch of prior draws (seed stream 10); the first n rows if n is given."""
    rng = np.random.default_rng(spec.seed_base + 10)
    th = prior_draw(rng, spec.batch, mc_range=spec.mc_range, spins=spec.spins)
    return th if n is None else th[:n]
