"""Green-Kubo transport coefficients from the per-step stress tensor and heat
flux (Section 3.1): the shear viscosity

    eta = 1/(k_B T V) int_0^tau <S_xy(t) S_xy(0)> dt

from the stress tensor S of eq. (50) (energy units, not divided by V), and
the thermal conductivity

    lambda = V/(3 k_B T^2) int_0^tau <J(0) . J(t)> dt

from the heat flux J of eq. (51).  Both integrals are cut at a finite lag
tau, the plateau the limit in the paper stands for; the running integral is
returned so the plateau can be judged.  Host-side analysis of a recorded
series (``rbsog_step`` fills ``stress`` and ``heat_flux`` of the energy
record): numpy only, no device work.

Units follow the library: S in eV, J in eV / (A^2 ps), time in ps, V in A^3,
T in K.  eta is returned in Pa s and lambda in W / (m K).
"""
from __future__ import annotations

import numpy as np

K_B = 8.617333262e-5  # eV / K
EV = 1.602176634e-19  # J
# eV ps / A^3 -> Pa s, and eV / (A ps K) -> W / (m K)
PA_S_PER_EV_PS_A3 = EV / 1e-30 * 1e-12
W_MK_PER_EV_A_PS_K = EV / (1e-10 * 1e-12)

_OFF_DIAG = {"xy": 3, "xz": 4, "yz": 5}  # positions in (xx, yy, zz, xy, xz, yz)


def autocorrelation(x: np.ndarray, n_lag: int) -> np.ndarray:
    """<x(0) . x(t)> for t = 0 .. n_lag-1 samples, averaged over every time
    origin, the components of a [T, d] series summed.  Computed through a
    zero-padded FFT (the same sums as the direct double loop)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    n = x.shape[0]
    if not 1 <= n_lag <= n:
        raise ValueError("need 1 <= n_lag <= number of samples")
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(x, m, axis=0)
    acf = np.fft.irfft(f * np.conj(f), m, axis=0)[:n_lag].sum(axis=1)
    return acf / (n - np.arange(n_lag))


def _running_integral(acf: np.ndarray, dt: float) -> np.ndarray:
    """Trapezoid rule from lag 0: entry k integrates over [0, k dt]."""
    out = np.zeros_like(acf)
    if len(acf) > 1:
        out[1:] = np.cumsum(0.5 * (acf[1:] + acf[:-1])) * dt
    return out


def viscosity(stress: np.ndarray, dt: float, volume: float, temperature: float, n_lag: int,
              components=("xy",)):
    """Shear viscosity from a [T, 6] series of S (xx, yy, zz, xy, xz, yz) sampled
    every dt ps.  components: the off-diagonal elements whose
    autocorrelations are averaged (the paper uses xy; all three of an
    isotropic fluid estimate the same eta).  Returns (eta in Pa s at the
    cut n_lag, running integral in Pa s for lags 0 .. n_lag-1)."""
    stress = np.asarray(stress, dtype=np.float64)
    if stress.ndim != 2 or stress.shape[1] != 6:
        raise ValueError("stress must be a [T, 6] series")
    acf = np.mean([autocorrelation(stress[:, _OFF_DIAG[c]], n_lag) for c in components], axis=0)
    run = _running_integral(acf, dt) / (K_B * temperature * volume) * PA_S_PER_EV_PS_A3
    return float(run[-1]), run


def thermal_conductivity(heat_flux: np.ndarray, dt: float, volume: float, temperature: float, n_lag: int):
    """Thermal conductivity from a [T, 3] series of J sampled every dt ps.
    Returns (lambda in W / (m K) at the cut n_lag, running integral)."""
    heat_flux = np.asarray(heat_flux, dtype=np.float64)
    if heat_flux.ndim != 2 or heat_flux.shape[1] != 3:
        raise ValueError("heat_flux must be a [T, 3] series")
    acf = autocorrelation(heat_flux, n_lag)
    run = _running_integral(acf, dt) * volume / (3.0 * K_B * temperature ** 2) * W_MK_PER_EV_A_PS_K
    return float(run[-1]), run
