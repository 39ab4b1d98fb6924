"""Green-Kubo helpers (Section 3.1) on synthetic series whose answers are
known: the time-origin averaged autocorrelation against the direct double
sum, and the integrals of AR(1) series, whose autocorrelation s^2 a^k has
the trapezoid integral dt s^2 (1 + a) / (2 (1 - a)) over a long window."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2512_24970_amd import green_kubo as G


def _ar1(rng, n, a, sigma, d):
    x = np.empty((n, d))
    x[0] = rng.normal(0.0, sigma, d)
    e = rng.normal(0.0, sigma * np.sqrt(1.0 - a * a), (n, d))
    for t in range(1, n):
        x[t] = a * x[t - 1] + e[t]
    return x


def test_autocorrelation_is_the_origin_averaged_double_sum():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(37, 3))
    acf = G.autocorrelation(x, 12)
    for k in range(12):
        direct = sum(float(x[t] @ x[t + k]) for t in range(37 - k)) / (37 - k)
        assert acf[k] == pytest.approx(direct, rel=1e-12, abs=1e-12)


def test_viscosity_of_an_ar1_stress_series():
    """S_xy an AR(1) series (a = 0.5, s = 2 eV): eta = 1/(k_B T V) * 1.5 dt s^2,
    in Pa s through 1 eV ps / A^3 = 0.1602176634 Pa s."""
    rng = np.random.default_rng(11)
    n, a, sig, dt, V, T = 400_000, 0.5, 2.0, 0.002, 1.0e5, 1200.0
    s = np.zeros((n, 6))
    s[:, 3] = _ar1(rng, n, a, sig, 1)[:, 0]
    s[:, 0] = 50.0  # the diagonal plays no part
    eta, run = G.viscosity(s, dt, V, T, n_lag=60)
    expect = 0.5 * dt * sig ** 2 * (1 + a) / (1 - a) / (8.617333262e-5 * T * V) * 0.1602176634
    assert eta == pytest.approx(expect, rel=0.05)
    assert run[0] == 0.0 and len(run) == 60
    # the plateau: once a^k has died away the last lags add only sampling
    # noise (about s^2 / sqrt(n) per lag)
    assert abs(run[-1] - run[40]) < 0.05 * abs(run[-1])
    # three off-diagonal components estimate the same coefficient
    s[:, 4] = _ar1(rng, n, a, sig, 1)[:, 0]
    s[:, 5] = _ar1(rng, n, a, sig, 1)[:, 0]
    eta3, _ = G.viscosity(s, dt, V, T, n_lag=60, components=("xy", "xz", "yz"))
    assert eta3 == pytest.approx(expect, rel=0.03)


def test_thermal_conductivity_of_an_ar1_heat_flux():
    """J with three independent AR(1) components (a = 0.8): <J(0).J(t)> =
    3 s^2 a^k, so lambda = V/(3 k_B T^2) * 3 * dt s^2 (1 + a)/(2 (1 - a)), in
    W/(m K) through 1 eV/(A ps K) = 1602.176634 W/(m K)."""
    rng = np.random.default_rng(12)
    n, a, sig, dt, V, T = 300_000, 0.8, 0.03, 0.001, 3.2e7, 1100.0
    J = _ar1(rng, n, a, sig, 3)
    lam, run = G.thermal_conductivity(J, dt, V, T, n_lag=120)
    expect = V / (3 * 8.617333262e-5 * T ** 2) * 3 * 0.5 * dt * sig ** 2 * (1 + a) / (1 - a) * 1602.176634
    assert lam == pytest.approx(expect, rel=0.05)
    assert np.all(np.diff(run[:10]) > 0)


def test_green_kubo_shapes_checked():
    with pytest.raises(ValueError):
        G.viscosity(np.zeros((10, 3)), 0.001, 1.0, 300.0, 5)
    with pytest.raises(ValueError):
        G.thermal_conductivity(np.zeros((10, 6)), 0.001, 1.0, 300.0, 5)
    with pytest.raises(ValueError):
        G.autocorrelation(np.zeros(10), 11)
