"""Force comparison bars shared by the GPU parity tests.

A force field is compared two ways: the relative RMS error
sqrt(sum |F - F_ref|^2 / sum |F_ref|^2) against the form's bar (1e-11 FP64,
1e-5 FP32-mixed), and the largest single-atom error max_i |F_i - F_ref,i|
against ATOM_FACTOR times that bar in units of the reference's RMS force
magnitude sqrt(mean_i |F_ref,i|^2), so one atom far off cannot hide inside a
norm that is small on average.
"""
from __future__ import annotations

import math

import numpy as np

ATOM_FACTOR = 10.0


def rel_rms(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return math.sqrt(float(((a - b) ** 2).sum()) / max(float((b ** 2).sum()), 1e-300))


def max_atom_rel(a, b) -> float:
    """max_i |a_i - b_i| / sqrt(mean_i |b_i|^2) over rows of [N][3] arrays."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 3)
    if len(b) == 0:
        return 0.0
    f_rms = math.sqrt(float((b ** 2).sum()) / len(b))
    return float(np.sqrt(((a - b) ** 2).sum(1)).max()) / max(f_rms, 1e-300)


def check_forces(a, b, tol: float, what: str = "") -> tuple:
    """Assert both bars; returns (relative RMS, largest atom error / F_rms)."""
    e = rel_rms(a, b)
    m = max_atom_rel(a, b)
    assert e <= tol, f"{what}: relative RMS {e:.3e} > {tol:.1e}"
    assert m <= ATOM_FACTOR * tol, f"{what}: atom error {m:.3e} F_rms > {ATOM_FACTOR * tol:.1e}"
    return e, m
