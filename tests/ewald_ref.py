"""Textbook Ewald summation for a periodic cubic/orthorhombic box (numpy).

Used by the CPU tests as an independent reference for the Coulomb energy and
forces: real-space erfc sum over image cells plus the reciprocal-space sum,
minus the self term, tinfoil boundary conditions.  Nothing here is shared
with the oracle or the GPU library.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc


def ewald(pos: np.ndarray, q: np.ndarray, box, k_e: float = 1.0, alpha: float | None = None,
          tol: float = 1e-14):
    pos = np.asarray(pos, float)
    q = np.asarray(q, float)
    L = np.asarray(box, float)
    V = float(np.prod(L))
    n = len(q)
    if alpha is None:
        alpha = 3.5 / L.min()
    # real space: images until erfc(alpha r) < tol
    rcut = math.sqrt(-math.log(tol)) / alpha + 1e-9
    nimg = [int(math.ceil(rcut / L[a])) for a in range(3)]
    E_real = 0.0
    F = np.zeros((n, 3))
    d0 = pos[:, None, :] - pos[None, :, :]
    two_a_sqpi = 2.0 * alpha / math.sqrt(math.pi)
    for ix in range(-nimg[0], nimg[0] + 1):
        for iy in range(-nimg[1], nimg[1] + 1):
            for iz in range(-nimg[2], nimg[2] + 1):
                shift = np.array([ix, iy, iz]) * L
                d = d0 + shift
                r = np.sqrt((d * d).sum(-1))
                if ix == 0 and iy == 0 and iz == 0:
                    np.fill_diagonal(r, np.inf)
                mask = r < rcut
                rr = np.where(mask, r, np.inf)
                qq = q[:, None] * q[None, :]
                e = np.where(mask, qq * erfc(alpha * rr) / rr, 0.0)
                E_real += 0.5 * e.sum()
                fmag = np.where(mask, qq * (erfc(alpha * rr) / rr ** 2 + two_a_sqpi * np.exp(-(alpha * rr) ** 2) / rr), 0.0)
                F += (fmag[:, :, None] * d / rr[:, :, None]).sum(1)
    # reciprocal space: exp(-k^2/(4 alpha^2)) < tol
    kmax = 2.0 * alpha * math.sqrt(-math.log(tol))
    nk = [int(math.floor(kmax * L[a] / (2 * math.pi))) for a in range(3)]
    mx, my, mz = np.meshgrid(*[np.arange(-nk[a], nk[a] + 1) for a in range(3)], indexing="ij")
    m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], 1)
    m = m[np.any(m != 0, axis=1)]
    k = 2 * math.pi * m / L
    k2 = (k * k).sum(1)
    keep = k2 <= kmax * kmax
    k, k2 = k[keep], k2[keep]
    coef = 4 * math.pi / V * np.exp(-k2 / (4 * alpha * alpha)) / k2
    E_rec = 0.0
    chunk = 4096
    for s in range(0, len(k), chunk):
        kk = k[s:s + chunk]
        th = pos @ kk.T  # (n, nk)
        c, sn = np.cos(th), np.sin(th)
        re = q @ c
        im = q @ sn
        cf = coef[s:s + chunk]
        E_rec += 0.5 * (cf * (re * re + im * im)).sum()
        # F_i = q_i sum_k coef k (sin th_i Re - cos th_i Im)
        g = (sn * re[None, :] - c * im[None, :]) * cf[None, :]
        F += q[:, None] * (g @ kk)
    E_self = -alpha / math.sqrt(math.pi) * (q * q).sum()
    E = E_real + E_rec + E_self
    return k_e * E, k_e * F
