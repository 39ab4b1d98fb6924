"""Seeded synthetic inputs: BMH parameter tables, rock-salt melts, velocities.

This module builds inputs only.  It holds none of the method's arithmetic and
is the one piece of code that the GPU library's tests and the CPU oracle
both use.  Every system is synthetic: a rock-salt lattice with seeded uniform
jitter and Maxwell-Boltzmann velocities, standing in for the paper's
NPT-equilibrated melts (Section 3), which are not available.

Parameter tables are the paper's: Table 1 (Tosi-Fumi NaCl) and Table 3
(LiCl-NaCl).  Masses are standard atomic weights (the paper gives none).
"""
from __future__ import annotations

import math

import numpy as np

# Coulomb constant e^2/(4 pi eps0) in eV*Angstrom (CODATA 2018).
COULOMB_K = 14.399645478425668
# Boltzmann constant in eV/K.
KB = 8.617333262e-5
# 1 eV/(Angstrom*amu) in Angstrom/ps^2.
ACC_UNIT = 9648.533212331

MASS = {"Li": 6.941, "Na": 22.98977, "K": 39.0983, "Cl": 35.453}

# Table 1: Tosi-Fumi parameters for molten NaCl (A eV, sigma A, C eV A^6, D eV A^8, rho A).
TABLE1 = {
    ("Na", "Na"): dict(A=0.303, sigma=2.340, C=1.049, D=0.499, rho=0.317),
    ("Na", "Cl"): dict(A=0.242, sigma=2.755, C=6.991, D=8.676, rho=0.317),
    ("Cl", "Cl"): dict(A=0.182, sigma=3.170, C=72.40, D=145.427, rho=0.317),
}

# Table 3: LiCl-NaCl parameters.
TABLE3 = {
    ("Li", "Li"): dict(A=0.4225, sigma=1.632, C=0.045625, D=0.01875, rho=0.3170),
    ("Li", "Na"): dict(A=0.334, sigma=1.986, C=0.218875, D=0.0968, rho=0.3185),
    ("Na", "Na"): dict(A=0.2640625, sigma=2.340, C=1.05, D=0.50, rho=0.3200),
    ("Li", "Cl"): dict(A=0.29046875, sigma=2.401, C=1.25, D=1.50, rho=0.3215),
    ("Na", "Cl"): dict(A=0.21125, sigma=2.755, C=7.00, D=8.6875, rho=0.3230),
    ("Cl", "Cl"): dict(A=0.1584375, sigma=3.170, C=71.328, D=143.281, rho=0.3261),
}

CHARGE = {"Li": 1.0, "Na": 1.0, "K": 1.0, "Cl": -1.0}


def species_block(names, table, element_of=None) -> dict:
    """Per-species charges and masses and per-pair BMH parameters for the
    species `names` (element_of maps a species name to the element whose
    parameters it uses, for duplicate slots)."""
    element_of = element_of or {n: n for n in names}
    S = len(names)
    out = {"names": list(names), "q": [], "mass": [], "A": [], "sigma": [], "rho": [], "C": [], "D": []}
    for a in names:
        ea = element_of[a]
        out["q"].append(CHARGE[ea])
        out["mass"].append(MASS[ea])
    for key in ("A", "sigma", "rho", "C", "D"):
        rows = []
        for a in names:
            row = []
            for b in names:
                ea, eb = element_of[a], element_of[b]
                e = table.get((ea, eb)) or table.get((eb, ea))
                row.append(float(e[key]))
            rows.append(row)
        out[key] = rows
    assert len(out["q"]) == S
    return out


def rocksalt(n_atoms: int, box: float, rng: np.random.Generator, jitter: float = 0.3):
    """Rock-salt sites on an n^3 grid (n the smallest even n with n^3 >= N),
    spacing box/n, cation where i+j+k is even.  When n^3 > N, N/2 sites of each
    parity are chosen at random.  Returns positions (wrapped to [0, box)) and a
    cation mask."""
    if n_atoms % 2:
        raise ValueError("rock-salt melts need an even atom count")
    n = 2
    while n ** 3 < n_atoms:
        n += 2
    a = box / n
    idx = np.arange(n ** 3, dtype=np.int64)
    i, j, k = idx // (n * n), (idx // n) % n, idx % n
    even = ((i + j + k) % 2) == 0
    half = n_atoms // 2
    cat_sites = idx[even]
    an_sites = idx[~even]
    if len(cat_sites) > half:
        cat_sites = np.sort(rng.choice(cat_sites, size=half, replace=False))
        an_sites = np.sort(rng.choice(an_sites, size=half, replace=False))
    sites = np.concatenate([cat_sites, an_sites])
    cation = np.concatenate([np.ones(half, bool), np.zeros(half, bool)])
    order = rng.permutation(len(sites))
    sites, cation = sites[order], cation[order]
    si, sj, sk = sites // (n * n), (sites // n) % n, sites % n
    pos = np.stack([(si + 0.5) * a, (sj + 0.5) * a, (sk + 0.5) * a], axis=1)
    pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    pos = np.mod(pos, box)
    pos[pos >= box] -= box
    return pos, cation


def maxwell_boltzmann(masses: np.ndarray, T: float, rng: np.random.Generator) -> np.ndarray:
    """Velocities (Angstrom/ps) at temperature T: Gaussian components, zero
    total momentum, rescaled to T exactly with 3N-3 degrees of freedom."""
    n = len(masses)
    sd = np.sqrt(KB * T * ACC_UNIT / masses)
    v = rng.normal(size=(n, 3)) * sd[:, None]
    if n > 1:
        p = (masses[:, None] * v).sum(axis=0) / masses.sum()
        v -= p
        ke = 0.5 * (masses[:, None] * v * v).sum() / ACC_UNIT
        t_now = 2.0 * ke / ((3 * n - 3) * KB)
        if t_now > 0:
            v *= math.sqrt(T / t_now)
    return v


def _melt(n_atoms, box, T, species, cation_types, cation_frac, seed, jitter=0.3):
    rng = np.random.default_rng(seed)
    pos, cation = rocksalt(n_atoms, box, rng, jitter)
    types = np.zeros(n_atoms, dtype=np.int32)
    anion_type = [i for i, q in enumerate(species["q"]) if q < 0][0]
    types[~cation] = anion_type
    ci = np.flatnonzero(cation)
    if len(cation_types) == 1:
        types[ci] = cation_types[0]
    else:
        u = rng.permutation(len(ci))
        bounds = np.floor(np.cumsum(cation_frac) * len(ci) + 0.5).astype(np.int64)
        start = 0
        for t, end in zip(cation_types, bounds):
            types[ci[u[start:end]]] = t
            start = end
    masses = np.array(species["mass"])[types]
    vel = maxwell_boltzmann(masses, T, rng)
    return types, pos, vel


BASE_SEED = 2512249700


def config(name: str, **over) -> dict:
    """A named synthetic workload: physical parameters plus per-atom inputs.

    nacl_512     molten NaCl 256+256, L = 25.2 A, 1200 K, Table 1, r_core 5, r_shell 10,
                 P_R 20, P_F 100
    nacl_32768   molten NaCl 16384+16384, L = 100.7 A, 1200 K, Table 1, P_R 20, P_F 200
    licl_nacl_1m 50:50 LiCl-NaCl melt with Table 3 parameters, N = 10^6, L = 329 A,
                 1150 K, r_core 5.5, r_shell 11, P_R 30, P_F 500; species slots
                 (Li, Na, Cl, Na2) with Na2 a second sodium slot of identical
                 parameters, holding half of the sodium ions
    nacl_5m      molten NaCl 2.5M+2.5M, L = 539 A, 1200 K, P_R 20, P_F 1000
    nacl_1024k   molten NaCl 512000+512000 at the 512-ion melt's density
                 (L = 317.5 A), 1200 K, Table 1, r_core 5, r_shell 10, P_R 30,
                 P_F 100: the size and batch sizes of the paper's timing table
    """
    table1 = species_block(["Na", "Cl"], TABLE1)
    if name == "nacl_512":
        d = dict(n=512, box=25.2, T=1200.0, species=table1, cat=[0], frac=[1.0],
                 r_core=5.0, r_shell=10.0, skin=1.0, p_r=20, p_f=100, seed=BASE_SEED + 1)
    elif name == "nacl_32768":
        d = dict(n=32768, box=100.7, T=1200.0, species=table1, cat=[0], frac=[1.0],
                 r_core=5.0, r_shell=10.0, skin=1.0, p_r=20, p_f=200, seed=BASE_SEED + 2)
    elif name == "licl_nacl_1m":
        sp = species_block(["Li", "Na", "Cl", "Na2"], TABLE3,
                           element_of={"Li": "Li", "Na": "Na", "Cl": "Cl", "Na2": "Na"})
        d = dict(n=1_000_000, box=329.0, T=1150.0, species=sp, cat=[0, 1, 3], frac=[0.5, 0.25, 0.25],
                 r_core=5.5, r_shell=11.0, skin=1.0, p_r=30, p_f=500, seed=BASE_SEED + 3)
    elif name == "nacl_5m":
        d = dict(n=5_000_000, box=539.0, T=1200.0, species=table1, cat=[0], frac=[1.0],
                 r_core=5.0, r_shell=10.0, skin=1.0, p_r=20, p_f=1000, seed=BASE_SEED + 5)
    elif name == "nacl_1024k":
        d = dict(n=1_024_000, box=25.2 * 2000.0 ** (1 / 3), T=1200.0, species=table1, cat=[0], frac=[1.0],
                 r_core=5.0, r_shell=10.0, skin=1.0, p_r=30, p_f=100, seed=BASE_SEED + 6)
    elif name == "nacl_small":
        # a few hundred ions in a box that still holds the 11 A list radius
        d = dict(n=216, box=22.5, T=1200.0, species=table1, cat=[0], frac=[1.0],
                 r_core=5.0, r_shell=10.0, skin=1.0, p_r=20, p_f=100, seed=BASE_SEED + 7)
    else:
        raise KeyError(name)
    d.update(over)
    box = d["box"]
    boxv = list(box) if isinstance(box, (list, tuple)) else [box, box, box]
    types, pos, vel = _melt(d["n"], boxv[0], d["T"], d["species"], d["cat"], d["frac"],
                            d.get("melt_seed", d["seed"]), d.get("jitter", 0.3))
    sysp = dict(species=d["species"], box=boxv, r_core=d["r_core"], r_shell=d["r_shell"], skin=d["skin"],
                p_r=d["p_r"], p_f=d["p_f"], seed=d["seed"], coulomb_k=COULOMB_K, dt=d.get("dt", 0.001),
                sog_eps=d.get("sog_eps", 1e-5), rebuild_every=d.get("rebuild_every", 10),
                replica=d.get("replica", 0))
    return dict(name=name, sys=sysp, types=types, pos=pos, vel=vel, T=d["T"])


def replica_batch(n_rep: int = 64, n_min: int = 512, n_max: int = 32768, density: float = 0.0319,
                  seed: int = BASE_SEED + 4) -> list:
    """A batch of molten-NaCl replicas of varied size (the batched workload).

    Replica r: N_r = 2 round(exp(U(ln n_min, ln n_max)) / 2) ions, cubic box
    L_r = (N_r / density)^(1/3), T_r ~ U(1100, 1400) K, Table 1, r_core 5,
    r_shell 10, skin 1, P_R 20, P_F 100.  All replicas share one Philox key
    (`seed`) and differ in their stream id (replica = r) and in the seed of
    their initial melt.  Returns one config dict per replica.
    """
    rng = np.random.default_rng(seed)
    sizes = 2 * np.round(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_rep)) / 2)
    temps = rng.uniform(1100.0, 1400.0, n_rep)
    out = []
    for r in range(n_rep):
        n = int(sizes[r])
        out.append(config("nacl_512", n=n, box=(n / density) ** (1.0 / 3.0), T=float(temps[r]), seed=seed,
                          replica=r, melt_seed=seed * 1000 + r))
    return out
