"""Python access to the double-precision CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers; the GPU library never
imports this package and shares no code with it.

Every function here only marshals arguments for the C oracle; the arithmetic
lives in ``oracle.c`` (Section 2 of arXiv:2512.24970, equations cited there).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MAXS = 8
MAXM = 511
TAG_SHELL = 2
TAG_KMODE = 3
TAG_SHELL_BUILD = 5
TAG_LANGEVIN = 6
THERMOSTATS = {"berendsen": 0, "nose_hoover": 1, "langevin": 2}


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (no fused multiply-add)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
               "-o", _LIB_PATH, os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


class Params(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32), ("p_r", C.c_int32), ("p_f", C.c_int32), ("M", C.c_int32),
        ("replica", C.c_uint32), ("rebuild_every", C.c_int32), ("seed", C.c_uint64),
        ("box", C.c_double * 3), ("r_core", C.c_double), ("r_shell", C.c_double), ("skin", C.c_double),
        ("coulomb_k", C.c_double), ("dt", C.c_double), ("sog_eps", C.c_double),
        ("b", C.c_double), ("s", C.c_double), ("x_c", C.c_double),
        ("w", C.c_double * (MAXM + 1)),
        ("q", C.c_double * MAXS), ("mass", C.c_double * MAXS),
        ("A", C.c_double * (MAXS * MAXS)), ("sig", C.c_double * (MAXS * MAXS)),
        ("rho", C.c_double * (MAXS * MAXS)), ("C", C.c_double * (MAXS * MAXS)),
        ("D", C.c_double * (MAXS * MAXS)),
        ("t_target", C.c_double), ("tau_t", C.c_double),
        ("shell_stored", C.c_int32), ("thermostat", C.c_int32),
        ("r_core_pair", C.c_double * (MAXS * MAXS)),
    ]


class Energy(C.Structure):
    _fields_ = [("u_core", C.c_double), ("u_shell", C.c_double), ("u_kspace", C.c_double),
                ("u_self", C.c_double), ("u_total", C.c_double), ("kinetic", C.c_double),
                ("p_corr", C.c_double * 3), ("e_thermostat", C.c_double), ("virial", C.c_double * 6),
                ("stress", C.c_double * 6), ("heat_flux", C.c_double * 3)]

    def as_dict(self) -> dict:
        return {"u_core": self.u_core, "u_shell": self.u_shell, "u_kspace": self.u_kspace,
                "u_self": self.u_self, "u_total": self.u_total, "kinetic": self.kinetic,
                "p_corr": list(self.p_corr), "e_thermostat": self.e_thermostat, "virial": list(self.virial),
                "stress": list(self.stress), "heat_flux": list(self.heat_flux)}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        u32p, i32p, dp = P(C.c_uint32), P(C.c_int32), P(C.c_double)
        sig = {
            "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
            "orc_stream_words": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, u32p]),
            "orc_bounded_from_words": (C.c_uint32, [u32p, C.c_int, C.c_uint32, P(C.c_int)]),
            "orc_sog_b_from_eps": (C.c_double, [C.c_double]),
            "orc_sog_xc": (C.c_double, [C.c_double, C.c_int]),
            "orc_sog_setup": (C.c_int, [P(Params)]),
            "orc_far": (C.c_double, [P(Params), C.c_double]),
            "orc_near": (C.c_double, [P(Params), C.c_double]),
            "orc_far_hat": (C.c_double, [P(Params), C.c_double]),
            "orc_far_hat_g": (C.c_double, [P(Params), C.c_double]),
            "orc_kspace_S": (C.c_double, [P(Params)]),
            "orc_kmodes": (C.c_int, [P(Params), C.c_uint64, i32p, dp]),
            "orc_create": (C.c_void_p, [P(Params), C.c_int32, i32p, dp, dp]),
            "orc_destroy": (None, [C.c_void_p]),
            "orc_build_lists": (C.c_int, [C.c_void_p]),
            "orc_list_counts": (C.c_int, [C.c_void_p, i32p, i32p]),
            "orc_list_atom": (C.c_int, [C.c_void_p, C.c_int32, i32p, i32p]),
            "orc_shell_ranks": (C.c_int, [C.c_void_p, C.c_int32, C.c_uint64, i32p]),
            "orc_scan_lists_atom": (C.c_int, [C.c_void_p, C.c_int32, i32p, i32p, i32p, i32p]),
            "orc_shell_ranks_count": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_uint64, i32p]),
            "orc_pair_force": (C.c_double, [P(Params), C.c_int32, C.c_int32, dp, dp]),
            "orc_forces": (C.c_int, [C.c_void_p, C.c_uint64, dp, P(Energy)]),
            "orc_forces_short": (C.c_int, [C.c_void_p, C.c_uint64, dp, dp, dp, dp]),
            "orc_forces_kspace": (C.c_int, [C.c_void_p, C.c_uint64, dp, dp, dp]),
            "orc_rho": (None, [C.c_void_p, C.c_int32, i32p, dp]),
            "orc_vv_steps": (C.c_int, [C.c_void_p, C.c_int32, P(Energy)]),
            "orc_get_state": (None, [C.c_void_p, dp, dp, dp, P(C.c_uint64)]),
            "orc_forces_short_atoms": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, i32p, dp]),
            "orc_rdf_counts": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.POINTER(C.c_uint64)]),
            "orc_kforce_atoms": (None, [C.c_void_p, C.c_int32, i32p, dp, C.c_double, C.c_int32, i32p, dp]),
            "orc_set_threads": (None, [C.c_int]),
            "orc_get_threads": (C.c_int, []),
            "orc_n_builds": (C.c_int64, [C.c_void_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def stream_words(seed: int, index: int, ev: int, tag: int, replica: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint32)
    lib().orc_stream_words(seed, index, ev, tag, replica, n, _ptr(out, C.c_uint32))
    return out


def bounded_from_words(words, rng: int):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    used = C.c_int(0)
    v = lib().orc_bounded_from_words(_ptr(w, C.c_uint32), len(w), rng, C.byref(used))
    return int(v), int(used.value)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def make_params(sysp: dict) -> Params:
    """Fill the C parameter block from a workload's physical parameters and run
    the SOG set-up (Section 2.1)."""
    p = Params()
    sp = sysp["species"]
    S = len(sp["q"])
    p.n_species = S
    p.p_r = int(sysp["p_r"])
    p.p_f = int(sysp["p_f"])
    p.replica = int(sysp.get("replica", 0))
    p.rebuild_every = int(sysp.get("rebuild_every", 10))
    p.seed = int(sysp["seed"])
    for a in range(3):
        p.box[a] = float(sysp["box"][a])
    p.r_core = float(sysp["r_core"])
    p.r_shell = float(sysp["r_shell"])
    p.skin = float(sysp["skin"])
    p.coulomb_k = float(sysp["coulomb_k"])
    p.dt = float(sysp.get("dt", 0.001))
    p.sog_eps = float(sysp.get("sog_eps", 1e-5))
    p.t_target = float(sysp.get("t_target", 0.0))
    p.tau_t = float(sysp.get("tau_t", 0.0))
    p.shell_stored = 1 if sysp.get("shell_stored", False) else 0
    p.thermostat = THERMOSTATS[sysp.get("thermostat", "berendsen")]
    rcp = sysp.get("r_core_pair")
    if rcp is not None:
        for i in range(S):
            for j in range(S):
                p.r_core_pair[i * MAXS + j] = float(rcp[i][j])
    for i in range(S):
        p.q[i] = float(sp["q"][i])
        p.mass[i] = float(sp["mass"][i])
        for j in range(S):
            t = i * MAXS + j
            p.A[t] = float(sp["A"][i][j])
            p.sig[t] = float(sp["sigma"][i][j])
            p.rho[t] = float(sp["rho"][i][j])
            p.C[t] = float(sp["C"][i][j])
            p.D[t] = float(sp["D"][i][j])
    rc = lib().orc_sog_setup(C.byref(p))
    if rc != 0:
        raise RuntimeError(f"oracle SOG set-up failed ({rc})")
    return p


def sog(p: Params) -> dict:
    return {"b": p.b, "s": p.s, "M": p.M, "x_c": p.x_c, "w": np.array(p.w[: p.M + 1])}


def far(p: Params, r: float) -> float:
    return lib().orc_far(C.byref(p), r)


def near(p: Params, r: float) -> float:
    return lib().orc_near(C.byref(p), r)


def far_hat(p: Params, k: float) -> float:
    return lib().orc_far_hat(C.byref(p), k)


def far_hat_g(p: Params, k: float) -> float:
    """-dF^/dk / k."""
    return lib().orc_far_hat_g(C.byref(p), k)


def pair_force(p: Params, ti: int, tj: int, d) -> tuple:
    """Force on i from j for displacement d = r_i - r_j, and the pair energy."""
    dd = np.ascontiguousarray(d, dtype=np.float64)
    f = np.zeros(3)
    u = lib().orc_pair_force(C.byref(p), ti, tj, _ptr(dd, C.c_double), _ptr(f, C.c_double))
    return f, u


def kspace_S(p: Params) -> float:
    return lib().orc_kspace_S(C.byref(p))


def kmodes(p: Params, ev: int):
    m = np.zeros((max(p.p_f, 1), 3), dtype=np.int32)
    S = C.c_double(0.0)
    lib().orc_kmodes(C.byref(p), ev, _ptr(m, C.c_int32), C.byref(S))
    return m[: p.p_f], S.value


class System:
    """A system held by the oracle: positions, velocities, lists, last force."""

    def __init__(self, sysp: dict, types: np.ndarray, pos: np.ndarray, vel: np.ndarray | None = None):
        self.params = make_params(sysp)
        self.n = int(len(types))
        self._types = np.ascontiguousarray(types, dtype=np.int32)
        self._pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        self._vel = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        vp = None if self._vel is None else _ptr(self._vel, C.c_double)
        self._h = lib().orc_create(C.byref(self.params), self.n, _ptr(self._types, C.c_int32),
                                   _ptr(self._pos, C.c_double), vp)
        self._lists = False

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_lists(self):
        lib().orc_build_lists(self._h)
        self._lists = True

    def _ensure_lists(self):
        if not self._lists:
            self.build_lists()

    def n_builds(self) -> int:
        return int(lib().orc_n_builds(self._h))

    def list_counts(self):
        self._ensure_lists()
        nc = np.zeros(self.n, dtype=np.int32)
        nk = np.zeros(self.n, dtype=np.int32)
        lib().orc_list_counts(self._h, _ptr(nc, C.c_int32), _ptr(nk, C.c_int32))
        return nc, nk

    def lists_of(self, i: int):
        nc, nk = self.list_counts()
        core = np.zeros(max(nc[i], 1), dtype=np.int32)
        cand = np.zeros(max(nk[i], 1), dtype=np.int32)
        lib().orc_list_atom(self._h, i, _ptr(core, C.c_int32), _ptr(cand, C.c_int32))
        return core[: nc[i]], cand[: nk[i]]

    def shell_ranks(self, i: int, ev: int) -> np.ndarray:
        self._ensure_lists()
        _, nk = self.list_counts()
        r = np.zeros(max(nk[i], 1), dtype=np.int32)
        k = lib().orc_shell_ranks(self._h, i, ev, _ptr(r, C.c_int32))
        return r[:k]

    def scan_lists_of(self, i: int):
        """Core and candidate lists of atom i by a scan over every atom (no
        full build): the same lists as lists_of, at any size."""
        nc = np.zeros(1, dtype=np.int32)
        nk = np.zeros(1, dtype=np.int32)
        null = C.POINTER(C.c_int32)()
        if lib().orc_scan_lists_atom(self._h, i, null, null, _ptr(nc, C.c_int32), _ptr(nk, C.c_int32)) != 0:
            raise ValueError("bad atom index")
        core = np.zeros(max(int(nc[0]), 1), dtype=np.int32)
        cand = np.zeros(max(int(nk[0]), 1), dtype=np.int32)
        lib().orc_scan_lists_atom(self._h, i, _ptr(core, C.c_int32), _ptr(cand, C.c_int32), _ptr(nc, C.c_int32),
                                  _ptr(nk, C.c_int32))
        return core[: nc[0]], cand[: nk[0]]

    def shell_ranks_count(self, i: int, n: int, ev: int) -> np.ndarray:
        """Shell ranks of atom i for a candidate count n (no lists needed)."""
        r = np.zeros(max(n, 1), dtype=np.int32)
        k = lib().orc_shell_ranks_count(self._h, i, n, ev, _ptr(r, C.c_int32))
        if k < 0:
            raise ValueError("bad atom index or count")
        return r[:k]

    def forces(self, ev: int):
        self._ensure_lists()
        f = np.zeros((self.n, 3))
        e = Energy()
        lib().orc_forces(self._h, ev, _ptr(f, C.c_double), C.byref(e))
        return f, e.as_dict()

    def forces_short(self, ev: int):
        self._ensure_lists()
        f = np.zeros((self.n, 3))
        uc, us = C.c_double(0), C.c_double(0)
        lib().orc_forces_short(self._h, ev, _ptr(f, C.c_double), C.byref(uc), C.byref(us), None)
        return f, uc.value, us.value

    def virial_parts(self, ev: int):
        """Virial W[6] (xx, yy, zz, xy, xz, yz) of the short-range and of the
        k-space estimator at evaluation ev."""
        self._ensure_lists()
        f = np.zeros((self.n, 3))
        uc, us, uk = C.c_double(0), C.c_double(0), C.c_double(0)
        ws = np.zeros(6)
        wk = np.zeros(6)
        lib().orc_forces_short(self._h, ev, _ptr(f, C.c_double), C.byref(uc), C.byref(us), _ptr(ws, C.c_double))
        lib().orc_forces_kspace(self._h, ev, _ptr(f, C.c_double), C.byref(uk), _ptr(wk, C.c_double))
        return ws, wk

    def forces_kspace(self, ev: int):
        f = np.zeros((self.n, 3))
        uk = C.c_double(0)
        lib().orc_forces_kspace(self._h, ev, _ptr(f, C.c_double), C.byref(uk), None)
        return f, uk.value

    def rho(self, m: np.ndarray) -> np.ndarray:
        m = np.ascontiguousarray(m, dtype=np.int32).reshape(-1, 3)
        out = np.zeros((len(m), 2))
        lib().orc_rho(self._h, len(m), _ptr(m, C.c_int32), _ptr(out, C.c_double))
        return out

    def rdf_counts(self, r_max: float, n_bins: int) -> np.ndarray:
        """Pair-distance histogram [S, S, n_bins] (ordered pairs, all by brute force)."""
        S = self.params.n_species
        out = np.zeros((S, S, n_bins), dtype=np.uint64)
        rc = lib().orc_rdf_counts(self._h, float(r_max), int(n_bins), _ptr(out, C.c_uint64))
        if rc != 0:
            raise ValueError("orc_rdf_counts: bad arguments")
        return out

    def forces_short_atoms(self, ev: int, sel) -> np.ndarray:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        f = np.zeros((len(sel), 3))
        rc = lib().orc_forces_short_atoms(self._h, ev, len(sel), _ptr(sel, C.c_int32), _ptr(f, C.c_double))
        if rc != 0:
            raise ValueError("bad atom index")
        return f

    def kforce_atoms(self, m: np.ndarray, rho: np.ndarray, coef_scale: float, sel) -> np.ndarray:
        m = np.ascontiguousarray(m, dtype=np.int32).reshape(-1, 3)
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1, 2)
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        f = np.zeros((len(sel), 3))
        lib().orc_kforce_atoms(self._h, len(m), _ptr(m, C.c_int32), _ptr(rho, C.c_double), coef_scale,
                               len(sel), _ptr(sel, C.c_int32), _ptr(f, C.c_double))
        return f

    def vv_steps(self, n: int) -> dict:
        self._ensure_lists()
        e = Energy()
        lib().orc_vv_steps(self._h, n, C.byref(e))
        return e.as_dict()

    def state(self):
        pos = np.zeros((self.n, 3))
        vel = np.zeros((self.n, 3))
        frc = np.zeros((self.n, 3))
        ev = C.c_uint64(0)
        lib().orc_get_state(self._h, _ptr(pos, C.c_double), _ptr(vel, C.c_double), _ptr(frc, C.c_double),
                            C.byref(ev))
        return pos, vel, frc, int(ev.value)
