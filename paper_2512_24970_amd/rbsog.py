"""ctypes binding of librbsog (C ABI in ``include/rbsog.h``).

Argument marshalling only: every step of the force evaluation runs in the
library's HIP kernels.  PyTorch provides device memory (tensors whose
``data_ptr()`` is passed through) and the stream.  Loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbsog.so")

MAX_SPECIES = 8
MAX_SOG = 512
FP64 = 0
MIXED = 1
FLAG_SHELL_STORED = 1  # shell batch drawn at the list build and kept (memory form)
FLAG_INT_PHASE = 2     # mixed form: k-space phases in 32-bit fixed point
THERMOSTATS = {"berendsen": 0, "nose_hoover": 1, "langevin": 2}

STATUS = {0: "OK", -1: "E_ARG", -2: "E_STATE", -3: "E_HIP", -4: "E_OOM", -5: "E_LIST_STALE",
          -6: "E_NONNEUTRAL", -7: "E_BOX", -8: "E_NONFINITE", -9: "E_CAPACITY"}


class RbsogError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Species(C.Structure):
    _fields_ = [("q", C.c_double), ("mass", C.c_double)]


class Pair(C.Structure):
    _fields_ = [("A", C.c_double), ("sigma", C.c_double), ("rho", C.c_double), ("C", C.c_double),
                ("D", C.c_double)]


class Params(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("n_species", C.c_int32), ("box", C.c_double * 3),
        ("species", Species * MAX_SPECIES), ("pair", Pair * (MAX_SPECIES * MAX_SPECIES)),
        ("r_core", C.c_double), ("r_shell", C.c_double), ("skin", C.c_double),
        ("p_r", C.c_int32), ("p_f", C.c_int32), ("sog_eps", C.c_double), ("dt", C.c_double),
        ("rebuild_every", C.c_int32), ("precision", C.c_int32), ("seed", C.c_uint64),
        ("replica", C.c_uint32), ("flags", C.c_uint32), ("coulomb_k", C.c_double),
        ("t_target", C.c_double), ("tau_t", C.c_double), ("thermostat", C.c_int32), ("reserved", C.c_int32),
        ("r_core_pair", C.c_double * (MAX_SPECIES * MAX_SPECIES)),
    ]


class Tuning(C.Structure):
    _fields_ = [("pair_block", C.c_int32), ("pair_ku", C.c_int32), ("rho_mpl", C.c_int32), ("kf_block", C.c_int32),
                ("kf_aux", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Energy(C.Structure):
    _fields_ = [("u_core", C.c_double), ("u_shell", C.c_double), ("u_kspace", C.c_double),
                ("u_self", C.c_double), ("u_total", C.c_double), ("kinetic", C.c_double),
                ("p_corr", C.c_double * 3), ("max_disp", C.c_double), ("n_builds", C.c_int64),
                ("e_thermostat", C.c_double), ("virial", C.c_double * 6), ("stress", C.c_double * 6),
                ("heat_flux", C.c_double * 3)]

    def as_dict(self) -> dict:
        arrays = ("p_corr", "virial", "stress", "heat_flux")
        return {k: (list(getattr(self, k)) if k in arrays else getattr(self, k)) for k, _ in self._fields_}


ABI = {
    # name: (restype, argtypes)
    "rbsog_version": (C.c_char_p, []),
    "rbsog_sog_params": (C.c_int, [C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int32]),
    "rbsog_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "rbsog_near_table": (C.c_int, [C.c_double, C.c_double, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32)]),
    "rbsog_destroy": (C.c_int, [C.c_void_p]),
    "rbsog_last_error": (C.c_char_p, [C.c_void_p]),
    "rbsog_set_system": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "rbsog_set_batch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int]),
    "rbsog_n_systems": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "rbsog_select_system": (C.c_int, [C.c_void_p, C.c_int32]),
    "rbsog_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "rbsog_set_tuning": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rbsog_get_tuning": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rbsog_use_graphs": (C.c_int, [C.c_void_p, C.c_int]),
    "rbsog_build_lists": (C.c_int, [C.c_void_p]),
    "rbsog_set_positions": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "rbsog_step_batch": (C.c_int, [C.c_void_p, C.c_int32]),
    "rbsog_get_shell_samples": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rbsog_compute_forces": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(Energy)]),
    "rbsog_get_force_parts": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rbsog_step": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Energy)]),
    "rbsog_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64), C.c_int]),
    "rbsog_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "rbsog_profile_read": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rbsog_get_list_counts": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rbsog_get_lists_of": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "rbsog_get_shell_ranks": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "rbsog_get_shell_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rbsog_rdf_counts": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_void_p]),
    "rbsog_rdf_counts_noalloc": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_void_p]),
    "rbsog_msd": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "rbsog_set_list_chunks": (C.c_int, [C.c_void_p, C.c_int32]),
    "rbsog_set_list_capacity": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32)]),
    "rbsog_get_kmodes": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(C.c_double)]),
    "rbsog_get_rho": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rbsog_get_sog": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_int32), C.c_void_p, C.c_int32]),
}

_lib = None


def lib():
    """Load librbsog.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2512_24970_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in ABI.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _np_ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


def make_params(sysp: dict, precision: int = FP64, n_atoms: int | None = None) -> Params:
    """The ABI parameter block from a workload's physical parameters."""
    p = Params()
    sp = sysp["species"]
    S = len(sp["q"])
    p.n_atoms = int(n_atoms if n_atoms is not None else sysp.get("n", 0))
    p.n_species = S
    for a in range(3):
        p.box[a] = float(sysp["box"][a])
    for i in range(S):
        p.species[i].q = float(sp["q"][i])
        p.species[i].mass = float(sp["mass"][i])
        for j in range(S):
            pr = p.pair[i * MAX_SPECIES + j]
            pr.A = float(sp["A"][i][j])
            pr.sigma = float(sp["sigma"][i][j])
            pr.rho = float(sp["rho"][i][j])
            pr.C = float(sp["C"][i][j])
            pr.D = float(sp["D"][i][j])
    p.r_core = float(sysp["r_core"])
    p.r_shell = float(sysp["r_shell"])
    p.skin = float(sysp["skin"])
    p.p_r = int(sysp["p_r"])
    p.p_f = int(sysp["p_f"])
    p.sog_eps = float(sysp.get("sog_eps", 1e-5))
    p.dt = float(sysp.get("dt", 0.001))
    p.rebuild_every = int(sysp.get("rebuild_every", 10))
    p.precision = int(precision)
    p.seed = int(sysp["seed"])
    p.replica = int(sysp.get("replica", 0))
    p.flags = (FLAG_SHELL_STORED if sysp.get("shell_stored", False) else 0) | \
        (FLAG_INT_PHASE if sysp.get("int_phase", False) else 0)
    p.coulomb_k = float(sysp["coulomb_k"])
    p.t_target = float(sysp.get("t_target", 0.0))
    p.tau_t = float(sysp.get("tau_t", 0.0))
    p.thermostat = THERMOSTATS[sysp.get("thermostat", "berendsen")]
    rcp = sysp.get("r_core_pair")
    if rcp is not None:
        for i in range(S):
            for j in range(S):
                p.r_core_pair[i * MAX_SPECIES + j] = float(rcp[i][j])
    return p


def rbsog_near_table(eps: float, r_shell: float) -> dict:
    """The mixed form's FP32 near-field table: e0, coef[n_intervals][8]."""
    e0, n = C.c_int32(), C.c_int32()
    rc = lib().rbsog_near_table(eps, r_shell, None, 0, C.byref(e0), C.byref(n))
    if rc != 0:
        raise RbsogError(rc, "rbsog_near_table failed")
    coef = np.zeros((max(n.value, 1), 8), np.float32)
    rc = lib().rbsog_near_table(eps, r_shell, _np_ptr(coef), coef.size, C.byref(e0), C.byref(n))
    if rc != 0:
        raise RbsogError(rc, "rbsog_near_table failed")
    return {"e0": e0.value, "coef": coef[: n.value]}


def rbsog_sog_params(eps: float, r_shell: float) -> dict:
    b, s, xc = C.c_double(), C.c_double(), C.c_double()
    M = C.c_int32()
    w = np.zeros(MAX_SOG)
    rc = lib().rbsog_sog_params(eps, r_shell, C.byref(b), C.byref(s), C.byref(xc), C.byref(M),
                                w.ctypes.data_as(C.POINTER(C.c_double)), MAX_SOG)
    if rc != 0:
        raise RbsogError(rc, "rbsog_sog_params failed")
    return {"b": b.value, "s": s.value, "x_c": xc.value, "M": M.value, "w": w[: M.value + 1].copy()}


class Context:
    """One rbsog_ctx: one system, or a batch of systems, on one device and
    stream.  Energies come back as one dict per system (a dict for a single
    system); per-atom arrays hold the systems' rows one after another."""

    def __init__(self, device: int = 0, stream=None):
        import torch  # device memory and streams come from torch
        self._torch = torch
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = C.c_void_p()
        self._check(lib().rbsog_create(C.byref(h), device, C.c_void_p(stream.cuda_stream)), "rbsog_create")
        self._h = h
        self.n = 0
        self.params = None
        self.params_list = []
        self.R = 0
        self.sel = 0

    def _check(self, rc: int, what: str):
        if rc != 0:
            msg = ""
            if getattr(self, "_h", None):
                m = lib().rbsog_last_error(self._h)
                msg = m.decode() if m else ""
            raise RbsogError(rc, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            lib().rbsog_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up --------------------------------------------------------------
    def rbsog_set_system(self, params: Params, types, pos, vel=None):
        """types/pos/vel: torch tensors on this device (int32 [N], float64 [N,3])."""
        t = self._torch
        types = t.as_tensor(types, dtype=t.int32, device=self.torch_device).contiguous()
        pos = t.as_tensor(pos, dtype=t.float64, device=self.torch_device).contiguous()
        vptr = None
        if vel is not None:
            vel = t.as_tensor(vel, dtype=t.float64, device=self.torch_device).contiguous()
            vptr = C.c_void_p(vel.data_ptr())
        params.n_atoms = int(types.numel())
        self._check(lib().rbsog_set_system(self._h, C.byref(params), C.c_void_p(types.data_ptr()),
                                           C.c_void_p(pos.data_ptr()), vptr, 1), "rbsog_set_system")
        self.n = int(types.numel())
        self.params = params
        self.params_list = [params]
        self.R = 1
        self.sel = 0

    def rbsog_set_batch(self, params_list, types, pos, vel=None):
        """params_list: one Params per system (n_atoms set); types/pos/vel:
        the systems' rows concatenated, torch tensors on this device."""
        t = self._torch
        types = t.as_tensor(types, dtype=t.int32, device=self.torch_device).contiguous()
        pos = t.as_tensor(pos, dtype=t.float64, device=self.torch_device).contiguous()
        vptr = None
        if vel is not None:
            vel = t.as_tensor(vel, dtype=t.float64, device=self.torch_device).contiguous()
            vptr = C.c_void_p(vel.data_ptr())
        R = len(params_list)
        arr = (Params * R)(*params_list)
        self._check(lib().rbsog_set_batch(self._h, R, arr, C.c_void_p(types.data_ptr()),
                                          C.c_void_p(pos.data_ptr()), vptr, 1), "rbsog_set_batch")
        self.n = int(types.numel())
        self.params_list = list(params_list)
        self.params = self.params_list[0]
        self.R = R
        self.sel = 0

    def rbsog_n_systems(self) -> int:
        n = C.c_int32()
        self._check(lib().rbsog_n_systems(self._h, C.byref(n)), "rbsog_n_systems")
        return int(n.value)

    def rbsog_select_system(self, r: int):
        self._check(lib().rbsog_select_system(self._h, r), "rbsog_select_system")
        self.sel = r

    def rbsog_autotune(self, reps: int = 3) -> dict:
        t = Tuning()
        self._check(lib().rbsog_autotune(self._h, reps, C.byref(t)), "rbsog_autotune")
        return t.as_dict()

    def rbsog_set_tuning(self, **kw):
        t = Tuning()
        self._check(lib().rbsog_get_tuning(self._h, C.byref(t)), "rbsog_get_tuning")
        for k, v in kw.items():
            setattr(t, k, int(v))
        self._check(lib().rbsog_set_tuning(self._h, C.byref(t)), "rbsog_set_tuning")

    def rbsog_get_tuning(self) -> dict:
        t = Tuning()
        self._check(lib().rbsog_get_tuning(self._h, C.byref(t)), "rbsog_get_tuning")
        return t.as_dict()

    def rbsog_use_graphs(self, on: bool = True):
        self._check(lib().rbsog_use_graphs(self._h, 1 if on else 0), "rbsog_use_graphs")

    def rbsog_set_list_capacity(self, cap_core: int, cap_cand: int):
        gc, gk = C.c_int32(), C.c_int32()
        self._check(lib().rbsog_set_list_capacity(self._h, cap_core, cap_cand, C.byref(gc), C.byref(gk)),
                    "rbsog_set_list_capacity")
        return gc.value, gk.value

    def rbsog_set_list_chunks(self, chunks: int):
        self._check(lib().rbsog_set_list_chunks(self._h, chunks), "rbsog_set_list_chunks")

    def _order_outputs(self):
        """Device outputs are written on the context's stream: make torch's
        current stream wait for them when the two differ."""
        cur = self._torch.cuda.current_stream(self.torch_device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    def _energies(self, e):
        out = [e[r].as_dict() for r in range(self.R)]
        return out[0] if self.R == 1 else out

    def rbsog_build_lists(self):
        self._check(lib().rbsog_build_lists(self._h), "rbsog_build_lists")

    def rbsog_set_positions(self, pos):
        """pos: [N, 3] float64 torch tensor on this device (user order)."""
        t = self._torch
        pos = t.as_tensor(pos, dtype=t.float64, device=self.torch_device).contiguous()
        self._check(lib().rbsog_set_positions(self._h, C.c_void_p(pos.data_ptr()), 1), "rbsog_set_positions")

    # -- evaluation ------------------------------------------------------------
    def rbsog_compute_forces(self, ev: int, want_energy: bool = True):
        t = self._torch
        f = t.empty((self.n, 3), dtype=t.float64, device=self.torch_device)
        e = (Energy * max(self.R, 1))()
        self._check(lib().rbsog_compute_forces(self._h, ev, C.c_void_p(f.data_ptr()),
                                               e if want_energy else None), "rbsog_compute_forces")
        self._order_outputs()
        return f, (self._energies(e) if want_energy else None)

    def rbsog_get_force_parts(self):
        t = self._torch
        fs = t.empty((self.n, 3), dtype=t.float64, device=self.torch_device)
        fk = t.empty((self.n, 3), dtype=t.float64, device=self.torch_device)
        self._check(lib().rbsog_get_force_parts(self._h, C.c_void_p(fs.data_ptr()), C.c_void_p(fk.data_ptr())),
                    "rbsog_get_force_parts")
        self._order_outputs()
        return fs, fk

    def rbsog_step(self, n_steps: int, want_energy: bool = True):
        e = (Energy * max(self.R, 1))()
        self._check(lib().rbsog_step(self._h, n_steps, e if want_energy else None), "rbsog_step")
        return self._energies(e) if want_energy else None

    def rbsog_step_batch(self, n_steps: int):
        self._check(lib().rbsog_step_batch(self._h, n_steps), "rbsog_step_batch")

    def rbsog_get_state(self):
        t = self._torch
        out = [t.empty((self.n, 3), dtype=t.float64, device=self.torch_device) for _ in range(3)]
        ev = C.c_uint64()
        self._check(lib().rbsog_get_state(self._h, *[C.c_void_p(o.data_ptr()) for o in out], C.byref(ev), 1),
                    "rbsog_get_state")
        self._order_outputs()
        return out[0], out[1], out[2], int(ev.value)

    # -- kernel timing -----------------------------------------------------------
    PHASES = ["build", "ksample", "pair", "rho", "reduce", "kforce", "integrate"]

    def rbsog_profile_enable(self, on=True):
        """on: True/1 every phase, 2 only the hot kernels' phases, False/0 off."""
        mode = int(on) if not isinstance(on, bool) else (1 if on else 0)
        self._check(lib().rbsog_profile_enable(self._h, mode), "rbsog_profile_enable")

    def rbsog_profile_read(self) -> dict:
        ms = np.zeros(len(self.PHASES))
        cnt = np.zeros(len(self.PHASES), np.int64)
        self._check(lib().rbsog_profile_read(self._h, _np_ptr(ms), _np_ptr(cnt)), "rbsog_profile_read")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.PHASES)}

    # -- parity exports (host arrays) of the selected system -----------------
    @property
    def _sel_n(self) -> int:
        return int(self.params_list[self.sel].n_atoms)

    def rbsog_get_list_counts(self):
        nc = np.zeros(self._sel_n, np.int32)
        nk = np.zeros(self._sel_n, np.int32)
        self._check(lib().rbsog_get_list_counts(self._h, _np_ptr(nc), _np_ptr(nk)), "rbsog_get_list_counts")
        return nc, nk

    def rbsog_get_lists_of(self, i: int, n_core: int, n_cand: int | None):
        """Core and candidate lists of atom i; n_cand None asks for no candidates."""
        core = np.zeros(max(n_core, 1), np.int32)
        cand = None if n_cand is None else np.zeros(max(n_cand, 1), np.int32)
        self._check(lib().rbsog_get_lists_of(self._h, i, _np_ptr(core), None if cand is None else _np_ptr(cand)),
                    "rbsog_get_lists_of")
        return core[:n_core], None if cand is None else cand[:n_cand]

    def rbsog_get_shell_ranks(self, ev: int):
        P = max(self.params_list[self.sel].p_r, 1)
        nr = np.zeros(self._sel_n, np.int32)
        r = np.zeros((self._sel_n, P), np.int32)
        self._check(lib().rbsog_get_shell_ranks(self._h, ev, _np_ptr(nr), _np_ptr(r)), "rbsog_get_shell_ranks")
        return nr, r

    def rbsog_get_shell_batch(self):
        P = max(self.params_list[self.sel].p_r, 1)
        nk = np.zeros(self._sel_n, np.int32)
        ids = np.zeros((self._sel_n, P), np.int32)
        self._check(lib().rbsog_get_shell_batch(self._h, _np_ptr(nk), _np_ptr(ids)), "rbsog_get_shell_batch")
        return nk, ids

    def rbsog_get_shell_samples(self):
        """(n_cand[N], ids[N, P_R]): the shell batch in use, neighbour ids sorted, -1 padded."""
        P = max(self.params_list[self.sel].p_r, 1)
        nk = np.zeros(self._sel_n, np.int32)
        ids = np.zeros((self._sel_n, P), np.int32)
        self._check(lib().rbsog_get_shell_samples(self._h, _np_ptr(nk), _np_ptr(ids)), "rbsog_get_shell_samples")
        return nk, ids

    def rbsog_rdf_counts(self, r_max: float, n_bins: int) -> np.ndarray:
        """Pair-distance histogram [S, S, n_bins] (uint64) of the selected system."""
        S = self.params_list[self.sel].n_species
        out = np.zeros((S, S, int(n_bins)), np.uint64)
        self._check(lib().rbsog_rdf_counts(self._h, float(r_max), int(n_bins), _np_ptr(out)), "rbsog_rdf_counts")
        return out

    def rbsog_rdf_counts_noalloc(self, r_max: float, n_bins: int) -> np.ndarray:
        """rbsog_rdf_counts through the allocation-free entry point."""
        S = self.params_list[self.sel].n_species
        out = np.zeros((S, S, int(n_bins)), np.uint64)
        self._check(lib().rbsog_rdf_counts_noalloc(self._h, float(r_max), int(n_bins), _np_ptr(out)),
                    "rbsog_rdf_counts_noalloc")
        return out

    def rbsog_msd(self, mark: bool = False) -> np.ndarray:
        """Per-species mean-square displacement (A^2) of the selected system since
        its marked origin; mark=True sets the origin at the current positions."""
        S = self.params_list[self.sel].n_species
        out = np.zeros(S, np.float64)
        self._check(lib().rbsog_msd(self._h, 1 if mark else 0, _np_ptr(out)), "rbsog_msd")
        return out

    def rbsog_get_kmodes(self, ev: int):
        p_f = self.params_list[self.sel].p_f
        m = np.zeros((max(p_f, 1), 3), np.int32)
        S = C.c_double()
        self._check(lib().rbsog_get_kmodes(self._h, ev, _np_ptr(m), C.byref(S)), "rbsog_get_kmodes")
        return m[:p_f], S.value

    def rbsog_get_rho(self, n_modes: int):
        rho = np.zeros((max(n_modes, 1), 2))
        self._check(lib().rbsog_get_rho(self._h, _np_ptr(rho)), "rbsog_get_rho")
        return rho[:n_modes]

    def rbsog_get_sog(self) -> dict:
        b, s, xc = C.c_double(), C.c_double(), C.c_double()
        M = C.c_int32()
        w = np.zeros(MAX_SOG)
        self._check(lib().rbsog_get_sog(self._h, C.byref(b), C.byref(s), C.byref(xc), C.byref(M), _np_ptr(w),
                                        MAX_SOG), "rbsog_get_sog")
        return {"b": b.value, "s": s.value, "x_c": xc.value, "M": M.value, "w": w[: M.value + 1].copy()}
