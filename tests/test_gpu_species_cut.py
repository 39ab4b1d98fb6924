"""Species-dependent core radii on the GPU against the oracle: lists
(bit-exact), shell ranks and stored batches (bit-exact), forces at the FP64
and mixed bars, for two- and four-species melts, and parameter checks."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle as O
from force_bars import check_forces
from paper_2512_24970_amd import rbsog as R
from paper_2512_24970_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-5
RCP2 = [[4.2, 5.6], [5.6, 6.4]]                      # Na-Na, Na-Cl, Cl-Cl
RCP4 = [[3.8, 4.6, 5.2, 4.6], [4.6, 5.0, 5.8, 5.0],  # Li, Na, Cl, Na2 (Na2 = Na)
        [5.2, 5.8, 6.3, 5.8], [4.6, 5.0, 5.8, 5.0]]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return math.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300))


def gpu_system(cfg, precision=R.FP64, **over):
    import torch
    sysp = dict(cfg["sys"], **over)
    ctx = R.Context(0)
    p = R.make_params(sysp, precision, n_atoms=len(cfg["types"]))
    dev = torch.device("cuda", 0)
    ctx.rbsog_set_system(p, torch.as_tensor(cfg["types"], device=dev), torch.as_tensor(cfg["pos"], device=dev),
                         torch.as_tensor(cfg["vel"], device=dev))
    return ctx, sysp


def _licl_small():
    n = 8000
    return W.config("licl_nacl_1m", n=n, box=329.0 * (n / 1e6) ** (1 / 3))


CASES = [("nacl_512", RCP2, R.FP64, TOL64), ("nacl_512", RCP2, R.MIXED, TOL32),
         ("nacl_32768", RCP2, R.FP64, TOL64), ("licl_8000", RCP4, R.FP64, TOL64),
         ("licl_8000", RCP4, R.MIXED, TOL32)]


@pytest.mark.parametrize("name,rcp,precision,tol", CASES)
def test_species_radii_lists_ranks_forces(name, rcp, precision, tol):
    _say(f"case: species radii {name} precision {precision}")
    cfg = _licl_small() if name == "licl_8000" else W.config(name)
    ctx, sysp = gpu_system(cfg, precision, r_core_pair=rcp)
    osys = O.System(sysp, cfg["types"], cfg["pos"], cfg["vel"])
    ncg, nkg = ctx.rbsog_get_list_counts()
    nco, nko = osys.list_counts()
    assert np.array_equal(ncg, nco) and np.array_equal(nkg, nko)
    rng = np.random.default_rng(3)
    atoms = rng.choice(len(cfg["types"]), 25, replace=False)
    for i in atoms:
        cg, kg = ctx.rbsog_get_lists_of(int(i), ncg[i], nkg[i])
        co, ko = osys.lists_of(int(i))
        assert np.array_equal(cg, np.sort(co)) and np.array_equal(kg, ko), int(i)
    nr, rk = ctx.rbsog_get_shell_ranks(3)
    for i in atoms:
        ro = osys.shell_ranks(int(i), 3)
        assert np.array_equal(rk[i, : nr[i]], ro), int(i)
    for ev in (0, 3):
        fg, eg = ctx.rbsog_compute_forces(ev)
        fo, eo = osys.forces(ev)
        e, m = check_forces(fg.cpu().numpy(), fo, tol, f"eval {ev}")
        _say(f"  eval {ev}: force rel rms {e:.2e}, worst atom {m:.2e} F_rms")
        for key in ("u_core", "u_shell"):
            assert eg[key] == pytest.approx(eo[key], rel=max(tol, 1e-12)), key


def test_species_radii_stored_batch():
    """The memory form with per-pair radii: stored batches bit-exact, forces."""
    _say("case: species radii stored batch nacl_32768")
    cfg = W.config("nacl_32768")
    ctx, sysp = gpu_system(cfg, R.FP64, r_core_pair=RCP2, shell_stored=True)
    osys = O.System(sysp, cfg["types"], cfg["pos"], cfg["vel"])
    nk_g, ids_g = ctx.rbsog_get_shell_batch()
    _, nk_o = osys.list_counts()
    assert np.array_equal(nk_g, nk_o)
    for i in np.random.default_rng(4).choice(len(cfg["types"]), 30, replace=False):
        _, cand = osys.lists_of(int(i))
        want = cand[osys.shell_ranks(int(i), 0)]
        assert np.array_equal(ids_g[i, : len(want)], want), int(i)
    fg, _ = ctx.rbsog_compute_forces(1)
    fo, _ = osys.forces(1)
    check_forces(fg.cpu().numpy(), fo, TOL64, "species radii")


def test_species_radii_rejected_when_invalid():
    import torch
    _say("case: species radii validation")
    cfg = W.config("nacl_512")
    dev = torch.device("cuda", 0)
    t = torch.as_tensor(cfg["types"], device=dev)
    x = torch.as_tensor(cfg["pos"], device=dev)
    ctx = R.Context(0)
    for bad in ([[4.0, 5.0], [5.5, 6.0]], [[4.0, 10.0], [10.0, 6.0]], [[4.0, -1.0], [-1.0, 6.0]]):
        with pytest.raises(R.RbsogError) as e:
            ctx.rbsog_set_system(R.make_params(dict(cfg["sys"], r_core_pair=bad), R.FP64, n_atoms=512), t, x)
        assert e.value.code == -1
