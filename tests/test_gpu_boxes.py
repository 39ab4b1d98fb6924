"""Orthorhombic boxes whose list grid is split along some axes and not
others: 101.25 x 22.5 x 45 A holds 9 x 1 x 4 list cells (an axis with fewer
than 3 list cells is not split, and its ordering grid has one cell), so the
cell sort's sub-cells, the staged region and the candidate order (ordering
cell, index) all meet both cases at once.  Lists bit-exact and forces
within the bars against the oracle, and a short trajectory with rebuilds."""
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
A0 = 2.8125  # rock-salt site spacing (A)
SITES = (36, 8, 16)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return math.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300))


def _ortho_melt(seed=17, T=1200.0, jitter=0.3):
    """Rock-salt sites on a 36 x 8 x 16 grid of spacing A0 with uniform jitter,
    Na where i+j+k is even, Maxwell-Boltzmann velocities: 4608 ions."""
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(m) for m in SITES], indexing="ij"), -1).reshape(-1, 3)
    box = np.array(SITES, dtype=float) * A0
    pos = (g + 0.5) * A0 + rng.uniform(-jitter, jitter, size=g.shape)
    pos = np.mod(pos, box)
    base = W.config("nacl_512")
    sp = base["sys"]["species"]
    na = sp["names"].index("Na")
    cl = sp["names"].index("Cl")
    types = np.where(g.sum(1) % 2 == 0, na, cl).astype(np.int32)
    vel = W.maxwell_boltzmann(np.array(sp["mass"])[types], T, rng)
    sysp = dict(base["sys"], box=[float(b) for b in box])
    return sysp, types, pos, vel


@pytest.fixture(scope="module")
def ortho():
    return _ortho_melt()


def _gpu(sysp, types, pos, vel, precision):
    import torch
    dev = torch.device("cuda", 0)
    ctx = R.Context(0)
    ctx.rbsog_set_system(R.make_params(sysp, precision, n_atoms=len(types)), torch.as_tensor(types, device=dev),
                         torch.as_tensor(pos, device=dev), torch.as_tensor(vel, device=dev))
    return ctx


def test_lists_identical_orthorhombic(ortho):
    sysp, types, pos, vel = ortho
    _say("case: lists orthorhombic 101.25 x 22.5 x 45")
    ctx = _gpu(sysp, types, pos, vel, R.FP64)
    osys = O.System(sysp, types, pos, vel)
    ncg, nkg = ctx.rbsog_get_list_counts()
    nco, nko = osys.list_counts()
    assert np.array_equal(ncg, nco)
    assert np.array_equal(nkg, nko)
    for i in np.random.default_rng(3).choice(len(types), 60, replace=False):
        cg, kg = ctx.rbsog_get_lists_of(int(i), ncg[i], nkg[i])
        co, ko = osys.lists_of(int(i))
        assert np.array_equal(cg, np.sort(co)), int(i)
        assert np.array_equal(kg, ko), int(i)


@pytest.mark.parametrize("precision,tol", [(R.FP64, TOL64), (R.MIXED, TOL32)])
def test_forces_orthorhombic(ortho, precision, tol):
    sysp, types, pos, vel = ortho
    _say(f"case: forces orthorhombic precision {precision}")
    ctx = _gpu(sysp, types, pos, vel, precision)
    osys = O.System(sysp, types, pos, vel)
    for ev in (0, 4):
        fg, eg = ctx.rbsog_compute_forces(ev)
        fo, eo = osys.forces(ev)
        e, m = check_forces(fg.cpu().numpy(), fo, tol, f"eval {ev}")
        _say(f"  eval {ev}: force rel rms {e:.2e}, worst atom {m:.2e} F_rms")
        assert eg["u_total"] == pytest.approx(eo["u_total"], rel=max(tol, 1e-12))


def test_trajectory_with_rebuilds_orthorhombic(ortho):
    """12 FP64 steps with skin 0.2 A and a scheduled rebuild every 5 steps."""
    sysp, types, pos, vel = ortho
    sysp = dict(sysp, skin=0.2, rebuild_every=5)
    _say("case: trajectory orthorhombic")
    ctx = _gpu(sysp, types, pos, vel, R.FP64)
    osys = O.System(sysp, types, pos, vel)
    ctx.rbsog_compute_forces(0, want_energy=False)
    osys.forces(0)
    eg = ctx.rbsog_step(12)
    eo = osys.vv_steps(12)
    assert eg["n_builds"] == osys.n_builds() >= 3
    pg, vg, _, _ = ctx.rbsog_get_state()
    po, vo, _, _ = osys.state()
    L = np.array(sysp["box"])
    d = pg.cpu().numpy() - po
    d -= L * np.rint(d / L)
    _say(f"  max |dx| {np.abs(d).max():.2e}, builds {eg['n_builds']}")
    assert np.abs(d).max() < 1e-9
    assert rel_rms(vg.cpu().numpy(), vo) < 1e-9
    assert eg["u_total"] == pytest.approx(eo["u_total"], rel=1e-9)
