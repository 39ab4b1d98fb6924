"""Capacity growth on the GPU: a compressed melt whose stencil overflows the
list kernel's staging (which then moves to its larger variants) and whose
candidate lists overflow their first capacity, against the oracle; and a
step call whose lists overflow mid-run and restart, bitwise equal to a run
that never overflowed."""
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return math.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300))


def gpu_system(cfg, precision=R.FP64, pos=None, **over):
    import torch
    sysp = dict(cfg["sys"], **over)
    ctx = R.Context(0)
    p = R.make_params(sysp, precision, n_atoms=len(cfg["types"]))
    dev = torch.device("cuda", 0)
    ctx.rbsog_set_system(p, torch.as_tensor(cfg["types"], device=dev),
                         torch.as_tensor(cfg["pos"] if pos is None else pos, device=dev),
                         torch.as_tensor(cfg["vel"], device=dev))
    return ctx, sysp


def test_compressed_melt_grows_staging_and_lists():
    """All 32768 ions squeezed into half the box along x: twice the density
    there, so the 27-cell stencils exceed the first two staging capacities
    and the candidate lists their first capacity.  Lists and forces still
    match the oracle."""
    _say("case: compressed nacl_32768 (x halved)")
    cfg = W.config("nacl_32768")
    pos = np.array(cfg["pos"], dtype=float)
    pos[:, 0] *= 0.5
    ctx, sysp = gpu_system(cfg, R.FP64, pos=pos)
    osys = O.System(sysp, cfg["types"], pos, cfg["vel"])
    ncg, nkg = ctx.rbsog_get_list_counts()
    nco, nko = osys.list_counts()
    _say(f"  largest core / candidate list: {nco.max()} / {nko.max()}")
    assert np.array_equal(ncg, nco) and np.array_equal(nkg, nko)
    for i in np.random.default_rng(2).choice(len(pos), 20, replace=False):
        cg, kg = ctx.rbsog_get_lists_of(int(i), ncg[i], nkg[i])
        co, ko = osys.lists_of(int(i))
        assert np.array_equal(cg, np.sort(co)) and np.array_equal(kg, ko)
    fg, _ = ctx.rbsog_compute_forces(1)
    fo, _ = osys.forces(1)
    e, m = check_forces(fg.cpu().numpy(), fo, 1e-11, "squeezed melt")
    _say(f"  force rel rms {e:.2e}, worst atom {m:.2e} F_rms")


def test_step_restart_after_overflow_is_transparent():
    """Lists sized to hold exactly the largest ones at the start overflow at
    a later rebuild inside rbsog_step; the call restarts from its starting
    state with larger lists and ends bitwise where a run with roomy lists
    ends."""
    _say("case: mid-run list overflow and restart, nacl_32768 fp64")
    cfg = W.config("nacl_32768")
    over = dict(skin=0.2, rebuild_every=3)
    a, _ = gpu_system(cfg, R.FP64, **over)
    b, _ = gpu_system(cfg, R.FP64, **over)
    nc, nk = b.rbsog_get_list_counts()
    # a list holds at most cap - 1 entries
    got = b.rbsog_set_list_capacity(int(nc.max()) + 1, int(nk.max()) + 1)
    _say(f"  tight capacities {got}")
    assert got == (int(nc.max()) + 1, int(nk.max()) + 1)
    ea = a.rbsog_step(20)
    eb = b.rbsog_step(20)
    _say(f"  builds: roomy {ea['n_builds']}, tight {eb['n_builds']}")
    assert eb["n_builds"] >= ea["n_builds"] + 2  # the capacity call's build and at least one restart
    pa, va, fa, _ = a.rbsog_get_state()
    pb, vb, fb, _ = b.rbsog_get_state()
    assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy())
    assert np.array_equal(va.cpu().numpy(), vb.cpu().numpy())
    assert np.array_equal(fa.cpu().numpy(), fb.cpu().numpy())
    assert ea["u_total"] == eb["u_total"]
