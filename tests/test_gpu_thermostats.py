"""Thermostats on the GPU against the oracle: Nose-Hoover (one variable,
Trotter half steps around the velocity-Verlet step) and Langevin (BAOAB,
Philox noise), trajectories through the C ABI; a batch mixing the three
thermostats equals its single-system runs bitwise."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle as O
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


def gpu_system(cfg, precision=R.FP64, **over):
    import torch
    sysp = dict(cfg["sys"], **over)
    ctx = R.Context(0)
    p = R.make_params(sysp, precision, n_atoms=len(cfg["types"]))
    dev = torch.device("cuda", 0)
    ctx.rbsog_set_system(p, torch.as_tensor(cfg["types"], device=dev), torch.as_tensor(cfg["pos"], device=dev),
                         torch.as_tensor(cfg["vel"], device=dev))
    return ctx, sysp


def _compare(ctx, osys, sysp, eg, eo, tol=1e-9):
    pg, vg, fg, _ = ctx.rbsog_get_state()
    po, vo, fo, _ = osys.state()
    L = np.array(sysp["box"])
    d = pg.cpu().numpy() - po
    d -= L * np.rint(d / L)
    _say(f"  max |dx| {np.abs(d).max():.2e}, v rel rms {rel_rms(vg.cpu().numpy(), vo):.2e}")
    assert np.abs(d).max() < tol
    assert rel_rms(vg.cpu().numpy(), vo) < tol
    assert rel_rms(fg.cpu().numpy(), fo) < tol
    assert eg["kinetic"] == pytest.approx(eo["kinetic"], rel=tol)
    assert eg["u_total"] == pytest.approx(eo["u_total"], rel=tol)


@pytest.fixture(scope="module")
def nacl512():
    return W.config("nacl_512")


def test_nose_hoover_trajectory_matches_oracle(nacl512):
    """15 steps toward T0 = 1000 K from the 1200 K melt, tau = 20 fs, in two
    calls (8 + 7 steps): positions, velocities (with the closing half step's
    factor), kinetic energy and the thermostat's energy track the oracle."""
    _say("case: nose-hoover 15 steps nacl_512")
    ctx, sysp = gpu_system(nacl512, t_target=1000.0, tau_t=0.02, thermostat="nose_hoover")
    osys = O.System(sysp, nacl512["types"], nacl512["pos"], nacl512["vel"])
    ctx.rbsog_compute_forces(0, want_energy=False)
    osys.forces(0)
    ctx.rbsog_step(8)
    eg = ctx.rbsog_step(7)
    eo = osys.vv_steps(15)
    _compare(ctx, osys, sysp, eg, eo)
    assert eo["e_thermostat"] != 0.0
    assert eg["e_thermostat"] == pytest.approx(eo["e_thermostat"], rel=1e-8)


def test_langevin_trajectory_matches_oracle(nacl512):
    """15 steps of BAOAB at 1200 K with tau = 20 fs: the noise is drawn from
    the same Philox streams on both sides."""
    _say("case: langevin 15 steps nacl_512")
    ctx, sysp = gpu_system(nacl512, t_target=1200.0, tau_t=0.02, thermostat="langevin")
    osys = O.System(sysp, nacl512["types"], nacl512["pos"], nacl512["vel"])
    ctx.rbsog_compute_forces(0, want_energy=False)
    osys.forces(0)
    eg = ctx.rbsog_step(15)
    eo = osys.vv_steps(15)
    _compare(ctx, osys, sysp, eg, eo)
    assert eg["e_thermostat"] == 0.0


def test_langevin_stored_mixed_holds_temperature():
    """The 32768-ion melt in the mixed form with the stored batch and a
    Langevin thermostat at 1200 K, tau = 10 fs: 200 steps stay near the
    target.  (The estimators' noise heats this system by about 3 K per step,
    so the friction holds T at about 1200 K + 3 K/fs / (2/tau); at tau = 50 fs
    it settles some 100 K above the target.)"""
    _say("case: langevin 200 steps nacl_32768 mixed stored")
    cfg = W.config("nacl_32768")
    n = len(cfg["types"])
    ctx, _ = gpu_system(cfg, R.MIXED, t_target=1200.0, tau_t=0.01, thermostat="langevin", shell_stored=True)
    Ts = []
    for _ in range(20):
        e = ctx.rbsog_step(10)
        Ts.append(2 * e["kinetic"] / ((3 * n - 3) * W.KB))
    _say(f"  T over the last 100 steps: {np.mean(Ts[10:]):.1f} K")
    assert abs(np.mean(Ts[10:]) - 1200.0) < 60.0


def test_batch_mixing_thermostats_equals_singles():
    """Berendsen, Nose-Hoover and Langevin systems in one context with step
    graphs: every system's trajectory equals its single-system run bitwise."""
    import torch
    _say("case: batch of three thermostats")
    dev = torch.device("cuda", 0)
    cfgs = [W.config("nacl_512"), W.config("nacl_512", melt_seed=9), W.config("nacl_small")]
    kinds = [dict(thermostat="berendsen", t_target=1100.0, tau_t=0.001),
             dict(thermostat="nose_hoover", t_target=1000.0, tau_t=0.02),
             dict(thermostat="langevin", t_target=1300.0, tau_t=0.01)]
    plist = [R.make_params(dict(c["sys"], replica=r, **k), R.MIXED, n_atoms=len(c["types"]))
             for r, (c, k) in enumerate(zip(cfgs, kinds))]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = R.Context(0, stream=st)
        ctx.rbsog_set_batch(plist, torch.as_tensor(np.concatenate([c["types"] for c in cfgs]), device=dev),
                            torch.as_tensor(np.concatenate([c["pos"] for c in cfgs]), device=dev),
                            torch.as_tensor(np.concatenate([c["vel"] for c in cfgs]), device=dev))
        ctx.rbsog_use_graphs(True)
        ctx.rbsog_step(6)
        eb = ctx.rbsog_step(6)
        pb, vb, _, _ = ctx.rbsog_get_state()
    off = 0
    for r, c in enumerate(cfgs):
        n = len(c["types"])
        one = R.Context(0)
        one.rbsog_set_system(plist[r], torch.as_tensor(c["types"], device=dev), torch.as_tensor(c["pos"], device=dev),
                             torch.as_tensor(c["vel"], device=dev))
        one.rbsog_step(6)
        e1 = one.rbsog_step(6)
        p1, v1, _, _ = one.rbsog_get_state()
        assert np.array_equal(pb.cpu().numpy()[off:off + n], p1.cpu().numpy()), r
        assert np.array_equal(vb.cpu().numpy()[off:off + n], v1.cpu().numpy()), r
        assert eb[r]["kinetic"] == e1["kinetic"] and eb[r]["e_thermostat"] == e1["e_thermostat"], r
        off += n


def test_unknown_thermostat_rejected(nacl512):
    import torch
    _say("case: unknown thermostat")
    dev = torch.device("cuda", 0)
    p = R.make_params(dict(nacl512["sys"], t_target=1000.0, tau_t=0.01), R.FP64, n_atoms=512)
    p.thermostat = 7
    ctx = R.Context(0)
    with pytest.raises(R.RbsogError) as e:
        ctx.rbsog_set_system(p, torch.as_tensor(nacl512["types"], device=dev),
                             torch.as_tensor(nacl512["pos"], device=dev))
    assert e.value.code == -1
