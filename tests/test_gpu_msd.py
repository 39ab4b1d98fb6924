"""Mean-square displacement (the MSD of Section 3.1) kept on the GPU from a
marked origin, against the oracle's trajectory unwrapped here with numpy
(the minimum image of each increment between samples, summed), per
species; a batch keeps each system's own origin; refusals."""
from __future__ import annotations

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


def _gpu(cfg, precision=R.FP64, **over):
    import torch
    sysp = dict(cfg["sys"], **over)
    ctx = R.Context(0)
    dev = torch.device("cuda", 0)
    ctx.rbsog_set_system(R.make_params(sysp, precision, n_atoms=len(cfg["types"])),
                         torch.as_tensor(cfg["types"], device=dev), torch.as_tensor(cfg["pos"], device=dev),
                         torch.as_tensor(cfg["vel"], device=dev))
    return ctx, sysp


def _unwrapped_msd(samples, types, L, S):
    D = np.zeros_like(samples[0])
    for a, b in zip(samples[:-1], samples[1:]):
        d = b - a
        d -= L * np.rint(d / L)
        D += d
    q = (D ** 2).sum(1)
    return np.array([q[types == s].mean() if (types == s).any() else 0.0 for s in range(S)])


@pytest.mark.parametrize("name", ["nacl_small", "nacl_512"])
def test_msd_matches_unwrapped_oracle_trajectory(name):
    """30 FP64 steps in blocks of 5 (ions cross the periodic boundary on
    the way): the GPU's per-species MSD after each block equals that of the
    oracle's positions unwrapped with numpy, to 1e-8 relative."""
    _say(f"case: msd {name}")
    cfg = W.config(name)
    ctx, sysp = _gpu(cfg)
    osys = O.System(sysp, cfg["types"], cfg["pos"], cfg["vel"])
    osys.forces(0)
    L = np.array(sysp["box"])
    S = len(sysp["species"]["q"])
    assert np.array_equal(ctx.rbsog_msd(mark=True), np.zeros(S))
    samples = [np.array(cfg["pos"], dtype=float) % L]
    for blk in range(6):
        ctx.rbsog_step(5)
        g = ctx.rbsog_msd()
        osys.vv_steps(5)
        samples.append(osys.state()[0])
        o = _unwrapped_msd(samples, cfg["types"], L, S)
        _say(f"  after {5 * (blk + 1)} steps: msd {g} (oracle {o})")
        assert np.all(g > 0)
        assert np.allclose(g, o, rtol=1e-8, atol=0.0)


def test_msd_in_a_batch_and_refusals():
    """Two systems of a batch keep their own origins (marked at different
    times); without a mark the call is refused."""
    import torch
    _say("case: msd batch")
    cfgs = [W.config("nacl_512"), W.config("nacl_small")]
    dev = torch.device("cuda", 0)
    plist = [R.make_params(dict(c["sys"], replica=r), R.FP64, n_atoms=len(c["types"])) for r, c in enumerate(cfgs)]
    ctx = R.Context(0)
    ctx.rbsog_set_batch(plist, torch.as_tensor(np.concatenate([c["types"] for c in cfgs]), device=dev),
                        torch.as_tensor(np.concatenate([c["pos"] for c in cfgs]), device=dev),
                        torch.as_tensor(np.concatenate([c["vel"] for c in cfgs]), device=dev))
    ctx.rbsog_select_system(1)
    with pytest.raises(R.RbsogError) as err:
        ctx.rbsog_msd()
    assert err.value.code == -2
    ctx.rbsog_select_system(0)
    ctx.rbsog_msd(mark=True)
    ctx.rbsog_step(4)
    ctx.rbsog_select_system(1)
    ctx.rbsog_msd(mark=True)
    ctx.rbsog_step(4)
    m1 = ctx.rbsog_msd()
    ctx.rbsog_select_system(0)
    m0 = ctx.rbsog_msd()
    # system 0 has moved for 8 steps, system 1 for 4: alone, each matches
    for r, (c, steps, m) in enumerate(zip(cfgs, (8, 4), (m0, m1))):
        one, _ = _gpu(c, replica=r)
        if steps == 4:
            one.rbsog_step(4)
        one.rbsog_msd(mark=True)
        one.rbsog_step(steps)
        assert np.array_equal(one.rbsog_msd(), m), r
