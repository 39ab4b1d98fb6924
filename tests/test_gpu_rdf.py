"""Radial distribution counts (the pair histogram behind the RDF of Section
3.1) from the GPU lists against the oracle's brute force over all pairs:
integer counts, so bit-exact.  Also after steps (the lists of an earlier
build, positions moved within the skin), with species-dependent core
radii, on an orthorhombic box, and at 10^6 ions the symmetry of the ordered
pair counts; the memory form and bad arguments are refused."""
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


@pytest.mark.parametrize("name,over,r_max,n_bins", [
    ("nacl_512", {}, 10.0, 100),
    ("nacl_512", {}, 7.3, 47),
    ("nacl_512_lattice", {}, 9.9, 90),
    ("licl_8000", {}, 11.0, 110),
    ("licl_8000", dict(r_core_pair=[[4.5, 5.0, 6.0, 5.0], [5.0, 5.5, 6.2, 5.5], [6.0, 6.2, 6.5, 6.2],
                                    [5.0, 5.5, 6.2, 5.5]]), 11.0, 64),
])
def test_rdf_counts_match_oracle(name, over, r_max, n_bins):
    _say(f"case: rdf {name} {over} r_max {r_max} bins {n_bins}")
    if name == "licl_8000":
        cfg = _licl_small()
    elif name == "nacl_512_lattice":
        cfg = W.config("nacl_512", jitter=0.0)
    else:
        cfg = W.config(name)
    ctx, sysp = gpu_system(cfg, **over)
    g = ctx.rbsog_rdf_counts(r_max, n_bins)
    osys = O.System(sysp, cfg["types"], cfg["pos"], cfg["vel"])
    o = osys.rdf_counts(r_max, n_bins)
    _say(f"  pairs {int(g.sum())} (oracle {int(o.sum())})")
    assert g.sum() > 0
    assert np.array_equal(g, o)


def test_rdf_counts_after_steps_and_on_an_orthorhombic_box():
    """12 mixed-form steps of the 512-ion melt (the lists hold pairs of the
    last build): counts at the final positions equal the oracle's; then a
    101.25 x 22.5 x 45 A box (list grid split along x and z only)."""
    import torch
    _say("case: rdf after steps, orthorhombic box")
    cfg = W.config("nacl_512")
    ctx, sysp = gpu_system(cfg, R.MIXED)
    e = ctx.rbsog_step(12)
    pos, vel, _, _ = ctx.rbsog_get_state()
    g = ctx.rbsog_rdf_counts(10.0, 80)
    o = O.System(sysp, cfg["types"], pos.cpu().numpy(), vel.cpu().numpy()).rdf_counts(10.0, 80)
    _say(f"  after 12 steps ({e['n_builds']} builds): pairs {int(g.sum())}")
    assert np.array_equal(g, o)
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_gpu_boxes import _ortho_melt
    sysp, types, pos, vel = _ortho_melt()
    dev = torch.device("cuda", 0)
    ctx2 = R.Context(0)
    ctx2.rbsog_set_system(R.make_params(sysp, R.FP64, n_atoms=len(types)), torch.as_tensor(types, device=dev),
                          torch.as_tensor(pos, device=dev), torch.as_tensor(vel, device=dev))
    g2 = ctx2.rbsog_rdf_counts(9.5, 95)
    o2 = O.System(sysp, types, pos, vel).rdf_counts(9.5, 95)
    assert np.array_equal(g2, o2)


def test_rdf_counts_full_size_symmetric_and_refusals():
    """10^6 ions: each unordered pair is counted from both ends, so the
    counts of (a, b) equal those of (b, a) bin by bin; the memory form and
    bad arguments are refused."""
    _say("case: rdf full size licl_nacl_1m")
    cfg = W.config("licl_nacl_1m")
    ctx, sysp = gpu_system(cfg, R.MIXED)
    g = ctx.rbsog_rdf_counts(11.0, 128)
    assert g.sum() > 100 * len(cfg["types"])
    assert np.array_equal(g, g.transpose(1, 0, 2))
    for bad in ((11.5, 64), (0.0, 64), (5.0, 0), (5.0, 2000)):
        with pytest.raises(R.RbsogError) as err:
            ctx.rbsog_rdf_counts(*bad)
        assert err.value.code == -1
    small = W.config("nacl_512")
    st, _ = gpu_system(small, shell_stored=True)
    with pytest.raises(R.RbsogError) as err:
        st.rbsog_rdf_counts(10.0, 10)
    assert err.value.code == -2
