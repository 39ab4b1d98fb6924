"""Memory form of the random batch list on the GPU (RBSOG_FLAG_SHELL_STORED):
the shell batch of eq. (25) is drawn at the list build, stored as P_R
entries per atom and kept until the next build (Section 2.4 bounds the list
at O(core + P_R) entries per atom).  Parity with the oracle's reading of the
same form: stored batches bit-exact as atom ids, forces to the FP64 / mixed
bars, trajectories with rebuilds, batches of systems, and the number of
build chunks changing no bit."""
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return math.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300))


def gpu_system(cfg, precision=R.FP64, chunks=None, **over):
    import torch
    sysp = dict(cfg["sys"], shell_stored=True, **over)
    ctx = R.Context(0)
    if chunks is not None:
        ctx.rbsog_set_list_chunks(chunks)
    p = R.make_params(sysp, precision, n_atoms=len(cfg["types"]))
    dev = torch.device("cuda", 0)
    ctx.rbsog_set_system(p, torch.as_tensor(cfg["types"], device=dev), torch.as_tensor(cfg["pos"], device=dev),
                         torch.as_tensor(cfg["vel"], device=dev))
    return ctx, sysp


def oracle_system(cfg, sysp):
    return O.System(sysp, cfg["types"], cfg["pos"], cfg["vel"])


def check_batches(ctx, osys, atoms):
    """Stored batch of each atom = the oracle's candidates at its ranks."""
    nk_g, ids_g = ctx.rbsog_get_shell_batch()
    _, nk_o = osys.list_counts()
    assert np.array_equal(nk_g, nk_o)
    P = ids_g.shape[1]
    for i in atoms:
        _, cand = osys.lists_of(int(i))
        want = cand[osys.shell_ranks(int(i), 0)]
        cnt = min(len(cand), P)
        assert np.array_equal(ids_g[i, :cnt], want), int(i)
        assert (ids_g[i, cnt:] == -1).all()


@pytest.fixture(scope="module")
def nacl512():
    return W.config("nacl_512")


@pytest.mark.parametrize("precision,tol", [(R.FP64, TOL64), (R.MIXED, TOL32)])
def test_stored_forces_and_batches_nacl512(nacl512, precision, tol):
    _say(f"case: stored batch nacl_512 precision {precision}")
    ctx, sysp = gpu_system(nacl512, precision)
    osys = oracle_system(nacl512, sysp)
    f_prev = None
    for ev in (0, 3, 40):
        fg, eg = ctx.rbsog_compute_forces(ev)
        fs_g, _ = ctx.rbsog_get_force_parts()
        fo, eo = osys.forces(ev)
        fso, _, _ = osys.forces_short(ev)
        e_tot, m_tot = check_forces(fg.cpu().numpy(), fo, tol, f"total, eval {ev}")
        e_s, m_s = check_forces(fs_g.cpu().numpy(), fso, tol, f"short, eval {ev}")
        _say(f"  eval {ev}: total {e_tot:.2e} short {e_s:.2e}; worst atom / F_rms {m_tot:.2e} {m_s:.2e}")
        for key in ("u_core", "u_shell", "u_kspace"):
            assert eg[key] == pytest.approx(eo[key], rel=max(tol, 1e-12), abs=1e-9), key
        # the batch is that of the build: the short-range part does not move
        fs = fs_g.cpu().numpy()
        if f_prev is not None:
            assert np.array_equal(fs, f_prev)
        f_prev = fs
    assert osys.n_builds() == 1
    check_batches(ctx, osys, range(512))


def test_stored_batch_exports_and_errors(nacl512):
    _say("case: stored batch exports and errors")
    import torch
    ctx, sysp = gpu_system(nacl512)
    nc, nk = ctx.rbsog_get_list_counts()
    core, _ = ctx.rbsog_get_lists_of(5, nc[5], None)
    osys = oracle_system(nacl512, sysp)
    co, _ = osys.lists_of(5)
    assert np.array_equal(core, np.sort(co))
    with pytest.raises(R.RbsogError) as e:
        ctx.rbsog_get_lists_of(5, nc[5], nk[5])  # candidate rows are not kept
    assert e.value.code == -2
    with pytest.raises(R.RbsogError) as e:
        ctx.rbsog_get_shell_ranks(0)
    assert e.value.code == -2
    dev = torch.device("cuda", 0)
    t = torch.as_tensor(nacl512["types"], device=dev)
    x = torch.as_tensor(nacl512["pos"], device=dev)
    bad = R.Context(0)
    with pytest.raises(R.RbsogError) as e:
        bad.rbsog_set_system(R.make_params(dict(sysp, p_r=0), R.FP64, n_atoms=512), t, x)
    assert e.value.code == -1
    p = R.make_params(sysp, R.FP64, n_atoms=512)
    p.flags = 6
    with pytest.raises(R.RbsogError) as e:
        bad.rbsog_set_system(p, t, x)
    assert e.value.code == -1
    with pytest.raises(R.RbsogError) as e:
        bad.rbsog_set_list_chunks(0)
    assert e.value.code == -1
    plain = R.Context(0)
    plain.rbsog_set_system(R.make_params(nacl512["sys"], R.FP64, n_atoms=512), t, x)
    with pytest.raises(R.RbsogError) as e:
        plain.rbsog_get_shell_batch()
    assert e.value.code == -2
    # a batch must agree on the flag
    pl = [R.make_params(sysp, R.FP64, n_atoms=512), R.make_params(nacl512["sys"], R.FP64, n_atoms=512)]
    with pytest.raises(R.RbsogError) as e:
        bad.rbsog_set_batch(pl, torch.cat([t, t]), torch.cat([x, x]))
    assert e.value.code == -1


@pytest.mark.parametrize("precision,tol", [(R.FP64, TOL64), (R.MIXED, TOL32)])
def test_stored_chunks_change_no_bit_nacl32768(precision, tol):
    """32768 ions (729 list cells): 1, 3, 8 and 64 build chunks give the same
    batches and the same force bits; sampled batches match the oracle."""
    _say(f"case: stored batch chunks nacl_32768 precision {precision}")
    cfg = W.config("nacl_32768")
    ref = None
    for K in (8, 1, 3, 64):
        ctx, sysp = gpu_system(cfg, precision, chunks=K)
        fg, _ = ctx.rbsog_compute_forces(2, want_energy=False)
        nk, ids = ctx.rbsog_get_shell_batch()
        got = (fg.cpu().numpy(), nk, ids)
        if ref is None:
            ref = got
            osys = oracle_system(cfg, sysp)
            rng = np.random.default_rng(11)
            check_batches(ctx, osys, rng.choice(len(cfg["types"]), 60, replace=False))
            fo, _ = osys.forces(2)
            e, m = check_forces(got[0], fo, tol, f"chunks {K}")
            _say(f"  chunks {K}: force rel rms {e:.2e}, worst atom {m:.2e} F_rms")
        else:
            _say(f"  chunks {K}: compared bitwise")
            assert all(np.array_equal(a, b) for a, b in zip(got, ref)), K


def test_stored_velocity_verlet_with_rebuilds_matches_oracle(nacl512):
    """15 steps with skin 0.2 A (rebuilds when an ion moved more than skin/2)
    and a scheduled rebuild every 4 steps: each build draws its batch from
    its own stream, on both sides."""
    _say("case: stored batch vv 15 steps nacl_512")
    ctx, sysp = gpu_system(nacl512, skin=0.2, rebuild_every=4)
    osys = oracle_system(nacl512, sysp)
    ctx.rbsog_compute_forces(0, want_energy=False)
    osys.forces(0)
    eg = ctx.rbsog_step(15)
    eo = osys.vv_steps(15)
    assert eg["n_builds"] == osys.n_builds() >= 4
    pg, vg, fg, _ = ctx.rbsog_get_state()
    po, vo, fo, _ = osys.state()
    L = np.array(sysp["box"])
    d = pg.cpu().numpy() - po
    d -= L * np.rint(d / L)
    assert np.abs(d).max() < 1e-9
    assert rel_rms(vg.cpu().numpy(), vo) < 1e-9
    assert rel_rms(fg.cpu().numpy(), fo) < 1e-9
    assert eg["u_total"] == pytest.approx(eo["u_total"], rel=1e-9)
    check_batches(ctx, osys, range(0, 512, 5))


def test_stored_batch_of_systems_equals_singles():
    """Four NaCl systems of different sizes in one context (graphs on) step
    exactly as each alone."""
    import torch
    _say("case: stored batch of 4 systems")
    dev = torch.device("cuda", 0)
    cfgs = [W.config("nacl_512"), W.config("nacl_32768"),
            W.config("nacl_512", melt_seed=5), W.config("nacl_small")]
    plist, types, pos, vel = [], [], [], []
    for r, c in enumerate(cfgs):
        sp = dict(c["sys"], shell_stored=True, replica=r, skin=0.5, rebuild_every=3)
        plist.append(R.make_params(sp, R.MIXED, n_atoms=len(c["types"])))
        types.append(c["types"])
        pos.append(c["pos"])
        vel.append(c["vel"])
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = R.Context(0, stream=st)
        ctx.rbsog_set_batch(plist, torch.as_tensor(np.concatenate(types), device=dev),
                            torch.as_tensor(np.concatenate(pos), device=dev),
                            torch.as_tensor(np.concatenate(vel), device=dev))
        ctx.rbsog_use_graphs(True)
        eb = ctx.rbsog_step(7)
        pb, vb, fb, _ = ctx.rbsog_get_state()
    off = 0
    for r, c in enumerate(cfgs):
        n = len(c["types"])
        one = R.Context(0)
        one.rbsog_set_system(plist[r], torch.as_tensor(c["types"], device=dev), torch.as_tensor(c["pos"], device=dev),
                             torch.as_tensor(c["vel"], device=dev))
        e1 = one.rbsog_step(7)
        p1, v1, f1, _ = one.rbsog_get_state()
        assert np.array_equal(pb.cpu().numpy()[off:off + n], p1.cpu().numpy()), r
        assert np.array_equal(fb.cpu().numpy()[off:off + n], f1.cpu().numpy()), r
        assert eb[r]["n_builds"] == e1["n_builds"] >= 2
        assert eb[r]["u_total"] == e1["u_total"]
        off += n


def test_stored_full_size_sampled_batches():
    """The 10^6-ion four-species workload at full size in the stored form (8
    build chunks): the batch drawn at build 0 for 40 random ions, as ids in
    ascending rank order, equals the oracle's candidates (found by a scan
    over all ions) at its ranks of build 0, and the candidate counts agree."""
    _say("case: stored full size batches licl_nacl_1m")
    cfg = W.config("licl_nacl_1m")
    n = len(cfg["types"])
    ctx, sysp = gpu_system(cfg, R.MIXED)
    osys = oracle_system(cfg, sysp)
    nk_g, ids_g = ctx.rbsog_get_shell_batch()
    P = ids_g.shape[1]
    for i in np.random.default_rng(13).choice(n, 40, replace=False):
        i = int(i)
        _, ko = osys.scan_lists_of(i)
        assert nk_g[i] == len(ko), i
        want = ko[osys.shell_ranks_count(i, len(ko), 0)]
        cnt = min(len(ko), P)
        assert np.array_equal(ids_g[i, :cnt], want), i
        assert (ids_g[i, cnt:] == -1).all()
    ctx.close()


@pytest.mark.parametrize("precision,tol", [(R.MIXED, TOL32), (R.FP64, TOL64)])
def test_stored_full_size_sampled_atoms(precision, tol):
    """The 10^6-ion four-species workload at full size in the stored form
    (8 build chunks): the short-range force of 300 sampled ions against the
    oracle computing them one by one with the batch of build 0."""
    _say(f"case: stored full size licl_nacl_1m precision {precision}")
    cfg = W.config("licl_nacl_1m")
    sysp = dict(cfg["sys"], shell_stored=True)
    osys = oracle_system(cfg, sysp)
    sel = np.sort(np.random.default_rng(7).choice(len(cfg["types"]), 300, replace=False)).astype(np.int32)
    fs_o = osys.forces_short_atoms(2, sel)
    ctx, _ = gpu_system(cfg, precision)
    ctx.rbsog_compute_forces(2, want_energy=False)
    fs_g, _ = ctx.rbsog_get_force_parts()
    e_s, m_s = check_forces(fs_g.cpu().numpy()[sel], fs_o, tol, "short, sampled atoms")
    _say(f"  sampled atoms: short {e_s:.2e}, worst atom {m_s:.2e} F_rms")
