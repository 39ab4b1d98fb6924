#!/usr/bin/env python3
"""Throughput of the IRBSOG step (force evaluation + velocity Verlet) on one GPU.

Workload (default): 50:50 LiCl-NaCl melt, N = 10^6 ions, L = 329 A, 1150 K,
r_core 5.5 A, r_shell 11 A, skin 1 A, P_R = 30, P_F = 500, lists rebuilt every
10 steps (earlier if an ion moved more than skin/2), synthetic rock-salt start
with jitter, Berendsen thermostat at 1150 K with tau = dt.  Both precision forms run:
FP32-mixed (the reported value) and plain FP64 (reported beside it).

A 5e6-ion NaCl melt (P_R 20, P_F 1000, mixed) runs after it, with the device
memory the library holds.  The batched form runs beside it: 64 molten-NaCl replicas of 566..32742 ions
(600664 in all) in one context, FP32-mixed, launch shapes autotuned, each step
replayed from a captured HIP graph; its aggregate atom-steps/s is reported
against the same replicas stepped one after another, each in its own context
with plain launches.

Prints one JSON line.  Each leg's rate is the median of `--repeats` timed
runs of `--steps` steps, and each leg states its FP32-mixed force error
against the FP64 path at its starting positions.  The roofline object
describes the dominant kernel of the reported form, timed with HIP events on
the library's stream during the timed steps, against per-form work models
(FP64 and FP32 flops separately, FP32 transcendentals, algorithmic HBM
bytes) stated below; where the committed counter summaries in profiles/ were
taken on the current kernel source, the measured VALU instruction mix and
HBM bytes stand beside the models.  The CPU baseline is the FP64 oracle on
a bounded sample of the same workload, plus direct timings of the 512- and
32768-ion melts at one thread and at all host threads.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz; the same
# rate holds for FP64 and for non-packed FP32 (packed FP32 is not used).
PEAK_VALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# VALU issue: one wave64 instruction per SIMD every 4 cycles, i.e. 256 x 4 x
# 16 lane-instructions per cycle at 2.4 GHz; an FP32 transcendental
# (v_exp, v_rsq, v_sin, v_cos) takes two of those slots: on this GPU a
# throughput probe (independent chains, all SIMDs busy) issues v_sin_f32 at
# 9.0 and v_exp_f32 at 8.3 cycles per wavefront instruction against 4.9 for
# v_fma_f64.
PEAK_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9
TRANS_SLOTS = 2

# Work models, FMA = 2 flops, a transcendental = 1 flop (and 4 issue slots).
# k-space kernels, per (atom, mode):
#   FP64 rho:     phase 5 (mul + 2 FMA), table sincos 18, accumulation 4       FP64 27
#   FP64 force:   phase 5, sincos 18, Im(e^{-i theta} rho) coef 3, sum 6       FP64 32
#   mixed rho:    phase 5, accumulation of four atoms' FP32 sums 0.5           FP64 5.5
#                 q cos, q sin (2 FMA), hardware sin + cos (2 transcendentals)  FP32 6
#   mixed force:  phase 5, sum of w m_a (3 FMA)                                FP64 11
#                 c A - s B (FMA + mul), sin + cos                             FP32 5
# pair kernel, per distance test (every core-list entry and every batch
# entry): FP64 form three differences and r^2 (8), the minimum image (9) in
# the wavefronts that touch the box edge (a quarter at the 10^6-ion size), so
# 10.25 FP64; mixed form the three scaled differences of 32-bit fixed-point
# records (integer subtractions, then 3 FP64 products) and r^2, 8 FP64;
# per evaluated pair: FP64 form 181 for the pair function (two
# software exponentials, the squaring chain of the narrow Gaussians, the
# 13-term polynomial of the wide ones, BMH terms) plus 6 to accumulate F;
# mixed form 40 FP32 for the table-driven pair function as compiled (rsqrt
# and two exponentials among them: 3 transcendentals) plus 6 FP64 to
# accumulate.  These per-pair constants were checked against the counted
# SQ_INSTS_VALU_FLOPS_FP64/FP32 of the kernels (within 15 %).
KSPACE_MODEL = {
    ("fp64", "rho"): (27.0, 0.0, 0.0), ("fp64", "kforce"): (32.0, 0.0, 0.0),
    ("mixed", "rho"): (5.5, 6.0, 2.0), ("mixed", "kforce"): (11.0, 5.0, 2.0),
}  # (FP64 flops, FP32 flops, FP32 transcendentals) per (atom, mode)
PAIR_MODEL = {
    "fp64": {"fp64_test": 10.25, "fp64_pair": 187.0, "fp32_pair": 0.0, "trans_pair": 0.0},
    "mixed": {"fp64_test": 8.0, "fp64_pair": 6.0, "fp32_pair": 40.0, "trans_pair": 3.0},
}


def _log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


TUNING_KEYS = ("pair_block", "pair_ku", "rho_mpl", "kf_block", "kf_aux")


def _force_err(a, b) -> dict:
    """FP32-mixed force a against the FP64 force b: relative RMS and the
    largest single-atom error in units of the RMS force."""
    d2 = ((a - b) ** 2).sum(1)
    f2 = (b ** 2).sum(1)
    return {"rel_rms": float(np.sqrt(d2.sum() / f2.sum())),
            "max_atom_over_f_rms": float(np.sqrt(d2.max() / f2.mean()))}


def form_error(cfg, mixed_only=None, **over) -> dict:
    """Both forms evaluate the force once (eval 0) at the workload's starting
    positions; the FP64 path is the reference (it matches the oracle to
    1e-11).  mixed_only: parameters set for the mixed form alone."""
    import torch
    from paper_2512_24970_amd import rbsog as R
    dev = torch.device("cuda", 0)
    sysp = dict(cfg["sys"], **over)
    out = {}
    for prec in (R.FP64, R.MIXED):
        ctx = R.Context(0)
        sp = dict(sysp, **(mixed_only or {})) if prec == R.MIXED else sysp
        ctx.rbsog_set_system(R.make_params(sp, prec, n_atoms=len(cfg["types"])),
                             torch.as_tensor(cfg["types"], device=dev), torch.as_tensor(cfg["pos"], device=dev),
                             torch.as_tensor(cfg["vel"], device=dev))
        f, _ = ctx.rbsog_compute_forces(0, want_energy=False)
        out[prec] = f.cpu().numpy()
        ctx.close()
        del f
    torch.cuda.empty_cache()
    return dict(_force_err(out[R.MIXED], out[R.FP64]), reference="fp64 path, eval 0, starting positions")


def batch_form_error(cfgs) -> dict:
    """form_error for a batch: both forms on the whole batch, the worst replica."""
    import torch
    from paper_2512_24970_amd import rbsog as R
    dev = torch.device("cuda", 0)
    out = {}
    for prec in (R.FP64, R.MIXED):
        ctx = R.Context(0)
        ctx.rbsog_set_batch([R.make_params(c["sys"], prec, n_atoms=len(c["types"])) for c in cfgs],
                            *_batch_inputs(cfgs, dev))
        f, _ = ctx.rbsog_compute_forces(0, want_energy=False)
        out[prec] = f.cpu().numpy()
        ctx.close()
    offs = np.cumsum([0] + [len(c["types"]) for c in cfgs])
    per = [_force_err(out[R.MIXED][a:b], out[R.FP64][a:b]) for a, b in zip(offs[:-1], offs[1:])]
    return dict(_force_err(out[R.MIXED], out[R.FP64]),
                worst_replica_rel_rms=max(x["rel_rms"] for x in per),
                reference="fp64 path, eval 0, starting positions")


def run_gpu(cfg, precision: str, steps: int, warmup: int, tuning: str = "auto", thermostat: str = "berendsen",
            tau: float | None = None, repeats: int = 5):
    import torch
    from paper_2512_24970_amd import rbsog as R
    dev = torch.device("cuda", 0)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info(dev)[0]
    ctx = R.Context(0)
    prec = R.MIXED if precision == "mixed" else R.FP64
    # the estimator's noise heats an NVE run at this size by several per cent
    # per step; the paper runs NVT, here a Berendsen thermostat with tau = dt
    sysp = dict(cfg["sys"], t_target=cfg["T"], tau_t=cfg["sys"]["dt"] if tau is None else tau,
                thermostat=thermostat)
    if precision != "mixed":
        sysp.pop("int_phase", None)  # an option of the mixed form
    p = R.make_params(sysp, prec, n_atoms=len(cfg["types"]))
    ctx.rbsog_set_system(p, torch.as_tensor(cfg["types"], device=dev), torch.as_tensor(cfg["pos"], device=dev),
                         torch.as_tensor(cfg["vel"], device=dev))
    if tuning == "auto":
        tuning = ctx.rbsog_autotune(3)
    else:
        ctx.rbsog_set_tuning(**dict(zip(TUNING_KEYS, (int(v) for v in tuning.split(",")))))
        tuning = ctx.rbsog_get_tuning()
    _log(f"[bench] {precision}: system set, tuning {tuning}, warmup {warmup} steps")
    f0, _ = ctx.rbsog_compute_forces(0, want_energy=False)
    f0 = f0.cpu().numpy()
    e0 = ctx.rbsog_step(warmup) if warmup > 0 else None
    # the timed steps bracket only the hot kernels with events (their live
    # durations give the roofline); every phase is timed on a short extra
    # run, since events around each phase cost a few per cent of a step
    ctx.rbsog_profile_read()
    ctx.rbsog_profile_enable(2)
    runs = []
    for _ in range(max(1, repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e1 = ctx.rbsog_step(steps)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    prof = ctx.rbsog_profile_read()
    phase_steps = min(steps, 30)
    ctx.rbsog_profile_enable(1)
    ctx.rbsog_step(phase_steps)
    prof_all = ctx.rbsog_profile_read()
    ctx.rbsog_profile_enable(False)
    # device memory held for the system: everything the library allocated
    # (torch's own cache emptied first)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    mem_gb = (free0 - torch.cuda.mem_get_info(dev)[0]) / 1e9
    n = len(cfg["types"])
    dt = float(np.median(runs))
    _log(f"[bench] {precision}: median of {len(runs)} x {steps} steps {dt:.3f} s -> {n * steps / dt:.4g} atom-steps/s")
    ctx.close()
    T = 2 * e1["kinetic"] / ((3 * n - 3) * 8.617333262e-5)
    return {"seconds": dt, "value": n * steps / dt, "ms_per_step": 1e3 * dt / steps, "phases": prof,
            "runs_ms_per_step": [round(1e3 * t / steps, 4) for t in runs],
            "phases_all": prof_all, "phase_steps": phase_steps,
            "energy": e1, "energy_warm": e0, "T_end": T, "force0": f0, "tuning": tuning,
            "device_mem_GB": round(mem_gb, 3)}


def _batch_inputs(cfgs, dev):
    import torch
    cat = lambda k: torch.as_tensor(np.concatenate([c[k] for c in cfgs]), device=dev)
    return cat("types"), cat("pos"), cat("vel")


def run_batch(n_rep: int, steps: int, warmup: int, repeats: int = 5):
    """Aggregate throughput of the batched form, and of the same replicas run
    one after another (own context each, plain launches)."""
    import torch
    from paper_2512_24970_amd import rbsog as R
    from paper_2512_24970_amd import workloads as W
    dev = torch.device("cuda", 0)
    cfgs = W.replica_batch(n_rep=n_rep)
    for c in cfgs:
        c["sys"] = dict(c["sys"], t_target=c["T"], tau_t=c["sys"]["dt"])
    n_tot = sum(len(c["types"]) for c in cfgs)
    stream = torch.cuda.Stream(device=dev)
    ctx = R.Context(0, stream=stream)
    plist = [R.make_params(c["sys"], R.MIXED, n_atoms=len(c["types"])) for c in cfgs]
    ctx.rbsog_set_batch(plist, *_batch_inputs(cfgs, dev))
    tuning = ctx.rbsog_autotune(3)
    ctx.rbsog_use_graphs(True)
    _log(f"[bench] batch: {n_rep} replicas, {n_tot} ions, tuning {tuning}; warmup {warmup} steps")
    ctx.rbsog_step(warmup)
    runs = []
    for _ in range(max(1, repeats)):
        stream.synchronize()
        t0 = time.perf_counter()
        e = ctx.rbsog_step(steps)
        stream.synchronize()
        runs.append(time.perf_counter() - t0)
    dt_b = float(np.median(runs))
    # kernel phases of the batched step (kernel by kernel while timed)
    ctx.rbsog_profile_read()
    ctx.rbsog_profile_enable(True)
    ctx.rbsog_step(10)
    prof = ctx.rbsog_profile_read()
    ctx.rbsog_profile_enable(False)
    ctx.close()
    _log(f"[bench] batch: {steps} steps in {dt_b:.3f} s -> {n_tot * steps / dt_b:.4g} atom-steps/s")
    # the same replicas, one context each, stepped one after another
    ctxs = []
    for c in cfgs:
        x = R.Context(0)
        x.rbsog_set_system(R.make_params(c["sys"], R.MIXED, n_atoms=len(c["types"])), *_batch_inputs([c], dev))
        x.rbsog_step(warmup, want_energy=False)
        ctxs.append(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x in ctxs:
        x.rbsog_step(steps, want_energy=False)
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    for x in ctxs:
        x.close()
    _log(f"[bench] sequential: {steps} steps x {n_rep} contexts in {dt_s:.3f} s -> "
         f"{n_tot * steps / dt_s:.4g} atom-steps/s")
    T = [2 * x["kinetic"] / ((3 * len(c["types"]) - 3) * 8.617333262e-5) for x, c in zip(e, cfgs)]
    err = batch_form_error(cfgs)
    return {
        "workload": f"nacl_replicas{n_rep}", "n_systems": n_rep, "n_atoms": n_tot,
        "mixed_vs_fp64_force": err,
        "runs_ms_per_step": [round(1e3 * t / steps, 4) for t in runs],
        "sizes": [int(len(c["types"])) for c in cfgs][:8] + ["..."],
        "form": "mixed", "value": n_tot * steps / dt_b, "unit": "atom-steps/s",
        "ms_per_step": 1e3 * dt_b / steps, "graph": True, "tuning": tuning,
        "sequential_value": n_tot * steps / dt_s, "sequential_ms_per_step": 1e3 * dt_s / steps,
        "speedup_vs_sequential": dt_s / dt_b,
        "phases_ms_per_step": {k: round(v[0] / 10, 4) for k, v in prof.items()},
        "T_end_K_range": [round(min(T), 1), round(max(T), 1)],
    }


KERNEL_OF_PHASE = {"pair": "k_pair", "rho": "k_rho", "kforce": "k_kforce"}


def phase_ms(res) -> dict:
    """Milliseconds per step of every phase, from the short all-phase run."""
    return {k: round(v[0] / res["phase_steps"], 4) for k, v in res["phases_all"].items()}


def pair_counts(sysp: dict, n: int) -> dict:
    """Per atom at the workload's density: distance tests (core-list entries
    plus batch entries) and evaluated pairs (inside r_core, plus the batch
    entries inside [r_core, r_shell))."""
    L = sysp["box"]
    rho_n = n / (L[0] * L[1] * L[2])
    rc, rs, sk, pr = sysp["r_core"], sysp["r_shell"], sysp["skin"], sysp["p_r"]
    v = lambda r: 4.0 / 3.0 * math.pi * r ** 3
    core_list = v(rc + sk) * rho_n
    core = v(rc) * rho_n
    cand = (v(rs + sk) - v(max(rc - sk, 0.0))) * rho_n
    valid = (v(rs) - v(rc)) * rho_n / cand
    batch = min(pr, cand) if pr > 0 else cand
    return {"core_list": core_list, "batch": batch, "tests": core_list + batch, "pairs": core + valid * batch}


def kernel_work(precision: str, phase: str, n: int, sysp: dict) -> dict:
    """Model work of one launch: FP64 flops, FP32 flops, FP32 transcendentals,
    algorithmic HBM bytes (each input read once, each output written once)."""
    if phase == "pair":
        c = pair_counts(sysp, n)
        m = PAIR_MODEL[precision]
        f64 = n * (c["tests"] * m["fp64_test"] + c["pairs"] * m["fp64_pair"])
        f32 = n * c["pairs"] * m["fp32_pair"]
        tr = n * c["pairs"] * m["trans_pair"]
        # own position record (FP64 32 B; the mixed form's fixed-point record
        # 16 B), list counts 8 B, core-list entries, one candidate index per
        # batch entry, short-range force 24 B
        rec = 16 if precision == "mixed" else 32
        hbm = n * (rec + 8 + 4 * c["core_list"] + 4 * c["batch"] + 24)
    else:
        am = float(n) * float(sysp["p_f"])
        a, b, t = KSPACE_MODEL[(precision, phase)]
        f64, f32, tr = am * a, am * b, am * t
        # positions once; the force kernel also writes the k-space force
        hbm = n * (32 + (24 if phase == "kforce" else 0))
    return {"fp64_flops": f64, "fp32_flops": f32, "trans": tr, "hbm_bytes": hbm}


def _profile_json(workload: str, tag: str):
    """The `<tag>_json:` line of profiles/<workload>_*.md taken on the current
    kernel source (else None)."""
    import hashlib
    src = os.path.join(HERE, "paper_2512_24970_amd", "csrc", "kernels.hip")
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    name = {"traffic": "traffic", "counters": "sq_counters"}[tag]
    path = os.path.join(HERE, "profiles", f"{workload}_{name}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith(f"{tag}_json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("source_sha1") == sha:
                return d
    return None


def kernel_roofline(precision: str, phase: str, ms: float, launches: int, n: int, sysp: dict,
                    workload: str) -> dict:
    avg = ms / launches * 1e-3
    w = kernel_work(precision, phase, n, sysp)
    flops = w["fp64_flops"] + w["fp32_flops"]
    ach = flops / avg / 1e12
    kern = KERNEL_OF_PHASE[phase]
    key = f"{kern}<{precision}>"
    out = {"bound": "alu", "kernel": kern, "achieved": round(ach, 3), "peak": PEAK_VALU_TFLOPS,
           "unit": "TFLOP/s", "frac": round(ach / PEAK_VALU_TFLOPS, 4), "traffic": None,
           "avg_launch_ms": round(ms / launches, 4), "launches": launches,
           "model": {"fp64_flops_per_launch": w["fp64_flops"], "fp32_flops_per_launch": w["fp32_flops"],
                     "fp64_tflops": round(w["fp64_flops"] / avg / 1e12, 3),
                     "fp32_tflops": round(w["fp32_flops"] / avg / 1e12, 3),
                     "fp32_trans_per_launch": w["trans"],
                     "fp32_trans_per_s": round(w["trans"] / avg, 1),
                     "hbm_bytes_per_launch": w["hbm_bytes"],
                     "hbm_GBps": round(w["hbm_bytes"] / avg / 1e9, 1)}}
    cnt = _profile_json(workload, "counters")
    if cnt and key in cnt.get("per_launch", {}):
        c = cnt["per_launch"][key]
        # VALU issue: lane-instructions, a transcendental taking two slots
        slots = c["valu_lane_instr"] + (TRANS_SLOTS - 1) * c["trans_lane_instr"]
        out["counted"] = {"fp64_flops_per_launch": c["fp64_flops"], "fp32_flops_per_launch": c["fp32_flops"],
                          "valu_lane_instr_per_launch": c["valu_lane_instr"],
                          "fp32_trans_lane_instr_per_launch": c["trans_lane_instr"],
                          "valu_issue_frac": round(slots / avg / PEAK_LANE_INSTR_PER_S, 4),
                          "flops_frac": round((c["fp64_flops"] + c["fp32_flops"]) / avg / 1e12
                                              / PEAK_VALU_TFLOPS, 4),
                          "model_over_counted_flops": round(flops / max(c["fp64_flops"] + c["fp32_flops"], 1), 3)}
        if "td_busy" in c:
            # the vector-memory path: L1 accesses (one per lane and cache
            # line of a load) and how busy the texture address and data
            # units were while the kernel ran alone
            out["counted"].update({"l1_accesses_per_launch": c["l1_accesses"],
                                   "l1_accesses_per_atom": round(c["l1_accesses"] / n, 2),
                                   "ta_busy_frac": c["ta_busy"], "td_busy_frac": c["td_busy"]})
    tr = _profile_json(workload, "traffic")
    if tr and key in tr.get("bytes_per_launch", {}):
        b = tr["bytes_per_launch"][key]
        out["traffic"] = b
        out["traffic_GBps"] = round(b / avg / 1e9, 1)
        out["traffic_frac_of_hbm_peak"] = round(b / avg / 1e9 / PEAK_HBM_GBS, 4)
        out["traffic_over_algorithmic"] = round(b / max(w["hbm_bytes"], 1), 3)
    return out


def roofline(precision: str, res: dict, n: int, sysp: dict, workload: str) -> dict:
    """The dominant kernel (largest time in the timed steps) and the others."""
    phases = {k: v for k, v in res["phases"].items() if k in KERNEL_OF_PHASE and v[1] > 0}
    lines = {k: kernel_roofline(precision, k, v[0], v[1], n, sysp, workload) for k, v in phases.items()}
    top = max(phases, key=lambda k: phases[k][0])
    out = dict(lines[top])
    out["others"] = {lines[k]["kernel"]: {key: lines[k][key] for key in
                                          ("achieved", "frac", "avg_launch_ms", "model", "counted", "traffic")
                                          if key in lines[k]}
                     for k in lines if k != top}
    # the k-space chain runs on a second stream beside the pair kernel, so
    # their launch durations overlap and each includes the other's share
    out["concurrent"] = "k_pair runs beside k_ksample + k_rho + k_kforce (second stream); durations overlap"
    return out


def apriori_model(sysp: dict, n: int, precision: str) -> dict:
    """The a-priori work model per atom-step this path was planned with:
    pairs x (~30 FP64 flops, 12 transcendentals) + 2 P_F x (~12 FP64 flops,
    2 transcendentals) in the mixed form; pairs x (60 + 12 x 50) + 2 P_F x
    (12 + 100) FP64 flops in the FP64 form (software exp and sincos counted
    as 25 FMAs); HBM bytes: positions read three times, type, velocity read
    and written, force and position written, the core list, P_R batch
    indices."""
    c = pair_counts(sysp, n)
    pf = float(sysp["p_f"])
    if precision == "mixed":
        f64 = c["pairs"] * 30 + 2 * pf * 12
        tr = c["pairs"] * 12 + 2 * pf * 2
    else:
        f64 = c["pairs"] * (60 + 12 * 50) + 2 * pf * (12 + 100)
        tr = 0.0
    hbm = 72 + 1 + 48 + 24 + 24 + 4 * c["core_list"] + 4 * c["batch"]
    return {"fp64_flops_per_atom_step": round(f64, 1), "fp32_trans_per_atom_step": round(tr, 1),
            "hbm_bytes_per_atom_step": round(hbm, 1)}


def copy_probe(nbytes: int, reps: int = 5) -> None:
    """A plain device copy of known size, to calibrate the HBM byte counters."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}))


def cpu_baseline(cfg, n_sample: int, ev: int = 1):
    """The oracle on a bounded sample of the workload: rho(k) over every atom
    (eq. 22), then the short-range (O(N) scan + batch) and k-space forces of
    n_sample atoms; one step's time is extrapolated as
    T_rho + (N / n_sample) (T_short + T_kforce)."""
    import oracle as O
    O.build(force=False)
    sysp = cfg["sys"]
    s = O.System(sysp, cfg["types"], cfg["pos"], cfg["vel"])
    n = len(cfg["types"])
    rng = np.random.default_rng(11)
    sel = np.sort(rng.choice(n, size=n_sample, replace=False)).astype(np.int32)
    m, S = O.kmodes(s.params, ev)
    t0 = time.perf_counter()
    rho = s.rho(m)
    t1 = time.perf_counter()
    s.forces_short_atoms(ev, sel)
    t2 = time.perf_counter()
    V = float(np.prod(sysp["box"]))
    s.kforce_atoms(m, rho, S / (len(m) * V), sel)
    t3 = time.perf_counter()
    t_step = (t1 - t0) + n / n_sample * ((t2 - t1) + (t3 - t2))
    threads = O.get_threads()
    s.close()
    return {"value": n / t_step, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle, rho(k) of all {n} atoms for {len(m)} modes ({t1 - t0:.2f} s) + short-range "
                       f"and k-space force of {n_sample} random atoms ({t3 - t1:.2f} s); an extrapolation to one "
                       f"step of all atoms, dominated by the oracle's brute-force O(N) neighbour search per atom, "
                       f"which the method amortises over list builds"),
            "extrapolated": True, "seconds_measured": round(t3 - t0, 3)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_direct(steps: int = 10) -> dict:
    """The oracle's full step timed directly on the 512- and 32768-ion melts
    (Table 1 NaCl, P_R 20, P_F 100 / 200), at one thread and at all host
    threads: the first force evaluation (which builds the lists by brute
    force), then `steps` velocity-Verlet steps (one rebuild period)."""
    import oracle as O
    from paper_2512_24970_amd import workloads as W
    O.build(force=False)
    all_threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    out = {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "threads_available": all_threads, "runs": []}
    for name in ("nacl_512", "nacl_32768"):
        cfg = W.config(name)
        n = len(cfg["types"])
        for th in (1, all_threads):
            O.set_threads(th)
            s = O.System(cfg["sys"], cfg["types"], cfg["pos"], cfg["vel"])
            t0 = time.perf_counter()
            s.forces(0)
            t1 = time.perf_counter()
            s.vv_steps(steps)
            t2 = time.perf_counter()
            s.close()
            per = (t2 - t1) / steps
            out["runs"].append({"workload": name, "n_atoms": n, "threads": th, "first_force_s": round(t1 - t0, 4),
                                "steps": steps, "s_per_step": round(per, 5), "atom_steps_per_s": round(n / per, 1)})
            _log(f"[bench] cpu oracle {name} threads {th}: {per:.4f} s/step")
    O.set_threads(0)
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="licl_nacl_1m")
    ap.add_argument("--forms", default="mixed,fp64", help="comma list of mixed,fp64; the first is reported")
    ap.add_argument("--cpu-sample", type=int, default=20000, help="atoms in the CPU-baseline sample (0: skip)")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a device copy of this many bytes")
    ap.add_argument("--batch", type=int, default=64, help="replicas in the batched-form leg (0: skip)")
    ap.add_argument("--large-steps", type=int, default=500,
                    help="timed steps of the 5e6-ion leg (0: skip)")
    ap.add_argument("--shell-stored", type=int, default=0,
                    help="1: the main legs use the memory form of the list (shell batch drawn at the build)")
    ap.add_argument("--int-phase-main", type=int, default=0,
                    help="1: the main legs use the fixed-point k-space phase (mixed form only)")
    ap.add_argument("--stored", type=int, default=1,
                    help="1: also time the memory form of the list (shell batch drawn at the build) "
                         "on the 1e6-ion workload and, with --large-steps, on the 5e6-ion melt")
    ap.add_argument("--int-phase", type=int, default=1,
                    help="1: also time the mixed form with the k-space phase in 32-bit fixed point")
    ap.add_argument("--thermo-steps", type=int, default=30,
                    help="timed steps of the Nose-Hoover and Langevin legs on the main workload (0: skip)")
    ap.add_argument("--paper-steps", type=int, default=100,
                    help="timed steps of the leg at the size and batch sizes of the paper's timing table (0: skip)")
    ap.add_argument("--repeats", type=int, default=5, help="timed runs per leg; the median is reported")
    ap.add_argument("--cpu-direct", type=int, default=1,
                    help="1: also time the oracle's full step on the 512- and 32768-ion melts at 1 and all threads")
    ap.add_argument("--form-errors", type=int, default=1,
                    help="1: state each leg's FP32-mixed force error against the FP64 path")
    ap.add_argument("--tuning", default="auto",
                    help="launch shapes of the single-system runs: auto (autotuned) or "
                         "pair_block,pair_ku,rho_mpl,kf_block,kf_aux")
    args = ap.parse_args()
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this build has no multi-GPU path.", file=sys.stderr)
        return 2

    from paper_2512_24970_amd import workloads as W
    t = time.perf_counter()
    cfg = W.config(args.workload)
    if args.shell_stored:
        cfg = dict(cfg, sys=dict(cfg["sys"], shell_stored=True))
    if args.int_phase_main:
        cfg = dict(cfg, sys=dict(cfg["sys"], int_phase=True))
    wl_key = args.workload + ("_stored" if args.shell_stored else "") + ("_intphase" if args.int_phase_main else "")
    n = len(cfg["types"])
    _log(f"[bench] workload {args.workload}: N={n} inputs in {time.perf_counter() - t:.1f} s")
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    results = {}
    for f in forms:
        results[f] = run_gpu(cfg, f, args.steps, args.warmup, args.tuning, repeats=args.repeats)
    head = forms[0]
    r = results[head]
    p_f = int(cfg["sys"]["p_f"])
    line = {
        "metric": "atom-steps/s (force+step) at N=1e6 NaCl, FP32-mixed vs FP64, % VALU peak",
        "value": r["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "n_atoms": n, "box_A": cfg["sys"]["box"][0], "T_K": cfg["T"],
            "species": cfg["sys"]["species"]["names"], "r_core": cfg["sys"]["r_core"],
            "r_shell": cfg["sys"]["r_shell"], "skin": cfg["sys"]["skin"], "p_r": cfg["sys"]["p_r"], "p_f": p_f,
            "rebuild_every": cfg["sys"]["rebuild_every"], "dt_ps": cfg["sys"]["dt"], "form": head,
            "shell_batch": "stored at the list build" if args.shell_stored else "drawn every evaluation",
        },
        "roofline": roofline(head, r, n, cfg["sys"], wl_key),
        "phases_ms_per_step": phase_ms(r),
        "runs_ms_per_step": r["runs_ms_per_step"],
        "apriori_model": apriori_model(cfg["sys"], n, head),
        "tuning": r["tuning"],
        "device_mem_GB": r["device_mem_GB"],
    }
    line["T_end_K"] = round(r["T_end"], 1)
    main_err = None
    if "mixed" in results and "fp64" in results:
        a, b = results["mixed"]["force0"], results["fp64"]["force0"]
        main_err = dict(_force_err(a, b), reference="fp64 path, eval 0, starting positions")
        line["mixed_vs_fp64_force_rel_rms"] = main_err["rel_rms"]
        line["mixed_vs_fp64_force"] = main_err
    for f in forms[1:]:
        rf = results[f]
        line[f] = {"value": rf["value"], "ms_per_step": rf["ms_per_step"], "T_end_K": round(rf["T_end"], 1),
                   "runs_ms_per_step": rf["runs_ms_per_step"], "tuning": rf["tuning"],
                   "roofline": roofline(f, rf, n, cfg["sys"], wl_key),
                   "apriori_model": apriori_model(cfg["sys"], n, f),
                   "phases_ms_per_step": phase_ms(rf)}
    if args.batch > 0:
        line["batch"] = run_batch(args.batch, args.steps, args.warmup, args.repeats)
    if args.large_steps > 0:
        # the 5e6-ion NaCl melt (P_F = 1000), mixed form
        t = time.perf_counter()
        big = W.config("nacl_5m")
        _log(f"[bench] large: N={len(big['types'])} inputs in {time.perf_counter() - t:.1f} s")
        rl = run_gpu(big, "mixed", args.large_steps, args.warmup, "auto", repeats=1)
        nb = len(big["types"])
        line["large"] = {"workload": "nacl_5m", "n_atoms": nb, "p_f": int(big["sys"]["p_f"]),
                         "mixed_vs_fp64_force": form_error(big) if args.form_errors else None,
                         "p_r": int(big["sys"]["p_r"]), "form": "mixed", "value": rl["value"],
                         "unit": "atom-steps/s", "steps": args.large_steps, "ms_per_step": rl["ms_per_step"],
                         "T_end_K": round(rl["T_end"], 1), "tuning": rl["tuning"],
                         "device_mem_GB": rl["device_mem_GB"],
                         "roofline": roofline("mixed", rl, nb, big["sys"], "nacl_5m"),
                         "phases_ms_per_step": phase_ms(rl)}
    if args.stored:
        # memory form of the random batch list: the shell batch is drawn at the
        # list build and kept until the next one (P_R entries per atom)
        def stored_leg(c, steps, wl, reps):
            cs = dict(c, sys=dict(c["sys"], shell_stored=True))
            rs = run_gpu(cs, "mixed", steps, args.warmup, "auto", repeats=reps)
            nn = len(c["types"])
            return {"workload": wl, "n_atoms": nn, "form": "mixed", "value": rs["value"], "unit": "atom-steps/s",
                    "mixed_vs_fp64_force": form_error(c, shell_stored=True) if args.form_errors else None,
                    "steps": steps, "ms_per_step": rs["ms_per_step"], "T_end_K": round(rs["T_end"], 1),
                    "tuning": rs["tuning"], "device_mem_GB": rs["device_mem_GB"],
                    "roofline": roofline("mixed", rs, nn, c["sys"], wl + "_stored"),
                    "phases_ms_per_step": phase_ms(rs)}
        line["stored"] = stored_leg(cfg, args.steps, args.workload, args.repeats)
        if args.large_steps > 0:
            line["stored"]["large"] = stored_leg(big, args.large_steps, "nacl_5m", 1)
    if args.int_phase:
        # the mixed form with the k-space phase reduced in 32-bit fixed point
        # instead of FP64 (same workload and protocol)
        ci = dict(cfg, sys=dict(cfg["sys"], int_phase=True))
        ri = run_gpu(ci, "mixed", args.steps, args.warmup, "auto", repeats=args.repeats)
        hot = {k: round(v[0] / max(v[1], 1), 4) for k, v in ri["phases"].items() if v[1] > 0}
        line["int_phase"] = {"workload": args.workload, "form": "mixed", "phase": "32-bit fixed point",
                             "value": ri["value"], "ms_per_step": ri["ms_per_step"],
                             "runs_ms_per_step": ri["runs_ms_per_step"], "tuning": ri["tuning"],
                             "hot_kernel_avg_launch_ms": hot, "phases_ms_per_step": phase_ms(ri),
                             "mixed_vs_fp64_force": form_error(cfg, mixed_only={"int_phase": True}) if args.form_errors else None}
    if args.paper_steps > 0:
        # Context, not the metric: molten NaCl at the size and batch sizes of
        # the paper's timing table (Section 3.2, Table 2: 1.024e6 ions,
        # P_R = 30, P_F = 100, r_core 5 A, r_shell 10 A), both forms, beside
        # that table's IRBSOG total of 9.04 ms per step on 1000 CPU cores
        # (LAMMPS, double precision, 2x Xeon Platinum 8358 per node).
        pc = W.config("nacl_1024k")
        npc = len(pc["types"])
        leg = {"workload": "nacl_1024k", "n_atoms": npc, "p_r": 30, "p_f": 100, "r_core_A": 5.0,
               "r_shell_A": 10.0, "unit": "atom-steps/s", "steps": args.paper_steps}
        for form in ("mixed", "fp64"):
            rp = run_gpu(pc, form, args.paper_steps, args.warmup, "auto", repeats=args.repeats)
            leg[form] = {"value": rp["value"], "ms_per_step": rp["ms_per_step"], "tuning": rp["tuning"],
                         "runs_ms_per_step": rp["runs_ms_per_step"], "phases_ms_per_step": phase_ms(rp)}
        if args.form_errors:
            leg["mixed_vs_fp64_force"] = form_error(pc)
        leg["paper_cpu_context"] = {"ms_per_step": 9.04, "atom_steps_per_s": round(npc / 9.04e-3, 1),
                                    "cores": 1000, "precision": "fp64",
                                    "hardware": "2x Intel Xeon Platinum 8358 per node", "source": "Table 2"}
        line["paper_workload"] = leg
    if args.thermo_steps > 0:
        # the other thermostats on the main workload (mixed form): Nose-Hoover
        # with tau = 10 fs; Langevin with friction 1/dt, since at this size a
        # looser Langevin bath (tau = 10 fs) lets the estimator's heating run
        # away within a few hundred steps
        line["thermostats"] = {}
        for kind, tau in (("nose_hoover", 0.01), ("langevin", float(cfg["sys"]["dt"]))):
            rt = run_gpu(cfg, "mixed", args.thermo_steps, args.warmup, "auto", kind, tau, repeats=args.repeats)
            line["thermostats"][kind] = {"tau_ps": tau, "value": rt["value"], "ms_per_step": rt["ms_per_step"],
                                         "mixed_vs_fp64_force": (dict(main_err, note="starting positions of the "
                                                                 "main leg") if main_err else None),
                                         "steps": args.thermo_steps, "T_end_K": round(rt["T_end"], 1),
                                         "phases_ms_per_step": phase_ms(rt)}
    if args.cpu_sample > 0:
        _log(f"[bench] cpu baseline: oracle on {args.cpu_sample} atoms")
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample)
        line["cpu_baseline"]["cpu_model"] = cpu_model()
        if args.cpu_direct:
            line["cpu_baseline"]["direct"] = cpu_direct()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
