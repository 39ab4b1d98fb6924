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

Prints one JSON line.  The roofline object describes the dominant kernel of
the reported form, timed with HIP events on the library's stream during the
timed steps; its algorithmic flop count per (atom, mode) pair is fixed below.
The CPU baseline is the FP64 oracle on a bounded sample of the same workload.
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

# Algorithmic flops per (atom, mode) pair, FMA = 2, as the kernels compute
# them (see the kernel comments):
#   FP64 k-space force: phase 5, table sincos 18, Im(e^{-i theta} rho) 3,
#                       accumulation 6                                  = 32
#   FP64 rho:           phase 5, sincos 18, accumulation 4              = 27
#   mixed k-space force: phase 5, turn reduction 2, sin + cos 2, 3, 6   = 18
#   mixed rho:           phase 5, reduction 2, sin + cos 2, accumulation 4 = 13
FLOPS_PER_PAIR = {
    ("fp64", "kforce"): 32, ("fp64", "rho"): 27,
    ("mixed", "kforce"): 18, ("mixed", "rho"): 13,
}


def _log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


TUNING_KEYS = ("pair_block", "pair_ku", "rho_mpl", "kf_block", "kf_aux")


def run_gpu(cfg, precision: str, steps: int, warmup: int, tuning: str = "auto", thermostat: str = "berendsen",
            tau: float | None = None):
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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e1 = ctx.rbsog_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
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
    dt = t1 - t0
    _log(f"[bench] {precision}: {steps} steps in {dt:.3f} s -> {n * steps / dt:.4g} atom-steps/s")
    ctx.close()
    T = 2 * e1["kinetic"] / ((3 * n - 3) * 8.617333262e-5)
    return {"seconds": dt, "value": n * steps / dt, "ms_per_step": 1e3 * dt / steps, "phases": prof,
            "phases_all": prof_all, "phase_steps": phase_steps,
            "energy": e1, "energy_warm": e0, "T_end": T, "force0": f0, "tuning": tuning,
            "device_mem_GB": round(mem_gb, 3)}


def _batch_inputs(cfgs, dev):
    import torch
    cat = lambda k: torch.as_tensor(np.concatenate([c[k] for c in cfgs]), device=dev)
    return cat("types"), cat("pos"), cat("vel")


def run_batch(n_rep: int, steps: int, warmup: int):
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
    stream.synchronize()
    t0 = time.perf_counter()
    e = ctx.rbsog_step(steps)
    stream.synchronize()
    dt_b = time.perf_counter() - t0
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
    return {
        "workload": f"nacl_replicas{n_rep}", "n_systems": n_rep, "n_atoms": n_tot,
        "sizes": [int(len(c["types"])) for c in cfgs][:8] + ["..."],
        "form": "mixed", "value": n_tot * steps / dt_b, "unit": "atom-steps/s",
        "ms_per_step": 1e3 * dt_b / steps, "graph": True, "tuning": tuning,
        "sequential_value": n_tot * steps / dt_s, "sequential_ms_per_step": 1e3 * dt_s / steps,
        "speedup_vs_sequential": dt_s / dt_b,
        "phases_ms_per_step": {k: round(v[0] / 10, 4) for k, v in prof.items()},
        "T_end_K_range": [round(min(T), 1), round(max(T), 1)],
    }


# Pair-kernel model (per atom, FMA = 2): a distance test is 17 flops (three
# differences, minimum image 9, r^2 5); an evaluated pair is 123 flops, with
# an FP64 exp counted as 20 and an rsqrt as 8 (two exps, five squarings, six
# Gaussian weights, a 13-term polynomial, BMH terms, force assembly).
FLOPS_TEST, FLOPS_PAIR = 17, 123

KERNEL_OF_PHASE = {"pair": "k_pair", "rho": "k_rho", "kforce": "k_kforce"}


def phase_ms(res) -> dict:
    """Milliseconds per step of every phase, from the short all-phase run."""
    return {k: round(v[0] / res["phase_steps"], 4) for k, v in res["phases_all"].items()}


def pair_flops_per_atom(sysp: dict, n: int) -> float:
    L = sysp["box"]
    rho_n = n / (L[0] * L[1] * L[2])
    rc, rs, sk, pr = sysp["r_core"], sysp["r_shell"], sysp["skin"], sysp["p_r"]
    v = lambda r: 4.0 / 3.0 * math.pi * r ** 3
    core_list = v(rc + sk) * rho_n
    core = v(rc) * rho_n
    cand = (v(rs + sk) - v(max(rc - sk, 0.0))) * rho_n
    valid = (v(rs) - v(rc)) * rho_n / cand
    batch = min(pr, cand) if pr > 0 else cand
    return (core_list + batch) * FLOPS_TEST + (core + valid * batch) * FLOPS_PAIR


def kernel_roofline(precision: str, phase: str, ms: float, launches: int, n: int, sysp: dict) -> dict:
    avg = ms / launches * 1e-3
    if phase == "pair":
        flops = pair_flops_per_atom(sysp, n) * n
    else:
        flops = FLOPS_PER_PAIR[(precision, phase)] * float(n) * float(sysp["p_f"])
    ach = flops / avg / 1e12
    return {"bound": "alu", "kernel": KERNEL_OF_PHASE[phase], "achieved": round(ach, 3), "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / PEAK_VALU_TFLOPS, 4), "traffic": None,
            "avg_launch_ms": round(ms / launches, 4), "launches": launches, "flops_per_launch": flops}


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(HERE, "profiles", f"{workload}_traffic.md")
    src = os.path.join(HERE, "paper_2512_24970_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    for line in open(path):
        if line.startswith("traffic_json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("source_sha1") == sha and kernel in d.get("bytes_per_launch", {}):
                return d["bytes_per_launch"][kernel]
    return None


def roofline(precision: str, res: dict, n: int, sysp: dict, workload: str) -> dict:
    """The dominant kernel (largest time in the timed steps) and the others."""
    phases = {k: v for k, v in res["phases"].items() if k in KERNEL_OF_PHASE and v[1] > 0}
    lines = {k: kernel_roofline(precision, k, v[0], v[1], n, sysp) for k, v in phases.items()}
    top = max(phases, key=lambda k: phases[k][0])
    out = dict(lines[top])
    out["traffic"] = traffic_from_profiles(out["kernel"] + ("<mixed>" if precision == "mixed" else "<fp64>"),
                                           workload)
    if out["traffic"]:
        # the measured HBM bytes against the HBM peak, beside the VALU view
        gbs = out["traffic"] / (out["avg_launch_ms"] * 1e-3) / 1e9
        out["traffic_GBps"] = round(gbs, 1)
        out["traffic_frac_of_hbm_peak"] = round(gbs / PEAK_HBM_GBS, 4)
    out["others"] = {lines[k]["kernel"]: {"achieved": lines[k]["achieved"], "frac": lines[k]["frac"],
                                         "avg_launch_ms": lines[k]["avg_launch_ms"]}
                     for k in lines if k != top}
    # the k-space chain runs on a second stream beside the pair kernel, so
    # their launch durations overlap and each includes the other's share
    out["concurrent"] = "k_pair runs beside k_ksample + k_rho + k_kforce (second stream); durations overlap"
    return out


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
                       f"and k-space force of {n_sample} random atoms ({t3 - t1:.2f} s, neighbours by O(N) scan), "
                       f"extrapolated to one step of all atoms"),
            "seconds_measured": round(t3 - t0, 3)}


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
    ap.add_argument("--stored", type=int, default=1,
                    help="1: also time the memory form of the list (shell batch drawn at the build) "
                         "on the 1e6-ion workload and, with --large-steps, on the 5e6-ion melt")
    ap.add_argument("--thermo-steps", type=int, default=30,
                    help="timed steps of the Nose-Hoover and Langevin legs on the main workload (0: skip)")
    ap.add_argument("--paper-steps", type=int, default=100,
                    help="timed steps of the leg at the size and batch sizes of the paper's timing table (0: skip)")
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
    wl_key = args.workload + ("_stored" if args.shell_stored else "")
    n = len(cfg["types"])
    _log(f"[bench] workload {args.workload}: N={n} inputs in {time.perf_counter() - t:.1f} s")
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    results = {}
    for f in forms:
        results[f] = run_gpu(cfg, f, args.steps, args.warmup, args.tuning)
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
        "tuning": r["tuning"],
        "device_mem_GB": r["device_mem_GB"],
    }
    line["T_end_K"] = round(r["T_end"], 1)
    if "mixed" in results and "fp64" in results:
        a, b = results["mixed"]["force0"], results["fp64"]["force0"]
        line["mixed_vs_fp64_force_rel_rms"] = float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))
    for f in forms[1:]:
        rf = results[f]
        line[f] = {"value": rf["value"], "ms_per_step": rf["ms_per_step"], "T_end_K": round(rf["T_end"], 1),
                   "tuning": rf["tuning"],
                   "roofline": roofline(f, rf, n, cfg["sys"], wl_key),
                   "phases_ms_per_step": phase_ms(rf)}
    if args.batch > 0:
        line["batch"] = run_batch(args.batch, args.steps, args.warmup)
    if args.large_steps > 0:
        # the 5e6-ion NaCl melt (P_F = 1000), mixed form
        t = time.perf_counter()
        big = W.config("nacl_5m")
        _log(f"[bench] large: N={len(big['types'])} inputs in {time.perf_counter() - t:.1f} s")
        rl = run_gpu(big, "mixed", args.large_steps, args.warmup, "auto")
        nb = len(big["types"])
        line["large"] = {"workload": "nacl_5m", "n_atoms": nb, "p_f": int(big["sys"]["p_f"]),
                         "p_r": int(big["sys"]["p_r"]), "form": "mixed", "value": rl["value"],
                         "unit": "atom-steps/s", "steps": args.large_steps, "ms_per_step": rl["ms_per_step"],
                         "T_end_K": round(rl["T_end"], 1), "tuning": rl["tuning"],
                         "device_mem_GB": rl["device_mem_GB"],
                         "roofline": roofline("mixed", rl, nb, big["sys"], "nacl_5m"),
                         "phases_ms_per_step": phase_ms(rl)}
    if args.stored:
        # memory form of the random batch list: the shell batch is drawn at the
        # list build and kept until the next one (P_R entries per atom)
        def stored_leg(c, steps, wl):
            cs = dict(c, sys=dict(c["sys"], shell_stored=True))
            rs = run_gpu(cs, "mixed", steps, args.warmup, "auto")
            nn = len(c["types"])
            return {"workload": wl, "n_atoms": nn, "form": "mixed", "value": rs["value"], "unit": "atom-steps/s",
                    "steps": steps, "ms_per_step": rs["ms_per_step"], "T_end_K": round(rs["T_end"], 1),
                    "tuning": rs["tuning"], "device_mem_GB": rs["device_mem_GB"],
                    "roofline": roofline("mixed", rs, nn, c["sys"], wl + "_stored"),
                    "phases_ms_per_step": phase_ms(rs)}
        line["stored"] = stored_leg(cfg, args.steps, args.workload)
        if args.large_steps > 0:
            line["stored"]["large"] = stored_leg(big, args.large_steps, "nacl_5m")
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
            rp = run_gpu(pc, form, args.paper_steps, args.warmup, "auto")
            leg[form] = {"value": rp["value"], "ms_per_step": rp["ms_per_step"], "tuning": rp["tuning"],
                         "phases_ms_per_step": phase_ms(rp)}
        leg["paper_cpu_context"] = {"ms_per_step": 9.04, "atom_steps_per_s": round(npc / 9.04e-3, 1),
                                    "cores": 1000, "precision": "fp64",
                                    "hardware": "2x Intel Xeon Platinum 8358 per node", "source": "Table 2"}
        line["paper_workload"] = leg
    if args.thermo_steps > 0:
        # the other thermostats on the main workload (mixed form), tau = 10 fs
        line["thermostats"] = {}
        for kind in ("nose_hoover", "langevin"):
            rt = run_gpu(cfg, "mixed", args.thermo_steps, args.warmup, "auto", kind, 0.01)
            line["thermostats"][kind] = {"tau_ps": 0.01, "value": rt["value"], "ms_per_step": rt["ms_per_step"],
                                         "steps": args.thermo_steps, "T_end_K": round(rt["T_end"], 1),
                                         "phases_ms_per_step": phase_ms(rt)}
    if args.cpu_sample > 0:
        _log(f"[bench] cpu baseline: oracle on {args.cpu_sample} atoms")
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
