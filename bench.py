"""Benchmark: PSO force-inversion generations on one MI355X.

One step = one PSO generation of the whole hot path over the workload's swarms: RK4 integration of
every particle's trajectory, lock-in projection and window misfit (one kernel), then personal and
swarm bests and the Eq. 8 move (one kernel).  Steps run inside the library's captured HIP graph
(afm_invert), inputs resident in HBM.

Headline workload: the uneven pixel batch -- 4096 independent pixel inversions of (H, E*) on the
point-mass DMT cantilever (k = 40 N/m, f0 = 300 kHz, Q = 400, A0 = 20 nm), each pixel with its own
E* (log-uniform 0.05-50 GPa), set-point (uniform 0.5-0.9 A0, separation found by the library's
amplitude-feedback search) and period count (uniform 100-2000, 256 RK4 steps each), 128
particles per pixel, noiseless synthetic targets from the plain FP64 GPU path at each pixel's
truth; FP32 integration with FP64 lock-in and misfit sums; all pixels' particles in one
persistent work-queue kernel per generation.

Prints one JSON line (metric RK4 steps/s; inversions/s beside it).  Also reported: the forward
kernel's roofline (FP32 VALU), the precision-path workload (1024 particles, 500 periods, noisy
target), the plain FP64 GPU path, a GPU-filling plain batch, time to inversion at equal misfit
accuracy, the adjoint, the 3-mode hybrid inversion, the paper's own inversions, and the oracle
timed on one host core with its extrapolated time to inversion for every workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published dense FP32 vector peak of MI355X, 157.3 TFLOP/s: 256 CUs x 4 SIMDs x 32 FMA lanes per
# cycle x 2 flop x 2.4 GHz.  Measured with the library (no packed FP32 instructions): a SIMD shared by
# four waves completes wave-wide FP32 VALU instructions faster than one per 4 cycles (3.4 cycles
# on average in the pixel-workload kernel, transcendentals included), so the published peak is
# the reference; a lone wave issues at most one instruction per 4 cycles (the small-batch
# ceiling below).
PEAK_FP32_PUBLISHED = 157.3e12
# one wave on its SIMD: 64 lanes x 2 flop every 4 cycles at 2.4 GHz
WAVE_ISSUE_FLOPS = 64 * 2 / 4 * 2.4e9
# FP32 flops per RK4 step of the point-mass DMT model, the algorithmic count of the hot-path scope
# (FMA = 2, add/mul = 1, rcp/sqrt = 1): 82.  Recounted from the kernel's own arithmetic: 68 with
# the far-field force only (what the method needs out of contact, and what a block that the
# contact bound clears executes), 96 for the branch-free block with both force pieces.
FLOPS_PER_STEP_DMT1 = 82
# HBM bytes per launch of a kernel from the FETCH_SIZE / WRITE_SIZE counter runs (scaled by a
# copy kernel of known size), valid only while the kernel sources are unchanged.
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_forward_queue_dmt1_c3_pmc.md")
PMC_SUMMARY_C2 = os.path.join(ROOT, "profiles", "k_forward_dmt1_c2_pmc.md")
KERNEL_SOURCES = ["forward_impl.hpp", "forward_dmt_mixed.hip", "rk4.hpp", "afm_internal.hpp"]


def counted_traffic(path=PMC_SUMMARY):
    """Counter-measured bytes per launch of a kernel, or None when its summary is missing or the
    kernel sources have changed since the counters were taken."""
    import hashlib
    import re

    try:
        text = open(path).read()
    except OSError:
        return None
    t = re.search(r"^traffic_bytes_per_launch:\s*(\d+)", text, re.M)
    h = re.search(r"^source_sha256:\s*([0-9a-f]{64})", text, re.M)
    if not (t and h):
        return None
    sha = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1109_0334_amd", "csrc", f), "rb") as fh:
            sha.update(fh.read())
    return int(t.group(1)) if sha.hexdigest() == h.group(1) else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision-path (c2), FP64, saturated and steady-exit legs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--pixel-steps", type=int, default=2)
    ap.add_argument("--no-more", action="store_true",
                    help="skip the time-to-inversion, gradient and 3-mode legs")
    ap.add_argument("--short-c5", action="store_true",
                    help="run 2 generations and one polish step of the 3-mode hybrid inversion")
    ap.add_argument("--gradient-probe", action="store_true",
                    help="run only the c4 adjoint leg (for profiling the adjoint kernel)")
    ap.add_argument("--queue-probe", action="store_true",
                    help="only build the pixel workload and run its work-queue forward launch "
                         "(afm_misfit_swarms) --steps times (for counter runs of that kernel)")
    ap.add_argument("--c2-probe", action="store_true",
                    help="only run the precision-path forward launch (afm_misfit) --steps times")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 256 MiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def _pixel_problem(afm, W, dev, S):
    """The first S pixels of the uneven-batching workload: per-pixel separations from their
    set-points (batched FP64 forward solves), parameters [12][S] and FP64 targets over each
    pixel's own period count."""
    import numpy as np
    import torch

    from paper_1109_0334_amd import setpoint

    cfg = W.config("c3")
    m = cfg["model"]
    pix = {k: v[:S] for k, v in W.pixels(cfg).items()}
    base = W.full_params(cfg)
    t0 = time.perf_counter()
    zc = setpoint.separations(afm, m, base, [2], [pix["Estar"]], pix["setpoint"], device=dev)
    t_sep = time.perf_counter() - t0
    good = np.isfinite(zc)
    sp = np.tile(base[:, None], (1, S)).astype(np.float64)
    sp = np.concatenate([sp, np.zeros((afm.MAX_PARAMS - sp.shape[0], S))], axis=0)
    sp[0] = np.where(good, zc, base[0])
    sp[2] = pix["Estar"]
    ref = afm.Plan(m, base, [(0, 0.0, 1.0, 0), (2, 0.0, 1.0, 0)], precision="fp64", device=dev)
    th = torch.tensor(np.stack([sp[0], sp[2]]), device=dev)
    cyc = torch.tensor(pix["cycles"], device=dev)
    U = ref.forward_batch(th, n_cycles=cyc, trace=True)["trace"].contiguous()
    return dict(cfg=cfg, m=m, base=base, pix=pix, U=U, cyc=cyc, spd=torch.tensor(sp, device=dev),
                t_sep=t_sep, good=good)


def headline_c3(afm, W, dev, K, Wu):
    """Uneven batching: 4096 pixel inversions of (H, E*) with per-pixel E*, set-point and period
    count (100..2000), 128 particles, through the persistent work-queue kernel; K generations
    timed as one graph replay, and the forward kernel alone (the same launch) with HIP events."""
    import numpy as np
    import torch

    cfg = W.config("c3")
    S, P = int(cfg["pixels"]), int(cfg["particles"])
    q = _pixel_problem(afm, W, dev, S)
    m, U, cyc, spd, pix = q["m"], q["U"], q["cyc"], q["spd"], q["pix"]
    N = m["steps_per_cycle"]
    free = W.free_index(cfg)
    plan = afm.Plan(m, q["base"], free, precision="mixed", device=dev)
    plan.invert(U, P, Wu, seed=0, n_cycles=cyc, swarm_params=spd)  # warm-up generations
    torch.cuda.synchronize()
    plan.invert(U, P, K, seed=0, n_cycles=cyc, swarm_params=spd)  # capture the K-generation graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = plan.invert(U, P, K, seed=0, n_cycles=cyc, swarm_params=spd)  # timed replay
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps_per_gen = float(P) * float(np.sum(pix["cycles"])) * N
    # the forward kernel alone: afm_misfit_swarms is the graph's forward launch (same kernel,
    # grid and queue), enqueued on torch's current stream, where the events are recorded
    th = torch.tensor(W.draw_free(cfg, S * P, 9).T.copy(), device=dev)
    plan.misfit_swarms(th, U, P, n_cycles=cyc, swarm_params=spd)  # builds the queue order
    torch.cuda.synchronize()
    k_ms = _event_ms(lambda: plan.misfit_swarms(th, U, P, n_cycles=cyc, swarm_params=spd), reps=5)
    flops = FLOPS_PER_STEP_DMT1 * steps_per_gen
    achieved = flops / (k_ms * 1e-3)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_PUBLISHED / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_PUBLISHED,
            "traffic": counted_traffic(PMC_SUMMARY),
            "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
            "kernel": "k_forward_queue<DMT,1 mode,mixed>", "kernel_ms": k_ms,
            "flops_per_step": FLOPS_PER_STEP_DMT1, "rk4_steps_per_launch": steps_per_gen,
            "flops_per_launch": flops,
            "occupancy": f"{S * P} trajectories = {S * P // 64} waves, 4 per SIMD in flight "
                         "(persistent grid of 4 x 256-lane workgroups per CU)"}
    # the same misfits as one plain-grid launch (per-lane period counts, no queue) for contrast
    tid = torch.arange(S, device=dev, dtype=torch.int32).repeat_interleave(P)
    ncl = cyc.repeat_interleave(P)
    plan.misfit(th, U, target_id=tid, n_cycles=ncl)  # launch-shape tuning
    grid_ms = _event_ms(lambda: plan.misfit(th, U, target_id=tid, n_cycles=ncl))
    return {"dt": dt, "steps_per_gen": steps_per_gen, "roofline": roof, "S": S, "P": P,
            "T": int(cfg["iters"]), "median_best_J": float(np.median(out["best_J"].cpu().numpy())),
            "plain_grid_forward_ms": grid_ms, "setup_separation_s": q["t_sep"],
            "pixels_without_setpoint_crossing": int((~q["good"]).sum()),
            "plan": plan, "q": q, "th": th, "ncl": ncl}


def steady_exit_leg(afm, W, dev, h, steps):
    """The pixel inversions with the adaptive steady-state exit (the period counts become caps)."""
    import numpy as np
    import torch

    cfg = W.config("c3")
    q, P = h["q"], h["P"]
    m, U, cyc, spd = q["m"], q["U"], q["cyc"], q["spd"]
    free = W.free_index(cfg)
    ms_plain = h["dt"] / max(1, h["K"]) * 1e3
    res = []
    for rtol in (1e-4, 1e-6):
        pex = afm.Plan(dict(m, steady_rtol=rtol), q["base"], free, precision="mixed", device=dev)
        pex.invert(U, P, steps, seed=0, n_cycles=cyc, swarm_params=spd)  # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        oex = pex.invert(U, P, steps, seed=0, n_cycles=cyc, swarm_params=spd)
        torch.cuda.synchronize()
        dtx = time.perf_counter() - t0
        used = pex.forward_steady(h["th"], n_cycles=h["ncl"])["periods"].double().sum().item()
        res.append({"steady_rtol": rtol, "ms_per_generation": dtx / steps * 1e3,
                    "speedup": ms_plain / (dtx / steps * 1e3),
                    "periods_saved": 1.0 - used / float(h["ncl"].double().sum().item()),
                    "median_best_J": float(np.median(oex["best_J"].cpu().numpy()))})
    return res


def c2_leg(afm, W, dev, K, Wu):
    """The precision-path workload: point-mass DMT, invert (H, E*, a0), 1024 particles, 500
    periods x 256 steps, noisy target; K generations as a graph replay, the forward kernel alone
    with HIP events, the plain FP64 forward and a GPU-filling batch of the same kernel."""
    import torch

    cfg = W.config("c2")
    m = cfg["model"]
    P = cfg["particles"]
    Wn = m["lockin_cycles"] * m["steps_per_cycle"]
    steps_per_traj = m["n_cycles"] * m["steps_per_cycle"]
    free = W.free_index(cfg)
    p_true = W.full_params(cfg)
    # target: plain FP64 GPU trace at the truth plus seeded measurement noise (setup, untimed)
    ref = afm.Plan(m, p_true, free, precision="fp64", device=dev)
    truth = torch.tensor([[cfg["truth"]["H"]], [cfg["truth"]["Estar"]], [cfg["truth"]["a0"]]],
                         dtype=torch.float64, device=dev)
    U = ref.forward_batch(truth, trace=True)["trace"] + torch.tensor(W.noise(cfg, Wn, 0), device=dev)
    U = U.contiguous()
    plan = afm.Plan(m, p_true, free, precision="mixed", device=dev)
    plan.invert(U, P, Wu, seed=cfg["seed"], cutoff=1e-3)
    torch.cuda.synchronize()
    out = plan.invert(U, P, K, seed=cfg["seed"], cutoff=1e-3)  # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = plan.invert(U, P, K, seed=cfg["seed"], cutoff=1e-3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    th_dev = torch.tensor(W.draw_free(cfg, P, 5).T.copy(), device=dev)
    plan.misfit(th_dev, U)
    torch.cuda.synchronize()
    k_ms = _event_ms(lambda: plan.misfit(th_dev, U), reps=max(3, min(K, 10)))
    flops = FLOPS_PER_STEP_DMT1 * P * steps_per_traj
    achieved = flops / (k_ms * 1e-3)
    res = {"workload": "c2-precision-path: point-mass DMT, invert (H, E*, a0), 1024 particles, "
                       "500 periods x 256 RK4 steps, noisy target",
           "generations": K, "ms_per_generation": dt / K * 1e3,
           "rk4_steps_per_s": P * steps_per_traj * K / dt,
           "inversions_per_s": 1.0 / (dt / K * cfg["iters"]),
           "best_J_after_steps": float(out["best_J"].item()),
           "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                        "peak": PEAK_FP32_PUBLISHED / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_FP32_PUBLISHED,
                        "traffic": counted_traffic(PMC_SUMMARY_C2),
                        "kernel": "k_forward<DMT,1 mode,mixed>", "kernel_ms": k_ms,
                        "flops_per_launch": flops,
                        "occupancy": f"{P} trajectories = {P // 64} waves on 1024 SIMDs, one "
                                     "wave per SIMD",
                        "wave_issue_ceiling_tflops": P // 64 * WAVE_ISSUE_FLOPS / 1e12,
                        "frac_of_wave_issue_ceiling": achieved / (P // 64 * WAVE_ISSUE_FLOPS)}}
    # plain FP64 per-particle forward on the same workload (one generation's misfits)
    plan64 = afm.Plan(m, p_true, free, precision="fp64", device=dev)
    plan64.misfit(th_dev, U)
    torch.cuda.synchronize()
    f64_ms = _event_ms(lambda: plan64.misfit(th_dev, U), reps=3)
    res["fp64_forward"] = {"kernel_ms": f64_ms,
                           "rk4_steps_per_s": P * steps_per_traj / (f64_ms * 1e-3),
                           "mixed_speedup": f64_ms / k_ms}
    # the same kernel on a batch that fills the GPU (4096 swarms x 128 particles, 40 periods)
    n_sat, nc_sat = 4096 * 128, 40
    plan_sat = afm.Plan(dict(m, n_cycles=nc_sat), p_true, free, precision="mixed", device=dev)
    th_sat = torch.tensor(W.draw_free(cfg, n_sat, 6).T.copy(), device=dev)
    tid = torch.zeros(n_sat, dtype=torch.int32, device=dev)
    plan_sat.misfit(th_sat, U, target_id=tid)
    torch.cuda.synchronize()
    sat_ms = _event_ms(lambda: plan_sat.misfit(th_sat, U, target_id=tid), reps=3)
    sat_steps = n_sat * nc_sat * m["steps_per_cycle"]
    sat_ach = FLOPS_PER_STEP_DMT1 * sat_steps / (sat_ms * 1e-3)
    res["saturated_forward"] = {
        "trajectories": n_sat, "periods": nc_sat, "kernel_ms": sat_ms,
        "rk4_steps_per_s": sat_steps / (sat_ms * 1e-3), "achieved_tflops": sat_ach / 1e12,
        "frac_published_peak": sat_ach / PEAK_FP32_PUBLISHED}
    return res, U, cfg


def pixel_time_to_inversion(afm, W, dev, S, cutoff):
    """Whole inversions (all generations) of the first S pixels, mixed vs plain FP64 forward:
    wall time, the generation at which each pixel's sqrt(best J) first reaches the cut-off."""
    import numpy as np
    import torch

    cfg = W.config("c3")
    P, T = int(cfg["particles"]), int(cfg["iters"])
    q = _pixel_problem(afm, W, dev, S)
    res = {"pixels": S, "generations": T, "cutoff_sqrtJ": cutoff}
    for prec in ("mixed", "fp64"):
        plan = afm.Plan(q["m"], q["base"], W.free_index(cfg), precision=prec, device=dev)
        kw = dict(seed=0, cutoff=cutoff, n_cycles=q["cyc"], swarm_params=q["spd"])
        plan.invert(q["U"], P, 2, **kw)  # workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = plan.invert(q["U"], P, T, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        gen = out["gen_to_cutoff"].cpu().numpy()
        ok = gen >= 0
        res[prec] = {"seconds_all_generations": dt, "fraction_reaching_cutoff": float(ok.mean()),
                     "median_generation_reaching_cutoff": float(np.median(gen[ok])) if ok.any() else None,
                     "seconds_to_cutoff_median": dt / T * (float(np.median(gen[ok])) + 1)
                     if ok.any() else None,
                     "median_final_best_J": float(np.median(out["best_J"].cpu().numpy()))}
    if res["mixed"]["seconds_to_cutoff_median"] and res["fp64"]["seconds_to_cutoff_median"]:
        res["fp64_over_mixed"] = (res["fp64"]["seconds_to_cutoff_median"]
                                  / res["mixed"]["seconds_to_cutoff_median"])
    return res


def _event_ms(fn, reps=1):
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_to_inversion(afm, W, dev, U, cfg):
    """Whole c2 inversions (all generations), mixed vs plain FP64 forward, at equal misfit
    accuracy.  The noisy target puts a floor under J, so the accuracy is stated relative to it:
    a first mixed run finds the floor J_f (its final best J); both precisions then run with the
    cut-off sqrt(J) <= sqrt((1 + e) J_f) for each excess e and report the generation and wall
    time that reach it."""
    import math

    import torch

    m, P, T = cfg["model"], cfg["particles"], cfg["iters"]
    plans = {prec: afm.Plan(m, W.full_params(cfg), W.free_index(cfg), precision=prec, device=dev)
             for prec in ("mixed", "fp64")}
    first = plans["mixed"].invert(U, P, T, seed=cfg["seed"], cutoff=0.0)
    floor = float(first["best_J"].item())
    res = {"generations": T, "J_floor": floor, "levels": []}
    for excess in (1e-2, 1e-4, 1e-5):
        cutoff = math.sqrt((1.0 + excess) * floor)
        lv = {"excess_over_floor": excess, "cutoff_sqrtJ": cutoff}
        for prec, plan in plans.items():
            plan.invert(U, P, 2, seed=cfg["seed"], cutoff=cutoff)  # workspace
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = plan.invert(U, P, T, seed=cfg["seed"], cutoff=cutoff)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            gen = int(out["gen_to_cutoff"].item())
            lv[prec] = {"seconds_all_generations": dt,
                        "generation_reaching_cutoff": gen,
                        "seconds_to_cutoff": dt / T * (gen + 1) if gen >= 0 else None,
                        "final_best_J": float(out["best_J"].item())}
        if lv["mixed"]["seconds_to_cutoff"] and lv["fp64"]["seconds_to_cutoff"]:
            lv["fp64_over_mixed"] = lv["fp64"]["seconds_to_cutoff"] / lv["mixed"]["seconds_to_cutoff"]
        res["levels"].append(lv)
    return res


def plain_method_leg(afm, W, dev):
    """c1: the plain method in FP64 -- 2 parameters (H, E*), 32 particles x 20 generations,
    100 periods x 200 steps, noiseless target (plain FP64 forward at the truth); whole
    inversions as graph replays, with the recovered parameters' errors."""
    import torch

    cfg = W.config("c1")
    m, free, base = cfg["model"], W.free_index(cfg), W.full_params(cfg)
    truth = [cfg["truth"]["H"], cfg["truth"]["Estar"]]
    ref = afm.Plan(m, base, free, precision="fp64", device=dev)
    U = ref.forward_batch(torch.tensor([[t] for t in truth], device=dev),
                          trace=True)["trace"].contiguous()
    res = {"workload": "c1: point-mass DMT, invert (H, E*), 32 particles x 20 generations, "
                       "100 periods x 200 steps, noiseless"}
    for prec in ("fp64", "mixed"):
        plan = afm.Plan(m, base, free, precision=prec, device=dev)
        P, T = int(cfg["particles"]), int(cfg["iters"])
        plan.invert(U, P, T, seed=cfg["seed"], cutoff=1e-2)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            out = plan.invert(U, P, T, seed=cfg["seed"], cutoff=1e-2)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        bt = out["best_theta"].cpu().numpy()[:, 0]
        res[prec] = {"ms_per_inversion": dt * 1e3,
                     "rk4_steps_per_s": P * T * m["n_cycles"] * m["steps_per_cycle"] / dt,
                     "best_J": float(out["best_J"].item()),
                     "generation_reaching_sqrtJ_0.01": int(out["gen_to_cutoff"].item()),
                     "rel_error_H": abs(bt[0] / truth[0] - 1),
                     "rel_error_Estar": abs(bt[1] / truth[1] - 1)}
    return res


def paper_solver_leg(afm, W, dev):
    """The paper's own forward-solve benchmark shape (Sec. 3.2): 960 independent solves of an
    eight-mode Euler-Bernoulli cantilever, ~1000 RK4 steps each (here 3 drive periods x 400
    steps, DMT tip force), one launch; tuned launch shape (one lane per mode where faster)."""
    import torch

    cfg = W.config("c2")
    eb = W.beam_modes(8)
    m = dict(cfg["model"], n_modes=8, q=[400.0] * 8, ratio=eb["ratio"], gain=eb["gain"],
             steps_per_cycle=400, n_cycles=3, lockin_cycles=1)
    free = W.free_index(cfg)
    plan = afm.Plan(m, W.full_params(cfg), free, precision="mixed", device=dev)
    n = 960
    th = torch.tensor(W.draw_free(cfg, n, 8).T.copy(), device=dev)
    plan.forward_batch(th)  # launch-shape tuning
    ms = _event_ms(lambda: plan.forward_batch(th), reps=5)
    steps = n * m["n_cycles"] * m["steps_per_cycle"]
    return {"workload": "960 solves, 8-mode EB beam, 3 periods x 400 RK4 steps, DMT, mixed",
            "ms_per_launch": ms, "trajectory_steps_per_s": steps / (ms * 1e-3),
            "mode_steps_per_s": 8 * steps / (ms * 1e-3),
            "paper": "960 solves of 8 modes x 1000 steps in 15.1 ms on a Quadro FX 5800 "
                     "(6.36e7 trajectory-steps/s), context only"}


def gradient_leg(afm, W, dev):
    """c4: discrete-adjoint gradients of 2048 Lennard-Jones-type points, 1000 periods x 256
    steps, at each checkpoint stride."""
    import torch

    cfg = W.config("c4")
    m, free, base = cfg["model"], W.free_index(cfg), W.full_params(cfg)
    n = int(cfg["points"])
    ref = afm.Plan(m, base, free, precision="fp64", device=dev)
    U = ref.forward_batch(torch.tensor([[base[f[0]]] for f in free], device=dev),
                          trace=True)["trace"].contiguous()
    th = torch.tensor(W.draw_free(cfg, n, 7).T.copy(), device=dev)
    plan = afm.Plan(m, base, free, precision="mixed", device=dev)
    steps = n * m["n_cycles"] * m["steps_per_cycle"]
    out = {"workload": "c4: 2048 LJ-type points (eps, r0, n, m), 1000 periods x 256 steps",
           "points": n}
    plan.misfit(th, U)  # launch-shape tuning
    fwd_ms = _event_ms(lambda: plan.misfit(th, U))
    out["forward_misfit_ms"] = fwd_ms
    for kc in cfg["ckpt_strides"]:
        plan.grad_batch(th, U, ckpt_stride=kc)
        ms = _event_ms(lambda: plan.grad_batch(th, U, ckpt_stride=kc))
        out[f"stride_{kc}"] = {"ms": ms, "gradients_per_s": n / (ms * 1e-3),
                               "over_forward": ms / fwd_ms}
    plan.grad_batch(th, U)  # autotuned stride
    ms = _event_ms(lambda: plan.grad_batch(th, U))
    out["autotuned"] = {"ms": ms, "gradients_per_s": n / (ms * 1e-3),
                        "forward_rk4_steps_per_s": steps / (ms * 1e-3)}
    return out


def three_mode_leg(afm, W, dev, full=True):
    """c5, the full hybrid inversion: 3-mode Kelvin-Voigt cantilever, 5 parameters (z_c, H, E*,
    a0, eta), 16384 particles x 300 generations, 2000 periods x 512 steps, then 10 L-BFGS steps
    on the discrete-adjoint gradient of the best 64 personal bests -- one captured graph.  The
    target is the plain FP64 GPU trace at the truth; reported: wall time, inversions/s, the
    recovered parameters against the truth and the oracle's misfit at the returned best.
    full=False runs 2 generations and one polish step and says so."""
    import numpy as np
    import torch

    import oracle

    cfg = W.config("c5")
    m, free, base = cfg["model"], W.free_index(cfg), W.full_params(cfg)
    P = int(cfg["particles"])
    T = int(cfg["iters"]) if full else 2
    ls, lk = (int(cfg["lbfgs_steps"]), int(cfg["lbfgs_topk"])) if full else (1, 64)
    ref = afm.Plan(m, base, free, precision="fp64", device=dev)
    U = ref.forward_batch(torch.tensor([[base[f[0]]] for f in free], device=dev),
                          trace=True)["trace"].contiguous()
    plan = afm.Plan(m, base, free, precision="mixed", device=dev)
    # generation time from a short graph replay (3 generations), for the split below
    plan.invert(U, P, 3, seed=0)  # launch-shape tuning, workspace, capture
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.invert(U, P, 3, seed=0)
    torch.cuda.synchronize()
    ms_gen = (time.perf_counter() - t1) / 3 * 1e3
    # the whole inversion: one call (graph capture, then the replay of T generations and the
    # polish of the best lk personal bests)
    t0 = time.perf_counter()
    out = plan.invert(U, P, T, seed=0, lbfgs_steps=ls, lbfgs_topk=lk)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dt_pso = ms_gen * 1e-3 * T
    bt = out["best_theta"].cpu().numpy()[:, 0]
    truth = np.array([base[f[0]] for f in free])
    p = base.copy()
    for j, f in enumerate(free):
        p[f[0]] = bt[j]
    o = oracle.forward(m, p, U.cpu().numpy()[0])
    steps = float(P) * T * m["n_cycles"] * m["steps_per_cycle"]
    return {"workload": "c5: 3-mode KV + vdW, invert (z_c, H, log E*, a0, log eta), 16384 "
                        "particles, 2000 periods x 512 steps, mixed, then L-BFGS on the best 64",
            "generations": T, "lbfgs_steps": ls, "lbfgs_topk": lk, "full_run": bool(full),
            "seconds_inversion": dt, "ms_per_generation": ms_gen,
            "seconds_pso_from_generation_time": dt_pso, "seconds_polish_remainder": dt - dt_pso,
            "inversions_per_s": 1.0 / dt, "rk4_steps_per_s_pso": steps / dt_pso,
            "best_J": float(out["best_J"].item()),
            "generation_reaching_cutoff": int(out["gen_to_cutoff"].item()),
            "oracle_J_at_best": o["J"], "oracle_status_at_best": int(o["status"]),
            "recovered": {f[0]: float(b) for f, b in zip(free, bt)},
            "relative_error": [float(abs(b / t - 1)) for b, t in zip(bt, truth)],
            "note": "seconds_inversion is one afm_invert call: graph capture, T generations, "
                    "polish; the split uses the generation time of a 3-generation replay"}


def paper_inversions_leg(afm, W, dev, swarms=64, particles=512):
    """The paper's own inversions (Sec. 4) on its 8-mode beam: base motion (1-D amplitude at two
    cut-offs, 2-D amplitude and frequency, 3-D chirp) and the spring and spring-damper samples.
    For each, `swarms` independent swarms of `particles` on one target (one graph launch; the
    swarms draw independent random streams) give the mean and variance of the generations to
    the cut-off, and a single swarm gives one inversion's time per generation.  Target: the
    plain FP64 GPU trace at the truth; inversion with the mixed forward."""
    import numpy as np
    import torch

    res = {}
    for case in W.PAPER_INVERSIONS:
        c = W.paper_inversion(case)
        m, cut = c["model"], c["cutoff"]
        gens = 40 if m["n_cycles"] == 1 else 60
        ref = afm.Plan(m, c["params"], [], precision="fp64", device=dev)
        U = ref.forward_batch(None, trace=True)["trace"].contiguous()
        plan = afm.Plan(m, c["params"], c["free"], precision="mixed", device=dev)
        Us = U.expand(swarms, -1).contiguous()
        plan.invert(Us, particles, gens, seed=7, cutoff=cut)  # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = plan.invert(Us, particles, gens, seed=7, cutoff=cut)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        gen = out["gen_to_cutoff"].cpu().numpy()
        bt = out["best_theta"].cpu().numpy()
        ng = gen[gen >= 0] + 1.0  # generations evaluated up to and including the cut-off one
        plan.invert(U, particles, gens, seed=7, cutoff=cut)  # capture (one swarm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.invert(U, particles, gens, seed=7, cutoff=cut)
        torch.cuda.synchronize()
        ms1 = (time.perf_counter() - t0) / gens * 1e3
        mean = float(ng.mean()) if ng.size else None
        # discrete adjoint over one swarm's worth of points drawn in the search box
        rng = np.random.default_rng(11)
        th = torch.tensor(np.stack([rng.uniform(lo, hi, particles) for _, lo, hi, _ in c["free"]]),
                          device=dev)
        plan.grad_batch(th, U)  # stride tuning
        grad_ms = _event_ms(lambda: plan.grad_batch(th, U))
        fwd_ms = _event_ms(lambda: plan.misfit(th, U))
        truth = [c["params"][f[0]] for f in c["free"]]
        err = [float(np.median(np.abs(bt[j] / truth[j] - 1))) for j in range(len(truth))]
        res[case] = {
            "law": m["law"], "free": [f[0] for f in c["free"]], "cutoff_sqrtJ": cut,
            "steps": m["n_cycles"] * m["steps_per_cycle"], "swarms": swarms,
            "particles": particles, "generations_run": gens, "converged_swarms": int(ng.size),
            "mean_generations_to_cutoff": mean,
            "var_generations_to_cutoff": float(ng.var()) if ng.size else None,
            "median_relative_error_of_best": err,
            "batch_ms_per_generation": dt / gens * 1e3,
            "single_inversion_ms_per_generation": ms1,
            "single_inversion_ms_to_cutoff": mean * ms1 if mean else None,
            "adjoint_ms_per_swarm": grad_ms, "adjoint_over_misfit": grad_ms / fwd_ms,
            "paper": c["paper"]}
    return {"workload": "App. A beam, 8 modes from rest, 4e-8 s RK4 steps; base motion or "
                        "sample law unknown; mixed", "cases": res}


def mode_convergence_leg(afm, W, dev):
    """The paper's mode-count study (Sec. 3.3): relative L2 distance of the 1000-step tip trace
    of the App. A beam truncated to m modes from the eight-mode trace, m = 1..7 (FP64)."""
    import numpy as np

    tr = {}
    for m in range(1, 9):
        c = W.mode_convergence(m)
        plan = afm.Plan(c["model"], c["params"], [], precision="fp64", device=dev)
        tr[m] = plan.forward_batch(None, trace=True)["trace"].cpu().numpy()[0]
    err = {m: float(np.linalg.norm(tr[m] - tr[8]) / np.linalg.norm(tr[8])) for m in range(1, 8)}
    return {"workload": "App. A beam, 1000 steps of 1e-7 s from rest, 5 nm base at 25.5 kHz",
            "relative_L2_vs_8_modes": err,
            "paper": "error falls with the mode count; four modes suffice for a sinusoidal base "
                     "(figure only); eight modes track the true solution to 3.3e-6"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(seconds):
    """The oracle (plain FP64, single thread) on the host: a bounded sample of the headline
    workload (pixel trajectories, each pixel's E* and period count, misfit against a window
    trace) until `seconds` of work; the c1 inversion in full; ns per RK4 step of each model
    (forward and adjoint); and each workload's time to inversion extrapolated from those by step
    count."""
    import numpy as np

    import oracle
    import workloads as W

    cfg = W.config("c3")
    m = cfg["model"]
    pix = W.pixels(cfg)
    base = W.full_params(cfg)  # the stored c3 separation (set-point 0.8) stands in for every pixel
    free = W.free_index(cfg)
    th = W.draw_free(cfg, 4000, 99)
    N = m["steps_per_cycle"]
    U = np.sin(np.arange(m["lockin_cycles"] * N) * (2 * np.pi / N)) * 1.6e-8
    t0 = time.perf_counter()
    n, steps = 0, 0
    while n < 4000:
        p = base.copy()
        p[2] = pix["Estar"][n]
        for j, f in enumerate(free):
            p[f[0]] = th[n, j]
        nc = int(pix["cycles"][n])
        oracle.forward(m, p, U, n_cycles=nc)
        steps += nc * N
        n += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    ns = {"dmt_point_mass": dt / steps * 1e9}
    # the plain method (c1) in full: one 32 x 20 inversion from the oracle's own noiseless target
    c1 = W.config("c1")
    m1, p1 = c1["model"], W.full_params(c1)
    U1 = oracle.forward(m1, p1, want_trace=True)["trace"]
    t1 = time.perf_counter()
    r1 = oracle.pso_invert(m1, p1, W.free_index(c1), U1, P=int(c1["particles"]),
                           T=int(c1["iters"]), seed=int(c1["seed"]))
    c1_s = time.perf_counter() - t1
    for name, key, cycles, reps in (("lj_point_mass", "c4", 40, 4), ("kv_3mode", "c5", 20, 2)):
        c = W.config(key)
        mm = dict(c["model"], n_cycles=cycles)
        pp = W.full_params(c)
        Uw = oracle.forward(mm, pp, want_trace=True)["trace"]
        t2 = time.perf_counter()
        for _ in range(reps):
            oracle.forward(mm, pp)
        ns[name] = (time.perf_counter() - t2) / (reps * cycles * mm["steps_per_cycle"]) * 1e9
        t2 = time.perf_counter()
        oracle.misfit_grad(mm, pp, Uw)
        ns[name + "_adjoint"] = (time.perf_counter() - t2) / (cycles * mm["steps_per_cycle"]) * 1e9
    # time to inversion of every workload on this core, extrapolated linearly by step count
    c2, c3, c4, c5 = (W.config(k) for k in ("c2", "c3", "c4", "c5"))

    def pso_steps(c, cycles_total):
        return float(c["particles"]) * c["iters"] * cycles_total * c["model"]["steps_per_cycle"]

    s2 = pso_steps(c2, c2["model"]["n_cycles"])
    s3 = pso_steps(c3, float(np.sum(pix["cycles"])))
    s4 = float(c4["points"]) * c4["model"]["n_cycles"] * c4["model"]["steps_per_cycle"]
    s5 = pso_steps(c5, c5["model"]["n_cycles"])
    s5_pol = float(c5["lbfgs_topk"]) * c5["lbfgs_steps"] * c5["model"]["n_cycles"] * \
        c5["model"]["steps_per_cycle"]  # one gradient and one trial misfit per L-BFGS step
    extrap = {
        "note": "extrapolated: oracle ns per RK4 step (above) x the workload's RK4 steps; "
                "one core; not run",
        "c2_inversion_s": s2 * ns["dmt_point_mass"] * 1e-9,
        "c3_all_4096_pixel_inversions_s": s3 * ns["dmt_point_mass"] * 1e-9,
        "c4_2048_gradients_s": s4 * ns["lj_point_mass_adjoint"] * 1e-9,
        "c5_inversion_s": (s5 * ns["kv_3mode"] + s5_pol * (ns["kv_3mode_adjoint"] + ns["kv_3mode"]))
        * 1e-9,
    }
    return {"value": steps / dt, "unit": "RK4 steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} trajectories of the pixel workload (the pixel's E* and period count, "
                      f"a particle drawn in the (H, E*) box, misfit over the last "
                      f"{m['lockin_cycles']} periods; {steps:.3g} RK4 steps), FP64, single "
                      f"thread, {dt:.1f} s",
            "ns_per_rk4_step": ns,
            "c1_full_inversion": {"seconds": c1_s, "best_J": r1["J"],
                                  "workload": "c1: 32 particles x 20 generations, 100 periods x "
                                              "200 steps, FP64, noiseless oracle target"},
            "time_to_inversion_extrapolated": extrap,
            "host_cpu": _cpu_model(), "host_logical_cpus": os.cpu_count()}


PAPER_CONTEXT = {
    "note": "the paper's own timings, other hardware and workloads; context, not a target",
    "gpu": "NVIDIA Quadro FX 5800 (240 cores), FP32",
    "cpu": "one core of a 2 GHz Xeon",
    "single_forward_solve_s": {"cpu": 0.482, "gpu": 0.0151},
    "batched": "960 solves (8 modes, 1000 RK4 steps) in 0.0151 s",
    "derived_gpu_trajectory_steps_per_s": 6.36e7,
    "derived_cpu_trajectory_steps_per_s": 2.07e3,
    "pso_generation_ms": 16,
}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the inversion path has no "
              "multi-GPU mode.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1109_0334_amd as afm
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "reps": 3}))
        return
    if args.gradient_probe:
        print(json.dumps(gradient_leg(afm, W, dev)))
        return
    if args.queue_probe:
        cfg = W.config("c3")
        S, P = int(cfg["pixels"]), int(cfg["particles"])
        q = _pixel_problem(afm, W, dev, S)
        plan = afm.Plan(q["m"], q["base"], W.free_index(cfg), precision="mixed", device=dev)
        th = torch.tensor(W.draw_free(cfg, S * P, 9).T.copy(), device=dev)
        ms = []
        for _ in range(max(1, args.steps)):
            ms.append(_event_ms(lambda: plan.misfit_swarms(th, q["U"], P, n_cycles=q["cyc"],
                                                           swarm_params=q["spd"])))
        print(json.dumps({"queue_probe_ms": ms}), flush=True)
        return
    if args.c2_probe:
        cfg = W.config("c2")
        m = cfg["model"]
        plan = afm.Plan(m, W.full_params(cfg), W.free_index(cfg), precision="mixed", device=dev)
        U = torch.zeros(1, m["lockin_cycles"] * m["steps_per_cycle"], dtype=torch.float64,
                        device=dev) + 1e-8
        th = torch.tensor(W.draw_free(cfg, cfg["particles"], 5).T.copy(), device=dev)
        plan.misfit(th, U)  # launch-shape tuning
        ms = [_event_ms(lambda: plan.misfit(th, U)) for _ in range(max(1, args.steps))]
        print(json.dumps({"c2_probe_ms": ms}), flush=True)
        return
    K, Wu = max(1, args.steps), max(1, args.warmup)
    h = headline_c3(afm, W, dev, K, Wu)
    h["K"] = K
    dt, S, P, T = h["dt"], h["S"], h["P"], h["T"]
    ms_step = dt / K * 1e3
    line = {
        "metric": "RK4 steps/s", "value": h["steps_per_gen"] * K / dt, "unit": "RK4 steps/s",
        "n_gpus": 1, "steps": K, "warmup": Wu, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "precision": "FP32 RK4 state (compensated), FP64 lock-in and misfit sums",
        "data": "synthetic",
        "config": {"workload": "c3-uneven-pixels: 4096 pixel inversions, point-mass DMT, invert "
                               "(H, log E*), per-pixel E*, set-point and period count "
                               "(U{100..2000} x 256 RK4 steps), 128 particles per pixel, "
                               "persistent work queue, graph-captured generations",
                   "pixels": S, "particles_per_pixel": P, "steps_per_period": 256,
                   "generations_per_inversion": T},
        "inversions_per_s": S / (ms_step * 1e-3 * T),
        "rk4_steps_per_generation": h["steps_per_gen"],
        "roofline": h["roofline"],
        "median_best_J_after_steps": h["median_best_J"],
        "plain_grid_forward_ms": h["plain_grid_forward_ms"],
        "setup_separation_s": h["setup_separation_s"],
        "pixels_without_setpoint_crossing": h["pixels_without_setpoint_crossing"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    U2 = cfg2 = None
    if not args.no_extras:
        c2, U2, cfg2 = c2_leg(afm, W, dev, K, Wu)
        line["c2_precision_path"] = c2
        line["steady_state_exit"] = steady_exit_leg(afm, W, dev, h, max(1, args.pixel_steps))
    if not args.no_more:
        if U2 is not None:
            line["time_to_inversion"] = time_to_inversion(afm, W, dev, U2, cfg2)
        line["time_to_inversion_pixels"] = pixel_time_to_inversion(afm, W, dev, 256, cutoff=1e-3)
        line["plain_method"] = plain_method_leg(afm, W, dev)
        line["paper_solver_shape"] = paper_solver_leg(afm, W, dev)
        line["gradients"] = gradient_leg(afm, W, dev)
        line["three_mode"] = three_mode_leg(afm, W, dev, full=not args.short_c5)
        line["paper_inversions"] = paper_inversions_leg(afm, W, dev)
        line["mode_convergence"] = mode_convergence_leg(afm, W, dev)
    line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
