"""Seeded synthetic workloads for the dynamic-AFM force inversion.

This module only describes inputs: cantilever and drive constants, force-law parameter boxes,
truth values, batch sizes and seeded random draws (NumPy PCG64).  It holds none of the method's
arithmetic (no integration, lock-in, misfit, set-point search or swarm update), so both the GPU
library's callers and the CPU oracle's callers can share it.

The five workloads follow the paper's setting -- a base-driven cantilever tapping a sample, a
parameterised tip-sample force, PSO over the force parameters (Sec. 2-4) -- with the force laws
the paper lists as its extension (adhesion / van der Waals, Sec. 5):

* ``c1`` point-mass DMT, invert (H, E*), 32 particles x 20 generations, 100 x 200 steps, FP64.
* ``c2`` point-mass DMT, invert (H, E*, a0), 1024 x 200, 500 x 256 steps, noisy target.
* ``c3`` 4096 pixel inversions of (H, E*) with per-pixel E*, set-point and cycle count.
* ``c4`` LJ-type law, 4 parameters, 2048 points for the adjoint gradient, 1000 x 256 steps.
* ``c5`` 3-mode beam, Kelvin-Voigt contact + vdW, 5 parameters, 16384 x 300, 2000 x 512 steps.

``paper_inversion`` describes the paper's own inversions (Sec. 4) on its 8-mode beam.

Separations z_c are *not* computed here: they follow from the set-point by the method's own
amplitude feedback and are stored in ``tests/golden/setpoint_zc.json`` by a script that calls
the oracle only.  Law parameter vectors hold z_c at index 0.
"""
from __future__ import annotations

import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
ZC_FILE = os.path.join(_HERE, "tests", "golden", "setpoint_zc.json")

NM = 1e-9
GPA = 1e9

LAW_PARAMS = {
    "dmt": ("zc", "H", "Estar", "a0", "R"),
    "lj": ("zc", "eps", "r0", "n", "m"),
    "kv": ("zc", "H", "Estar", "a0", "R", "eta"),
    "hooke": ("zc", "ks"),
    "sd": ("zc", "ks", "zeta_s"),
    "none": ("zc",),
}

# Point-mass cantilever of the DMT workloads: k = 40 N/m, f0 = 300 kHz, Q = 400, driven at f0
# with free amplitude A0 = 20 nm; tip radius 10 nm.
_PM = dict(n_modes=1, law="dmt", k=40.0, f0=300e3, drive_freq=300e3, q=[400.0], ratio=[1.0],
           gain=[1.0], free_amplitude=20 * NM, ic="free_steady", div_limit=100.0)

_DMT_TRUTH = dict(H=6.4e-20, Estar=1.0 * GPA, a0=0.3 * NM, R=10 * NM)

CONFIGS = {
    "c1": dict(
        model=dict(_PM, steps_per_cycle=200, n_cycles=100, lockin_cycles=20),
        truth=dict(_DMT_TRUTH), setpoint=0.8,
        free=[("H", 1e-20, 1e-19, False), ("Estar", 0.1 * GPA, 10 * GPA, False)],
        particles=32, iters=20, seed=0, noise=0.0, precision="fp64"),
    "c2": dict(
        model=dict(_PM, steps_per_cycle=256, n_cycles=500, lockin_cycles=20),
        truth=dict(_DMT_TRUTH), setpoint=0.8,
        free=[("H", 1e-20, 1e-19, False), ("Estar", 0.1 * GPA, 10 * GPA, False),
              ("a0", 0.1 * NM, 0.5 * NM, False)],
        particles=1024, iters=200, seed=0, noise=0.05 * NM, precision="mixed"),
    "c3": dict(
        model=dict(_PM, steps_per_cycle=256, n_cycles=2000, lockin_cycles=20),
        truth=dict(_DMT_TRUTH), setpoint=0.8,
        free=[("H", 1e-20, 1e-19, False), ("Estar", 0.05 * GPA, 50 * GPA, True)],
        particles=128, iters=100, seed=0, noise=0.0, precision="mixed",
        pixels=4096, estar_range=(0.05 * GPA, 50 * GPA), setpoint_range=(0.5, 0.9),
        cycles_range=(100, 2000)),
    "c4": dict(
        model=dict(_PM, law="lj", ic="rest", steps_per_cycle=256, n_cycles=1000,
                   lockin_cycles=20),
        truth=dict(eps=1.25e-19, r0=0.35 * NM, n=10.0, m=5.5), setpoint=0.8,
        free=[("eps", 0.5e-19, 2.0e-19, False), ("r0", 0.2 * NM, 0.5 * NM, False),
              ("n", 8.0, 12.0, False), ("m", 4.0, 7.0, False)],
        points=2048, seed=0, noise=0.0, precision="mixed", ckpt_strides=(16, 64, 256)),
    "c5": dict(
        model=dict(_PM, law="kv", n_modes=3, q=[400.0, 400.0, 400.0], ratio=[1.0, 6.27, 17.55],
                   gain=None, steps_per_cycle=512, n_cycles=2000, lockin_cycles=20),
        truth=dict(H=6.4e-20, Estar=0.1 * GPA, a0=0.3 * NM, R=10 * NM, eta=10.0),
        setpoint=0.8,
        free=[("zc", -5 * NM, 5 * NM, False), ("H", 1e-20, 1e-19, False),
              ("Estar", 0.01 * GPA, 1.0 * GPA, True), ("a0", 0.1 * NM, 0.5 * NM, False),
              ("eta", 1.0, 100.0, True)],
        particles=16384, iters=300, seed=0, noise=0.0, precision="mixed", lbfgs_steps=10,
        lbfgs_topk=64),
}


# The paper's own inversions (Sec. 4) on its App. A cantilever -- 8 Euler-Bernoulli modes,
# first at 25468.9 Hz, L = 525 um, E = 1.76e11 Pa, section 35 x 5 um, so k = 3 E I / L^3 with
# I = w h^3 / 12 -- started at rest, RK4 steps of 4e-8 s (1000 per period of a 25 kHz time unit),
# misfit over the whole trajectory.  The paper gives no damping for this beam: Q = 400 per mode.
# It states 512 particles for the 1-D runs; every case uses the same.
#
# Base motion (Sec. 4.1): y_b = a sin(2 pi (f + g t) t) (Eq. 9 with g = 0, Eq. 10) is the
# unknown; a free tip (no force law, z_c = 0), n_t = 1000 steps.
#
# Sample (Sec. 4.2, 4.3): the base motion is known -- App. A's drive, 5 nm at 25.5 kHz -- and the
# tip meets a Hooke spring (Eq. 11) or spring-damper (Eq. 12) sample h = 50 nm away
# (z_c = h; the gap closes when the tip deflects 50 nm towards the sample); n_t = 10000 steps
# (the top of the range Sec. 4.1 tried), so that the tip, ringing up from rest, presses into the
# sample over the later periods.  The printed spring-damper truth zeta_s = 0.1 N s/m (box
# [0, 2]) puts zeta_s dt / m_1 near 77 for this beam, far outside explicit RK4's stability
# interval: every trajectory in contact diverges, the truth included.  zeta_s and its box are
# scaled by 1e-4 (truth 1e-5 N s/m, box [0, 2e-4]), the largest power of ten that keeps the box
# stable.
_EB_I = 35e-6 * 5e-6**3 / 12.0
_BEAM = dict(n_modes=8, law="none", k=3.0 * 1.76e11 * _EB_I / 525e-6**3, f0=25468.9,
             drive_freq=25e3, q=[400.0] * 8, free_amplitude=20 * NM, ic="rest", div_limit=1e4,
             steps_per_cycle=1000, n_cycles=1, lockin_cycles=1, drive="params")
_APP_A_DRIVE = (5 * NM, 25500.0, 0.0)

PAPER_INVERSIONS = {
    "1d": dict(base=(2 * NM, 25600.0, 0.0), free=[(8, 0.0, 100 * NM, False)], cutoff=1e-2,
               paper=dict(generations=3.0, ms=48.0, note="mean, 512 particles, cut-off 0.01")),
    "1d_tight": dict(base=(2 * NM, 25600.0, 0.0), free=[(8, 0.0, 100 * NM, False)],
                     cutoff=1e-3, paper=dict(generations=7.99, ms=128.0, note="cut-off 0.001")),
    "2d": dict(base=(2 * NM, 25600.0, 0.0),
               free=[(8, 0.0, 100 * NM, False), (9, 25100.0, 26100.0, False)], cutoff=1e-2,
               paper=dict(generations=19.0458, ms=320.0, note="a and f, a 1000 Hz box")),
    "3d_chirp": dict(base=(2 * NM, 10e3, 2e7),
                     free=[(8, 0.0, 100 * NM, False), (9, 7500.0, 12500.0, False),
                           (10, 1.9e7, 2.1e7, False)], cutoff=1e-2,
                     paper=dict(generations=14.9, ms=240.0, note="a, f, g (chirp)")),
    "spring": dict(law="hooke", law_params=(50 * NM, 4.0), base=_APP_A_DRIVE, n_cycles=10,
                   free=[(0, 0.0, 100 * NM, False), (1, 0.0, 25.0, False)], cutoff=5e-4,
                   paper=dict(generations=18.0, ms=288.0,
                              note="h and k unknown, cut-off J_L2 = 0.0005; box not printed")),
    "spring_damper": dict(law="sd", law_params=(50 * NM, 4.0, 1e-5), base=_APP_A_DRIVE,
                          n_cycles=10, free=[(1, 0.0, 25.0, False), (2, 0.0, 2e-4, False)],
                          cutoff=5e-4,
                          paper=dict(generations=16.0, ms=256.0,
                                     note="k and zeta_s unknown, h known; zeta_s scaled 1e-4")),
}
BASE_MOTION = ("1d", "1d_tight", "2d", "3d_chirp")


def paper_inversion(case: str) -> dict:
    """One of the paper's inversions: model, full 12-entry parameter vector at the truth (the
    law's first, z_c at 0; a, f, g at 8, 9, 10), free-parameter spec, cut-off on sqrt(J)."""
    c = PAPER_INVERSIONS[case]
    eb = beam_modes(8)
    nc = int(c.get("n_cycles", 1))
    model = dict(_BEAM, law=c.get("law", "none"), ratio=list(eb["ratio"]), gain=list(eb["gain"]),
                 n_cycles=nc, lockin_cycles=nc)
    p = np.zeros(12)
    lp = c.get("law_params", (0.0,))
    p[: len(lp)] = lp
    p[8], p[9], p[10] = c["base"]
    return dict(model=model, params=p, free=[tuple(f) for f in c["free"]], cutoff=c["cutoff"],
                paper=dict(c["paper"]))


def mode_convergence(n_modes: int) -> dict:
    """The paper's mode-count study (Sec. 3.3): the App. A beam truncated to its first n_modes
    modes, 1000 RK4 steps of 1e-7 s from rest (two periods of a 20 kHz time unit, 500 steps
    each), App. A's sinusoidal base motion (5 nm at 25.5 kHz), no tip force; the whole trace is
    compared against the eight-mode one.  Returns dict(model, params)."""
    eb = beam_modes(8)
    model = dict(_BEAM, n_modes=n_modes, q=[400.0] * n_modes, ratio=list(eb["ratio"][:n_modes]),
                 gain=list(eb["gain"][:n_modes]), drive_freq=20e3, steps_per_cycle=500,
                 n_cycles=2, lockin_cycles=2)
    p = np.zeros(12)
    p[8], p[9], p[10] = _APP_A_DRIVE
    return dict(model=model, params=p)


def base_motion(case: str) -> dict:
    """One of the paper's base-motion problems (Sec. 4.1); see paper_inversion."""
    assert case in BASE_MOTION
    return paper_inversion(case)


def stored_setpoints() -> dict:
    """Separations and modal gains written by tests/golden/make_setpoints.py (oracle only)."""
    with open(ZC_FILE) as f:
        return json.load(f)


def beam_modes(n: int) -> dict:
    """Stored frequency ratios and base-drive gains of the first n Euler-Bernoulli modes."""
    return stored_setpoints()[f"eb{n}"]


def config(name: str, **overrides) -> dict:
    """A deep-enough copy of a workload with its stored z_c (and 3-mode gains) filled in."""
    c = json.loads(json.dumps(CONFIGS[name]))
    c["free"] = [tuple(f) for f in c["free"]]
    st = stored_setpoints() if os.path.exists(ZC_FILE) else {}
    rec = st.get(name, {})
    if c["model"].get("gain") is None:
        c["model"]["gain"] = rec.get("gain", [1.0] * c["model"]["n_modes"])
    c["zc"] = rec.get("zc")
    for k, v in overrides.items():
        if k in c["model"]:
            c["model"][k] = v
        else:
            c[k] = v
    return c


def law_names(cfg) -> tuple:
    return LAW_PARAMS[cfg["model"]["law"]]


def full_params(cfg, zc=None, **vals) -> np.ndarray:
    """Full law parameter vector (z_c first) from the truth values with overrides."""
    names = law_names(cfg)
    d = dict(cfg["truth"])
    d["zc"] = cfg["zc"] if zc is None else zc
    d.update(vals)
    return np.array([float(d[n]) for n in names])


def free_index(cfg) -> list:
    """[(index into the full vector, lo, hi, log_scale)] for the free parameters.  For laws
    whose z_c is free, the z_c box is relative to the stored separation."""
    names = law_names(cfg)
    out = []
    for name, lo, hi, lg in cfg["free"]:
        if name == "zc":
            lo, hi = cfg["zc"] + lo, cfg["zc"] + hi
        out.append((names.index(name), lo, hi, lg))
    return out


def draw_free(cfg, n: int, seed: int) -> np.ndarray:
    """n seeded points from the free-parameter box ([n][D]; log-scaled ones log-uniform)."""
    rng = np.random.default_rng(seed)
    cols = []
    for _, lo, hi, lg in free_index(cfg):
        u = rng.random(n)
        cols.append(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo))) if lg else lo + u * (hi - lo))
    return np.stack(cols, axis=1)


def noise(cfg, W: int, seed: int) -> np.ndarray:
    """Gaussian measurement noise (sigma from the workload) added to a synthetic target."""
    sig = float(cfg.get("noise", 0.0))
    if sig == 0.0:
        return np.zeros(W)
    return np.random.default_rng(seed + 7919).normal(0.0, sig, W)


def pixels(cfg, seed: int = 0) -> dict:
    """Per-pixel draws of the uneven-batching workload: E* log-uniform, set-point uniform,
    cycle count uniform on the integers."""
    rng = np.random.default_rng(seed + 104729)
    S = int(cfg["pixels"])
    lo, hi = cfg["estar_range"]
    estar = np.exp(np.log(lo) + rng.random(S) * (np.log(hi) - np.log(lo)))
    s_lo, s_hi = cfg["setpoint_range"]
    setpoint = s_lo + rng.random(S) * (s_hi - s_lo)
    c_lo, c_hi = cfg["cycles_range"]
    cycles = rng.integers(c_lo, c_hi + 1, S).astype(np.int32)
    return {"Estar": estar, "setpoint": setpoint, "cycles": cycles}
