"""Tip-sample separation from an amplitude set-point, for many pixels at once.

Dynamic AFM holds the oscillation amplitude at a set-point by feedback on the separation
(paper Sec. 1).  Given each pixel's force-law parameters and set-point s, this finds the
separation z_c at which the steady amplitude equals s * A0, the way an approach curve does:
z_c steps down from A0 + 2 nm in 0.25 nm steps until the amplitude first drops below the
set-point, then the bracket is narrowed by 16-point sections.  Every amplitude is a forward solve
of the library (afm_forward_batch) over many periods; all pixels and all trial separations of a
round go in one launch.
"""
from __future__ import annotations

import numpy as np


def separations(afm, model, base, pixel_free, pixel_values, setpoint, *, precision="fp64",
                periods=3000, lockin=2, step=0.25e-9, rounds=6, sections=16, device="cuda"):
    """z_c [S] for S pixels.

    model: model dict; base: full parameter vector (z_c entry ignored); pixel_free: law-parameter
    indices that vary per pixel; pixel_values: [len(pixel_free)][S] their values; setpoint: [S].
    """
    import torch

    pixel_values = np.atleast_2d(np.asarray(pixel_values, np.float64))
    setpoint = np.asarray(setpoint, np.float64)
    S = setpoint.shape[0]
    A0 = float(model["free_amplitude"])
    m = dict(model, n_cycles=int(periods), lockin_cycles=int(lockin))
    free = [(0, 0.0, 1.0, False)] + [(int(q), 0.0, 1.0, False) for q in pixel_free]
    plan = afm.Plan(m, base, free, precision=precision, device=device)
    # each round is one long launch of a new size: skip the launch-shape tuning (which would
    # run it once per candidate) and take GPU-filling 4-wave workgroups
    plan.set_launch_shape(256, 1)

    def amplitudes(z):  # z: [S][k] -> A [S][k]
        k = z.shape[1]
        theta = np.empty((1 + len(pixel_free), S * k))
        theta[0] = z.reshape(-1)
        for j in range(len(pixel_free)):
            theta[1 + j] = np.repeat(pixel_values[j], k)
        r = plan.forward_batch(torch.tensor(theta, device=device))
        A = r["amp"].cpu().numpy().reshape(S, k)
        return np.where(r["status"].cpu().numpy().reshape(S, k) == 0, A, -np.inf)

    target = setpoint * A0
    grid = A0 + 2e-9 - step * np.arange(int((A0 + 2e-9) / step))
    A = amplitudes(np.tile(grid, (S, 1)))
    below = A < target[:, None]
    first = np.argmax(below, axis=1)
    ok = below.any(axis=1) & (first > 0)
    lo = np.where(ok, grid[np.maximum(first, 1)], np.nan)        # amplitude below the set-point
    hi = np.where(ok, grid[np.maximum(first, 1) - 1], np.nan)    # amplitude above it
    for _ in range(rounds):
        frac = (np.arange(1, sections + 1) / (sections + 1))
        z = lo[:, None] + (hi - lo)[:, None] * frac[None, :]
        A = amplitudes(np.nan_to_num(z))
        above = A >= target[:, None]
        # the bracket keeps the last trial below the set-point and the first one above it
        idx = np.argmax(above, axis=1)
        any_above = above.any(axis=1)
        new_hi = np.where(any_above, z[np.arange(S), idx], hi)
        new_lo = np.where(any_above, np.where(idx > 0, z[np.arange(S), np.maximum(idx - 1, 0)], lo),
                          z[:, -1])
        lo, hi = new_lo, new_hi
    return 0.5 * (lo + hi)
