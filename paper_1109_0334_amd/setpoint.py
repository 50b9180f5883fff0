"""Tip-sample separation from an amplitude set-point, for many pixels at once.

Argument marshalling for ``afm_separations`` (include/afm.h): dynamic AFM holds the oscillation
amplitude at a set-point by feedback on the separation (paper Sec. 1); the library finds, for
each pixel, the separation z_c at which the steady amplitude equals s * A0 the way an approach
curve does (grid from A0 + 2 nm down, then 16-point sections of the bracket), all on the GPU.
"""
from __future__ import annotations

import numpy as np


def separations(afm, model, base, pixel_free, pixel_values, setpoint, *, periods=3000, lockin=2,
                step=0.25e-9, rounds=6, device="cuda"):
    """z_c [S] (numpy, m) for S pixels.

    model: model dict; base: full parameter vector (z_c entry ignored); pixel_free: law-parameter
    indices that vary per pixel; pixel_values: [len(pixel_free)][S] their values; setpoint: [S].
    """
    pixel_values = np.atleast_2d(np.asarray(pixel_values, np.float64))
    setpoint = np.asarray(setpoint, np.float64)
    S = setpoint.shape[0]
    params = np.tile(np.zeros(afm.MAX_PARAMS), (S, 1)).T.copy()
    b = np.asarray(base, np.float64)
    params[:b.size] = b[:, None]
    for j, q in enumerate(pixel_free):
        params[int(q)] = pixel_values[j]
    plan = afm.Plan(model, base, (), precision="fp64", device=device)
    zc = plan.separations(setpoint, params, periods=periods, lockin=lockin, step=step,
                          rounds=rounds)
    out = zc.cpu().numpy()
    plan.close()
    return out
