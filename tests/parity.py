"""Helpers for GPU-vs-oracle parity tests: tolerances and the conditioning filter.

Tolerances (per result, against the FP64 oracle):
* amplitude: 1e-5 relative; phase: 1e-4 rad;
* misfit: |J_gpu - J_orc| <= 1e-4 J_orc + 2 sqrt(J_orc) eps_u + eps_u^2 with eps_u = 1e-5, the
  change of J = |U - u|^2/|U|^2 that a relative deflection error eps_u produces (a pure relative
  bound is meaningless as J -> 0);
* plain FP64 path: 1e-9 relative amplitude, 1e-9 rad phase (rounding-order differences only).

A trajectory counts toward mixed-precision parity only if the FP64 oracle itself is well
conditioned there: moving the initial deflection by 1e-9 A0 must change the amplitude by less
than 1e-7 relative (near a separatrix between tapping branches FP32 rounding may pick the other
branch).  Excluded fractions are reported by the tests.
"""
import numpy as np

A_RTOL = 1e-5
PHI_ATOL = 1e-4
EPS_U = 1e-5
FP64_RTOL = 1e-9


def misfit_tol(Jo):
    Jo = np.asarray(Jo, dtype=np.float64)
    return 1e-4 * Jo + 2 * np.sqrt(Jo) * EPS_U + EPS_U**2


def wrap(dphi):
    return np.angle(np.exp(1j * np.asarray(dphi)))


def well_conditioned(orc, model, p):
    """Oracle amplitude is insensitive (1e-7) to a 1e-9 A0 change of the initial deflection."""
    y0 = orc.initial_state(model)
    r0 = orc.forward(model, p)
    y1 = y0.copy()
    y1[0] += 1e-9 * model["free_amplitude"]
    W = orc.window_len(model)
    st, u, _, _ = orc.trajectory(model, p, y0=y1, n_out=W)
    if st or r0["status"]:
        return True
    A1, _ = orc.lockin(u, model["steps_per_cycle"], 1)
    return abs(A1 - r0["A"]) <= 1e-7 * abs(r0["A"])


def oracle_batch(orc, model, P, target=None, n_cycles=None):
    """Oracle forward solves for rows of P ([n][nparams])."""
    n = P.shape[0]
    out = {k: np.empty(n) for k in ("A", "phi", "J")}
    out["status"] = np.empty(n, np.int32)
    for i in range(n):
        nc = None if n_cycles is None else int(n_cycles[i])
        r = orc.forward(model, P[i], target, n_cycles=nc)
        for k in ("A", "phi", "J", "status"):
            out[k][i] = r[k]
    return out


def full_from_free(base, free, theta):
    """[n][nparams] full parameter rows from the base vector and theta [D][n]."""
    theta = np.atleast_2d(theta)
    P = np.tile(np.asarray(base, np.float64), (theta.shape[1], 1))
    for j, f in enumerate(free):
        P[:, f[0]] = theta[j]
    return P
