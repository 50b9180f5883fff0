"""Helpers for GPU-vs-oracle parity tests: tolerances and the conditioning filter.

Tolerances (per result, against the FP64 oracle):
* amplitude: |dA| <= max(1e-5 A, 5e-6 A0).  The state of every trajectory is O(A0) (the gap or
  deflection swings over ~A0 whatever the final amplitude), so the FP32 resolution of the
  amplitude is set by A0: for a trajectory trapped at small amplitude the stated 1e-5 relative
  bound would ask for more than FP32 can hold; 5e-6 A0 (1e-4 nm at A0 = 20 nm) is the floor;
* phase: |dphi| <= max(1e-4, 5e-6 A0 / A) rad (the same deflection floor seen as a phase);
* misfit: |J_gpu - J_orc| <= 1e-4 J_orc + 2 sqrt(J_orc) eps_u + eps_u^2 with eps_u = 1e-5, the
  change of J = |U - u|^2/|U|^2 that a relative deflection error eps_u produces (a pure relative
  bound is meaningless as J -> 0);
* plain FP64 path: 1e-9 relative amplitude, 1e-9 rad phase (rounding-order differences only).

A trajectory counts toward mixed-precision parity only if the FP64 oracle itself is well
conditioned there: changing any force-law constant by 1e-7 relative (about two FP32 ulps, the
resolution at which an FP32 solver holds the problem's data) must move the oracle's amplitude by
at most 1e-7 relative and its phase by at most 1e-6 rad -- a hundredth of the tolerance.  Where a
discrete orbit is that sensitive (steep contact walls resolved by few steps) no FP32 solver can
promise the tolerance.  Excluded fractions are printed and bounded by each test.  Only the law's
constants (parameter slots 0 .. 7) are perturbed: the base-motion parameters of a
parameter-driven base (slots 8 .. 10) are not FP32 data of the kernel -- it forms their phase in
FP64 -- and their amplitude enters the response linearly.
"""
import numpy as np

A_RTOL = 1e-5
A_FLOOR = 5e-6   # times A0
PHI_ATOL = 1e-4
EPS_U = 1e-5
FP64_RTOL = 1e-9


def misfit_tol(Jo):
    Jo = np.asarray(Jo, dtype=np.float64)
    return 1e-4 * Jo + 2 * np.sqrt(Jo) * EPS_U + EPS_U**2


def wrap(dphi):
    return np.angle(np.exp(1j * np.asarray(dphi)))


def amp_ok(Ag, Ao, A0):
    return np.abs(Ag - Ao) <= np.maximum(A_RTOL * np.abs(Ao), A_FLOOR * A0)


def phase_ok(pg, po, Ao, A0):
    return np.abs(wrap(pg - po)) <= np.maximum(PHI_ATOL, A_FLOOR * A0 / np.abs(Ao))


def well_conditioned(orc, model, p, rel=1e-7):
    """Oracle (A, phi) move by <= 1e-7 A and 1e-6 rad under a `rel` change of any law constant."""
    r0 = orc.forward(model, p)
    if r0["status"]:
        return True
    for j in range(min(len(p), 8)):
        if p[j] == 0:
            continue
        for sgn in (1.0, -1.0):
            q = np.array(p, dtype=np.float64)
            q[j] *= 1.0 + sgn * rel
            r = orc.forward(model, q)
            if r["status"] != 0:
                return False
            if abs(r["A"] / r0["A"] - 1) > 1e-7 or abs(wrap(r["phi"] - r0["phi"])) > 1e-6:
                return False
    return True


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


def compare_mixed(orc, model, P, o, A, phi, st, J=None, tag="", n_cycles=None):
    """Classify each trajectory as passing, excluded (ill-conditioned oracle) or failing.

    Failure (a non-zero status word) must agree except on excluded trajectories -- which bit is
    set may differ: a blow-up that FP64 reports as non-finite can stay finite but huge in FP32;
    amplitude, phase and (if given) misfit must meet the tolerances above.  Returns (failing indices, excluded indices)."""
    A0 = model["free_amplitude"]
    n = len(A)
    bad = np.zeros(n, bool)
    both_ok = (st == 0) & (o["status"] == 0)
    bad |= (st != 0) != (o["status"] != 0)
    bad[both_ok] |= ~amp_ok(A[both_ok], o["A"][both_ok], A0)
    bad[both_ok] |= ~phase_ok(phi[both_ok], o["phi"][both_ok], o["A"][both_ok], A0)
    if J is not None:
        bad[both_ok] |= np.abs(J[both_ok] - o["J"][both_ok]) > misfit_tol(o["J"][both_ok])
    excluded, failing = [], []
    for i in np.flatnonzero(bad):
        m = model if n_cycles is None else dict(model, n_cycles=int(n_cycles[i]))
        (failing if well_conditioned(orc, m, P[i]) else excluded).append(int(i))
    if both_ok.any():
        eA = np.abs(A[both_ok] / o["A"][both_ok] - 1)
        eP = np.abs(wrap(phi[both_ok] - o["phi"][both_ok]))
        print(f"{tag}: n {n}, max |dA|/A {eA.max():.2e} (median {np.median(eA):.1e}), max |dphi| "
              f"{eP.max():.2e} (median {np.median(eP):.1e}), excluded {len(excluded)}, "
              f"failing {len(failing)}")
    return failing, excluded


def grad_sensitivity(orc, model, p, target, free, rel):
    """Largest norm-wise relative change (normalised coordinates) of the oracle's gradient under
    a `rel` relative change of any one law constant."""
    st, J0, g0 = orc.misfit_grad(model, p, target)
    if st:
        return 0.0
    idx = [f[0] for f in free]
    scale = np.array([p[f[0]] * np.log(f[2] / f[1]) if f[3] else f[2] - f[1] for f in free])
    gz0 = g0[idx] * scale
    worst = 0.0
    for j in range(len(p)):
        if p[j] == 0:
            continue
        for sgn in (1.0, -1.0):
            q = np.array(p, dtype=np.float64)
            q[j] *= 1.0 + sgn * rel
            st, J, g = orc.misfit_grad(model, q, target)
            if st:
                return np.inf
            worst = max(worst, np.linalg.norm(g[idx] * scale - gz0) / np.linalg.norm(gz0))
    return worst


# Gradient tolerance.  The mixed adjoint is the exact gradient of the FP32 trajectory, which
# behaves like the exact trajectory with its data moved by up to ~1e-5 relative (its constants
# are FP32-rounded and its amplitude and phase errors, <= 3e-6 and <= 3e-5 rad on the C2 box,
# match such a move).  Where the misfit landscape is finely corrugated the exact gradient itself
# swings under such a move, so the tolerance of a point is the larger of 1e-3 and three times
# the oracle gradient's own change under a 1e-5 relative change of its data.  The FP64 path is
# held to 1e-6, widened the same way with a 1e-10 relative change.
GRAD_TOL, GRAD_REL = 1e-3, 1e-5
GRAD_TOL64, GRAD_REL64 = 1e-6, 1e-10


def grad_tolerance(orc, model, p, target, free, fp64=False):
    tol, rel = (GRAD_TOL64, GRAD_REL64) if fp64 else (GRAD_TOL, GRAD_REL)
    return max(tol, 3.0 * grad_sensitivity(orc, model, p, target, free, rel))
