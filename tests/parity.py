"""Helpers for GPU-vs-oracle parity tests: tolerances and the conditioning filters.

Forward tolerances (per result, against the FP64 oracle; the stated bars):
* amplitude: |dA| <= 1e-5 A;
* phase: |dphi| <= 1e-4 rad;
* misfit: |J_gpu - J_orc| <= 1e-4 J_orc + 2 sqrt(J_orc) eps_u + eps_u^2 with eps_u = 1e-5, the
  change of J = |U - u|^2/|U|^2 that a relative deflection error eps_u produces (a pure relative
  bound is meaningless as J -> 0);
* plain FP64 path: 1e-9 relative amplitude, 1e-9 rad phase (rounding-order differences only).
Small orbits: for a trajectory whose oracle amplitude is below A0/4 (a tip trapped at small
amplitude), the amplitude bar is max(1e-5 A, 5e-6 A0) and the phase bar max(1e-4, 5e-6 A0/A)
rad.  The state of every trajectory swings over ~A0 (the gap or the deflection) whatever its
final amplitude, so FP32 resolves that amplitude only to a fraction of A0; the floor never
applies at A >= A0/4, where 1e-5 A >= 2.5e-6 A0.  Every comparison also counts the trajectories
that meet the bars without any floor (`strict`), and the tests bound that count from below.

Conditioning: a mixed-precision mismatch is excused only where the FP64 oracle itself is ill
conditioned at the resolution at which an FP32 solver holds the problem's data: changing any
force-law constant by 1e-7 relative (about two FP32 ulps) moves the oracle's amplitude by more
than 1e-7 relative or its phase by more than 1e-6 rad -- a hundredth of the tolerance -- or
changes whether the oracle's trajectory fails.  Whether a trajectory fails at all (it becomes
non-finite or diverges, e.g. crashing through a steep wall the time step barely resolves) is a
yes/no event: where the GPU and the oracle disagree on it, the disagreement is excused only if
the oracle's own verdict changes when its initial state moves by at most 1e-5 A0, the amount by
which a solver that meets the amplitude bar may move the orbit.  For every
excused trajectory the comparison also reports the measurement behind that reading: how far the
oracle moves when its law constants are rounded to FP32 (with FP64 arithmetic), next to the GPU's
error.  Excluded counts are bounded by each test.  Only the law's constants (parameter slots
0 .. 7) are perturbed: the base-motion parameters of a parameter-driven base (slots 8 .. 10) are
not FP32 data of the kernel -- it forms their phase in FP64 -- and their amplitude enters the
response linearly.

Gradient (reading G18): norm-wise in normalised coordinates against the oracle's exact discrete
adjoint, on retained points.  FP64 path: 1e-6, a point retained when the oracle's gradient moves
by at most a third of that under a 1e-10 relative change of any law constant.  Mixed path: a
point is retained when the oracle's gradient moves by at most a third of 1e-3 under a 1e-7
relative change of any law constant (the FP32 resolution of the data) and responds about
linearly beyond, up to 1e-5 (a faster response means a change of that size crosses a kink of
the misfit: contact onset, the attraction frozen in contact); on retained points the mixed
gradient must be within 5e-3 of the oracle's and within 1e-3 at the median -- the FP32
trajectory's own deviation from the FP64 one moves the exact gradient of the map by that much
over the long horizons (measured: the FP64 path, same kernels, meets 1e-10 there).  Excluded
points are counted and bounded by each test; no tolerance depends on the point.  A status
mismatch is excused as for the forward solve.
"""
import numpy as np

A_RTOL = 1e-5
A_FLOOR = 5e-6   # times A0, below A0/4 only
SMALL_ORBIT = 0.25  # times A0
PHI_ATOL = 1e-4
EPS_U = 1e-5
FP64_RTOL = 1e-9


def misfit_tol(Jo):
    Jo = np.asarray(Jo, dtype=np.float64)
    return 1e-4 * Jo + 2 * np.sqrt(Jo) * EPS_U + EPS_U**2


def wrap(dphi):
    return np.angle(np.exp(1j * np.asarray(dphi)))


def _small(Ao, A0):
    return np.abs(Ao) < SMALL_ORBIT * A0


def amp_ok(Ag, Ao, A0):
    bar = np.where(_small(Ao, A0), np.maximum(A_RTOL * np.abs(Ao), A_FLOOR * A0),
                   A_RTOL * np.abs(Ao))
    return np.abs(Ag - Ao) <= bar


def phase_ok(pg, po, Ao, A0):
    bar = np.where(_small(Ao, A0), np.maximum(PHI_ATOL, A_FLOOR * A0 / np.abs(Ao)), PHI_ATOL)
    return np.abs(wrap(pg - po)) <= bar


def strict_ok(Ag, Ao, pg, po, Jg=None, Jo=None):
    """The stated bars with no floor."""
    ok = (np.abs(Ag - Ao) <= A_RTOL * np.abs(Ao)) & (np.abs(wrap(pg - po)) <= PHI_ATOL)
    if Jg is not None:
        ok &= np.abs(Jg - Jo) <= misfit_tol(Jo)
    return ok


def well_conditioned(orc, model, p, rel=1e-7):
    """Oracle (A, phi) move by <= 1e-7 A and 1e-6 rad under a `rel` change of any law constant,
    and its failure status does not change (a trajectory that fails only for some of those
    data, e.g. one that crashes through a singular wall, is ill conditioned)."""
    r0 = orc.forward(model, p)
    for j in range(min(len(p), 8)):
        if p[j] == 0:
            continue
        for sgn in (1.0, -1.0):
            q = np.array(p, dtype=np.float64)
            q[j] *= 1.0 + sgn * rel
            r = orc.forward(model, q)
            if (r["status"] != 0) != (r0["status"] != 0):
                return False
            if r0["status"]:
                continue
            if abs(r["A"] / r0["A"] - 1) > 1e-7 or abs(wrap(r["phi"] - r0["phi"])) > 1e-6:
                return False
    return True


FATE_RELS = (1e-7, 2e-7, 5e-7, 1e-6, 2e-6, 5e-6, 1e-5)


def fate_conditioned(orc, model, p):
    """Whether the oracle's failure status (a trajectory that becomes non-finite or diverges,
    e.g. crashing through a steep wall that the time step barely resolves) is decided at the
    solver's resolution: it must not change when the initial deflection or rate of the first mode
    moves by up to 1e-5 A0 (a solver meeting the amplitude bar may move the orbit that far), nor
    when a law constant changes by up to 1e-5 relative (the deviation of the FP32 trajectory from
    the FP64 one is of that size).  Tried at 1, 2 and 5 x 1e-7 .. 1e-5, both signs."""
    st0 = orc.forward(model, p)["status"] != 0
    A0 = model["free_amplitude"]
    wd = 2 * np.pi * model.get("drive_freq", model["f0"])
    y00 = np.asarray(orc.initial_state(model), dtype=np.float64)
    nm = len(y00) // 2
    for rel in FATE_RELS:
        for k, scale in ((0, A0), (nm, A0 * wd)):
            for sgn in (1.0, -1.0):
                y0 = y00.copy()
                y0[k] += sgn * rel * scale
                st = orc.trajectory(model, p, y0=y0, n_out=1)[0]
                if (st != 0) != st0:
                    return False
        for j in range(min(len(p), 8)):
            if p[j] == 0:
                continue
            for sgn in (1.0, -1.0):
                q = np.array(p, dtype=np.float64)
                q[j] *= 1.0 + sgn * rel
                if (orc.forward(model, q)["status"] != 0) != st0:
                    return False
    return True


def fp32_data_shift(orc, model, p):
    """How far the FP64 oracle's (A, phi) move when its law constants are rounded to FP32:
    (|dA|/A, |dphi|), or (inf, inf) if the rounded problem fails."""
    r0 = orc.forward(model, p)
    q = np.array(p, dtype=np.float64)
    q[:8] = q[:8].astype(np.float32).astype(np.float64)
    r = orc.forward(model, q)
    if r0["status"] or r["status"]:
        return np.inf, np.inf
    return abs(r["A"] / r0["A"] - 1), abs(wrap(r["phi"] - r0["phi"]))


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


def compare_mixed(orc, model, P, o, A, phi, st, J=None, tag="", n_cycles=None,
                  max_excluded=0, min_strict=None):
    """Classify each trajectory as passing, excluded (ill-conditioned oracle) or failing, and
    count the trajectories that meet the bars without the small-orbit floor.

    Failure (a non-zero status word) must agree except on excluded trajectories -- which bit is
    set may differ: a blow-up that FP64 reports as non-finite can stay finite but huge in FP32;
    amplitude, phase and (if given) misfit must meet the tolerances above.  Asserts that nothing
    fails, that at most max_excluded trajectories are excluded and, if min_strict is given, that
    at least that many meet the strict bars.  Returns (failing, excluded, n_strict)."""
    A0 = model["free_amplitude"]
    n = len(A)
    bad = np.zeros(n, bool)
    both_ok = (st == 0) & (o["status"] == 0)
    bad |= (st != 0) != (o["status"] != 0)
    bad[both_ok] |= ~amp_ok(A[both_ok], o["A"][both_ok], A0)
    bad[both_ok] |= ~phase_ok(phi[both_ok], o["phi"][both_ok], o["A"][both_ok], A0)
    if J is not None:
        bad[both_ok] |= np.abs(J[both_ok] - o["J"][both_ok]) > misfit_tol(o["J"][both_ok])
    strict = np.zeros(n, bool)
    strict[both_ok] = strict_ok(A[both_ok], o["A"][both_ok], phi[both_ok], o["phi"][both_ok],
                                None if J is None else J[both_ok],
                                None if J is None else o["J"][both_ok])
    both_failed = (st != 0) & (o["status"] != 0)
    excluded, failing = [], []
    for i in np.flatnonzero(bad):
        m = model if n_cycles is None else dict(model, n_cycles=int(n_cycles[i]))
        ok_i = well_conditioned(orc, m, P[i])
        if ok_i and (st[i] != 0) != (o["status"][i] != 0):
            ok_i = fate_conditioned(orc, m, P[i])
        (failing if ok_i else excluded).append(int(i))
    n_strict = int(strict.sum())
    if both_ok.any():
        eA = np.abs(A[both_ok] / o["A"][both_ok] - 1)
        eP = np.abs(wrap(phi[both_ok] - o["phi"][both_ok]))
        print(f"{tag}: n {n}, max |dA|/A {eA.max():.2e} (median {np.median(eA):.1e}), max |dphi| "
              f"{eP.max():.2e} (median {np.median(eP):.1e}); strict bars met by {n_strict} of "
              f"{int(both_ok.sum())} finite ({int(both_failed.sum())} fail on both sides), "
              f"excluded {len(excluded)}, failing {len(failing)}")
    for i in excluded:
        m = model if n_cycles is None else dict(model, n_cycles=int(n_cycles[i]))
        sA, sP = fp32_data_shift(orc, m, P[i])
        gA = abs(A[i] / o["A"][i] - 1) if both_ok[i] else np.nan
        gP = abs(wrap(phi[i] - o["phi"][i])) if both_ok[i] else np.nan
        print(f"  {tag} excluded {i}: gpu |dA|/A {gA:.1e} |dphi| {gP:.1e}; oracle with FP32 "
              f"law constants |dA|/A {sA:.1e} |dphi| {sP:.1e}; status gpu {st[i]} oracle "
              f"{o['status'][i]}")
    assert not failing, (tag, failing)
    assert len(excluded) <= max_excluded, (tag, excluded)
    if min_strict is not None:
        assert n_strict >= min_strict, (tag, n_strict, min_strict)
    return failing, excluded, n_strict


def _zscale(free, p):
    return np.array([p[f[0]] * np.log(f[2] / f[1]) if f[3] else f[2] - f[1] for f in free])


def grad_sensitivity(orc, model, p, target, free, rel):
    """Largest norm-wise relative change (normalised coordinates) of the oracle's gradient under
    a `rel` relative change of any one law constant."""
    st, J0, g0 = orc.misfit_grad(model, p, target)
    if st:
        return 0.0
    idx = [f[0] for f in free]
    scale = _zscale(free, p)
    gz0 = g0[idx] * scale
    worst = 0.0
    for j in range(min(len(p), 8)):
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


GRAD_TOL = 1e-3
GRAD_TOL64 = 1e-6
# The mixed adjoint is the exact derivative of the FP32 discrete map, whose trajectory deviates
# from the FP64 one by about as much as a 1e-6 .. 1e-5 relative change of the data does (the
# forward tests measure |dA|/A up to 7e-6).  Over the long horizons that deviation alone moves
# the gradient by up to a few 1e-3 on points whose gradient is smooth in the data: the mixed
# path is held to GRAD_TOL_MIXED on retained points and to GRAD_TOL at their median (the FP64
# path is held to GRAD_TOL64).
GRAD_TOL_MIXED = 5e-3
# A retained point's gradient must be determined at the FP32 resolution of the data and respond
# smoothly beyond it: it moves by at most GRAD_TOL / 3 under a 1e-7 relative change of any law
# constant, and from 1e-7 to 1e-6 and from 1e-6 to 1e-5 its response grows by at most 3x the
# linear factor of 10 (plus a floor of a hundredth of the scaled bar).  A faster growth means
# that a change of that size -- the deviation of the FP32 trajectory from the FP64 one is of
# that size -- crosses a kink of the misfit (contact onset, the attraction frozen in contact).
# FP64: GRAD_TOL64 / 3 under 1e-10.
GRAD_RELS = (1e-7, 1e-6, 1e-5)
GRAD_RELS64 = (1e-10,)


def grad_retained(orc, model, p, target, free, fp64=False):
    """Whether the oracle's gradient at p is determined at the solver's resolution (see above).
    A point whose oracle trajectory fails has no gradient and is not retained."""
    if orc.misfit_grad(model, p, target)[0]:
        return False
    if fp64:
        return grad_sensitivity(orc, model, p, target, free, GRAD_RELS64[0]) <= GRAD_TOL64 / 3.0
    prev = grad_sensitivity(orc, model, p, target, free, GRAD_RELS[0])
    if prev > GRAD_TOL / 3.0:
        return False
    for rel in GRAD_RELS[1:]:
        s = grad_sensitivity(orc, model, p, target, free, rel)
        if s > 30.0 * prev + rel / 1e-7 * GRAD_TOL / 300.0:
            return False
        prev = s
    return True


def grad_retained_many(orc, model, P, target, free, fp64=False, threads=16):
    """grad_retained for every row of P, on a thread pool (the oracle releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(threads) as ex:
        return np.array(list(ex.map(lambda p: grad_retained(orc, model, p, target, free, fp64),
                                    list(P))))


def oracle_grads_many(orc, model, P, free, target, threads=16):
    """(J [n], g [D][n] over the free parameters, status [n]) of the oracle at the rows of P."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda p: orc.misfit_grad(model, p, target), list(P)))
    st = np.array([r[0] for r in res], np.int32)
    J = np.array([r[1] for r in res])
    g = np.array([[r[2][f[0]] for r in res] for f in free])
    return J, g, st
