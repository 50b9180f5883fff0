"""Pins of the oracle's particle swarm (paper Sec. 3.4, Eq. 8) and of whole inversions."""
import numpy as np
import pytest

import workloads as W


def _sphere(z, centre):
    return np.sum((z - centre[:, None]) ** 2, axis=0)


@pytest.mark.parametrize("D", [1, 2, 5])
def test_pso_converges_on_shifted_sphere(orc, D):
    """On a shifted quadratic the constriction-coefficient swarm converges to the minimum; the
    swarm invariants hold at every generation."""
    P, T = 24, 300
    centre = np.linspace(0.2, 0.8, D)
    sw = orc.Swarm(D, P, 1, seed=123)
    prev_pbest = np.full(P, np.inf)
    for t in range(T):
        J = _sphere(sw.z, centre)
        sw.update(J, t, t == T - 1, cutoff=1e-4)
        assert np.all(sw.pbest_J <= prev_pbest)
        prev_pbest = sw.pbest_J.copy()
        best = int(np.argmin(sw.pbest_J))  # lowest index among ties
        assert sw.gbest_J[0] == sw.pbest_J[best]
        np.testing.assert_array_equal(sw.gbest_z[:, 0], sw.pbest_z[:, best])
        assert np.all(sw.z >= 0) and np.all(sw.z <= 1)
        assert np.all(np.abs(sw.v) <= 1.0)
    assert sw.gbest_J[0] < 1e-8
    assert 0 <= sw.gen_to_cutoff[0] < T


def test_pso_init_uniform(orc):
    sw = orc.Swarm(2, 3, 2, seed=(7 << 32) | 9)
    for s in range(2):
        for p in range(3):
            for j in range(2):
                g = s * 3 + p
                rz = orc.draw((7 << 32) | 9, s, 0, p, j, 1)
                rv = orc.draw((7 << 32) | 9, s, 0, p, j, 2)
                z0 = orc.u53(rz[0], rz[1])
                assert sw.z[j, g] == z0 and sw.pbest_z[j, g] == z0
                assert sw.v[j, g] == orc.u53(rv[0], rv[1]) - z0
    assert np.all(np.isinf(sw.pbest_J)) and np.all(sw.gen_to_cutoff == -1)


def test_pso_step_follows_eq8(orc):
    """One move, checked against Eq. 8 evaluated independently in NumPy with the same draws."""
    D, P, S, seed = 3, 5, 2, 42
    sw = orc.Swarm(D, P, S, seed)
    rng = np.random.default_rng(0)
    J = rng.random(S * P)
    J[3] = np.nan  # non-finite misfits never become a best
    z0, v0 = sw.z.copy(), sw.v.copy()
    sw.update(J, 0, False)
    pso = orc.PSO_DEFAULTS
    for s in range(S):
        Js = np.where(np.isfinite(J[s * P:(s + 1) * P]), J[s * P:(s + 1) * P], np.inf)
        b = int(np.argmin(Js))
        assert sw.gbest_J[s] == Js[b]
        for p in range(P):
            g = s * P + p
            for j in range(D):
                r = orc.draw(seed, s, 0, p, j, 0)
                r1, r2 = orc.u53(r[0], r[1]), orc.u53(r[2], r[3])
                pb = z0[j, g] if np.isfinite(Js[p]) else z0[j, g]
                v = pso["w"] * v0[j, g] + pso["c1"] * r1 * (pb - z0[j, g]) + \
                    pso["c2"] * r2 * (z0[j, s * P + b] - z0[j, g])
                v = min(max(v, -1.0), 1.0)
                z = z0[j, g] + v
                if z < 0 or z > 1:
                    z, v = min(max(z, 0.0), 1.0), 0.0
                assert abs(sw.z[j, g] - z) < 1e-15 and abs(sw.v[j, g] - v) < 1e-15
    assert np.isinf(sw.pbest_J[3])


def _small_dmt():
    c = W.config("c1")
    m = dict(c["model"], steps_per_cycle=64, n_cycles=40, lockin_cycles=5)
    return c, m


def test_noiseless_recovery_tiny_swarm_and_lbfgs(orc):
    """Noiseless target at the truth: an 8 x 10 swarm then L-BFGS on the adjoint gradient
    recovers (H, E*) to 1e-6 relative.  E* spans two decades, so it is searched in log
    coordinates (the time-domain misfit is corrugated along E*)."""
    c, m = _small_dmt()
    ptrue = W.full_params(c)
    U = orc.forward(m, ptrue, want_trace=True)["trace"]
    free = W.free_index(c)
    free[1] = (free[1][0], free[1][1], free[1][2], True)
    for seed in (0, 1, 2):
        res = orc.pso_invert(m, ptrue, free, U, P=8, T=10, seed=seed, cutoff=1e-3)
        assert np.all(np.diff(res["hist"]) <= 0)
        z, J = orc.lbfgs(m, ptrue, free, U, res["z"], 40)
        theta = [orc.z_to_theta(z[j], *free[j][1:]) for j in range(len(free))]
        assert J < 1e-20
        assert abs(theta[0] / ptrue[1] - 1) < 1e-6 and abs(theta[1] / ptrue[2] - 1) < 1e-6


@pytest.mark.slow
def test_pso_optimum_vs_brute_force_grid(orc):
    """2-D misfit landscape of (H, log E*) on a 48 x 48 grid: a 32 x 30 swarm reaches a misfit no
    worse than the grid's best, and its E* lies within one grid cell of the grid's.  (Over this
    short horizon the misfit is nearly flat along H, so only E* is located by the grid.)"""
    c, m = _small_dmt()
    ptrue = W.full_params(c)
    U = orc.forward(m, ptrue, want_trace=True)["trace"]
    free = W.free_index(c)
    free[1] = (free[1][0], free[1][1], free[1][2], True)
    n = 48
    zs = (np.arange(n) + 0.5) / n
    best = (np.inf, None)
    for z1 in zs:
        for z2 in zs:
            p = ptrue.copy()
            p[free[0][0]] = orc.z_to_theta(z1, *free[0][1:])
            p[free[1][0]] = orc.z_to_theta(z2, *free[1][1:])
            J = orc.forward(m, p, U)["J"]
            if J < best[0]:
                best = (J, (z1, z2))
    for seed in (0, 1):
        res = orc.pso_invert(m, ptrue, free, U, P=32, T=30, seed=seed)
        assert res["J"] <= best[0]
        assert abs(res["z"][1] - best[1][1]) <= 1.0 / n
