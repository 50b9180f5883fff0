"""GPU swarm kernels and whole inversions against the oracle.

The swarm update is FP64 with a fixed evaluation order and no contraction, and both sides draw
from Philox4x32-10 with the same stream layout, so given identical misfits the GPU swarm must
equal the oracle's bit for bit."""
import numpy as np
import pytest

import parity as PT
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def afm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1109_0334_amd as afm

    afm.lib()
    return afm


def _swarm_arrays(sw):
    return {k: getattr(sw, k).cpu().numpy() for k in
            ("z", "v", "pbest_z", "pbest_J", "gbest_z", "gbest_J", "gen_to_cutoff")}


def _assert_same(gpu, orc_sw):
    for k, g in gpu.items():
        o = getattr(orc_sw, k)
        assert g.shape == o.shape, k
        assert np.array_equal(g.view(np.uint8), np.ascontiguousarray(o).view(np.uint8)), k


@pytest.mark.parametrize("D,P,S", [(3, 70, 3), (2, 128, 5), (5, 300, 1), (1, 1, 2)])
def test_pso_bit_exact(afm, orc, D, P, S):
    c = W.config("c2")
    free = [(1 + j % 3, 0.0, 1.0, 0) for j in range(D)]
    base = W.full_params(c)
    if D > 3:
        c5 = W.config("c5")
        base, free = W.full_params(c5), W.free_index(c5)[:D]
        model = c5["model"]
    else:
        model = c["model"]
        free = W.free_index(c)[:D]
    plan = afm.Plan(model, base, free, precision="mixed")
    seed = (0xABCDEF << 32) | 12345
    sw = plan.swarm_init(P, S, seed)
    osw = orc.Swarm(D, P, S, seed)
    _assert_same(_swarm_arrays(sw), osw)
    rng = np.random.default_rng(D * 100 + P)
    for it in range(6):
        J = rng.random(S * P)
        J[rng.random(S * P) < 0.05] = np.nan
        J[rng.random(S * P) < 0.05] = np.inf
        if it == 2:
            J[:] = J[0]  # all tied: the lowest index wins
        last = it == 5
        plan.pso_step(sw, J, seed, it, last, cutoff=0.2)
        osw.update(J, it, last, cutoff=0.2)
        _assert_same(_swarm_arrays(sw), osw)
    # theta is the SI image of z
    th = sw.theta.cpu().numpy()
    for j, f in enumerate(free):
        ref = np.array([orc.z_to_theta(z, f[1], f[2], f[3]) for z in osw.z[j]])
        np.testing.assert_allclose(th[j], ref, rtol=1e-14)


def test_invert_c1_fp64_matches_oracle(afm, orc):
    """C1 end to end with the plain FP64 forward: same swarm trajectory as the oracle (misfits
    agree to ~1e-12, far below any gap between particles), so the same best point."""
    c = W.config("c1")
    m = c["model"]
    U = orc.forward(m, W.full_params(c), want_trace=True)["trace"]
    plan = afm.Plan(m, W.full_params(c), W.free_index(c), precision="fp64")
    out = plan.invert(U[None, :], c["particles"], c["iters"], seed=c["seed"], cutoff=1e-2)
    ores = orc.pso_invert(m, W.full_params(c), W.free_index(c), U, c["particles"], c["iters"],
                          c["seed"], cutoff=1e-2)
    bt = out["best_theta"].cpu().numpy()[:, 0]
    zt = [orc.z_to_theta(ores["z"][j], *W.free_index(c)[j][1:]) for j in range(2)]
    np.testing.assert_allclose(bt, zt, rtol=1e-12)
    assert abs(out["best_J"].item() - ores["J"]) <= 1e-9 * ores["J"] + 1e-15
    assert out["gen_to_cutoff"].item() == ores["gen_to_cutoff"]


def test_invert_replay_is_deterministic(afm, orc):
    """A cached graph replays to identical results, with eager work between the replays."""
    import torch

    c = W.config("c1")
    m = dict(c["model"], n_cycles=60)
    U = orc.forward(m, W.full_params(c), want_trace=True)["trace"]
    plan = afm.Plan(m, W.full_params(c), W.free_index(c), precision="mixed")
    targets = torch.tensor(np.stack([U, U * 0.97]), device="cuda")
    res = []
    for rep in range(3):
        out = plan.invert(targets, 16, 6, seed=3, cutoff=1e-2)
        torch.cuda.synchronize()
        res.append({k: v.cpu().numpy().copy() for k, v in out.items()})
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del junk
    for r in res[1:]:
        for k in r:
            assert np.array_equal(r[k], res[0][k]), k


def test_invert_c2_small_recovers_truth(afm, orc):
    """Mixed path, noiseless C2-shaped target (shortened run): the swarm lands near the truth
    and its best misfit matches the oracle's misfit at that point."""
    c = W.config("c2")
    m = dict(c["model"], n_cycles=150)
    p_true = W.full_params(c)
    U = orc.forward(m, p_true, want_trace=True)["trace"]
    free = W.free_index(c)
    free[1] = (free[1][0], free[1][1], free[1][2], True)  # E* searched in log coordinates
    plan = afm.Plan(m, p_true, free, precision="mixed")
    out = plan.invert(U[None, :], 256, 40, seed=1, cutoff=1e-3)
    bt = out["best_theta"].cpu().numpy()[:, 0]
    p = p_true.copy()
    for j, f in enumerate(free):
        p[f[0]] = bt[j]
    Jo = orc.forward(m, p, U)["J"]
    Jg = out["best_J"].item()
    assert abs(Jg - Jo) <= PT.misfit_tol(Jo)
    assert Jo < 1e-4
    assert abs(bt[1] / c["truth"]["Estar"] - 1) < 0.05


def test_invert_uneven_queue_matches_oracle(afm, orc):
    """Several pixels with their own period counts, separations and stiffnesses (the persistent
    work-queue path, a ragged 70-particle swarm = 2 queue items per pixel), FP64 forward: every
    swarm follows the oracle swarm step for step."""
    import torch

    c = W.config("c1")
    m = dict(c["model"], steps_per_cycle=64, n_cycles=40, lockin_cycles=5)
    free = W.free_index(c)
    S, P, T, seed = 3, 70, 5, 11
    cyc = np.array([40, 25, 33], np.int32)
    zcs = [14.6e-9, 15.0e-9, 14.2e-9]
    estar = [1.0e9, 2.5e9, 0.6e9]
    base = W.full_params(c)
    sp = np.zeros((afm.MAX_PARAMS, S))
    for s in range(S):
        sp[:5, s] = base
        sp[0, s], sp[2, s] = zcs[s], estar[s]
    U = np.stack([orc.forward(dict(m, n_cycles=int(cyc[s])), sp[:5, s], want_trace=True)["trace"]
                  for s in range(S)])
    plan = afm.Plan(m, base, free, precision="fp64")
    out = plan.invert(U, P, T, seed=seed, cutoff=1e-2, n_cycles=cyc, swarm_params=sp)
    bt, bJ = out["best_theta"].cpu().numpy(), out["best_J"].cpu().numpy()
    gen = out["gen_to_cutoff"].cpu().numpy()
    sw = orc.Swarm(len(free), P, S, seed)
    for t in range(T):
        J = np.empty(S * P)
        for s in range(S):
            ms = dict(m, n_cycles=int(cyc[s]))
            for p in range(P):
                q = sp[:5, s].copy()
                for j, f in enumerate(free):
                    q[f[0]] = orc.z_to_theta(sw.z[j, s * P + p], *f[1:])
                J[s * P + p] = orc.forward(ms, q, U[s])["J"]
        sw.update(J, t, t == T - 1, cutoff=1e-2)
    for s in range(S):
        zt = [orc.z_to_theta(sw.gbest_z[j, s], *free[j][1:]) for j in range(len(free))]
        np.testing.assert_allclose(bt[:, s], zt, rtol=1e-12)
        assert abs(bJ[s] - sw.gbest_J[s]) <= 1e-9 * sw.gbest_J[s] + 1e-15
        assert gen[s] == sw.gen_to_cutoff[s]


def test_invert_degenerate_shapes(afm, orc):
    """One particle, one generation, two swarms (FP64 forward): the best is the initial particle,
    exactly as the oracle draws it."""
    c = W.config("c1")
    m = dict(c["model"], n_cycles=30, lockin_cycles=3)
    U = orc.forward(m, W.full_params(c), want_trace=True)["trace"]
    plan = afm.Plan(m, W.full_params(c), W.free_index(c), precision="fp64")
    out = plan.invert(np.stack([U, 0.9 * U]), 1, 1, seed=5, cutoff=1e-2)
    sw = orc.Swarm(2, 1, 2, 5)
    J = np.empty(2)
    for s, Us in enumerate((U, 0.9 * U)):
        q = W.full_params(c).copy()
        for j, f in enumerate(W.free_index(c)):
            q[f[0]] = orc.z_to_theta(sw.z[j, s], *f[1:])
        J[s] = orc.forward(m, q, Us)["J"]
    sw.update(J, 0, True, cutoff=1e-2)
    bt = out["best_theta"].cpu().numpy()
    for s in range(2):
        zt = [orc.z_to_theta(sw.gbest_z[j, s], *W.free_index(c)[j][1:]) for j in range(2)]
        np.testing.assert_allclose(bt[:, s], zt, rtol=1e-12)
        assert abs(out["best_J"].cpu().numpy()[s] - sw.gbest_J[s]) <= 1e-9 * sw.gbest_J[s]


def test_invert_bad_pixel_does_not_touch_the_others(afm, orc):
    """A pixel whose period count is shorter than the lock-in window gets status BAD_INPUT for
    every particle (best J = inf, cut-off never reached); every other pixel's swarm is
    bit-identical to a run where that pixel was valid (swarms are independent streams)."""
    c = W.config("c1")
    m = dict(c["model"], steps_per_cycle=64, n_cycles=40, lockin_cycles=5)
    free = W.free_index(c)
    base = W.full_params(c)
    U = orc.forward(m, base, want_trace=True)["trace"]
    targets = np.stack([U, U, U])
    res = []
    for cyc in ([40, 25, 33], [40, 3, 33]):
        plan = afm.Plan(m, base, free, precision="mixed")
        out = plan.invert(targets, 70, 4, seed=9, cutoff=1e-2, n_cycles=np.array(cyc, np.int32))
        res.append({k: v.cpu().numpy() for k, v in out.items()})
    for k in res[0]:
        assert np.array_equal(res[0][k][..., [0, 2]], res[1][k][..., [0, 2]]), k
    assert np.isinf(res[1]["best_J"][1]) and res[1]["gen_to_cutoff"][1] == -1
