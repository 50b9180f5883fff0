"""The adaptive steady-state exit on the GPU (steady_rtol > 0: a trajectory ends its transient
after the first period whose end point (u, u'/wd) moved by less than steady_rtol of its size
since the previous period's end; the period count is the cap), against the oracle.

* FP64: every trajectory exits at the oracle's period and its amplitude, phase and misfit match;
* mixed: the FP32 trajectory is not the FP64 one, so its exit period may differ from the
  oracle's where the test is close: the oracle's own test at the GPU's exit period must pass
  within a small slack (and fail at every earlier period by as much); the results equal the
  oracle's plain solve with the window at the GPU's period, to the mixed tolerances;
* the work-queue path of an inversion with per-swarm caps (the lane-refill kernel) follows the
  oracle's swarm step for step (FP64) and equals a swarm stepped from the one-lane kernel's
  misfits bit for bit (mixed and FP64);
* point deflections use the same per-lane window; the adjoint reports unsupported."""
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


def _case(rtol, n_cycles=1200, N=128, lockin=5):
    c = W.config("c2")
    m = dict(c["model"], n_cycles=n_cycles, steps_per_cycle=N, lockin_cycles=lockin,
             steady_rtol=rtol)
    return c, m


def _amp(u, N):
    k = np.arange(1, len(u) + 1) % N
    X = 2.0 / len(u) * np.sum(u * np.cos(2 * np.pi * k / N))
    Y = 2.0 / len(u) * np.sum(u * np.sin(2 * np.pi * k / N))
    return np.hypot(X, Y)


@pytest.mark.parametrize("rtol", [1e-3, 1e-4, 1e-5])
def test_fp64_exits_where_the_oracle_does(afm, orc, rtol):
    c, m = _case(rtol)
    base, free = W.full_params(c), W.free_index(c)
    th = W.draw_free(c, 16, 31).T.copy()
    U = orc.forward(dict(m, steady_rtol=0.0), base, want_trace=True)["trace"]
    plan = afm.Plan(m, base, free, precision="fp64")
    r = plan.forward_steady(th, trace=True)
    J, _ = plan.misfit(th, U[None, :])
    per, A, ph, st = (r[k].cpu().numpy() for k in ("periods", "amp", "phase", "status"))
    P = PT.full_from_free(base, free, th)
    saved = []
    for i in range(th.shape[1]):
        o = orc.forward_steady(m, P[i], rtol, U, want_trace=True)
        assert st[i] == o["status"] and per[i] == o["periods"], (i, per[i], o["periods"])
        if st[i]:
            continue
        assert abs(A[i] / o["A"] - 1) < 1e-9 and abs(ph[i] - o["phi"]) < 1e-9
        assert abs(J.cpu().numpy()[i] - o["J"]) <= 1e-9 * o["J"] + 1e-15
        np.testing.assert_allclose(r["trace"].cpu().numpy()[i], o["trace"], rtol=0,
                                   atol=1e-9 * np.max(np.abs(o["trace"])))
        saved.append(1 - per[i] / m["n_cycles"])
    print(f"rtol {rtol:g}: periods saved per trajectory {np.mean(saved):.2f}")
    assert np.mean(saved) > 0.05  # the exit did trigger


@pytest.mark.parametrize("rtol", [1e-3, 1e-4])
def test_mixed_exit_matches_the_oracle_test(afm, orc, rtol):
    import torch

    c, m = _case(rtol, n_cycles=900)
    base, free = W.full_params(c), W.free_index(c)
    N, L, nc = m["steps_per_cycle"], m["lockin_cycles"], m["n_cycles"]
    th = W.draw_free(c, 12, 32).T.copy()
    plan = afm.Plan(m, base, free, precision="mixed")
    r = plan.forward_steady(torch.tensor(th, device="cuda"))
    per, A, ph, st = (r[k].cpu().numpy() for k in ("periods", "amp", "phase", "status"))
    P = PT.full_from_free(base, free, th)
    wd = 2 * np.pi * m["drive_freq"]
    m0 = dict(m, steady_rtol=0.0)
    same = 0
    for i in range(th.shape[1]):
        if st[i]:
            continue
        so, u, ud, _ = orc.trajectory(m0, P[i], n_out=nc * N, want_rate=True)
        y0 = orc.initial_state(m0)
        Pu = np.r_[y0[0], u[N - 1::N]]
        Pv = np.r_[y0[1], ud[N - 1::N]] / wd
        crit = np.hypot(np.diff(Pu), np.diff(Pv)) / (rtol * np.hypot(Pu[1:], Pv[1:]))
        Tg = per[i] - L
        if Tg < nc - L:
            assert crit[Tg - 1] < 1.05, (i, Tg, crit[Tg - 1])
        assert np.all(crit[:Tg - 1] > 0.95), (i, Tg)
        same += int(Tg == (np.argmax(crit[:nc - L] < 1) + 1 if np.any(crit[:nc - L] < 1) else nc - L))
        o = orc.forward(m0, P[i], n_cycles=int(per[i]))
        mi = dict(m0, n_cycles=int(per[i]))
        assert PT.amp_ok(A[i], o["A"], m["free_amplitude"]) or not PT.well_conditioned(orc, mi, P[i])
        assert PT.phase_ok(ph[i], o["phi"], o["A"], m["free_amplitude"]) or \
            not PT.well_conditioned(orc, mi, P[i])
    print(f"rtol {rtol:g}: {same} of {th.shape[1]} exit at the oracle's period")


def test_queue_inversion_follows_oracle_swarm(afm, orc):
    import torch

    c = W.config("c1")
    m = dict(c["model"], steps_per_cycle=64, n_cycles=400, lockin_cycles=5, steady_rtol=1e-5)
    free = W.free_index(c)
    S, P, T, seed = 2, 16, 3, 12
    cyc = np.array([400, 250], np.int32)
    base = W.full_params(c)
    sp = np.zeros((afm.MAX_PARAMS, S))
    sp[:5] = base[:, None]
    sp[2] = [1.0e9, 2.5e9]
    U = np.stack([orc.forward(dict(m, steady_rtol=0.0, n_cycles=int(cyc[s])), sp[:5, s],
                              want_trace=True)["trace"] for s in range(S)])
    plan = afm.Plan(m, base, free, precision="fp64")
    out = plan.invert(U, P, T, seed=seed, cutoff=1e-2, n_cycles=cyc, swarm_params=sp)
    bt, bJ = out["best_theta"].cpu().numpy(), out["best_J"].cpu().numpy()
    sw = orc.Swarm(len(free), P, S, seed)
    for t in range(T):
        J = np.empty(S * P)
        for s in range(S):
            for p in range(P):
                q = sp[:5, s].copy()
                for j, f in enumerate(free):
                    q[f[0]] = orc.z_to_theta(sw.z[j, s * P + p], *f[1:])
                J[s * P + p] = orc.forward_steady(m, q, 1e-5, U[s], n_cycles=int(cyc[s]))["J"]
        sw.update(J, t, t == T - 1, cutoff=1e-2)
    for s in range(S):
        zt = [orc.z_to_theta(sw.gbest_z[j, s], *free[j][1:]) for j in range(len(free))]
        np.testing.assert_allclose(bt[:, s], zt, rtol=1e-12)
        assert abs(bJ[s] - sw.gbest_J[s]) <= 1e-9 * sw.gbest_J[s] + 1e-15


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_lane_refill_equals_plain_kernel(afm, prec):
    """The inversion's lane-refill kernel (work-queue batches with the exit) gives the same bits
    as the one-lane kernel: the swarm it drives equals a swarm stepped from afm_misfit (plain
    launch, per-trajectory caps and target rows) and afm_pso_step.  Ragged swarms (70 particles:
    a padded second chunk) and a pixel whose cap is below the window (bad input) included."""
    import torch

    c = W.config("c1")
    m = dict(c["model"], steps_per_cycle=64, n_cycles=450, lockin_cycles=5, steady_rtol=1e-5)
    free = W.free_index(c)
    S, P, T, seed = 5, 70, 4, 21
    cyc = np.array([300, 120, 450, 200, 3], np.int32)
    base = W.full_params(c)
    rng = np.random.default_rng(3)
    Wn = m["lockin_cycles"] * m["steps_per_cycle"]
    U = np.stack([1.6e-8 * np.sin(2 * np.pi * np.arange(1, Wn + 1) / 64 - rng.uniform(0.5, 1.5))
                  for _ in range(S)])
    plan = afm.Plan(m, base, free, precision=prec)
    out = plan.invert(U, P, T, seed=seed, cutoff=1e-2, n_cycles=cyc)
    sw = plan.swarm_init(P, S, seed)
    tid = torch.arange(S, dtype=torch.int32, device="cuda").repeat_interleave(P)
    ncl = torch.tensor(cyc, device="cuda").repeat_interleave(P)
    Ud = torch.tensor(U, device="cuda")
    for t in range(T):
        J, _ = plan.misfit(sw.theta, Ud, target_id=tid, n_cycles=ncl)
        plan.pso_step(sw, J, seed, t, t == T - 1, cutoff=1e-2)
    torch.cuda.synchronize()
    assert np.array_equal(out["best_J"].cpu().numpy().view(np.uint8),
                          sw.gbest_J.cpu().numpy().view(np.uint8))
    assert np.array_equal(out["gen_to_cutoff"].cpu().numpy(), sw.gen_to_cutoff.cpu().numpy())
    assert np.isinf(out["best_J"].cpu().numpy()[4])


def test_points_and_adjoint(afm):
    import torch

    c, m = _case(1e-5, n_cycles=600)
    plan = afm.Plan(m, W.full_params(c), W.free_index(c), precision="mixed")
    th = torch.tensor(W.draw_free(c, 40, 33).T.copy(), device="cuda")
    r = plan.forward_steady(th)
    q = plan.forward_points(th, np.ones((1, 1)))
    ok = r["status"].cpu().numpy() == 0
    d = np.abs(q["amp"].cpu().numpy()[0, ok] - r["amp"].cpu().numpy()[ok])
    assert np.max(d) < 1e-12 * m["free_amplitude"]
    U = torch.zeros(1, plan.W, dtype=torch.float64, device="cuda") + 1e-9
    with pytest.raises(afm.AfmError, match="status 4"):
        plan.grad_batch(th, U)
