"""The adaptive steady-state exit on the GPU (steady_rtol > 0: a trajectory ends its transient
after the first period whose lock-in amplitude differs from the previous period's by less than
steady_rtol relative; the period count is the cap), against the oracle.

* FP64: every trajectory exits at the oracle's period and its amplitude, phase and misfit match;
* mixed: the FP32 trajectory is not the FP64 one, so its exit period is its own: a plain dump of
  the same GPU trajectory (bit-identical steps) gives, through numpy's one-period lock-in, the
  period the kernel must have picked; the results equal the oracle's plain solve with the window
  at that period, to the mixed tolerances;
* the work-queue path of an inversion with per-swarm caps follows the oracle's swarm step for
  step (FP64);
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


@pytest.mark.parametrize("rtol", [1e-4, 1e-6])
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


@pytest.mark.parametrize("rtol", [1e-4, 1e-6])
def test_mixed_exit_is_consistent_with_its_own_trajectory(afm, orc, rtol):
    import torch

    c, m = _case(rtol, n_cycles=900)
    base, free = W.full_params(c), W.free_index(c)
    N, L, nc = m["steps_per_cycle"], m["lockin_cycles"], m["n_cycles"]
    th = torch.tensor(W.draw_free(c, 12, 32).T.copy(), device="cuda")
    plan = afm.Plan(m, base, free, precision="mixed")
    r = plan.forward_steady(th)
    per, A, ph, st = (r[k].cpu().numpy() for k in ("periods", "amp", "phase", "status"))
    # the same trajectories without the exit, every sample in the window
    dump = afm.Plan(dict(m, steady_rtol=0.0, lockin_cycles=nc), base, free, precision="mixed")
    tr = dump.forward_batch(th, trace=True)["trace"].cpu().numpy()
    P = PT.full_from_free(base, free, th.cpu().numpy())
    for i in range(th.shape[1]):
        if st[i]:
            continue
        amps = [_amp(tr[i, k * N:(k + 1) * N], N) for k in range(nc)]
        T = nc - L
        for k in range(1, nc - L):
            crit = abs(amps[k] - amps[k - 1]) / (rtol * amps[k])
            if abs(crit - 1) < 1e-6:
                pytest.skip("borderline decision for this point; choose another draw")
            if crit < 1:
                T = k + 1
                break
        assert per[i] == T + L, (i, per[i], T + L)
        o = orc.forward(dict(m, steady_rtol=0.0), P[i], n_cycles=int(per[i]))
        assert PT.amp_ok(A[i], o["A"], m["free_amplitude"]) or \
            not PT.well_conditioned(orc, dict(m, steady_rtol=0.0, n_cycles=int(per[i])), P[i])
        assert PT.phase_ok(ph[i], o["phi"], o["A"], m["free_amplitude"]) or \
            not PT.well_conditioned(orc, dict(m, steady_rtol=0.0, n_cycles=int(per[i])), P[i])


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
