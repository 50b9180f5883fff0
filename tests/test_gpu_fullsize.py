"""Parity at the workloads' full sizes, in the launch configurations the benchmark times, on
sampled outputs the oracle recomputes one by one.

* uneven pixels: 4096 pixels x 128 particles, periods 100..2000, one generation through the
  persistent work queue (afm_invert); three pixels' whole swarms recomputed by the oracle;
* LJ-type gradients: 2048 points x 1000 periods x 256 steps (afm_grad_batch, tuned stride);
* 3-mode Kelvin-Voigt: 16384 particles x 2000 periods x 512 steps (afm_misfit), and the adjoint
  of 64 such points (the polish batch).

Targets are synthetic sinusoids from seeded draws (inputs only; neither side's arithmetic)."""
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


def _sine_targets(m, amps, phases):
    N = m["steps_per_cycle"]
    k = np.arange(1, m["lockin_cycles"] * N + 1)
    return np.stack([a * np.sin(2 * np.pi * k / N - p) for a, p in zip(amps, phases)])


def test_c3_full_size_queue_sampled(afm, orc):
    import torch

    c = W.config("c3")
    m = c["model"]
    S, P = int(c["pixels"]), int(c["particles"])
    pix = W.pixels(c)
    rng = np.random.default_rng(77)
    A0 = m["free_amplitude"]
    base = W.full_params(c)
    sp = np.zeros((afm.MAX_PARAMS, S))
    sp[: len(base)] = base[:, None]
    sp[0] = pix["setpoint"] * A0 + rng.uniform(-0.5e-9, 0.5e-9, S)  # separations near the set-point
    sp[2] = pix["Estar"]
    U = _sine_targets(m, pix["setpoint"] * A0, rng.uniform(0.5, 1.5, S))
    free = W.free_index(c)
    plan = afm.Plan(m, base, free, precision="mixed")
    out = plan.invert(torch.tensor(U, device="cuda"), P, 1, seed=4, n_cycles=pix["cycles"],
                      swarm_params=torch.tensor(sp, device="cuda"))
    bJ = out["best_J"].cpu().numpy()
    bt = out["best_theta"].cpu().numpy()
    sw = orc.Swarm(len(free), P, S, 4)
    for s in np.argsort(pix["cycles"], kind="stable")[:3]:
        ms = dict(m, n_cycles=int(pix["cycles"][s]))
        J = np.empty(P)
        Ps = np.empty((P, len(base)))
        for p in range(P):
            q = sp[: len(base), s].copy()
            for j, f in enumerate(free):
                q[f[0]] = orc.z_to_theta(sw.z[j, s * P + p], *f[1:])
            Ps[p] = q
            J[p] = orc.forward(ms, q, U[s])["J"]
        k = int(np.argmin(J))
        print(f"pixel {s} ({pix['cycles'][s]} periods): gpu best J {bJ[s]:.6e}, oracle {J[k]:.6e}")
        assert abs(bJ[s] - J[k]) <= PT.misfit_tol(J[k]) or not PT.well_conditioned(orc, ms, Ps[k])
        gap = np.sort(J)[1] - J[k]
        if gap > 2 * PT.misfit_tol(J[k]):  # unique best: the GPU must pick the same particle
            np.testing.assert_allclose(bt[:, s], [Ps[k][f[0]] for f in free], rtol=1e-12)


C4_FULL_MIN_RETAINED = 8


def W_len(m):
    return m["lockin_cycles"] * m["steps_per_cycle"]


def _grad_check(orc, m, P, free, U, J, dJ, st, th, tag):
    """Sampled points of a full-size gradient launch against the oracle: retained points (see
    parity.py) to 1e-3; returns (retained, excluded) counts."""
    zs = np.stack([(np.log(f[2] / f[1]) * th[j] if f[3] else (f[2] - f[1]) * np.ones_like(th[j]))
                   for j, f in enumerate(free)])
    keep = PT.grad_retained_many(orc, m, P, U, free)
    failing, n_keep = [], 0
    for i in range(P.shape[0]):
        sto, Jo, gf = orc.misfit_grad(m, P[i], U)
        go = np.array([gf[f[0]] for f in free])
        assert (st[i] != 0) == (sto != 0) or not PT.fate_conditioned(orc, m, P[i])
        if st[i] or sto:
            continue
        assert abs(J[i] - Jo) <= PT.misfit_tol(Jo) or not PT.well_conditioned(orc, m, P[i])
        e = np.linalg.norm((dJ[:, i] - go) * zs[:, i]) / np.linalg.norm(go * zs[:, i])
        print(f"{tag} point {i}: rel err {e:.2e} ({'retained' if keep[i] else 'excluded'})")
        n_keep += int(keep[i])
        if keep[i] and e > PT.GRAD_TOL_MIXED:
            failing.append((i, e))
    assert not failing, failing
    return n_keep, int(P.shape[0] - n_keep)


def test_c4_full_size_gradient_sampled(afm, orc):
    c = W.config("c4")
    m, base, free = c["model"], W.full_params(c), W.free_index(c)
    n = int(c["points"])
    th = W.draw_free(c, n, 7).T.copy()
    U = orc.forward(m, base, want_trace=True)["trace"] + W.noise(dict(noise=0.05e-9), W_len(m), 5)
    plan = afm.Plan(m, base, free, precision="mixed")
    J, dJ, st = (x.cpu().numpy() for x in plan.grad_batch(th, U[None, :]))
    # a small part of this box is retained at the full 1000-period horizon
    idx = np.random.default_rng(8).choice(n, 64, replace=False)
    P = PT.full_from_free(base, free, th[:, idx])
    n_keep, n_ex = _grad_check(orc, m, P, free, U, J[idx], dJ[:, idx], st[idx], th[:, idx],
                               "c4 full")
    print(f"c4 full: {n_keep} of 64 sampled points retained, {n_ex} excluded")
    assert n_keep >= C4_FULL_MIN_RETAINED


def test_c5_full_size_forward_and_polish_gradient_sampled(afm, orc):
    c = W.config("c5")
    m, base, free = c["model"], W.full_params(c), W.free_index(c)
    U = _sine_targets(m, [0.8 * m["free_amplitude"]], [1.2])[0]
    plan = afm.Plan(m, base, free, precision="mixed")
    n = int(c["particles"])
    th = W.draw_free(c, n, 9).T.copy()
    J, st = (x.cpu().numpy() for x in plan.misfit(th, U[None, :]))
    idx = np.random.default_rng(10).choice(n, 4, replace=False)
    P = PT.full_from_free(base, free, th[:, idx])
    o = PT.oracle_batch(orc, m, P, target=U)
    for k, i in enumerate(idx):
        print(f"c5 full forward {i}: gpu J {J[i]:.6e} oracle {o['J'][k]:.6e} status {st[i]}")
        assert (st[i] != 0) == (o["status"][k] != 0) or not PT.well_conditioned(orc, m, P[k])
        if st[i] == 0 and o["status"][k] == 0:
            assert abs(J[i] - o["J"][k]) <= PT.misfit_tol(o["J"][k]) or \
                not PT.well_conditioned(orc, m, P[k])
    k64 = int(c["lbfgs_topk"])
    th64 = th[:, :k64].copy()
    Jg, dJ, stg = (x.cpu().numpy() for x in plan.grad_batch(th64, U[None, :]))
    assert np.array_equal(Jg, J[:k64])  # the adjoint's forward pass is afm_misfit's arithmetic
    P2 = PT.full_from_free(base, free, th64[:, :2])
    _grad_check(orc, m, P2, free, U, Jg[:2], dJ[:, :2], stg[:2], th64[:, :2], "c5 full")
