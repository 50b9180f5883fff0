"""GPU parity of the forward solve (afm_forward_batch / afm_misfit) against the FP64 oracle."""
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


def _plan(afm, cfg, precision, model=None, params=None, free=None):
    model = model or cfg["model"]
    params = W.full_params(cfg) if params is None else params
    free = W.free_index(cfg) if free is None else free
    return afm.Plan(model, params, free, precision=precision)


def _theta(cfg, n, seed):
    return W.draw_free(cfg, n, seed).T.copy()  # [D][n]


def test_forward_fp64_c1(afm, orc):
    """Plain FP64 path, C1 shape (100 periods x 200 steps), 67 points (a ragged second wave)."""
    c = W.config("c1")
    plan = _plan(afm, c, "fp64")
    th = _theta(c, 67, 1)
    r = plan.forward_batch(th)
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, c["model"], P)
    st = r["status"].cpu().numpy()
    assert np.array_equal(st, o["status"])
    A, phi = r["amp"].cpu().numpy(), r["phase"].cpu().numpy()
    np.testing.assert_allclose(A, o["A"], rtol=PT.FP64_RTOL)
    assert np.max(np.abs(PT.wrap(phi - o["phi"]))) < PT.FP64_RTOL


def test_forward_mixed_c2(afm, orc):
    """Mixed path, C2 shape (500 periods x 256 steps), 130 points from the C2 prior."""
    c = W.config("c2")
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 130, 2)
    r = plan.forward_batch(th)
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, c["model"], P)
    A, phi = r["amp"].cpu().numpy(), r["phase"].cpu().numpy()
    assert np.array_equal(r["status"].cpu().numpy(), o["status"])
    bad = (np.abs(A / o["A"] - 1) > PT.A_RTOL) | (np.abs(PT.wrap(phi - o["phi"])) > PT.PHI_ATOL)
    excluded = [i for i in np.flatnonzero(bad) if not PT.well_conditioned(orc, c["model"], P[i])]
    failing = sorted(set(np.flatnonzero(bad)) - set(excluded))
    print(f"mixed C2: max |dA|/A {np.max(np.abs(A / o['A'] - 1)):.2e}, max |dphi| "
          f"{np.max(np.abs(PT.wrap(phi - o['phi']))):.2e}, excluded {len(excluded)}/130")
    assert not failing, [(i, A[i], o["A"][i], phi[i], o["phi"][i]) for i in failing]
    assert len(excluded) <= 3


def test_misfit_mixed_c2_noisy_target(afm, orc):
    """Misfit against a noisy target made by the oracle at the truth (inverse-crime avoidance:
    the measured trace comes from the other implementation)."""
    c = W.config("c2")
    m = c["model"]
    Wn = orc.window_len(m)
    U = orc.forward(m, W.full_params(c), want_trace=True)["trace"] + W.noise(c, Wn, 0)
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 70, 3)
    th[:, 0] = [c["truth"]["H"], c["truth"]["Estar"], c["truth"]["a0"]]  # the truth itself
    J, st = plan.misfit(th, U[None, :])
    J = J.cpu().numpy()
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, m, P, target=U)
    assert np.array_equal(st.cpu().numpy(), o["status"])
    err = np.abs(J - o["J"])
    ok = err <= PT.misfit_tol(o["J"])
    for i in np.flatnonzero(~ok):
        assert not PT.well_conditioned(orc, m, P[i]), (i, J[i], o["J"][i])
    assert ok.sum() >= 68


def test_trace_and_lockin_fp64(afm, orc):
    """Window trace output (FP64 path) equals the oracle's deflection samples."""
    c = W.config("c1")
    plan = _plan(afm, c, "fp64")
    th = _theta(c, 5, 4)
    r = plan.forward_batch(th, trace=True)
    tr = r["trace"].cpu().numpy()
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    A0 = c["model"]["free_amplitude"]
    for i in range(5):
        ref = orc.forward(c["model"], P[i], want_trace=True)["trace"]
        assert np.max(np.abs(tr[i] - ref)) < 1e-9 * A0


@pytest.mark.parametrize("law", ["lj", "kv3", "hooke", "sd", "none", "dmt3"])
def test_forward_mixed_other_laws(afm, orc, law):
    if law == "lj":
        c = W.config("c4")
        m = dict(c["model"], n_cycles=600)
        base = W.full_params(c)
        free = W.free_index(c)
        th = _theta(c, 24, 5)
    elif law in ("kv3", "dmt3"):
        c = W.config("c5")
        m = dict(c["model"], n_cycles=150)
        if law == "dmt3":
            m["law"] = "dmt"
        base = W.full_params(c)[: 5 if law == "dmt3" else 6]
        free = [f for f in W.free_index(c) if f[0] < len(base)]
        th = np.stack([np.random.default_rng(6).uniform(f[1], f[2], 12) if not f[3] else
                       np.exp(np.random.default_rng(6).uniform(np.log(f[1]), np.log(f[2]), 12))
                       for f in free])
    else:
        c = W.config("c1")
        m = dict(c["model"], law=law, n_cycles=200, steps_per_cycle=128)
        zc = 15e-9
        base = {"hooke": [zc, 4.0], "sd": [zc, 4.0, 0.1e-6], "none": [zc]}[law]
        free = {"hooke": [(1, 0.5, 20.0, 0)], "sd": [(1, 0.5, 20.0, 0), (2, 1e-8, 1e-6, 1)],
                "none": [(0, 10e-9, 30e-9, 0)]}[law]
        rng = np.random.default_rng(7)
        th = np.stack([rng.uniform(f[1], f[2], 20) for f in free])
    plan = afm.Plan(m, base, free, precision="mixed")
    r = plan.forward_batch(th)
    P = PT.full_from_free(base, free, th)
    o = PT.oracle_batch(orc, m, P)
    A, phi = r["amp"].cpu().numpy(), r["phase"].cpu().numpy()
    st = r["status"].cpu().numpy()
    assert np.array_equal(st, o["status"])
    ok = st == 0
    bad = ok & ((np.abs(A / o["A"] - 1) > PT.A_RTOL) | (np.abs(PT.wrap(phi - o["phi"])) > PT.PHI_ATOL))
    print(f"{law}: max |dA|/A {np.nanmax(np.abs(A[ok] / o['A'][ok] - 1)):.2e}, max |dphi| "
          f"{np.nanmax(np.abs(PT.wrap(phi[ok] - o['phi'][ok]))):.2e}")
    for i in np.flatnonzero(bad):
        assert not PT.well_conditioned(orc, m, P[i]), (law, i, A[i], o["A"][i], phi[i], o["phi"][i])
    assert bad.sum() <= max(1, len(A) // 10)


def test_failure_status_matches_oracle(afm, orc):
    c = W.config("c1")
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 4, 8)
    th[1, 1] = 1e15  # E* far beyond RK4's stability limit
    th[0, 2] = np.nan
    r = plan.forward_batch(th)
    J, stJ = plan.misfit(th, np.ones((1, orc.window_len(c["model"]))))
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, c["model"], P)
    st = r["status"].cpu().numpy()
    assert (st[1] != 0) and (o["status"][1] != 0)
    assert st[2] == o["status"][2] == 1
    assert st[0] == o["status"][0] == 0
    A = r["amp"].cpu().numpy()
    assert np.isnan(A[1]) and np.isnan(A[2])
    Jc = J.cpu().numpy()
    assert np.isinf(Jc[1]) and np.isinf(Jc[2]) and np.isfinite(Jc[0])


def test_empty_and_single(afm, orc):
    c = W.config("c1")
    plan = _plan(afm, c, "mixed")
    r = plan.forward_batch(np.zeros((2, 0)))
    assert r["amp"].numel() == 0
    th = _theta(c, 1, 9)
    r = plan.forward_batch(th)
    o = orc.forward(c["model"], PT.full_from_free(W.full_params(c), W.free_index(c), th)[0])
    assert abs(r["amp"].item() / o["A"] - 1) < PT.A_RTOL


def test_per_trajectory_cycles(afm, orc):
    """Uneven cycle counts within one launch (the pixel workload's shape)."""
    c = W.config("c2")
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 40, 10)
    cyc = np.random.default_rng(11).integers(100, 400, 40).astype(np.int32)
    r = plan.forward_batch(th, n_cycles=cyc)
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, c["model"], P, n_cycles=cyc)
    A, phi = r["amp"].cpu().numpy(), r["phase"].cpu().numpy()
    bad = (np.abs(A / o["A"] - 1) > PT.A_RTOL) | (np.abs(PT.wrap(phi - o["phi"])) > PT.PHI_ATOL)
    for i in np.flatnonzero(bad):
        assert not PT.well_conditioned(orc, c["model"], P[i])


def test_full_size_c2_sampled(afm, orc):
    """The benchmark's launch: 1024 particles of C2 at full length in one misfit call; 8 sampled
    particles recomputed by the oracle one by one."""
    c = W.config("c2")
    m = c["model"]
    U = orc.forward(m, W.full_params(c), want_trace=True)["trace"] + W.noise(c, orc.window_len(m), 0)
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 1024, 12)
    J, st = plan.misfit(th, U[None, :])
    J = J.cpu().numpy()
    idx = np.random.default_rng(13).choice(1024, 8, replace=False)
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th[:, idx])
    o = PT.oracle_batch(orc, m, P, target=U)
    err = np.abs(J[idx] - o["J"])
    for k in np.flatnonzero(err > PT.misfit_tol(o["J"])):
        assert not PT.well_conditioned(orc, m, P[k])
