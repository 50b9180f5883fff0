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


def _np(r):
    return r["amp"].cpu().numpy(), r["phase"].cpu().numpy(), r["status"].cpu().numpy()


def test_forward_fp64_c1(afm, orc):
    """Plain FP64 path, C1 shape (100 periods x 200 steps), 67 points (a ragged second wave)."""
    c = W.config("c1")
    plan = _plan(afm, c, "fp64")
    th = _theta(c, 67, 1)
    A, phi, st = _np(plan.forward_batch(th))
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, c["model"], P)
    assert np.array_equal(st, o["status"])
    np.testing.assert_allclose(A, o["A"], rtol=PT.FP64_RTOL)
    assert np.max(np.abs(PT.wrap(phi - o["phi"]))) < PT.FP64_RTOL


def test_forward_mixed_c2(afm, orc):
    """Mixed path, C2 shape (500 periods x 256 steps), 130 points from the C2 prior."""
    c = W.config("c2")
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 130, 2)
    A, phi, st = _np(plan.forward_batch(th))
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, c["model"], P)
    PT.compare_mixed(orc, c["model"], P, o, A, phi, st, tag="mixed C2", max_excluded=1,
                     min_strict=128)


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
    A, phi, _ = _np(plan.forward_batch(th))
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, m, P, target=U)
    PT.compare_mixed(orc, m, P, o, A, phi, st.cpu().numpy(), J=J.cpu().numpy(), tag="misfit C2",
                     max_excluded=1, min_strict=68)


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


def _law_case(law):
    if law in ("lj", "lj512"):
        c = W.config("c4")
        m = dict(c["model"])
        if law == "lj512":
            m.update(steps_per_cycle=512, n_cycles=600)
        return m, W.full_params(c), W.free_index(c), _theta(c, 24, 5)
    if law in ("kv3", "dmt3"):
        c = W.config("c5")
        m = dict(c["model"], n_cycles=150)
        if law == "dmt3":
            m["law"] = "dmt"
        base = W.full_params(c)[: 5 if law == "dmt3" else 6]
        free = [f for f in W.free_index(c) if f[0] < len(base)]
        rng = np.random.default_rng(6)
        th = np.stack([np.exp(rng.uniform(np.log(f[1]), np.log(f[2]), 12)) if f[3] else
                       rng.uniform(f[1], f[2], 12) for f in free])
        return m, base, free, th
    c = W.config("c1")
    m = dict(c["model"], law=law, n_cycles=200, steps_per_cycle=128)
    zc = 15e-9
    base = {"hooke": [zc, 4.0], "sd": [zc, 4.0, 0.1e-6], "none": [zc]}[law]
    free = {"hooke": [(1, 0.5, 20.0, 0)], "sd": [(1, 0.5, 20.0, 0), (2, 1e-8, 1e-6, 1)],
            "none": [(0, 10e-9, 30e-9, 0)]}[law]
    rng = np.random.default_rng(7)
    th = np.stack([rng.uniform(f[1], f[2], 20) for f in free])
    return m, base, free, th


# Allowed excluded (ill-conditioned) trajectories and required strict-bar counts per case (the
# measured counts with a margin of one or two).  The LJ workload at 256 steps per period resolves
# its steep repulsive wall with few steps: 3 of its 24 points are excluded (two whose steady orbit
# moves with the data at the 1e-7 level, one whose crash through the wall flips with its initial
# state); at 512 steps it behaves like the other laws.
_EXCLUDE = {"lj": 4, "lj512": 1, "kv3": 1, "dmt3": 1, "hooke": 1, "sd": 1, "none": 0}
_MIN_STRICT = {"lj": 19, "lj512": 23, "kv3": 10, "dmt3": 10, "hooke": 19, "sd": 19, "none": 19}


@pytest.mark.parametrize("law", ["lj", "lj512", "kv3", "hooke", "sd", "none", "dmt3"])
def test_forward_mixed_other_laws(afm, orc, law):
    m, base, free, th = _law_case(law)
    plan = afm.Plan(m, base, free, precision="mixed")
    A, phi, st = _np(plan.forward_batch(th))
    P = PT.full_from_free(base, free, th)
    o = PT.oracle_batch(orc, m, P)
    PT.compare_mixed(orc, m, P, o, A, phi, st, tag=law, max_excluded=_EXCLUDE[law],
                     min_strict=_MIN_STRICT[law])


@pytest.mark.parametrize("law", ["lj", "kv3"])
def test_forward_fp64_other_laws(afm, orc, law):
    m, base, free, th = _law_case(law)
    plan = afm.Plan(m, base, free, precision="fp64")
    A, phi, st = _np(plan.forward_batch(th))
    P = PT.full_from_free(base, free, th)
    o = PT.oracle_batch(orc, m, P)
    ok = (st == 0) & (o["status"] == 0)
    assert np.array_equal(st, o["status"])
    eA = np.abs(A[ok] / o["A"][ok] - 1)
    eP = np.abs(PT.wrap(phi[ok] - o["phi"][ok]))
    print(f"fp64 {law}: max |dA|/A {eA.max():.1e}, max |dphi| {eP.max():.1e}")
    # rounding-order differences are amplified on the ill-conditioned LJ orbits
    assert np.median(eA) < 1e-12 and np.median(eP) < 1e-10
    assert eA.max() < 1e-6 and eP.max() < 1e-4


def test_failure_status_matches_oracle(afm, orc):
    c = W.config("c1")
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 4, 8)
    th[1, 1] = 1e15  # E* far beyond RK4's stability limit
    th[0, 2] = np.nan
    A, phi, st = _np(plan.forward_batch(th))
    J, stJ = plan.misfit(th, np.ones((1, orc.window_len(c["model"]))))
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, c["model"], P)
    assert (st[1] != 0) and (o["status"][1] != 0)
    assert st[2] == o["status"][2] == 1
    assert st[0] == o["status"][0] == 0
    assert np.isnan(A[1]) and np.isnan(A[2])
    Jc = J.cpu().numpy()
    assert np.isinf(Jc[1]) and np.isinf(Jc[2]) and np.isfinite(Jc[0])


def test_bad_inputs_flagged(afm, orc):
    """Out-of-range target rows and period counts below the lock-in window are flagged, not
    integrated (and never read out of bounds)."""
    c = W.config("c1")
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 3, 14)
    U = np.ones((2, orc.window_len(c["model"])))
    J, st = plan.misfit(th, U, target_id=[0, 2, -1])
    st = st.cpu().numpy()
    assert st[0] == 0 and st[1] == afm.ST_BAD_INPUT and st[2] == afm.ST_BAD_INPUT
    assert np.isinf(J.cpu().numpy()[1:]).all()
    A, phi, st = _np(plan.forward_batch(th, n_cycles=[100, 19, 20]))
    assert st.tolist() == [0, afm.ST_BAD_INPUT, 0]


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
    A, phi, st = _np(plan.forward_batch(th, n_cycles=cyc))
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, c["model"], P, n_cycles=cyc)
    PT.compare_mixed(orc, c["model"], P, o, A, phi, st, tag="uneven", n_cycles=cyc,
                     max_excluded=3, min_strict=35)


def test_full_size_c2_sampled(afm, orc):
    """The benchmark's launch: 1024 particles of C2 at full length in one misfit call; 16 sampled
    particles recomputed by the oracle one by one."""
    c = W.config("c2")
    m = c["model"]
    U = orc.forward(m, W.full_params(c), want_trace=True)["trace"] + W.noise(c, orc.window_len(m), 0)
    plan = _plan(afm, c, "mixed")
    th = _theta(c, 1024, 12)
    J, st = plan.misfit(th, U[None, :])
    J, st = J.cpu().numpy(), st.cpu().numpy()
    idx = np.random.default_rng(13).choice(1024, 16, replace=False)
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th[:, idx])
    o = PT.oracle_batch(orc, m, P, target=U)
    assert np.array_equal(st[idx], o["status"])
    err = np.abs(J[idx] - o["J"])
    for k in np.flatnonzero(err > PT.misfit_tol(o["J"])):
        assert not PT.well_conditioned(orc, m, P[k])


def test_saturating_batch_sampled(afm, orc):
    """A GPU-filling launch (4-wave blocks, branching force law): 131072 trajectories of 40
    periods; 16 sampled trajectories recomputed by the oracle."""
    c = W.config("c2")
    m = dict(c["model"], n_cycles=40)
    plan = _plan(afm, c, "mixed", model=m)
    n = 131072
    th = _theta(c, n, 15)
    A, phi, st = _np(plan.forward_batch(th))
    idx = np.random.default_rng(16).choice(n, 16, replace=False)
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th[:, idx])
    o = PT.oracle_batch(orc, m, P)
    PT.compare_mixed(orc, m, P, o, A[idx], phi[idx], st[idx], tag="saturating", max_excluded=1,
                     min_strict=15)


@pytest.mark.parametrize("N", [4, 5, 203, 4096])
def test_steps_per_period_edges(afm, orc, N):
    """Step counts at the validated limits (4 and 4096) and ones the 4-step inner blocks do not
    divide (5, 203), plain FP64 path, 67 points (a ragged second wave): equal to the oracle to
    rounding; the status (a step of a quarter period can blow up in contact) equal too."""
    c = W.config("c1")
    nc = max(3, 40000 // N)
    m = dict(c["model"], steps_per_cycle=N, n_cycles=nc, lockin_cycles=2)
    plan = _plan(afm, c, "fp64", model=m)
    th = _theta(c, 67, 20 + N)
    A, phi, st = _np(plan.forward_batch(th))
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, m, P)
    assert np.array_equal(st, o["status"])
    ok = st == 0
    np.testing.assert_allclose(A[ok], o["A"][ok], rtol=PT.FP64_RTOL)
    assert np.max(np.abs(PT.wrap(phi[ok] - o["phi"][ok])), initial=0.0) < PT.FP64_RTOL


@pytest.mark.parametrize("N", [203, 4096])
def test_steps_per_period_edges_mixed(afm, orc, N):
    """The same step counts on the mixed path (remainder steps after the 4-step blocks)."""
    c = W.config("c2")
    nc = max(4, 60000 // N)
    m = dict(c["model"], steps_per_cycle=N, n_cycles=nc, lockin_cycles=2)
    plan = _plan(afm, c, "mixed", model=m)
    th = _theta(c, 40, 30 + N)
    A, phi, st = _np(plan.forward_batch(th))
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th)
    o = PT.oracle_batch(orc, m, P)
    PT.compare_mixed(orc, m, P, o, A, phi, st, tag=f"N={N}", max_excluded=1, min_strict=38)


@pytest.mark.parametrize("precision,n,nc", [("mixed", 1000, 60), ("fp64", 333, 40),
                                            ("mixed", 3000, 24), ("mixed", 70000, 24)])
def test_launch_shapes_bit_identical(afm, orc, precision, n, nc):
    """Every launch shape (64 / 128 / 256 lanes x 1 / 2 trajectories per lane) gives the same
    bits as the autotuned launch, on ragged batches (partial workgroups, half-filled lane
    pairs) below and above the large-batch switch; sampled trajectories match the oracle.  At
    3000 trajectories the shapes with at most 32 workgroups run packed onto one XCD and the
    others on the plain grid."""
    import torch

    c = W.config("c2")
    m = dict(c["model"], n_cycles=nc)
    U = orc.forward(m, W.full_params(c), want_trace=True)["trace"]
    plan = _plan(afm, c, precision, model=m)
    th = torch.tensor(_theta(c, n, 40 + n), device="cuda")
    ref_J, ref_st = (x.cpu().numpy() for x in plan.misfit(th, U[None, :]))
    ref = {k: v.cpu().numpy() for k, v in plan.forward_batch(th, trace=n <= 1000).items()
           if v is not None}
    for block in (64, 128, 256):
        for tpl in (1, 2):
            plan.set_launch_shape(block, tpl)
            J, st = (x.cpu().numpy() for x in plan.misfit(th, U[None, :]))
            assert np.array_equal(J.view(np.uint64), ref_J.view(np.uint64)), (block, tpl)
            assert np.array_equal(st, ref_st), (block, tpl)
            r = plan.forward_batch(th, trace=n <= 1000)
            for k, v in r.items():
                if v is None:
                    continue
                a = v.cpu().numpy()
                assert np.array_equal(a.view(np.uint8), ref[k].view(np.uint8)), (block, tpl, k)
    plan.set_launch_shape(0)
    idx = np.random.default_rng(n).choice(n, 12, replace=False)
    P = PT.full_from_free(W.full_params(c), W.free_index(c), th.cpu().numpy()[:, idx])
    o = PT.oracle_batch(orc, m, P, target=U)
    assert np.array_equal(ref_st[idx], o["status"])
    tol = (lambda Jo: 1e-9 * Jo + 1e-15) if precision == "fp64" else PT.misfit_tol
    for k in np.flatnonzero(np.abs(ref_J[idx] - o["J"]) > tol(o["J"])):
        assert precision == "mixed" and not PT.well_conditioned(orc, m, P[k])


@pytest.mark.gpu
@pytest.mark.parametrize("n", [65, 1000, 16384, 16385])
def test_lane_order_is_invisible(afm, n):
    """The small-batch kernel assigns trajectories to lanes in contact-key order (65 to 16384
    trajectories; 16385 runs unordered): permuting the inputs permutes the outputs bit for bit,
    and equal keys (duplicated parameter columns) still cover every trajectory once."""
    import torch

    c = W.config("c2")
    m = dict(c["model"], n_cycles=40)
    plan = _plan(afm, c, "mixed", model=m)
    th = _theta(c, n, 70 + n)
    th[:, : n // 4] = th[:, n // 4: 2 * (n // 4)]  # ties in the ordering key
    perm = np.random.default_rng(n).permutation(n)
    a = plan.forward_batch(torch.tensor(th, device="cuda"))
    b = plan.forward_batch(torch.tensor(np.ascontiguousarray(th[:, perm]), device="cuda"))
    for k in ("amp", "phase", "status"):
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.array_equal(x[perm].view(np.uint8), y.view(np.uint8)), k
    st = a["status"].cpu().numpy()
    assert np.isin(st, [0, 1, 2]).all() and (st == 0).mean() > 0.9  # every slot written


@pytest.mark.parametrize("nm,law", [(2, "dmt"), (3, "kv"), (4, "kv"), (5, "dmt"), (6, "kv"),
                                    (7, "kv"), (8, "kv")])
def test_mode_parallel_bit_identical(afm, orc, nm, law):
    """Mode-parallel launches (one lane per mode, butterfly sums over the group) give the same
    bits as one lane per trajectory, on a ragged batch (partial workgroups); sampled points
    match the oracle."""
    import torch

    c = W.config("c5")
    if nm >= 5:  # the paper's Euler-Bernoulli beam, its first nm modes
        eb = orc.eb_modes(nm, 501)
        ratio, gains = list(eb["ratio"]), list(eb["gain"])
    else:
        ratio = [1.0, 6.27, 17.55, 34.39][:nm]
        gains = c["model"]["gain"] if nm == 3 else [1.566, -0.868, 0.509, -0.36][:nm]
    m = dict(c["model"], law=law, n_modes=nm, q=[400.0] * nm, ratio=ratio, gain=gains,
             n_cycles=60)
    npar = 5 if law == "dmt" else 6
    base = W.full_params(c)[:npar]
    free = [f for f in W.free_index(c) if f[0] < npar]
    rng = np.random.default_rng(50 + nm)
    n = 333
    th = np.stack([np.exp(rng.uniform(np.log(f[1]), np.log(f[2]), n)) if f[3] else
                   rng.uniform(f[1], f[2], n) for f in free])
    U = orc.forward(m, base, want_trace=True)["trace"]
    plan = afm.Plan(m, base, free, precision="mixed")
    thd = torch.tensor(th, device="cuda")
    plan.set_launch_shape(64, 1)
    ref_J = plan.misfit(thd, U[None, :])[0].cpu().numpy()
    ref = {k: v.cpu().numpy() for k, v in plan.forward_batch(thd, trace=True).items()}
    for block in (64, 128, 256):
        plan.set_launch_shape(block, 0)
        J = plan.misfit(thd, U[None, :])[0].cpu().numpy()
        assert np.array_equal(J.view(np.uint64), ref_J.view(np.uint64)), block
        r = plan.forward_batch(thd, trace=True)
        for k, v in r.items():
            assert np.array_equal(v.cpu().numpy().view(np.uint8), ref[k].view(np.uint8)), (block, k)
    idx = rng.choice(n, 6, replace=False)
    P = PT.full_from_free(base, free, th[:, idx])
    o = PT.oracle_batch(orc, m, P)
    PT.compare_mixed(orc, m, P, o, ref["amp"][idx], ref["phase"][idx], ref["status"][idx],
                     tag=f"{nm}-mode {law}", max_excluded=1, min_strict=5)


def test_misfit_swarms_work_queue(afm, orc):
    """afm_misfit_swarms (one generation's forward of afm_invert) on 37 swarms of 100 points with
    uneven period counts and per-swarm separations: the persistent work queue gives the bits of
    afm_misfit with per-point target rows, period counts and parameters (the plain one-lane
    launch, same force form below 65536 trajectories), and sampled points match the oracle; a
    second call reuses the queue order."""
    import torch

    c = W.config("c2")
    m = dict(c["model"], n_cycles=300)
    S, P = 37, 100
    base, free = W.full_params(c), W.free_index(c)
    rng = np.random.default_rng(70)
    cyc = torch.tensor(rng.integers(20, 300, S).astype(np.int32), device="cuda")
    sp = np.zeros((12, S))
    sp[:len(base)] = np.asarray(base)[:, None]
    sp[0] = rng.uniform(13e-9, 16e-9, S)
    U = np.stack([orc.forward(dict(m, n_cycles=int(n)), sp[:len(base), s], want_trace=True)["trace"]
                  for s, n in zip(range(S), cyc.cpu().numpy())])
    th = _theta(c, S * P, 71)
    plan = afm.Plan(m, base, free, precision="mixed")
    J1, st1 = (x.cpu().numpy() for x in plan.misfit_swarms(th, U, P, n_cycles=cyc, swarm_params=sp))
    J2, st2 = (x.cpu().numpy() for x in plan.misfit_swarms(th, U, P, n_cycles=cyc, swarm_params=sp))
    assert np.array_equal(J1.view(np.uint64), J2.view(np.uint64)) and np.array_equal(st1, st2)
    tid = np.repeat(np.arange(S, dtype=np.int32), P)
    ncl = np.repeat(cyc.cpu().numpy(), P)
    # afm_misfit with the same per-point inputs: per-point parameters go in through theta
    # (z_c is not free here), so compare against a plan whose free set includes z_c
    free_z = [(0, 1e-9, 30e-9, 0)] + free
    plan_z = afm.Plan(m, base, free_z, precision="mixed")
    thz = np.vstack([np.repeat(sp[0], P)[None, :], th])
    Jm, stm = (x.cpu().numpy() for x in plan_z.misfit(thz, U, target_id=tid, n_cycles=ncl))
    assert np.array_equal(stm, st1)
    assert np.array_equal(Jm.view(np.uint64), J1.view(np.uint64))
    idx = rng.choice(S * P, 12, replace=False)
    for i in idx:
        s = i // P
        p = sp[:len(base), s].copy()
        for j, f in enumerate(free):
            p[f[0]] = th[j, i]
        o = orc.forward(dict(m, n_cycles=int(ncl[i])), p, U[s])
        assert (st1[i] != 0) == (o["status"] != 0)
        if st1[i] == 0:
            assert abs(J1[i] - o["J"]) <= PT.misfit_tol(o["J"]) or \
                not PT.well_conditioned(orc, dict(m, n_cycles=int(ncl[i])), p)


def test_force_forms_bit_identical(afm):
    """The forms of the FP32 DMT contact force give the same bits on the same tapping
    trajectories, since each adds the contact piece where a lane needs it and nothing (or an
    exact zero) elsewhere: the work queue with more items than 4 x CUs (wave-uniform skip of the
    contact piece per RK4 stage) and with fewer (four-step blocks without it where no lane can
    reach contact), the plain launch above the large-batch switch (the per-stage skip) and below
    it (the block form, lanes in contact-key order)."""
    import torch

    c = W.config("c3")
    m = dict(c["model"], n_cycles=60)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    P = 128
    S = max(2 * n_cu + 6, 520)  # 2 items per swarm: more items than 4 waves per CU
    n = S * P
    assert n >= 65536  # the plain launch of all of them takes the per-lane branching form
    base, free = W.full_params(c), W.free_index(c)
    rng = np.random.default_rng(81)
    cyc = rng.integers(20, 61, S).astype(np.int32)
    sp = np.zeros((afm.MAX_PARAMS, S))
    sp[: len(base)] = base[:, None]
    sp[0] = rng.uniform(9e-9, 17e-9, S)  # 0.45 .. 0.85 A0: every swarm taps
    N, Wn = m["steps_per_cycle"], m["lockin_cycles"] * m["steps_per_cycle"]
    k = np.arange(1, Wn + 1)
    U = np.stack([a * np.sin(2 * np.pi * k / N - ph)
                  for a, ph in zip(sp[0], rng.uniform(0.5, 1.5, S))])
    th = _theta(c, n, 82)
    plan = afm.Plan(m, base, free, precision="mixed")
    cyc_d = torch.tensor(cyc, device="cuda")
    Jq, sq = (x.cpu().numpy() for x in plan.misfit_swarms(th, U, P, n_cycles=cyc_d,
                                                           swarm_params=sp))
    s_small = 40  # 80 items: the under-filled queue
    Jb, sb = (x.cpu().numpy() for x in plan.misfit_swarms(
        np.ascontiguousarray(th[:, : s_small * P]), U[:s_small], P,
        n_cycles=cyc_d[:s_small].clone(), swarm_params=np.ascontiguousarray(sp[:, :s_small])))
    plan_z = afm.Plan(m, base, [(0, 1e-9, 30e-9, 0)] + free, precision="mixed")
    thz = np.vstack([np.repeat(sp[0], P)[None, :], th])
    tid = np.repeat(np.arange(S, dtype=np.int32), P)
    ncl = np.repeat(cyc, P)
    Jp, stp = (x.cpu().numpy() for x in plan_z.misfit(thz, U, target_id=tid, n_cycles=ncl))
    m_small = s_small * P
    Js, sts = (x.cpu().numpy() for x in plan_z.misfit(
        np.ascontiguousarray(thz[:, :m_small]), U[:s_small], target_id=tid[:m_small],
        n_cycles=ncl[:m_small]))
    assert (sq == 0).mean() > 0.99
    for name, J, st in (("plain large", Jp, stp), ("queue block", Jb, sb),
                        ("plain block", Js, sts)):
        r = slice(0, J.size)
        assert np.array_equal(st, sq[r]), name
        assert np.array_equal(J.view(np.uint64), Jq[r].view(np.uint64)), name


def test_int32_batch_limits_are_refused(afm):
    """Swarm batches index their points with 32-bit integers: 2^31 points (one more than an
    int32 holds) are refused with AFM_ERR_INVALID before any pointer is read or anything is
    enqueued, by afm_misfit_swarms, afm_invert and afm_swarm_init alike."""
    import ctypes as C

    c = W.config("c2")
    plan = _plan(afm, c, "mixed", model=dict(c["model"], n_cycles=40))
    L = afm.lib()
    S, P = 1 << 16, 1 << 15
    assert L.afm_misfit_swarms(plan._h, S, P, None, None, None, None, None, None, None) == 1
    assert b"too large" in L.afm_last_error()
    assert L.afm_invert(plan._h, S, None, None, None, P, 1, 0, 0.0, 0, 0, None, None, None,
                        None) == 1
    assert b"too large" in L.afm_last_error()
    sw = afm._Swarm(n_dim=plan.n_free, particles=P, swarms=S)
    assert L.afm_swarm_init(plan._h, C.byref(sw), 0, None) == 1
    assert b"too large" in L.afm_last_error()
    plan.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_kv_point_mass_block_form(afm, orc, precision):
    """Point-mass Kelvin-Voigt batches of 65 to 16384 trajectories run the block-level contact
    test with lanes in contact-key order: their misfits equal those of the gradient's forward
    pass (the branch-free form) bit for bit, a permuted batch permutes them bit for bit, and
    sampled points match the oracle."""
    import torch

    c = W.config("c2")
    m = dict(c["model"], law="kv", n_cycles=80)
    base = np.append(W.full_params(c), 10.0)  # (z_c, H, E*, a0, R) of c2, eta = 10 Pa s
    free = [(1, 1e-20, 1e-19, 0), (2, 0.1e9, 10e9, 1), (5, 1.0, 100.0, 1)]
    n = 1000
    rng = np.random.default_rng(91)
    th = np.stack([np.exp(rng.uniform(np.log(f[1]), np.log(f[2]), n)) if f[3] else
                   rng.uniform(f[1], f[2], n) for f in free])
    U = orc.forward(m, base, want_trace=True)["trace"]
    plan = afm.Plan(m, base, free, precision=precision)
    thd = torch.tensor(th, device="cuda")
    J, st = (x.cpu().numpy() for x in plan.misfit(thd, U[None, :]))
    Jg, _, stg = (x.cpu().numpy() for x in plan.grad_batch(thd, U[None, :]))
    assert np.array_equal(st, stg) and (st == 0).mean() > 0.95
    assert np.array_equal(J.view(np.uint64), Jg.view(np.uint64))
    perm = rng.permutation(n)
    Jp = plan.misfit(torch.tensor(np.ascontiguousarray(th[:, perm]), device="cuda"),
                     U[None, :])[0].cpu().numpy()
    assert np.array_equal(J[perm].view(np.uint64), Jp.view(np.uint64))
    idx = rng.choice(n, 8, replace=False)
    P = PT.full_from_free(base, free, th[:, idx])
    o = PT.oracle_batch(orc, m, P, target=U)
    tol = (lambda Jo: 1e-9 * Jo + 1e-15) if precision == "fp64" else PT.misfit_tol
    assert np.array_equal(st[idx], o["status"])
    for k in np.flatnonzero(np.abs(J[idx] - o["J"]) > tol(o["J"])):
        assert precision == "mixed" and not PT.well_conditioned(orc, m, P[k])


@pytest.mark.parametrize("nm,law", [(2, "dmt"), (3, "kv")])
def test_mode_parallel_block_form_fp64(afm, nm, law):
    """FP64 mode-parallel batches run the block-level contact test too: one lane per mode gives
    the bits of one lane per trajectory (the branch-free form) on tapping trajectories."""
    import torch

    c = W.config("c5")
    ratio = [1.0, 6.27, 17.55][:nm]
    gains = c["model"]["gain"] if nm == 3 else [1.566, -0.868]
    m = dict(c["model"], law=law, n_modes=nm, q=[400.0] * nm, ratio=ratio, gain=gains,
             n_cycles=40)
    npar = 5 if law == "dmt" else 6
    base = W.full_params(c)[:npar]
    free = [f for f in W.free_index(c) if f[0] < npar]
    rng = np.random.default_rng(60 + nm)
    n = 200
    th = np.stack([np.exp(rng.uniform(np.log(f[1]), np.log(f[2]), n)) if f[3] else
                   rng.uniform(f[1], f[2], n) for f in free])
    plan = afm.Plan(m, base, free, precision="fp64")
    thd = torch.tensor(th, device="cuda")
    plan.set_launch_shape(64, 1)
    ref = {k: v.cpu().numpy() for k, v in plan.forward_batch(thd).items() if v is not None}
    assert (ref["status"] == 0).mean() > 0.9
    plan.set_launch_shape(64, 0)
    r = {k: v.cpu().numpy() for k, v in plan.forward_batch(thd).items() if v is not None}
    for k in ref:
        assert np.array_equal(r[k].view(np.uint8), ref[k].view(np.uint8)), k
