"""Deflection at points along the beam (afm_forward_points; the paper's deflection points,
Sec. 3.2) against the oracle.

* seeded weights (the computation is linear in any weights, so physical mode shapes add
  nothing to the check), 3-mode Kelvin-Voigt and the 8-mode beam with a parameter-driven base,
  mixed and FP64: each point's amplitude, phase and window trace;
* weights of one are the tip: the same amplitude and phase as afm_forward_batch;
* a batch too large for one workspace chunk gives the same bits as small batches of the same
  points (chunk offsets), and a diverging trajectory gives NaN at every point."""
import numpy as np
import pytest

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


def _kv3(n_cycles=30, lockin=5):
    c = W.config("c5")
    return c, dict(c["model"], n_cycles=n_cycles, lockin_cycles=lockin, steps_per_cycle=256)


def _check(afm, orc, m, base, free, th, w, prec, tag):
    import torch

    plan = afm.Plan(m, base, free, precision=prec)
    r = plan.forward_points(torch.tensor(th, device="cuda"), w, trace=True)
    A, ph, st = (r[k].cpu().numpy() for k in ("amp", "phase", "status"))
    tr = r["trace"].cpu().numpy()
    A0 = m["free_amplitude"]
    worst = 0.0
    for j in range(th.shape[1]):
        p = np.array(base, dtype=np.float64)
        for d, f in enumerate(free):
            p[f[0]] = th[d, j]
        o = orc.forward_points(m, p, w, want_trace=True)
        assert (st[j] != 0) == (o["status"] != 0), (tag, j)
        if st[j]:
            assert np.all(np.isnan(A[:, j])) and np.all(np.isnan(tr[:, j]))
            continue
        for k in range(w.shape[0]):
            scale = np.max(np.abs(o["trace"][k])) + A0 * np.max(np.abs(w[k])) * 1e-3
            e = np.max(np.abs(tr[k, j] - o["trace"][k])) / scale
            worst = max(worst, e)
            if prec == "fp64":
                assert e <= 1e-9, (tag, j, k, e)
                assert abs(A[k, j] - o["A"][k]) <= 1e-9 * scale
            else:
                assert e <= 2e-5, (tag, j, k, e)
                floor = 5e-6 * A0 * np.max(np.abs(w[k]))
                assert abs(A[k, j] - o["A"][k]) <= max(1e-5 * o["A"][k], floor), (tag, j, k)
                dphi = np.angle(np.exp(1j * (ph[k, j] - o["phi"][k])))
                assert abs(dphi) <= max(1e-4, floor / o["A"][k]), (tag, j, k)
    print(f"{tag}: worst trace error {worst:.2e} of the point's scale")


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_points_kv3(afm, orc, prec):
    c, m = _kv3()
    base, free = W.full_params(c), W.free_index(c)
    th = W.draw_free(c, 9, 21).T.copy()
    w = np.vstack([np.ones(3), np.random.default_rng(5).uniform(-1.5, 1.5, (3, 3))])
    _check(afm, orc, m, base, free, th, w, prec, f"3-mode KV {prec}")


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_points_beam8_parameter_drive(afm, orc, prec):
    c = W.paper_inversion("3d_chirp")
    m = dict(c["model"], n_cycles=2, lockin_cycles=2, steps_per_cycle=500)
    rng = np.random.default_rng(6)
    th = np.stack([rng.uniform(lo, hi, 7) for _, lo, hi, _ in c["free"]])
    w = rng.uniform(-1.0, 1.0, (3, 8))
    _check(afm, orc, m, c["params"], c["free"], th, w, prec, f"8-mode chirp {prec}")


def test_unit_weights_are_the_tip(afm):
    import torch

    c, m = _kv3()
    plan = afm.Plan(m, W.full_params(c), W.free_index(c), precision="mixed")
    th = torch.tensor(W.draw_free(c, 100, 22).T.copy(), device="cuda")
    r = plan.forward_points(th, np.ones((1, 3)))
    f = plan.forward_batch(th)
    ok = f["status"].cpu().numpy() == 0
    assert np.array_equal(r["status"].cpu().numpy(), f["status"].cpu().numpy())
    A0 = m["free_amplitude"]
    assert np.max(np.abs(r["amp"].cpu().numpy()[0, ok] - f["amp"].cpu().numpy()[ok])) < 1e-12 * A0
    dphi = r["phase"].cpu().numpy()[0, ok] - f["phase"].cpu().numpy()[ok]
    assert np.max(np.abs(np.angle(np.exp(1j * dphi)))) < 1e-9


def test_chunked_batch_matches_small_batches(afm):
    """8 modes x 20 x 256 window samples x 8 B = 328 KB per trajectory: 7000 trajectories need
    three workspace chunks; every point of every chunk equals a small batch's, bit for bit."""
    import torch

    c = W.config("c5")
    eb = W.beam_modes(8)
    m = dict(c["model"], n_modes=8, q=[400.0] * 8, ratio=list(eb["ratio"]),
             gain=list(eb["gain"]), n_cycles=22, lockin_cycles=20, steps_per_cycle=256)
    plan = afm.Plan(m, W.full_params(c), W.free_index(c), precision="mixed")
    n = 7000
    th = W.draw_free(c, n, 23).T.copy()
    th[1, 5] = 1e-12  # a destabilising point stays NaN wherever it falls
    w = np.random.default_rng(7).uniform(-1, 1, (2, 8))
    big = plan.forward_points(torch.tensor(th, device="cuda"), w, trace=False)
    Ab, Pb, Sb = (big[k].cpu().numpy() for k in ("amp", "phase", "status"))
    for lo in (0, 3270, 3290, 6900):
        sl = slice(lo, lo + 100)
        r = plan.forward_points(torch.tensor(th[:, sl].copy(), device="cuda"), w)
        assert np.array_equal(r["status"].cpu().numpy(), Sb[sl])
        assert np.array_equal(r["amp"].cpu().numpy().view(np.uint8), Ab[:, sl].copy().view(np.uint8))
        assert np.array_equal(r["phase"].cpu().numpy().view(np.uint8), Pb[:, sl].copy().view(np.uint8))
    bad = Sb != 0
    assert np.all(np.isnan(Ab[:, bad]))


def test_arguments_checked(afm):
    import torch

    c, m = _kv3()
    plan = afm.Plan(m, W.full_params(c), W.free_index(c), precision="mixed")
    th = torch.tensor(W.draw_free(c, 4, 24).T.copy(), device="cuda")
    with pytest.raises(afm.AfmError, match="status 1"):
        plan.forward_points(th, np.ones((17, 3)))
    with pytest.raises(afm.AfmError, match="status 1"):
        plan.forward_points(th, np.full((1, 3), np.nan))
    r = plan.forward_points(th[:, :0], np.ones((1, 3)))
    assert r["amp"].shape == (1, 0)


def test_points_then_polish_then_points_on_one_plan(afm):
    """The point workspace and the polish workspace are separate plan buffers: growing the
    polish workspace between two afm_forward_points calls must leave the second call's results
    equal to the first's, bit for bit, and closing the plan must release each buffer once."""
    import torch

    c, m = _kv3(n_cycles=12, lockin=4)
    base, free = W.full_params(c), W.free_index(c)
    plan = afm.Plan(m, base, free, precision="mixed")
    th = torch.tensor(W.draw_free(c, 64, 25).T.copy(), device="cuda")
    w = np.random.default_rng(8).uniform(-1.0, 1.0, (2, 3))
    first = plan.forward_points(th, w, trace=True)
    first = {k: v.cpu().numpy() for k, v in first.items()}
    U = plan.forward_batch(th[:, :1], trace=True)["trace"]
    for n in (4, 96):  # the second polish grows its workspace
        z = torch.tensor(np.random.default_rng(n).uniform(0.2, 0.8, (len(free), n)), device="cuda")
        plan.polish(z, U, steps=2)
    second = plan.forward_points(th, w, trace=True)
    torch.cuda.synchronize()
    for k in ("amp", "phase", "status", "trace"):
        assert np.array_equal(second[k].cpu().numpy().view(np.uint8), first[k].view(np.uint8)), k
    plan.close()
