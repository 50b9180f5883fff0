"""GPU discrete adjoint (afm_grad_batch) against the oracle's adjoint and finite differences.

Errors are norm-wise in normalised coordinates, |g - g_ref|_2 / |g_ref|_2 per parameter point
with g_z = dJ/dz = dJ/dtheta * dtheta/dz over the search box.  A point passes when its error is
below its tolerance: 1e-3 (mixed) or 1e-6 (FP64), widened where the oracle's own gradient
changes by more than a third of that under FP32-sized (resp. FP64-sized) changes of the data
(see parity.py).  The tests print how many points needed the widened tolerance."""
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


def _zscale(free, theta):
    """dtheta/dz per free parameter at theta [D][n]."""
    out = np.empty_like(theta)
    for j, (_, lo, hi, lg) in enumerate(free):
        out[j] = theta[j] * np.log(hi / lo) if lg else (hi - lo)
    return out


def _oracle_grads(orc, m, P, free, U):
    g = np.empty((len(free), P.shape[0]))
    J = np.empty(P.shape[0])
    st = np.empty(P.shape[0], np.int32)
    for i in range(P.shape[0]):
        st[i], J[i], gf = orc.misfit_grad(m, P[i], U)
        g[:, i] = [gf[f[0]] for f in free]
    return J, g, st


def _case(name):
    if name == "dmt-c2":
        c = W.config("c2")
        m = c["model"]
        th = W.draw_free(c, 33, 21).T.copy()
        return c, m, W.full_params(c), W.free_index(c), th
    if name == "lj-c4":
        c = W.config("c4")
        return c, c["model"], W.full_params(c), W.free_index(c), W.draw_free(c, 20, 22).T.copy()
    if name == "kv3-c5":
        c = W.config("c5")
        m = dict(c["model"], n_cycles=120)
        free = W.free_index(c)
        rng = np.random.default_rng(23)
        th = np.stack([np.exp(rng.uniform(np.log(f[1]), np.log(f[2]), 10)) if f[3] else
                       rng.uniform(f[1], f[2], 10) for f in free])
        return c, m, W.full_params(c), free, th
    raise KeyError(name)


def _target(orc, c, m, base):
    U = orc.forward(m, base, want_trace=True)["trace"]
    return U + W.noise(dict(noise=0.05e-9), len(U), 5)


def test_grad_fp64_matches_oracle_adjoint(afm, orc):
    c = W.config("c2")
    m = dict(c["model"], n_cycles=60)
    base, free = W.full_params(c), W.free_index(c)
    th = W.draw_free(c, 20, 20).T.copy()
    U = _target(orc, c, m, base)
    plan = afm.Plan(m, base, free, precision="fp64")
    J, dJ, st = plan.grad_batch(th, U[None, :], ckpt_stride=16)
    J, dJ, st = J.cpu().numpy(), dJ.cpu().numpy(), st.cpu().numpy()
    P = PT.full_from_free(base, free, th)
    Jo, go, sto = _oracle_grads(orc, m, P, free, U)
    assert np.array_equal(st, sto)
    np.testing.assert_allclose(J, Jo, rtol=1e-9)
    zs = _zscale(free, th)
    err = np.linalg.norm((dJ - go) * zs, axis=0) / np.linalg.norm(go * zs, axis=0)
    print(f"fp64 adjoint: max rel err {err.max():.2e}")
    assert err.max() < 1e-7


@pytest.mark.parametrize("name", ["dmt-c2", "lj-c4", "kv3-c5"])
def test_grad_mixed_matches_oracle_adjoint(afm, orc, name):
    c, m, base, free, th = _case(name)
    U = _target(orc, c, m, base)
    plan = afm.Plan(m, base, free, precision="mixed")
    J, dJ, st = plan.grad_batch(th, U[None, :])
    J, dJ, st = J.cpu().numpy(), dJ.cpu().numpy(), st.cpu().numpy()
    Jm, _ = plan.misfit(th, U[None, :])
    assert np.array_equal(J, Jm.cpu().numpy())  # same forward arithmetic as afm_misfit
    P = PT.full_from_free(base, free, th)
    Jo, go, sto = _oracle_grads(orc, m, P, free, U)
    zs = _zscale(free, th)
    ok = (st == 0) & (sto == 0)
    assert np.array_equal(st != 0, sto != 0) or all(
        PT.grad_tolerance(orc, m, P[i], U, free) > PT.GRAD_TOL for i in np.flatnonzero(st != sto))
    err = np.full(len(J), np.nan)
    err[ok] = np.linalg.norm((dJ[:, ok] - go[:, ok]) * zs[:, ok], axis=0) / \
        np.linalg.norm(go[:, ok] * zs[:, ok], axis=0)
    widened, failing = 0, []
    for i in np.flatnonzero(ok & (err > PT.GRAD_TOL)):
        tol = PT.grad_tolerance(orc, m, P[i], U, free)
        widened += 1
        if err[i] > tol:
            failing.append((int(i), err[i], tol))
    print(f"{name}: n {len(J)}, median rel err {np.nanmedian(err):.2e}, max {np.nanmax(err):.2e}, "
          f"within 1e-3 {int(np.sum(err[ok] <= PT.GRAD_TOL))}, needed a widened tolerance "
          f"{widened}, failing {len(failing)}")
    assert not failing, failing


def test_grad_mixed_vs_central_differences(afm, orc):
    """Central differences of the FP64 oracle misfit agree with the GPU adjoint to 1e-3
    (norm-wise, normalised coordinates) on well-conditioned points (a 100-period horizon, where
    most of the box is well conditioned).  The differences are Richardson-extrapolated from
    h = 1e-4 and 5e-5 relative: a plain central difference at 1e-4 carries an O(h^2) truncation
    error that alone reaches 1e-3 where the misfit is strongly curved."""
    c, m, base, free, th = _case("dmt-c2")
    m = dict(m, n_cycles=100)
    U = _target(orc, c, m, base)
    plan = afm.Plan(m, base, free, precision="mixed")
    _, dJ, st = plan.grad_batch(th, U[None, :])
    dJ, st = dJ.cpu().numpy(), st.cpu().numpy()
    P = PT.full_from_free(base, free, th)
    zs = _zscale(free, th)
    checked = 0
    for i in range(th.shape[1]):
        if checked == 6:
            break
        if st[i] != 0 or PT.grad_tolerance(orc, m, P[i], U, free) > PT.GRAD_TOL:
            continue
        fd = np.empty(len(free))
        for j, f in enumerate(free):
            cd = []
            for rel in (1e-4, 5e-5):
                hj = rel * abs(P[i, f[0]])
                pp, pm = P[i].copy(), P[i].copy()
                pp[f[0]] += hj
                pm[f[0]] -= hj
                cd.append((orc.forward(m, pp, U)["J"] - orc.forward(m, pm, U)["J"]) / (2 * hj))
            fd[j] = (4.0 * cd[1] - cd[0]) / 3.0
        e = np.linalg.norm((dJ[:, i] - fd) * zs[:, i]) / np.linalg.norm(fd * zs[:, i])
        print(f"point {i}: adjoint vs central differences {e:.2e}")
        assert e < 1e-3, (i, dJ[:, i], fd)
        checked += 1
    assert checked >= 4


def test_ckpt_stride_invariance(afm, orc):
    """The recomputation is bit-identical and the reverse walk visits the steps in the same
    order for every stride, so J and dJ are independent of the checkpoint stride bit for bit."""
    c = W.config("c2")
    m = dict(c["model"], n_cycles=50)
    base, free = W.full_params(c), W.free_index(c)
    th = W.draw_free(c, 70, 24).T.copy()
    U = _target(orc, c, m, base)
    plan = afm.Plan(m, base, free, precision="mixed")
    ref = None
    for kc in (1, 7, 64, 256, 50 * 256, 0):
        J, dJ, st = plan.grad_batch(th, U[None, :], ckpt_stride=kc)
        J, dJ = J.cpu().numpy(), dJ.cpu().numpy()
        if ref is None:
            ref = (J, dJ)
            continue
        assert np.array_equal(J, ref[0]), kc
        assert np.array_equal(dJ, ref[1]), (kc, np.max(np.abs(dJ / ref[1] - 1)))


def test_autograd_function(afm, orc):
    import torch

    c = W.config("c2")
    m = dict(c["model"], n_cycles=40)
    base, free = W.full_params(c), W.free_index(c)
    th = torch.tensor(W.draw_free(c, 9, 25).T.copy(), device="cuda", requires_grad=True)
    U = torch.tensor(_target(orc, c, m, base)[None, :], device="cuda")
    plan = afm.Plan(m, base, free, precision="mixed")
    J = afm.misfit_fn().apply(th, plan, U)
    w = torch.arange(1, 10, dtype=torch.float64, device="cuda")
    (w * J).sum().backward()
    _, dJ, _ = plan.grad_batch(th.detach(), U)
    torch.testing.assert_close(th.grad, w[None, :] * dJ, rtol=0, atol=0)
    Jm, _ = plan.misfit(th.detach(), U)
    assert torch.equal(J.detach(), Jm)


def test_grad_fp64_other_laws(afm, orc):
    """FP64 adjoint for LJ (full C4 length) and the 3-mode Kelvin-Voigt beam: no exclusions."""
    for name in ("lj-c4", "kv3-c5"):
        c, m, base, free, th = _case(name)
        th = th[:, :6]
        U = _target(orc, c, m, base)
        plan = afm.Plan(m, base, free, precision="fp64")
        J, dJ, st = plan.grad_batch(th, U[None, :], ckpt_stride=256)
        J, dJ, st = J.cpu().numpy(), dJ.cpu().numpy(), st.cpu().numpy()
        P = PT.full_from_free(base, free, th)
        Jo, go, sto = _oracle_grads(orc, m, P, free, U)
        assert np.array_equal(st, sto)
        ok = st == 0
        zs = _zscale(free, th)
        err = np.linalg.norm((dJ[:, ok] - go[:, ok]) * zs[:, ok], axis=0) / \
            np.linalg.norm(go[:, ok] * zs[:, ok], axis=0)
        print(f"fp64 {name}: median rel err {np.median(err):.2e}, max {err.max():.2e}")
        for k, i in enumerate(np.flatnonzero(ok)):
            if err[k] > PT.GRAD_TOL64:
                assert err[k] <= PT.grad_tolerance(orc, m, P[i], U, free, fp64=True), (name, i)


@pytest.mark.parametrize("nm", [2, 3, 4, 5, 6, 7, 8])
def test_grad_mode_parallel_bit_identical(afm, orc, nm):
    """The mode-parallel adjoint (one lane per mode; small batches) returns the same bits at
    every checkpoint stride as one lane per trajectory (explicit stride above 16384 points);
    J equals afm_misfit's."""
    c = W.config("c5")
    if nm >= 5:
        eb = orc.eb_modes(nm, 501)
        ratio, gains = list(eb["ratio"]), list(eb["gain"])
    else:
        ratio = [1.0, 6.27, 17.55, 34.39][:nm]
        gains = c["model"]["gain"] if nm == 3 else [1.566, -0.868, 0.509, -0.36][:nm]
    m = dict(c["model"], n_modes=nm, q=[400.0] * nm, ratio=ratio, gain=gains, n_cycles=40)
    base, free = W.full_params(c), W.free_index(c)
    rng = np.random.default_rng(60 + nm)
    n = 37
    th = np.stack([np.exp(rng.uniform(np.log(f[1]), np.log(f[2]), n)) if f[3] else
                   rng.uniform(f[1], f[2], n) for f in free])
    U = _target(orc, c, m, base)
    plan = afm.Plan(m, base, free, precision="mixed")
    ref = None
    for kc in (16, 64, 256):
        r = [x.cpu().numpy() for x in plan.grad_batch(th, U[None, :], ckpt_stride=kc)]
        if ref is None:
            ref = r
        for a, b in zip(r, ref):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), kc
    Jm, _ = plan.misfit(th, U[None, :])
    assert np.array_equal(ref[0], Jm.cpu().numpy())
    # above 16384 trajectories an explicit stride runs one lane per trajectory: the same points
    # repeated past that size must give the same bits as the mode-parallel small batch
    big = np.tile(th, (1, 16400 // n + 1))
    rb = [x.cpu().numpy() for x in plan.grad_batch(big, U[None, :], ckpt_stride=64)]
    assert np.array_equal(rb[0][:n].view(np.uint8), ref[0].view(np.uint8))
    assert np.array_equal(rb[1][:, :n].view(np.uint8), ref[1].view(np.uint8))
    assert np.array_equal(rb[2][:n], ref[2])


def test_grad_eight_modes_matches_oracle_adjoint(afm, orc):
    """The paper's eight-mode beam with the Kelvin-Voigt law: mixed adjoint against the oracle's
    exact discrete adjoint (conditioning-aware tolerance), 6 points, 60 periods x 512 steps."""
    c = W.config("c5")
    eb = orc.eb_modes(8, 501)
    m = dict(c["model"], n_modes=8, q=[400.0] * 8, ratio=list(eb["ratio"]),
             gain=list(eb["gain"]), n_cycles=60)
    base, free = W.full_params(c), W.free_index(c)
    rng = np.random.default_rng(88)
    th = np.stack([np.exp(rng.uniform(np.log(f[1]), np.log(f[2]), 6)) if f[3] else
                   rng.uniform(f[1], f[2], 6) for f in free])
    U = _target(orc, c, m, base)
    plan = afm.Plan(m, base, free, precision="mixed")
    J, dJ, st = (x.cpu().numpy() for x in plan.grad_batch(th, U[None, :]))
    P = PT.full_from_free(base, free, th)
    Jo, go, sto = _oracle_grads(orc, m, P, free, U)
    zs = _zscale(free, th)
    for i in range(6):
        assert (st[i] != 0) == (sto[i] != 0)
        if st[i]:
            continue
        assert abs(J[i] - Jo[i]) <= PT.misfit_tol(Jo[i]) or not PT.well_conditioned(orc, m, P[i])
        e = np.linalg.norm((dJ[:, i] - go[:, i]) * zs[:, i]) / np.linalg.norm(go[:, i] * zs[:, i])
        tol = PT.GRAD_TOL if e <= PT.GRAD_TOL else PT.grad_tolerance(orc, m, P[i], U, free)
        print(f"8-mode point {i}: rel err {e:.2e} (tolerance {tol:.1e})")
        assert e <= tol
