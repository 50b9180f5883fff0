"""Pins of the oracle's parameter-driven base motion (the base-motion and chirp inversions of
Sec. 4): the chirp of Eq. 10, y_b = a sin(2 pi (f + g t) t), with a, f, g per trajectory (p[8],
p[9], p[10]).

* with f at the nominal frequency, no chirp and a the amplitude the free amplitude sets, the
  trajectory equals the fixed-drive one (a different code path of the same motion);
* the response of the linear cantilever is linear in a;
* off resonance, the long-run response is the closed-form steady state at f (Eq. 2 with the
  tip force off), fitted by least squares at f from the trajectory;
* a chirp's response matches an independent adaptive integrator (scipy's DOP853) of the same
  motion written in absolute coordinates, where only y_b and its rate enter: this fixes the
  sign and form of the base acceleration the oracle derives for the chirp;
* the reverse-mode gradient with respect to a, f, g equals the complex-step derivative of an
  independent restatement of the discrete map."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp


def _model(N=256, n_cycles=40, lockin=20, drive="params", q=400.0):
    return dict(n_modes=1, law="none", k=40.0, f0=300e3, drive_freq=300e3, q=[q], ratio=[1.0],
                gain=[1.0], free_amplitude=20e-9, steps_per_cycle=N, n_cycles=n_cycles,
                lockin_cycles=lockin, ic="rest", div_limit=100.0, drive=drive)


def _p(a, f, g=0.0):
    p = np.zeros(12)
    p[8], p[9], p[10] = a, f, g
    return p


def test_matches_fixed_drive(orc):
    m_tab = _model(drive="table")
    a = orc.base_amplitude(m_tab)
    st0, u0, _, y0 = orc.trajectory(m_tab, [0.0], n_out=5120)
    st1, u1, _, y1 = orc.trajectory(_model(), _p(a, 300e3), n_out=5120)
    assert st0 == 0 and st1 == 0
    scale = np.max(np.abs(u0))
    assert np.max(np.abs(u1 - u0)) < 1e-11 * scale


def test_linear_in_amplitude(orc):
    m = _model(n_cycles=10, lockin=10)
    _, u1, _, _ = orc.trajectory(m, _p(0.05e-9, 290e3, 1e9), n_out=2560)
    _, u3, _, _ = orc.trajectory(m, _p(0.15e-9, 290e3, 1e9), n_out=2560)
    assert np.max(np.abs(u3 - 3.0 * u1)) < 1e-12 * np.max(np.abs(u3))


@pytest.mark.parametrize("fr", [0.9, 1.07])
def test_off_resonance_steady_state(orc, fr):
    q = 20.0  # fast ring-down so that 600 periods reach the steady state to ~1e-12
    m = _model(N=256, n_cycles=600, lockin=20, q=q)
    a, f = 0.3e-9, 300e3 * fr
    st, u, _, _ = orc.trajectory(m, _p(a, f), n_out=20 * 256)
    assert st == 0
    h = 1.0 / (300e3 * 256)
    n = np.arange(600 * 256 - 20 * 256 + 1, 600 * 256 + 1)
    t = n * h
    B = np.stack([np.sin(2 * np.pi * f * t), np.cos(2 * np.pi * f * t)], axis=1)
    c, *_ = np.linalg.lstsq(B, u, rcond=None)
    A_fit = np.hypot(*c)
    w0, wd = 2 * np.pi * 300e3, 2 * np.pi * f
    A_closed = a * wd**2 / abs(w0**2 - wd**2 + 1j * w0 * wd / q)
    assert abs(A_fit / A_closed - 1) < 1e-7
    assert np.max(np.abs(B @ c - u)) < 1e-7 * A_closed


def test_chirp_against_adaptive_integrator(orc):
    q, f0 = 50.0, 300e3
    a, f, g = 0.4e-9, 280e3, 1e9  # instantaneous f + 2 g t: 280 -> 480 kHz over the 30 periods
    m = _model(N=1024, n_cycles=30, lockin=30, q=q)
    st, u, ud, yend = orc.trajectory(m, _p(a, f, g), n_out=1, want_rate=True)
    assert st == 0
    w0 = 2 * np.pi * f0
    T = 30 / f0

    # the same motion in absolute coordinates X = q + y_b, which needs only y_b and its rate:
    # X'' = -w0^2 (X - y_b) - (w0/Q) (X' - y_b'), so the base acceleration never appears
    def base(t):
        phi = 2 * np.pi * (f + g * t) * t
        return a * np.sin(phi), a * 2 * np.pi * (f + 2 * g * t) * np.cos(phi)

    def rhs(t, y):
        yb, ybd = base(t)
        return [y[1], -w0 * w0 * (y[0] - yb) - (w0 / q) * (y[1] - ybd)]

    yb0, ybd0 = base(0.0)
    sol = solve_ivp(rhs, (0.0, T), [yb0, ybd0], method="DOP853", rtol=1e-12, atol=1e-24)
    ybT, ybdT = base(T)
    ref = np.array([sol.y[0, -1] - ybT, sol.y[1, -1] - ybdT])
    # the chirp term 4 pi g cos(phi) is ~4e-3 of the base acceleration here, so a wrong sign or
    # a missing term would show at ~4e-3 a Q; RK4 at 1024 steps per period is good to ~1e-9
    assert abs(yend[0] - ref[0]) < 1e-7 * a * q
    assert abs(yend[1] - ref[1]) < 1e-7 * a * q * w0


@pytest.mark.parametrize("case", ["none1", "dmt1", "kv3"])
def test_misfit_gradient_matches_complex_step(orc, case):
    """The oracle's reverse-mode gradient with respect to the base motion's a, f, g (and the law's
    constants) equals the complex-step derivative of an independent restatement of the same
    discrete map (tests/cs_model.py)."""
    import cs_model

    if case == "kv3":
        m = dict(_model(N=64, n_cycles=6, lockin=2), law="kv", n_modes=3, q=[400.0] * 3,
                 ratio=[1.0, 6.27, 17.55], gain=[1.565984, -0.867872, 0.508851])
        p = _p(0.3e-9, 297e3, 2e9)
        p[:6] = [3e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9, 10.0]
    else:
        m = dict(_model(N=64, n_cycles=6, lockin=2), law=case[:-1])
        p = _p(0.3e-9, 297e3, 2e9)
        p[:5] = [3e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9] if case == "dmt1" else [3e-9, 0, 0, 0, 0]
    tr = orc.forward(m, p, want_trace=True)["trace"]
    U = 0.9 * tr + 1e-10
    st, J, g = orc.misfit_grad(m, p, U)
    assert st == 0
    Jc, gc = cs_model.gradient(m, list(p), list(U), [0.0] * (2 * m["n_modes"]), 0.0)
    assert abs(J / Jc - 1) < 1e-12
    for j in (8, 9, 10):
        assert abs(g[j] - gc[j]) <= 1e-8 * abs(gc[j]), (j, g[j], gc[j])
    law_slots = {"none1": [0], "dmt1": [0, 1, 2, 3], "kv3": [0, 1, 2, 3, 5]}[case]
    for j in law_slots:
        assert abs(g[j] - gc[j]) <= 1e-8 * max(abs(gc[j]), 1e-30), (j, g[j], gc[j])
