"""Pins of the oracle's integrator on the linear driven cantilever (tip force switched off).

With F = 0 the model is the damped, base-driven oscillator of Eq. 2, whose steady state has a
closed form and whose RK4 discretisation is an affine map with a closed form too.  The paper
validates its solvers against analytic solutions for sinusoidal base motion (Sec. 3.3).
"""
import numpy as np
import pytest

import workloads as W


def _linear_model(n_modes=1, ratio=(1.0,), gain=(1.0,), q=(400.0,), N=64, drive_ratio=1.0,
                  n_cycles=40, lockin=20):
    return dict(n_modes=n_modes, law="none", k=40.0, f0=300e3, drive_freq=300e3 * drive_ratio,
                q=list(q), ratio=list(ratio), gain=list(gain), free_amplitude=20e-9,
                steps_per_cycle=N, n_cycles=n_cycles, lockin_cycles=lockin, ic="free_steady",
                div_limit=100.0)


def _continuous_steady(m):
    """Closed-form steady response u = A sin(wd t - phi) of the linear modal equations."""
    wd = 2 * np.pi * m["drive_freq"]
    H = 0j
    for i in range(m["n_modes"]):
        wi = 2 * np.pi * m["f0"] * m["ratio"][i]
        H += m["gain"][i] * wd**2 / (wi**2 - wd**2 + 1j * wi * wd / m["q"][i])
    return abs(H), -np.angle(H)


def _state_scale(m):
    """Natural size of each state component: A0 for deflections, w_d A0 for rates."""
    nm = m["n_modes"]
    A0, wd = m["free_amplitude"], 2 * np.pi * m["drive_freq"]
    return np.concatenate([np.full(nm, A0), np.full(nm, wd * A0)])


def _rk4_affine_period(m, a):
    """N-step map y -> Phi y + C of classical RK4 on y' = L y + g(t), from the RK4 stability
    polynomial and its forcing form: one step is y+ = R(Z) y + h/6 [(I + Z + Z^2/2 + Z^3/4) g0
    + (4I + 2Z + Z^2/2) g_half + g1], Z = h L, R(Z) = I + Z + Z^2/2 + Z^3/6 + Z^4/24."""
    nm = m["n_modes"]
    w0 = 2 * np.pi * m["f0"]
    wd = 2 * np.pi * m["drive_freq"]
    N = m["steps_per_cycle"]
    h = 1.0 / (m["drive_freq"] * N)
    w = np.array([w0 * r for r in m["ratio"]])
    c = w / np.array(m["q"])
    L = np.zeros((2 * nm, 2 * nm))
    L[:nm, nm:] = np.eye(nm)
    L[nm:, :nm] = -np.diag(w**2)
    L[nm:, nm:] = -np.diag(c)
    I = np.eye(2 * nm)
    Z = h * L
    R = I + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    B0 = I + Z + Z @ Z / 2 + Z @ Z @ Z / 4
    Bh = 4 * I + 2 * Z + Z @ Z / 2
    gv = np.concatenate([np.zeros(nm), np.array(m["gain"])]) * a * wd**2

    def g(t):
        return gv * np.sin(wd * t)

    Phi, C = I.copy(), np.zeros(2 * nm)
    for n in range(N):
        t = n * h
        cn = h / 6 * (B0 @ g(t) + Bh @ g(t + h / 2) + g(t + h))
        Phi = R @ Phi
        C = R @ C + cn
    return Phi, C


@pytest.mark.parametrize("drive_ratio", [1.0, 0.93])
def test_discrete_periodic_orbit(orc, drive_ratio):
    """The oracle started on the exact periodic orbit of the RK4 map returns to it after every
    period (a wrong stage time, sign or weight breaks this at O(h) or worse)."""
    m = _linear_model(N=64, drive_ratio=drive_ratio)
    a = orc.base_amplitude(m)
    Phi, C = _rk4_affine_period(m, a)
    ystar = np.linalg.solve(np.eye(len(C)) - Phi, C)
    for nc in (1, 7):
        st, u, _, yend = orc.trajectory(m, [0.0], n_cycles=nc, y0=ystar, n_out=1)
        assert st == 0
        assert np.all(np.abs(yend - ystar) < 1e-12 * _state_scale(m))


def test_periodic_orbit_three_modes(orc):
    m = _linear_model(n_modes=3, ratio=(1.0, 6.27, 17.55), gain=(1.565984, -0.867872, 0.508851),
                      q=(400.0, 300.0, 200.0), N=128, drive_ratio=1.0)
    a = orc.base_amplitude(m)
    Phi, C = _rk4_affine_period(m, a)
    ystar = np.linalg.solve(np.eye(len(C)) - Phi, C)
    st, _, _, yend = orc.trajectory(m, [0.0], n_cycles=3, y0=ystar, n_out=1)
    assert st == 0
    assert np.all(np.abs(yend - ystar) < 1e-12 * _state_scale(m))


@pytest.mark.parametrize("n_modes", [1, 3])
def test_free_amplitude_and_phase_closed_form(orc, n_modes):
    """Free steady state: lock-in amplitude equals the set free amplitude A0 and the phase the
    closed-form one (pi/2 for a point mass driven at resonance), up to the RK4 error."""
    if n_modes == 1:
        m = _linear_model(N=256, n_cycles=30, lockin=20)
    else:
        m = _linear_model(n_modes=3, ratio=(1.0, 6.27, 17.55),
                          gain=(1.565984, -0.867872, 0.508851), q=(400.0,) * 3, N=512,
                          n_cycles=30, lockin=20)
    A_c, phi_c = _continuous_steady(m)
    a = orc.base_amplitude(m)
    assert abs(a * A_c / m["free_amplitude"] - 1) < 1e-14
    r = orc.forward(m, [0.0])
    assert r["status"] == 0
    assert abs(r["A"] / m["free_amplitude"] - 1) < 2e-7
    assert abs(r["phi"] - phi_c) < 2e-6
    if n_modes == 1:
        assert abs(phi_c - np.pi / 2) < 1e-15


def test_point_mass_resonance_ic(orc):
    """At resonance the free steady state starts at the bottom of the swing: u = -A0, u' = 0."""
    m = _linear_model()
    y = orc.initial_state(m)
    assert abs(y[0] + 20e-9) < 1e-22 and abs(y[1]) < 1e-12
    assert abs(orc.base_amplitude(m) - 20e-9 / 400) < 1e-24


def test_fourth_order_convergence(orc):
    """Off resonance, from the exact discrete orbit: the periodic orbit's lock-in amplitude and
    phase approach the continuous closed form with error ratio ~16 per step halving."""
    errs = []
    for N in (32, 64, 128):
        m = _linear_model(N=N, drive_ratio=0.97, n_cycles=1, lockin=1)
        a = orc.base_amplitude(m)
        Phi, C = _rk4_affine_period(m, a)
        ystar = np.linalg.solve(np.eye(len(C)) - Phi, C)
        st, u, _, _ = orc.trajectory(m, [0.0], n_cycles=1, y0=ystar, n_out=N)
        A, phi = orc.lockin(u, N, 1)
        A_c, phi_c = _continuous_steady(m)
        errs.append(abs(A - a * A_c) / (a * A_c) + abs(phi - phi_c))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 14.0 < r1 < 18.0 and 14.0 < r2 < 18.0, (errs, r1, r2)


def test_rest_ic_rings_up(orc):
    """From rest the resonant response grows as A0 (1 - exp(-pi n / Q)) (envelope of the
    linear oscillator); after 3Q/pi cycles it is within 5.5% of A0."""
    m = _linear_model(N=64, n_cycles=382, lockin=1)
    m["ic"] = "rest"
    r = orc.forward(m, [0.0])
    expect = 1 - np.exp(-np.pi * 381.5 / 400.0)
    assert abs(r["A"] / 20e-9 - expect) < 2e-3


def test_workload_linear_limit(orc):
    """The stored workloads reduce to the free oscillator when the tip is far away."""
    c = W.config("c1")
    p = W.full_params(c, zc=1e-6)
    r = orc.forward(c["model"], p)
    assert abs(r["A"] / c["model"]["free_amplitude"] - 1) < 1e-5


def _eight_modes(orc, **kw):
    eb = orc.eb_modes(8, 501)
    return _linear_model(n_modes=8, ratio=tuple(eb["ratio"]), gain=tuple(eb["gain"]),
                         q=(400.0,) * 8, **kw)


def test_periodic_orbit_eight_modes(orc):
    """The paper's eight-mode beam (Sec. 3.2): the oracle returns to the exact periodic orbit of
    the RK4 map after each period (N = 512 keeps the eighth mode inside RK4's stability
    interval, h w_8 = 1.94)."""
    m = _eight_modes(orc, N=512, drive_ratio=1.0)
    a = orc.base_amplitude(m)
    Phi, C = _rk4_affine_period(m, a)
    ystar = np.linalg.solve(np.eye(len(C)) - Phi, C)
    st, _, _, yend = orc.trajectory(m, [0.0], n_cycles=2, y0=ystar, n_out=1)
    assert st == 0
    assert np.all(np.abs(yend - ystar) < 1e-11 * _state_scale(m))


def test_free_amplitude_closed_form_eight_modes(orc):
    m = _eight_modes(orc, N=1024, n_cycles=30, lockin=20)
    A_c, phi_c = _continuous_steady(m)
    a = orc.base_amplitude(m)
    assert abs(a * A_c / m["free_amplitude"] - 1) < 1e-13
    r = orc.forward(m, [0.0])
    assert r["status"] == 0
    assert abs(r["A"] / m["free_amplitude"] - 1) < 2e-7
    assert abs(r["phi"] - phi_c) < 2e-6
