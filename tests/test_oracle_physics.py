"""Physical pins of the oracle with tip-sample forces: energy balance, the Cleveland relation for
conservative forces at resonance, dissipation sign for Kelvin-Voigt contact, the set-point
separation, and failure reporting."""
import numpy as np
import pytest

import workloads as W


def _steady_window(orc, m, p, N, nc=3000, periods=20):
    m = dict(m, steps_per_cycle=N, n_cycles=nc, lockin_cycles=periods)
    Wn = periods * N
    st, u, ud, _ = orc.trajectory(m, p, want_rate=True, n_out=Wn)
    assert st == 0
    h = 1.0 / (m["drive_freq"] * N)
    t = (nc * N - Wn + 1 + np.arange(Wn)) * h
    return m, u, ud, t, h


def _works(orc, m, u, ud, t, h):
    """Drive work of the base acceleration and damping loss over whole periods (rectangle rule
    on a periodic integrand): W_drive = int u' M a wd^2 sin(wd t), W_damp = int M (w0/Q) u'^2."""
    w0, wd = 2 * np.pi * m["f0"], 2 * np.pi * m["drive_freq"]
    M = m["k"] / w0**2
    a = orc.base_amplitude(m)
    Wd = np.sum(ud * M * a * wd**2 * np.sin(wd * t)) * h
    Wdamp = np.sum(M * w0 / m["q"][0] * ud**2) * h
    return Wd, Wdamp


def test_energy_balance_conservative_dmt(orc):
    """At steady state a conservative tip force does no net work per period, so the drive work
    equals the damping loss; the imbalance falls with the step (quadrature of a kinked force)."""
    c = W.config("c1")
    p = W.full_params(c)
    imb = []
    for N in (256, 512):
        m, u, ud, t, h = _steady_window(orc, c["model"], p, N)
        Wd, Wdamp = _works(orc, m, u, ud, t, h)
        imb.append(abs(Wd - Wdamp) / Wdamp)
    assert imb[0] < 2e-4 and imb[1] < 3e-5 and imb[1] < imb[0] / 4, imb


def test_energy_balance_free(orc):
    c = W.config("c1")
    m = dict(c["model"], law="none")
    m, u, ud, t, h = _steady_window(orc, m, [0.0], 256, nc=40)
    Wd, Wdamp = _works(orc, m, u, ud, t, h)
    assert abs(Wd - Wdamp) / Wdamp < 1e-7  # O((wd h)^4) discretisation of the orbit


def test_cleveland_relation(orc):
    """Conservative interaction, drive at resonance: sin(phi) = A / A0 (energy balance in the
    harmonic approximation; the relation the paper's phase-imaging citation rests on)."""
    c = W.config("c2")
    for zc in (c["zc"], c["zc"] + 2e-9):
        r = orc.forward(dict(c["model"], n_cycles=3000), W.full_params(c, zc=zc))
        assert abs(np.sin(r["phi"]) - r["A"] / c["model"]["free_amplitude"]) < 1e-3


def test_kelvin_voigt_dissipates(orc):
    """With contact viscosity the drive work exceeds the cantilever's damping loss by the work of
    the viscous force -eta sqrt(R delta) d' over the period, and sin(phi) > A/A0."""
    c = W.config("c1")
    m = dict(c["model"], law="kv")
    p = np.concatenate([W.full_params(c), [5.0]])  # eta = 5 Pa s
    m, u, ud, t, h = _steady_window(orc, m, p, 512)
    Wd, Wdamp = _works(orc, m, u, ud, t, h)
    zc, a0, R, eta = p[0], p[3], p[4], p[5]
    d = zc + u
    Fv = np.where(d <= a0, -eta * np.sqrt(R * np.clip(a0 - d, 0, None)) * ud, 0.0)
    Wv = -np.sum(Fv * ud) * h
    assert Wv > 0 and Wd > Wdamp
    assert abs(Wd - Wdamp - Wv) / Wdamp < 3e-5
    A, phi = orc.lockin(u, 512, 1)
    assert np.sin(phi) > A / m["free_amplitude"]


@pytest.mark.parametrize("name", ["c1", "c2", "c4"])
def test_setpoint_separation(orc, name):
    """The stored separation gives steady amplitude setpoint * A0 (to 1e-9 A0), and 0.25 nm
    further away the amplitude is above the set-point (first crossing of an approach)."""
    c = W.config(name)
    m = c["model"]
    A, _ = orc.steady_amplitude(m, W.full_params(c))
    assert abs(A - c["setpoint"] * m["free_amplitude"]) < 1.5e-9 * m["free_amplitude"]
    A2, _ = orc.steady_amplitude(m, W.full_params(c, zc=c["zc"] + 0.25e-9))
    assert A2 > c["setpoint"] * m["free_amplitude"]


def test_force_laws_values(orc):
    """Continuity and limits of the laws."""
    dmt = dict(law="dmt")
    H, E, a0, R = 6.4e-20, 1e9, 0.3e-9, 10e-9
    p = [0.0, H, E, a0, R]
    assert orc.force(dmt, p, a0 * 1.0000001) == pytest.approx(orc.force(dmt, p, a0), rel=1e-6)
    assert orc.force(dmt, p, 2e-9) == pytest.approx(-H * R / (6 * 4e-18), rel=1e-15)
    assert orc.force(dmt, p, a0 - 1e-9) > 0
    lj = dict(law="lj")
    eps, r0, n, mm = 1.25e-19, 0.35e-9, 10.0, 5.5
    q = [0.0, eps, r0, n, mm]
    assert abs(orc.force(lj, q, r0)) < 1e-25  # force vanishes at the potential minimum
    # F = -dU/dd with U(r0) = -eps: integrate F from r0 outwards to "infinity"
    ds = np.geomspace(r0, 2000 * r0, 200001)
    F = np.array([orc.force(lj, q, x) for x in ds])
    work = np.sum(0.5 * (F[1:] + F[:-1]) * np.diff(ds))
    assert work == pytest.approx(-eps, rel=1e-4)
    assert np.isnan(orc.force(lj, q, -1e-10))
    sd = dict(law="sd")
    assert orc.force(sd, [0.0, 4.0, 0.1], -1e-9, 2.0) == pytest.approx(4e-9 - 0.2)
    assert orc.force(sd, [0.0, 4.0, 0.1], 1e-9, 2.0) == 0.0


def test_failure_status(orc):
    c = W.config("c1")
    m = c["model"]
    p = W.full_params(c, Estar=1e15)  # contact stiffness far beyond RK4's stability limit
    r = orc.forward(m, p, target=np.ones(4000))
    assert r["status"] != 0 and r["J"] == np.inf and np.isnan(r["A"])
    p = W.full_params(c, H=np.nan)
    r = orc.forward(m, p)
    assert r["status"] & 1 and np.isnan(r["phi"])
