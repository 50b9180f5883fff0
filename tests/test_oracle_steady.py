"""Pins of the oracle's adaptive steady-state exit (the uneven-pixel workload's period counts
"until the steady-state tolerance is met"; the cap is the period count): the transient ends
after the first period whose stroboscopic point P = (u, u'/wd) at the period's end moved by less
than rtol |P| from the previous period's end (the initial state before the first period).

* rtol = 0 never exits early: identical to the plain forward solve;
* a huge rtol exits after the first period: identical to a plain solve of 1 + lockin periods;
* brute force: from a dump of the whole trajectory with its rate, the period-end points give
  the first period meeting the test; the oracle integrates exactly that many transient periods,
  and its window is the following lockin periods of the dump;
* a trajectory that diverges reports its status and NaN."""
import numpy as np
import pytest

import workloads as W


def _amp(u, N):
    k = np.arange(1, len(u) + 1) % N
    X = 2.0 / len(u) * np.sum(u * np.cos(2 * np.pi * k / N))
    Y = 2.0 / len(u) * np.sum(u * np.sin(2 * np.pi * k / N))
    return np.hypot(X, Y), np.arctan2(-X, Y)


def _case(n_cycles=1200, N=128, lockin=5):
    c = W.config("c2")
    m = dict(c["model"], n_cycles=n_cycles, steps_per_cycle=N, lockin_cycles=lockin)
    return m, W.full_params(c)


def test_zero_tolerance_is_the_plain_solve(orc):
    m, p = _case(n_cycles=120)
    U = np.ones(m["lockin_cycles"] * m["steps_per_cycle"]) * 1e-8
    a = orc.forward(m, p, U, want_trace=True)
    b = orc.forward_steady(m, p, 0.0, U, want_trace=True)
    assert b["periods"] == 120 and a["status"] == b["status"] == 0
    assert (a["A"], a["phi"], a["J"]) == (b["A"], b["phi"], b["J"])
    assert np.array_equal(a["trace"], b["trace"])


def test_huge_tolerance_stops_after_one_period(orc):
    m, p = _case(n_cycles=120)
    b = orc.forward_steady(m, p, 1e9, want_trace=True)
    a = orc.forward(dict(m, n_cycles=1 + m["lockin_cycles"]), p, want_trace=True)
    assert b["periods"] == 1 + m["lockin_cycles"]
    assert (a["A"], a["phi"]) == (b["A"], b["phi"])
    assert np.array_equal(a["trace"], b["trace"])


@pytest.mark.parametrize("rtol", [1e-3, 1e-4, 1e-5, 1e-6])
def test_exit_period_by_brute_force(orc, rtol):
    m, p = _case()
    N, L, nc = m["steps_per_cycle"], m["lockin_cycles"], m["n_cycles"]
    st, u, ud, _ = orc.trajectory(m, p, n_out=nc * N, want_rate=True)  # after steps 1 .. nc N
    assert st == 0
    wd = 2 * np.pi * m["drive_freq"]
    y0 = orc.initial_state(m)
    Pu = np.r_[y0[:1].sum(), u[N - 1::N]]       # period ends 0 .. nc (0: the initial state)
    Pv = np.r_[y0[1:].sum(), ud[N - 1::N]] / wd
    T = nc - L
    for c in range(0, nc - L):
        crit = np.hypot(Pu[c + 1] - Pu[c], Pv[c + 1] - Pv[c]) / (rtol * np.hypot(Pu[c + 1], Pv[c + 1]))
        assert abs(crit - 1) > 1e-6, "borderline decision; choose another tolerance"
        if crit < 1:
            T = c + 1
            break
    r = orc.forward_steady(m, p, rtol, want_trace=True)
    assert r["periods"] == T + L
    np.testing.assert_allclose(r["trace"], u[T * N:(T + L) * N], rtol=0, atol=1e-24)
    A, phi = _amp(u[T * N:(T + L) * N], N)
    assert abs(r["A"] / A - 1) < 1e-12 and abs(r["phi"] - phi) < 1e-12
    print(f"rtol {rtol:g}: transient {T} of {nc - L} periods")


def test_divergence_reports_nan(orc):
    m, p = _case(n_cycles=40)
    q = p.copy()
    q[2] = 1e18  # an absurd stiffness: the explicit scheme blows up in contact
    r = orc.forward_steady(m, q, 1e-6, want_trace=True)
    if r["status"] == 0:
        pytest.skip("this stiffness did not destabilise the scheme")
    assert np.isnan(r["A"]) and np.isinf(r["J"]) and np.all(np.isnan(r["trace"]))
