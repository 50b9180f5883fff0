"""Pins of the oracle's deflection at points along the beam (the paper's n_dp deflection
points, Sec. 3.2; u(x) = sum_i q_i Phi_i(x) / Phi_i(L) from App. B's modal expansion, Eq. 13).

* weights of one at every mode are the tip itself: amplitude, phase and trace equal the tip
  outputs bit for bit;
* the clamped base does not move: weights Phi_i(0) = 0 give an identically zero trace;
* the trace is linear in the weights;
* the free linear beam's steady state at x = L/4, L/2, 3L/4 is the closed form
  |a sum_i w_i H_i| with H_i = gamma_i wd^2 / (w_i^2 - wd^2 + i w_i wd / Q_i), phase -arg(.),
  up to the RK4 error (the mode shapes from the oracle's Eq. 6 with the corrected G, pinned
  elsewhere against App. A)."""
import numpy as np
import pytest


def _model(n_modes=3, law="none", N=512, n_cycles=30, lockin=20, ic="free_steady"):
    return dict(n_modes=n_modes, law=law, k=40.0, f0=300e3, drive_freq=300e3,
                q=[400.0] * n_modes, ratio=[1.0, 6.27, 17.55][:n_modes],
                gain=[1.565984, -0.867872, 0.508851][:n_modes], free_amplitude=20e-9,
                steps_per_cycle=N, n_cycles=n_cycles, lockin_cycles=lockin, ic=ic,
                div_limit=100.0)


def _weights(orc, xs, n_modes=3):
    eb = orc.eb_modes(n_modes, 501)
    return np.array([[orc.lib().orc_eb_shape(b, x) / orc.lib().orc_eb_shape(b, 1.0)
                      for b in eb["betaL"]] for x in xs])


def test_unit_weights_are_the_tip(orc):
    m = _model(law="dmt", ic="free_steady")
    p = [14.5e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9]
    r = orc.forward(m, p, want_trace=True)
    q = orc.forward_points(m, p, np.ones((2, 3)), want_trace=True)
    assert q["status"] == r["status"] == 0
    for k in range(2):
        assert q["A"][k] == r["A"] and q["phi"][k] == r["phi"]
        assert np.array_equal(q["trace"][k], r["trace"])


def test_clamped_base_is_still(orc):
    w = _weights(orc, [0.0])
    assert np.max(np.abs(w)) < 1e-12
    q = orc.forward_points(_model(), [0.0], np.zeros((1, 3)), want_trace=True)
    assert np.all(q["trace"] == 0.0) and q["A"][0] == 0.0


def test_linear_in_weights(orc):
    m = _model(law="dmt", n_cycles=40, lockin=5)
    p = [14.5e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9]
    w1, w2 = np.array([[0.3, -0.2, 0.9]]), np.array([[0.5, 0.7, -0.1]])
    t1 = orc.forward_points(m, p, w1, want_trace=True)["trace"][0]
    t2 = orc.forward_points(m, p, w2, want_trace=True)["trace"][0]
    t12 = orc.forward_points(m, p, w1 + w2, want_trace=True)["trace"][0]
    assert np.max(np.abs(t12 - (t1 + t2))) < 1e-14 * np.max(np.abs(t12))


@pytest.mark.parametrize("x", [0.25, 0.5, 0.75])
def test_free_beam_points_closed_form(orc, x):
    m = _model()
    w = _weights(orc, [x])[0]
    a = orc.base_amplitude(m)
    wd = 2 * np.pi * m["drive_freq"]
    H = 0j
    for i in range(3):
        wi = 2 * np.pi * m["f0"] * m["ratio"][i]
        H += w[i] * m["gain"][i] * wd**2 / (wi**2 - wd**2 + 1j * wi * wd / m["q"][i])
    A_c, phi_c = a * abs(H), -np.angle(H)
    q = orc.forward_points(m, [0.0], w[None, :])
    assert q["status"] == 0
    assert abs(q["A"][0] / A_c - 1) < 2e-7
    assert abs(q["phi"][0] - phi_c) < 2e-6
