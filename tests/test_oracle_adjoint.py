"""Pins of the oracle's discrete adjoint (reverse-mode gradient of the RK4 window misfit).

Checked against complex-step derivatives of the same discrete map (exact to rounding) and,
for smooth laws, central finite differences.
"""
import numpy as np
import pytest

import cs_model
import workloads as W


def _small(name, N, nc, lockin, law=None, **extra):
    c = W.config(name)
    m = dict(c["model"], steps_per_cycle=N, n_cycles=nc, lockin_cycles=lockin)
    if law:
        m["law"] = law
    m.update(extra)
    return c, m


def _target(orc, m, p):
    r = orc.forward(m, p, want_trace=True)
    assert r["status"] == 0
    return r["trace"]


CASES = [
    # name, law, N, cycles, lockin, parameter vector builder, target offsets
    ("dmt", "c1", None, 64, 30, 4, lambda c: W.full_params(c, H=7.1e-20, Estar=1.3e9, a0=0.27e-9)),
    ("lj", "c4", None, 128, 40, 4,
     lambda c: W.full_params(c, zc=20.3e-9, eps=1.1e-19, r0=0.37e-9, n=9.5, m=5.0)),
    ("kv", "c1", "kv", 64, 30, 4,
     lambda c: np.concatenate([W.full_params(c, Estar=0.8e9), [7.0]])),
    ("sd", "c1", "sd", 64, 30, 4, lambda c: np.array([5e-9, 4.0, 0.1e-6])),
    ("kv3", "c5", None, 128, 12, 3,
     lambda c: W.full_params(c, Estar=0.12e9, eta=12.0)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adjoint_matches_complex_step(orc, case):
    tag, name, law, N, nc, lockin, build = case
    c, m = _small(name, N, nc, lockin, law=law)
    if tag in ("sd", "lj"):
        m["ic"] = "free_steady"  # short runs: start at full amplitude so that the tip taps
    p = build(c)
    ptrue = p.copy()
    ptrue[0] *= 1.01  # target from a nearby separation so that J > 0
    U = _target(orc, m, ptrue)
    st, J, g = orc.misfit_grad(m, p, U)
    assert st == 0 and J > 0
    y0 = orc.initial_state(m)
    a = orc.base_amplitude(m)
    Jc, gc = cs_model.gradient(m, list(p), list(U), list(y0), a)
    assert abs(Jc - J) <= 1e-10 * J
    scale = np.abs(np.array(gc) * np.where(p != 0, p, 1.0))  # sensitivity per relative change
    for j in range(len(p)):
        assert abs(g[j] - gc[j]) * abs(p[j] if p[j] else 1.0) <= 1e-8 * scale.max() + 1e-300, (
            tag, j, g[j], gc[j])


def test_adjoint_matches_central_differences_lj(orc):
    """Smooth law: central differences with h = 1e-4 relative agree to 1e-5 relative (their
    O(h^2) truncation error; the complex-step test above is the tight check)."""
    c, m = _small("c4", 128, 40, 4, ic="free_steady")
    p = W.full_params(c, zc=20.3e-9, eps=1.1e-19, r0=0.37e-9, n=9.5, m=5.0)
    U = _target(orc, m, W.full_params(c, zc=20.3e-9))
    st, J, g = orc.misfit_grad(m, p, U)

    def fd(j, rel):
        hj = rel * abs(p[j])
        pp, pm = p.copy(), p.copy()
        pp[j] += hj
        pm[j] -= hj
        return (orc.forward(m, pp, U)["J"] - orc.forward(m, pm, U)["J"]) / (2 * hj)

    for j in range(1, 5):
        e4 = abs(fd(j, 1e-4) - g[j])
        assert e4 <= 1e-5 * abs(g[j]), (j, e4, g[j])


def test_gradient_vanishes_at_truth(orc):
    """Noiseless target at the truth: J = 0 and dJ/dp = 0 (minimum of a sum of squares)."""
    c, m = _small("c1", 64, 30, 4)
    p = W.full_params(c)
    U = _target(orc, m, p)
    st, J, g = orc.misfit_grad(m, p, U)
    assert J == 0.0 and np.all(g == 0.0)
