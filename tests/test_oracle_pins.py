"""Pins of the oracle's coordinate map and of the stored set-point separations.

* orc_z_to_theta maps the normalised search coordinate z in [0, 1] onto the search box (the
  PSO of Sec. 3.4 moves particles in that box): linear lo + z (hi - lo), or geometric
  lo (hi/lo)^z for log-scaled parameters.  Pinned by its values at the box ends and the middle
  (arithmetic resp. geometric mean) and, for the geometric map, by the constant ratio of
  neighbouring values.
* orc_dtheta_dz, the chain-rule factor of the L-BFGS polish, is pinned by complex-step
  derivatives of an independent restatement of the map (numpy complex powers).
* The stored separation z_c of each workload is where the steady amplitude equals the
  set-point (the amplitude feedback of Sec. 1).  orc_steady_amplitude stops on its own
  one-period amplitude change; here an independent long run -- a plain forward solve of 4000
  periods with the 20-period lock-in -- must give A = s A0 at the stored z_c.
"""
import numpy as np
import pytest

import workloads as W

BOXES = [(1e-20, 1e-19, 0), (0.05e9, 50e9, 1), (0.1e-9, 0.5e-9, 0), (1.0, 100.0, 1),
         (-5e-9, 5e-9, 0), (0.0, 25.0, 0), (0.01e9, 1.0e9, 1)]


@pytest.mark.parametrize("lo,hi,lg", BOXES)
def test_z_to_theta_ends_and_middle(orc, lo, hi, lg):
    t0, t1, th = (orc.z_to_theta(z, lo, hi, lg) for z in (0.0, 1.0, 0.5))
    # the geometric map forms exp(log lo + ...): exact up to a few ulps of the exponent
    assert t0 == pytest.approx(lo, rel=1e-14 if lg else 0.0, abs=0.0 if lo or lg else 1e-300)
    assert t1 == pytest.approx(hi, rel=1e-14 if lg else 4e-16)
    mid = np.sqrt(lo * hi) if lg else 0.5 * (lo + hi)
    assert th == pytest.approx(mid, rel=4e-15, abs=1e-30 * abs(hi))
    zs = np.linspace(0.0, 1.0, 41)
    t = np.array([orc.z_to_theta(z, lo, hi, lg) for z in zs])
    assert np.all(np.diff(t) > 0)
    if lg:  # equal steps in z multiply theta by the same factor (hi/lo)^(1/40)
        np.testing.assert_allclose(t[1:] / t[:-1], (hi / lo) ** (1 / 40), rtol=1e-13)
    else:   # and add the same amount on the linear map
        np.testing.assert_allclose(np.diff(t), (hi - lo) / 40, rtol=1e-9)


@pytest.mark.parametrize("lo,hi,lg", BOXES)
def test_dtheta_dz_complex_step(orc, lo, hi, lg):
    def theta(z):  # restated: z -> lo (hi/lo)^z, or lo + z (hi - lo)
        return lo * (hi / lo) ** z if lg else lo + z * (hi - lo)

    h = 1e-30
    for z in (0.0, 0.13, 0.5, 0.77, 1.0):
        ref = (theta(complex(z, h))).imag / h
        assert orc.dtheta_dz(z, lo, hi, lg) == pytest.approx(ref, rel=1e-13)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["c1", "c2", "c4", "c5"])
def test_stored_separation_gives_the_setpoint(orc, name):
    """c3 shares c2's cantilever, truth and set-point (its stored z_c is c2's)."""
    c = W.config(name)
    m = dict(c["model"], n_cycles=4000)
    p = W.full_params(c)
    r = orc.forward(m, p)
    A0 = m["free_amplitude"]
    print(f"{name}: z_c {p[0]:.6e} m, A after 4000 periods {r['A']:.12e} m, "
          f"(A - s A0) / A0 = {(r['A'] - c['setpoint'] * A0) / A0:.2e}")
    assert r["status"] == 0
    assert abs(r["A"] - c["setpoint"] * A0) <= 1e-7 * A0
