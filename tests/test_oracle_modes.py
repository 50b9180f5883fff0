"""Pins of the Euler-Bernoulli modal set-up (paper Sec. 3.2 Eq. 6-7, Appendix A)."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_first_natural_frequency_appendix_a(orc):
    """omega_1 = beta_1^2 sqrt(EI / (mu L^4)) with the Appendix A cantilever gives the printed
    first natural frequency 25468.9 Hz."""
    g = json.load(open(os.path.join(HERE, "golden", "appendix_a_cantilever.json")))
    Ival = g["width_m"] * g["height_m"] ** 3 / 12
    assert abs(Ival / (g["inertia_printed"] * 1e-22) - 1) < 1e-5
    bL = orc.eb_root(1)
    beta = bL / g["length_m"]
    f1 = beta**2 * np.sqrt(g["youngs_modulus_Pa"] * Ival / g["mass_per_length_kg_per_m"]) / (2 * np.pi)
    assert abs(f1 - g["first_natural_frequency_Hz"]) < 0.05


def test_roots_solve_frequency_equation(orc):
    for i in range(1, 9):
        x = orc.eb_root(i)
        assert abs(np.cos(x) * np.cosh(x) + 1) < 1e-9 * np.cosh(x)
        assert (i - 1) * np.pi < x < i * np.pi


def _deriv(f, x, k, h=1e-3):
    """k-th derivative by central differences of the given stencil (k <= 3)."""
    if k == 1:
        return (f(x + h) - f(x - h)) / (2 * h)
    if k == 2:
        return (f(x + h) - 2 * f(x) + f(x - h)) / h**2
    return (f(x + 2 * h) - 2 * f(x + h) + 2 * f(x - h) - f(x - 2 * h)) / (2 * h**3)


def test_shape_boundary_conditions(orc):
    """Clamped base Phi(0) = Phi'(0) = 0 and free tip Phi''(L) = Phi'''(L) = 0 (shapes are
    evaluated past x = L by the same formula for the one-sided stencil)."""
    for i in (1, 2, 3, 4):
        bL = orc.eb_root(i)
        f = lambda xi: orc.eb_shape(bL, xi)  # noqa: E731
        scale = abs(f(1.0))
        assert abs(f(0.0)) < 1e-12 * scale
        # central differences with h = 1e-3 carry an O(h^2 bL^{k+2}) truncation error
        assert abs(_deriv(f, 0.0, 1)) < 1e-5 * scale * bL**3
        assert abs(_deriv(f, 1.0, 2)) < 1e-5 * scale * bL**4
        assert abs(_deriv(f, 1.0, 3)) < 1e-5 * scale * bL**5


def test_printed_G_denominator_violates_free_end(orc):
    """With the minus sign printed in Eq. 7's denominator the free-end moment does not vanish:
    the plus sign is the reading that satisfies the boundary conditions."""
    bL = orc.eb_root(1)
    e = np.exp(-bL)
    G_printed = (2 * e * np.sin(bL) - e * e + 1) / (2 * e * np.cos(bL) - e * e + 1)

    def shape(xi, G):
        bx = bL * xi
        return (2 * np.sin(bx) - 2 * G * np.cos(bx) + (G - 1) * np.exp(bx) + (G + 1) * np.exp(-bx)) / 2

    f = lambda xi: shape(xi, G_printed)  # noqa: E731
    assert abs(_deriv(f, 1.0, 2)) > 0.05 * abs(f(1.0)) * bL**2  # ~1000x the tolerance above


def test_modal_mass_orthogonality_and_gains(orc):
    """Tip-normalised modes: int Phi^2 dx = L/4 for every mode, int Phi_i Phi_j = 0, frequency
    ratios (beta_i/beta_1)^2 round to the 3-mode workload's 6.27 and 17.55."""
    eb = orc.eb_modes(4, 501)
    np.testing.assert_allclose(eb["mass"], 0.25, rtol=1e-8)
    assert round(eb["ratio"][1], 2) == 6.27 and round(eb["ratio"][2], 2) == 17.55
    xs = np.linspace(0, 1, 2001)
    w = np.ones_like(xs)
    w[1:-1:2], w[2:-1:2] = 4, 2
    w *= (xs[1] - xs[0]) / 3
    sh = [np.array([orc.eb_shape(b, x) for x in xs]) / orc.eb_shape(b, 1.0) for b in eb["betaL"]]
    for i in range(4):
        for j in range(i + 1, 4):
            assert abs(np.sum(w * sh[i] * sh[j])) < 1e-9
    for i in range(4):
        assert abs(np.sum(w * sh[i]) / np.sum(w * sh[i] ** 2) - eb["gain"][i]) < 1e-8
    # a uniform distributed load on a point-mass-equivalent mode 1 has gain above 1
    assert 1.5 < eb["gain"][0] < 1.6 and eb["gain"][1] < 0 < eb["gain"][2]
