"""Complex-step differentiation of the window misfit (test helper, pure Python).

J(p + i h e_j) = J(p) + i h dJ/dp_j + O(h^2) for a real-analytic J, so Im(J)/h with h = 1e-30 is
the derivative to rounding, with no subtractive cancellation (Squire & Trapp 1998).  The model
below is the modal cantilever with tip force F(d, d'; p) restated with complex parameters; branch
conditions (contact or not) are decided on real parts, so the derivative is that of the piece the
trajectory is on.  The initial state and base amplitude do not depend on p and are taken as
inputs.  Used only to check the oracle's reverse-mode gradient; small sizes only.
"""
import cmath
import math


def _force(law, p, d, dd):
    if law == "dmt" or law == "kv":
        zc, H, E, a0, R = p[:5]
        if d.real > a0.real:
            F = -H * R / (6 * d * d)
        else:
            dl = a0 - d
            F = -H * R / (6 * a0 * a0) + 4.0 / 3.0 * E * cmath.sqrt(R) * dl * cmath.sqrt(dl)
            if law == "kv":
                F += -p[5] * cmath.sqrt(R * dl) * dd
        return F
    if law == "lj":
        zc, eps, r0, n, m = p[:5]
        s = r0 / d
        ls = cmath.log(s)
        return eps * (n * m / (n - m)) / d * (cmath.exp(n * ls) - cmath.exp(m * ls))
    if law == "sd":
        return (-p[1] * d - p[2] * dd) if d.real < 0 else 0j
    if law == "hooke":
        return (-p[1] * d) if d.real < 0 else 0j
    return 0j


def misfit(model, p, U, y0, a, n_cycles=None):
    """Window misfit J = sum (U - u)^2 / sum U^2 of the RK4 trajectory, complex arithmetic."""
    nm = model["n_modes"]
    law = model["law"]
    N = model["steps_per_cycle"]
    nc = model["n_cycles"] if n_cycles is None else n_cycles
    Wn = model["lockin_cycles"] * N
    w0 = 2 * math.pi * model["f0"]
    wd = 2 * math.pi * model["drive_freq"]
    M = model["k"] / w0**2
    w = [w0 * r for r in model["ratio"][:nm]]
    c = [w[i] / model["q"][i] for i in range(nm)]
    g = model["gain"][:nm]
    h = 1.0 / (model["drive_freq"] * N)
    p = [complex(x) for x in p]

    params_drive = model.get("drive", "table") == "params"

    def rhs(t, y):
        u = sum(y[:nm])
        ud = sum(y[nm:])
        F = _force(law, p, p[0] + u, ud)
        if params_drive:  # Eq. 10 with (a, f, g) = p[8], p[9], p[10]: -y_b''
            ab, fb, gb = p[8], p[9], p[10]
            phi = 2 * math.pi * (fb + gb * t) * t
            wb = 2 * math.pi * (fb + 2 * gb * t)
            drive = ab * (wb * wb * cmath.sin(phi) - 4 * math.pi * gb * cmath.cos(phi))
        else:
            drive = a * wd * wd * math.sin(wd * t)
        return [y[nm + i] for i in range(nm)] + [
            -w[i] * w[i] * y[i] - c[i] * y[nm + i] + F / M + g[i] * drive for i in range(nm)]

    y = [complex(v) for v in y0]
    num = 0j
    den = 0.0
    first = nc * N - Wn + 1
    for n in range(nc * N):
        t = n * h
        k1 = rhs(t, y)
        k2 = rhs(t + h / 2, [y[i] + h / 2 * k1[i] for i in range(2 * nm)])
        k3 = rhs(t + h / 2, [y[i] + h / 2 * k2[i] for i in range(2 * nm)])
        k4 = rhs(t + h, [y[i] + h * k3[i] for i in range(2 * nm)])
        y = [y[i] + h / 6 * (k1[i] + 2 * k2[i] + 2 * k3[i] + k4[i]) for i in range(2 * nm)]
        if n + 1 >= first:
            e = U[n + 1 - first] - sum(y[:nm])
            num += e * e
            den += U[n + 1 - first] ** 2
    return num / den


def gradient(model, p, U, y0, a, hstep=1e-30):
    """Complex-step gradient of misfit() over every entry of p; returns (J, [dJ/dp_j])."""
    out = []
    J0 = None
    for j in range(len(p)):
        q = [complex(x) for x in p]
        q[j] += 1j * hstep
        Jc = misfit(model, q, U, y0, a)
        J0 = Jc.real
        out.append(Jc.imag / hstep)
    return J0, out
