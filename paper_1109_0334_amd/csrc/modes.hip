// modes.hip -- host-side modal set-up of a uniform clamped-free Euler-Bernoulli cantilever
// (Sec. 3.2 "Computational issues", Eq. 6-7; App. B): eigenvalues by Newton's method, mode
// shapes in the overflow-free exponential form, normalisation integrals by Simpson's rule.
// Produces the frequency ratios and base-drive gains of tip-normalised modes that afm_problem
// takes, and the first natural frequency from the beam's properties.  Host code only.
#include <cmath>
#include <vector>

#include "afm_internal.hpp"

namespace afm {

namespace {

// i-th root (i = 1, 2, ...) of cos(z) cosh(z) + 1 = 0, found as a root of the bounded form
// cos(z) + 1/cosh(z) = 0 (same roots, no overflow) by Newton's method from (2i - 1) pi / 2,
// which for i >= 2 lies within 0.06 of the root; the first root (1.8751) is started at 1.9.
double clamped_free_root(int i) {
    double z = i == 1 ? 1.9 : (2.0 * i - 1.0) * M_PI / 2.0;
    for (int it = 0; it < 100; ++it) {
        const double ch = std::cosh(z);
        const double f = std::cos(z) + 1.0 / ch;
        const double df = -std::sin(z) - std::tanh(z) / ch;
        const double dz = f / df;
        z -= dz;
        if (std::fabs(dz) <= 1e-15 * z) break;
    }
    return z;
}

// Eq. 6 at s = x / L in [0, 1] for b = beta L, with Eq. 7's G whose denominator reads
// 2 e^{-b} cos(b) + e^{-2b} + 1 (the printed minus sign on e^{-2b} breaks the free-end
// conditions).  The growing term (G - 1) e^{b s} is formed as
// 2 (sin b - cos b - e^{-b}) e^{b (s - 1)} / den, which never overflows and does not lose
// G - 1 to cancellation.
double mode_shape(double b, double s) {
    const double e1 = std::exp(-b), e2 = e1 * e1;
    const double den = 2.0 * e1 * std::cos(b) + e2 + 1.0;
    const double G = (2.0 * e1 * std::sin(b) - e2 + 1.0) / den;
    const double grow = 2.0 * (std::sin(b) - std::cos(b) - e1) * std::exp(b * (s - 1.0)) / den;
    return 0.5 * (2.0 * std::sin(b * s) - 2.0 * G * std::cos(b * s) + grow +
                  (G + 1.0) * std::exp(-b * s));
}

}  // namespace

}  // namespace afm

extern "C" {

afm_status afm_beam_modes(int32_t n_modes, int32_t n_points, double E, double I, double mu,
                          double L, double *ratio, double *gain, double *f1) {
    using namespace afm;
    if (n_modes < 1 || n_modes > AFM_MAX_MODES)
        return fail(AFM_ERR_INVALID, "afm_beam_modes: n_modes must be in [1, 8]");
    if (n_points < 3 || n_points % 2 == 0)
        return fail(AFM_ERR_INVALID, "afm_beam_modes: n_points must be odd and >= 3");
    if (!ratio || !gain) return fail(AFM_ERR_INVALID, "afm_beam_modes: ratio and gain are required");
    std::vector<double> b(n_modes);
    for (int i = 0; i < n_modes; ++i) b[i] = clamped_free_root(i + 1);
    const double ds = 1.0 / (n_points - 1);
    for (int i = 0; i < n_modes; ++i) {
        // Simpson's rule over s in [0, 1] for the integrals of phi and phi^2, phi = Phi / Phi(1)
        const double tip = mode_shape(b[i], 1.0);
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < n_points; ++k) {
            const double w = (k == 0 || k == n_points - 1) ? 1.0 : (k % 2 ? 4.0 : 2.0);
            const double ph = mode_shape(b[i], k * ds) / tip;
            s1 += w * ph;
            s2 += w * ph * ph;
        }
        // the common factor ds / 3 (and L) cancels in the ratio
        gain[i] = s1 / s2;
        ratio[i] = (b[i] / b[0]) * (b[i] / b[0]);
    }
    if (f1) {
        if (E > 0 && I > 0 && mu > 0 && L > 0)
            *f1 = b[0] * b[0] * std::sqrt(E * I / (mu * L * L * L * L)) / (2.0 * M_PI);
        else
            *f1 = NAN;
    }
    return AFM_OK;
}

afm_status afm_beam_shapes(int32_t n_modes, int32_t n_x, const double *x, double *w) {
    using namespace afm;
    if (n_modes < 1 || n_modes > AFM_MAX_MODES)
        return fail(AFM_ERR_INVALID, "afm_beam_shapes: n_modes must be in [1, 8]");
    if (n_x < 0 || (n_x > 0 && (!x || !w)))
        return fail(AFM_ERR_INVALID, "afm_beam_shapes: x and w are required");
    for (int k = 0; k < n_x; ++k)
        if (!(x[k] >= 0.0 && x[k] <= 1.0))
            return fail(AFM_ERR_INVALID, "afm_beam_shapes: points must lie in [0, 1]");
    for (int i = 0; i < n_modes; ++i) {
        const double b = clamped_free_root(i + 1);
        const double tip = mode_shape(b, 1.0);
        for (int k = 0; k < n_x; ++k) w[k * n_modes + i] = mode_shape(b, x[k]) / tip;
    }
    return AFM_OK;
}

}  // extern "C"
