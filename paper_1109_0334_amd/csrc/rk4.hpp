// rk4.hpp -- the RK4 step of the non-dimensional modal system, shared by the forward and the
// adjoint kernels (the adjoint recomputes trajectory segments with exactly this code, so the
// recomputed states are bit-identical to the forward pass).
#pragma once

#include "afm_internal.hpp"

namespace afm {

// Mode 1 is carried as the tip-sample gap g = z_c + x_1 rather than as x_1: the force laws are
// steepest exactly where the gap is small, and there an FP32 gap keeps full relative precision
// (forming z_c + x_1 from two ~A0-sized numbers would lose it).  The restoring force of mode 1
// uses x_1 = g - z_c, which needs only absolute precision.
//
// Sum over modes in the order a butterfly over the lanes of a mode-parallel group produces:
// sequential up to three modes ((x0 + x1) + x2, the missing fourth lane adding an exact zero),
// pairwise for four to eight (lanes without a mode add exact zeros: five modes give
// ((x0 + x1) + (x2 + x3)) + x4).  The one-lane and the mode-parallel kernels use this same
// order, so they compute identical bits.
template <int NM, typename R>
__device__ __forceinline__ R mode_sum(const R (&x)[NM]) {
    if constexpr (NM > 4) {
        const R lo = (x[0] + x[1]) + (x[2] + x[3]);
        if constexpr (NM == 5) return lo + x[4];
        else if constexpr (NM == 6) return lo + (x[4] + x[5]);
        else if constexpr (NM == 7) return lo + ((x[4] + x[5]) + x[6]);
        else return lo + ((x[4] + x[5]) + (x[6] + x[7]));
    } else if constexpr (NM == 4) {
        return (x[0] + x[1]) + (x[2] + x[3]);
    } else {
        R d = x[0];
#pragma unroll
        for (int i = 1; i < NM; ++i) d += x[i];
        return d;
    }
}

// Slopes of the modal system at state (g, x_2.., v_1..): returns the accelerations a_i.
template <int NM, int FM, typename R, class L>
__device__ __forceinline__ void accel(const L &law, const R (&x)[NM], const R (&v)[NM],
                                      const R (&om2)[NM], const R (&cd)[NM], const R (&gn)[NM],
                                      R D, R (&a)[NM]) {
    const R d = mode_sum<NM>(x);
    R dd = R(0);
    if constexpr (L::kRate) dd = mode_sum<NM>(v);
    if constexpr (NM == 1) {
        // point mass: the drive table already carries the mode's gain.  The restoring term keeps
        // its own (g - z_c): folding om2 z_c into the drive values instead would round the small
        // drive (a = A0/Q) against a z_c-sized sum, the same error every period, which the
        // resonance then amplifies by Q.
        a[0] = Ops<R>::fma(-om2[0], x[0] - law.zc,
                           Ops<R>::fma(-cd[0], v[0], law.template add<FM>(d, dd, D)));
    } else {
        const R F = law.template add<FM>(d, dd, R(0));
        a[0] = Ops<R>::fma(-om2[0], x[0] - law.zc, Ops<R>::fma(-cd[0], v[0], Ops<R>::fma(gn[0], D, F)));
#pragma unroll
        for (int i = 1; i < NM; ++i)
            a[i] = Ops<R>::fma(-om2[i], x[i], Ops<R>::fma(-cd[i], v[i], Ops<R>::fma(gn[i], D, F)));
    }
}

// One classical RK4 step, c = (0, 1/2, 1/2, 1), b = (1/6, 1/3, 1/3, 1/6).  D0, D1, D2 are the
// drive terms at t, t + h/2, t + h.  COMP: Kahan-compensated update of the state.
template <int NM, bool COMP, int FM, typename R, class L>
__device__ __forceinline__ void rk4_step(const L &law, R (&x)[NM], R (&v)[NM], R (&cx)[NM],
                                         R (&cv)[NM], const R (&om2)[NM], const R (&cd)[NM],
                                         const R (&gn)[NM], R h, R h2, R h6, R D0, R D1, R D2) {
    R a[NM], sx[NM], sv[NM], xs[NM], vs[NM];
    accel<NM, FM>(law, x, v, om2, cd, gn, D0, a);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        sx[i] = v[i];
        sv[i] = a[i];
        xs[i] = Ops<R>::fma(h2, v[i], x[i]);
        vs[i] = Ops<R>::fma(h2, a[i], v[i]);
    }
    accel<NM, FM>(law, xs, vs, om2, cd, gn, D1, a);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        const R kx = vs[i];
        sx[i] = Ops<R>::fma(R(2), kx, sx[i]);
        sv[i] = Ops<R>::fma(R(2), a[i], sv[i]);
        xs[i] = Ops<R>::fma(h2, kx, x[i]);
        vs[i] = Ops<R>::fma(h2, a[i], v[i]);
    }
    accel<NM, FM>(law, xs, vs, om2, cd, gn, D1, a);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        const R kx = vs[i];
        sx[i] = Ops<R>::fma(R(2), kx, sx[i]);
        sv[i] = Ops<R>::fma(R(2), a[i], sv[i]);
        xs[i] = Ops<R>::fma(h, kx, x[i]);
        vs[i] = Ops<R>::fma(h, a[i], v[i]);
    }
    accel<NM, FM>(law, xs, vs, om2, cd, gn, D2, a);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        sx[i] += vs[i];
        sv[i] += a[i];
        if constexpr (COMP) {
            const R dx = Ops<R>::fma(h6, sx[i], -cx[i]);
            const R tx = x[i] + dx;
            cx[i] = (tx - x[i]) - dx;
            x[i] = tx;
            const R dv = Ops<R>::fma(h6, sv[i], -cv[i]);
            const R tv = v[i] + dv;
            cv[i] = (tv - v[i]) - dv;
            v[i] = tv;
        } else {
            x[i] = Ops<R>::fma(h6, sx[i], x[i]);
            v[i] = Ops<R>::fma(h6, sv[i], v[i]);
        }
    }
}

// Base motion from a trajectory's own parameters: the chirp of Eq. 10 (g = 0 gives Eq. 9), with
// a, f, g in parameter slots 8, 9, 10.  at(j) is the drive term -y_b'' / wd^2 in nm at half-step
// j (time j h / 2, i.e. s = j / (2 N) drive periods): phase in revolutions rho = s (r0 + gam s),
// rate w = r0 + 2 gam s in units of wd, term amp (w^2 sin(2 pi rho) - (gam / pi) cos(2 pi rho)),
// r0 = f / f_d, gam = g / f_d^2.  The phase is formed and reduced to [-1/2, 1/2] in FP64 (it
// reaches thousands of revolutions), the sine and cosine are taken in R.
template <typename R>
struct DriveP {
    double c1 = 0, c2 = 0, c3 = 0, r0 = 0;  // rho = j (c1 + j c2), w = r0 + j c3
    R amp = R(0), kg = R(0);
    DriveP() = default;
    __device__ DriveP(const double (&p)[kMaxParams], const KConst &K, int nm) {
        const double inv2n = 1.0 / (2.0 * K.N);
        const double gam = p[AFM_P_BASE_G] / (K.fref * K.fref);
        r0 = p[AFM_P_BASE_F] / K.fref;
        c1 = r0 * inv2n;
        c2 = gam * inv2n * inv2n;
        c3 = 2.0 * gam * inv2n;
        // a point mass carries its gain in the drive term (as the fixed drive table does)
        amp = (R)(p[AFM_P_BASE_A] * 1e9 * (nm == 1 ? K.gain[0] : 1.0));
        kg = (R)(gam / M_PI);
    }
    __device__ __forceinline__ R at(double j) const {
        const double rho = j * __builtin_fma(j, c2, c1);
        const double r = rho - __builtin_rint(rho);
        const R w = (R)__builtin_fma(j, c3, r0);
        R sn, cs;
        if constexpr (std::is_same<R, float>::value) sincospif(2.0f * (float)r, &sn, &cs);
        else sincospi(2.0 * r, &sn, &cs);
        return amp * Ops<R>::fma(w * w, sn, -(kg * cs));
    }
};

// Derivatives of the drive term DriveP::at(j) with respect to the base motion's a (m), f (Hz)
// and g (Hz/s), in FP64, for the adjoint: with s = j / (2 N) periods, rho = s (r0 + gam s),
// w = r0 + 2 gam s, D = amp (w^2 sin(2 pi rho) - kg cos(2 pi rho)), amp = a 1e9 G,
// r0 = f / f_d, gam = g / f_d^2, kg = gam / pi:
//   dD/da = 1e9 G (w^2 sin - kg cos),
//   dD/df = amp (2 w sin / f_d + 2 pi (w^2 cos + kg sin) s / f_d),
//   dD/dg = amp (4 w s sin / f_d^2 + 2 pi (w^2 cos + kg sin) s^2 / f_d^2 - cos / (pi f_d^2)).
struct DriveGrad {
    double inv2n = 0, fref = 0, r0 = 0, gam = 0, kg = 0, scale = 0, amp = 0;
    DriveGrad() = default;
    __device__ DriveGrad(const double (&p)[kMaxParams], const KConst &K, int nm) {
        inv2n = 1.0 / (2.0 * K.N);
        fref = K.fref;
        r0 = p[AFM_P_BASE_F] / fref;
        gam = p[AFM_P_BASE_G] / (fref * fref);
        kg = gam / M_PI;
        scale = 1e9 * (nm == 1 ? K.gain[0] : 1.0);
        amp = p[AFM_P_BASE_A] * scale;
    }
    __device__ void at(double j, double (&dD)[3]) const {
        const double s = j * inv2n;
        const double rho = s * __builtin_fma(gam, s, r0);
        double sn, cs;
        sincospi(2.0 * (rho - __builtin_rint(rho)), &sn, &cs);
        const double w = __builtin_fma(2.0 * gam, s, r0);
        const double core = __builtin_fma(w * w, cs, kg * sn);  // w^2 cos + kg sin
        dD[0] = scale * __builtin_fma(w * w, sn, -(kg * cs));
        dD[1] = amp * (2.0 * w * sn + 2.0 * M_PI * core * s) / fref;
        dD[2] = amp * (4.0 * w * s * sn + 2.0 * M_PI * core * s * s - cs / M_PI) / (fref * fref);
    }
};

// Tip deflection u = g - z_c + x_2 + ... in FP64, including the Kahan residuals (the compensated
// state is x - c).
template <int NM, bool COMP, typename R>
__device__ __forceinline__ double sample(const R (&x)[NM], const R (&cx)[NM], double zc) {
    double u = -zc;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        u += (double)x[i];
        if constexpr (COMP) u -= (double)cx[i];
    }
    return u;
}

// ------------------------------------------------------------------------------------------
// Mode-parallel form (the paper's own mapping of modes to threads, Sec. 3.2): the G lanes of a
// group (G = 2 for two modes, 4 for three or four, 8 for five to eight) hold one trajectory, lane q its mode q (a
// lane without a mode carries an exact zero).  The gap and gap rate are butterfly sums over the
// group (DPP lane swaps, so the sum costs one add per butterfly level); every lane evaluates the
// force law on the same sums and advances only its own mode.

// Butterfly sum over the G lanes of a group; every lane gets the same bits.
// DPP controls: quad_perm [1,0,3,2] swaps neighbours, quad_perm [2,3,0,1] swaps pairs,
// row_half_mirror reverses each 8-lane half-row (after the two quad levels every lane of a quad
// holds the quad's sum, so the mirror brings in the other quad's).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    float s = v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                      0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    if constexpr (G >= 4)
        s = s + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                    0, __builtin_bit_cast(int, s), 0x4E, 0xF, 0xF, false));
    if constexpr (G == 8)
        s = s + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                    0, __builtin_bit_cast(int, s), 0x141, 0xF, 0xF, false));
    return s;
}

template <int CTRL>
__device__ __forceinline__ double dpp_swap(double a) {
    const long long b = __builtin_bit_cast(long long, a);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned int)hi << 32) |
                                                  (unsigned int)lo));
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
    double s = v + dpp_swap<0xB1>(v);
    if constexpr (G >= 4) s = s + dpp_swap<0x4E>(s);
    if constexpr (G == 8) s = s + dpp_swap<0x141>(s);
    return s;
}

// One lane's mode constants: the restoring, damping and drive coefficients of its mode, the
// offset of its coordinate (z_c for mode 1, carried as the gap) and the force weight (1 for a
// real mode, 0 for a lane without one).
template <typename R>
struct ModeLane {
    R om2, cd, gn, zoff, w;
};

// The block-level contact test of a mode-parallel group (the point mass's BlockBound, mode by
// mode): over a block of four steps the acceleration of mode q stays within
// u |x_q - zoff| + v |v_q| + f fmax + c0, with u, v, f, c0 the point-mass coefficients of its
// frequency, damping and drive gain; the group sum of these bounds bounds the gap's, and since
// every stage of every mode takes the same RK4 weights, no stage gap falls below
// g - 4h max(0, 4h A* - g') (g, g' the gap and its rate).  A lane without a mode has zero
// coefficients.  ok is false, for every lane, when some mode is too fast for the bound at this
// step (denominator below 0.2): then the test always answers "near".
template <typename R>
struct ModeBound {
    R u = R(0), v = R(0), f = R(0), c0 = R(0), h4 = R(0);
    bool ok = false;
    __device__ ModeBound(const KConst &K, int nm, int q) {
        const double hh = K.h;
        ok = true;
        for (int i = 0; i < nm; ++i)
            ok = ok && 1.0 - 16.0 * hh * hh * K.om2[i] - 4.0 * hh * K.cdamp[i] >= 0.2;
        h4 = (R)(4.0 * hh * 1.02);
        if (q < nm) {
            const double o2 = K.om2[q], c = K.cdamp[q];
            const double den = 1.0 - 16.0 * hh * hh * o2 - 4.0 * hh * c;
            const double qf = den >= 0.2 ? 1.02 / den : 0.0;
            u = (R)(o2 * qf);
            v = (R)((4.0 * hh * o2 + c) * qf);
            f = (R)qf;
            c0 = den >= 0.2 ? (R)(::fabs(K.gain[q]) * K.dmax * qf) : (R)INFINITY;
        }
    }
};

// Whether no group of the wave can come within the law's dskip of contact during the next four
// steps (wave-uniform).  NaN states count as near.
template <int G, typename R, class L>
__device__ __forceinline__ bool group_far(const L &law, const ModeLane<R> &ml,
                                          const ModeBound<R> &mb, R x, R v) {
    if (!mb.ok) return false;
    const R Tq = Ops<R>::fma(mb.u, Ops<R>::abs(x - ml.zoff),
                             Ops<R>::fma(mb.v, Ops<R>::abs(v), Ops<R>::fma(mb.f, law.fmax, mb.c0)));
    const R Am = group_sum<G>(Tq);
    const R g = group_sum<G>(x), vg = group_sum<G>(v);
    const R reach = Ops<R>::fma(mb.h4, Ops<R>::max(Ops<R>::fma(mb.h4, Am, -vg), R(0)), R(1e-3));
    return __builtin_amdgcn_ballot_w64(!(g - reach > law.dskip)) == 0;
}

template <int NM, int G, int FM, typename R, class L>
__device__ __forceinline__ R accel_mp(const L &law, const ModeLane<R> &ml, R x, R v, R D) {
    const R d = group_sum<G>(x);
    R dd = R(0);
    if constexpr (L::kRate) dd = group_sum<G>(v);
    R F = law.template add<FM>(d, dd, R(0));
    if constexpr (NM < G) F *= ml.w;
    return Ops<R>::fma(-ml.om2, x - ml.zoff, Ops<R>::fma(-ml.cd, v, Ops<R>::fma(ml.gn, D, F)));
}

// The RK4 step of rk4_step for this lane's mode (same operations, same order).
template <int NM, int G, bool COMP, int FM, typename R, class L>
__device__ __forceinline__ void rk4_step_mp(const L &law, const ModeLane<R> &ml, R &x, R &v,
                                            R &cx, R &cv, R h, R h2, R h6, R D0, R D1, R D2) {
    R a = accel_mp<NM, G, FM>(law, ml, x, v, D0);
    R sx = v, sv = a;
    R xs = Ops<R>::fma(h2, v, x), vs = Ops<R>::fma(h2, a, v);
    a = accel_mp<NM, G, FM>(law, ml, xs, vs, D1);
    {
        const R kx = vs;
        sx = Ops<R>::fma(R(2), kx, sx);
        sv = Ops<R>::fma(R(2), a, sv);
        xs = Ops<R>::fma(h2, kx, x);
        vs = Ops<R>::fma(h2, a, v);
    }
    a = accel_mp<NM, G, FM>(law, ml, xs, vs, D1);
    {
        const R kx = vs;
        sx = Ops<R>::fma(R(2), kx, sx);
        sv = Ops<R>::fma(R(2), a, sv);
        xs = Ops<R>::fma(h, kx, x);
        vs = Ops<R>::fma(h, a, v);
    }
    a = accel_mp<NM, G, FM>(law, ml, xs, vs, D2);
    sx += vs;
    sv += a;
    if constexpr (COMP) {
        const R dx = Ops<R>::fma(h6, sx, -cx);
        const R tx = x + dx;
        cx = (tx - x) - dx;
        x = tx;
        const R dv = Ops<R>::fma(h6, sv, -cv);
        const R tv = v + dv;
        cv = (tv - v) - dv;
        v = tv;
    } else {
        x = Ops<R>::fma(h6, sx, x);
        v = Ops<R>::fma(h6, sv, v);
    }
}

// The tip deflection of `sample` from the group's lanes (gathered; the same sequence of FP64
// additions), identical in every lane of the group.
template <int NM, bool COMP, typename R>
__device__ __forceinline__ double sample_mp(R x, R cx, double zc, int group_base) {
    double u = -zc;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        u += (double)__shfl(x, group_base + i, 64);
        if constexpr (COMP) u -= (double)__shfl(cx, group_base + i, 64);
    }
    return u;
}

}  // namespace afm
