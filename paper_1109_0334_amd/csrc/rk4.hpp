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
// Slopes of the modal system at state (g, x_2.., v_1..): returns the accelerations a_i.
template <int NM, int FM, typename R, class L>
__device__ __forceinline__ void accel(const L &law, const R (&x)[NM], const R (&v)[NM],
                                      const R (&om2)[NM], const R (&cd)[NM], const R (&gn)[NM],
                                      R D, R (&a)[NM]) {
    R d = x[0];
#pragma unroll
    for (int i = 1; i < NM; ++i) d += x[i];
    R dd = R(0);
    if constexpr (L::kRate) {
        dd = v[0];
#pragma unroll
        for (int i = 1; i < NM; ++i) dd += v[i];
    }
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

}  // namespace afm
