// grad.hip -- discrete adjoint of the RK4 trajectory and window misfit (afm_grad_batch).
//
// The paper inverts with a gradient-free swarm (Sec. 3.4); its misfit J (Eq. 5) is nonetheless a
// smooth function of the force parameters along most of the search box, so its exact gradient is
// used here to polish swarm optima.  The gradient is that of the discrete map the forward kernel
// computes: reverse-mode differentiation of the classical RK4 steps (stages reversed in the
// order 4, 3, 2, 1) and of the window misfit.
//
// One lane owns one trajectory.  Forward pass: integrate as the forward kernel does, writing the
// full FP32 state (including the Kahan residuals) to an HBM checkpoint every `kc` steps.
// Reverse sweep, segment by segment from the end: reload the checkpoint, recompute the
// segment's states with the forward code (bit-identical) into a segment buffer, then walk the
// segment backwards applying the transposed stage Jacobians.  The adjoint state is FP32; the
// sensitivities to the law's constants are summed over a step's four stages in FP32 and
// accumulated across steps in FP64 (so the result is independent of the checkpoint stride), and
// are mapped to SI parameter derivatives by the chain rule at the end.
// Buffers are structure-of-arrays over lanes ([slot][variable][n]) so every access coalesces.
#include <cmath>

#include "rk4.hpp"

namespace afm {

namespace {

// dJ contributions of one stage: kb = adjoint of the stage slope k = f(Y).  Adds
// (df/dy)^T kb to Yb, and (dF/dc)^T S, (dF/dd)^T S to the constant and z_c sensitivities.
template <int NM, class L, typename R>
__device__ __forceinline__ void stage_vjp(const R (&kbx)[NM], const R (&kbv)[NM], R Fd, R Fdd,
                                          const R (&dc)[L::NC], const R (&om2)[NM],
                                          const R (&cd)[NM], R (&Ybx)[NM], R (&Ybv)[NM],
                                          R (&gsf)[L::NC], R &gzf) {
    const R S = mode_sum<NM>(kbv);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        Ybx[i] = Ops<R>::fma(-om2[i], kbv[i], Fd * S);
        Ybv[i] = Ops<R>::fma(-cd[i], kbv[i], Ops<R>::fma(Fdd, S, kbx[i]));
    }
#pragma unroll
    for (int k = 0; k < L::NC; ++k) gsf[k] = Ops<R>::fma(S, dc[k], gsf[k]);
    gzf = Ops<R>::fma(S, Fd, gzf);
}

// Slopes at a stage state (x = gap for mode 1), with the force partials for the adjoint.
template <int NM, class L, typename R>
__device__ __forceinline__ void stage_eval(const L &law, const R (&x)[NM], const R (&v)[NM],
                                           const R (&om2)[NM], const R (&cd)[NM],
                                           const R (&gn)[NM], R D, R (&a)[NM], R &Fd, R &Fdd,
                                           R (&dc)[L::NC]) {
    const R d = mode_sum<NM>(x);
    const R dd = mode_sum<NM>(v);
    const R F = law.grad(d, dd, Fd, Fdd, dc);
    if constexpr (NM == 1) {
        a[0] = Ops<R>::fma(-om2[0], x[0] - law.zc, Ops<R>::fma(-cd[0], v[0], F + D));
    } else {
        a[0] = Ops<R>::fma(-om2[0], x[0] - law.zc, Ops<R>::fma(-cd[0], v[0], Ops<R>::fma(gn[0], D, F)));
#pragma unroll
        for (int i = 1; i < NM; ++i)
            a[i] = Ops<R>::fma(-om2[i], x[i], Ops<R>::fma(-cd[i], v[i], Ops<R>::fma(gn[i], D, F)));
    }
}

// Adjoint of a stage's drive term D from the adjoint of its velocity slopes: D enters slope i
// with the mode's gain (a point mass carries its gain in D itself).
template <int NM, typename R>
__device__ __forceinline__ R drive_adjoint(const R (&kbv)[NM], const R (&gn)[NM]) {
    if constexpr (NM == 1) {
        return kbv[0];
    } else {
        R d = R(0);
#pragma unroll
        for (int i = 0; i < NM; ++i) d = Ops<R>::fma(gn[i], kbv[i], d);
        return d;
    }
}

// Reverse one RK4 step y_n -> y_{n+1}: on entry (xb, vb) = dJ/dy_{n+1}, on exit dJ/dy_n.  DP:
// also accumulates the adjoints of the step's drive terms D0, D1 (two stages), D2 into Db.
template <int NM, class L, bool DP = false, typename R>
__device__ __forceinline__ void reverse_step(const L &law, const R (&x)[NM], const R (&v)[NM],
                                             R (&xb)[NM], R (&vb)[NM], const R (&om2)[NM],
                                             const R (&cd)[NM], const R (&gn)[NM], R h, R h2,
                                             R h3, R h6, R D0, R D1, R D2, R (&gsf)[L::NC],
                                             R &gzf, R (&Db)[3]) {
    // recompute the four stage states and the force partials there
    R a1[NM], a2[NM], a3[NM], a4[NM], Y[NM], V2[NM], V3[NM], V4[NM];
    R Fd1, Fdd1, Fd2, Fdd2, Fd3, Fdd3, Fd4, Fdd4;
    R dc1[L::NC], dc2[L::NC], dc3[L::NC], dc4[L::NC];
    stage_eval<NM>(law, x, v, om2, cd, gn, D0, a1, Fd1, Fdd1, dc1);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        Y[i] = Ops<R>::fma(h2, v[i], x[i]);
        V2[i] = Ops<R>::fma(h2, a1[i], v[i]);
    }
    stage_eval<NM>(law, Y, V2, om2, cd, gn, D1, a2, Fd2, Fdd2, dc2);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        Y[i] = Ops<R>::fma(h2, V2[i], x[i]);
        V3[i] = Ops<R>::fma(h2, a2[i], v[i]);
    }
    stage_eval<NM>(law, Y, V3, om2, cd, gn, D1, a3, Fd3, Fdd3, dc3);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        Y[i] = Ops<R>::fma(h, V3[i], x[i]);
        V4[i] = Ops<R>::fma(h, a3[i], v[i]);
    }
    stage_eval<NM>(law, Y, V4, om2, cd, gn, D2, a4, Fd4, Fdd4, dc4);
    // stage adjoints: kb_i = h (b_i yb + a_{i+1,i} Yb_{i+1})
    R kbx[NM], kbv[NM], Ybx[NM], Ybv[NM], sx[NM], sv[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        kbx[i] = h6 * xb[i];
        kbv[i] = h6 * vb[i];
    }
    if constexpr (DP) Db[2] += drive_adjoint<NM>(kbv, gn);
    stage_vjp<NM, L>(kbx, kbv, Fd4, Fdd4, dc4, om2, cd, Ybx, Ybv, gsf, gzf);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        sx[i] = Ybx[i];
        sv[i] = Ybv[i];
        kbx[i] = Ops<R>::fma(h3, xb[i], h * Ybx[i]);
        kbv[i] = Ops<R>::fma(h3, vb[i], h * Ybv[i]);
    }
    if constexpr (DP) Db[1] += drive_adjoint<NM>(kbv, gn);
    stage_vjp<NM, L>(kbx, kbv, Fd3, Fdd3, dc3, om2, cd, Ybx, Ybv, gsf, gzf);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        sx[i] += Ybx[i];
        sv[i] += Ybv[i];
        kbx[i] = Ops<R>::fma(h3, xb[i], h2 * Ybx[i]);
        kbv[i] = Ops<R>::fma(h3, vb[i], h2 * Ybv[i]);
    }
    if constexpr (DP) Db[1] += drive_adjoint<NM>(kbv, gn);
    stage_vjp<NM, L>(kbx, kbv, Fd2, Fdd2, dc2, om2, cd, Ybx, Ybv, gsf, gzf);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        sx[i] += Ybx[i];
        sv[i] += Ybv[i];
        kbx[i] = Ops<R>::fma(h6, xb[i], h2 * Ybx[i]);
        kbv[i] = Ops<R>::fma(h6, vb[i], h2 * Ybv[i]);
    }
    if constexpr (DP) Db[0] += drive_adjoint<NM>(kbv, gn);
    stage_vjp<NM, L>(kbx, kbv, Fd1, Fdd1, dc1, om2, cd, Ybx, Ybv, gsf, gzf);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        xb[i] += sx[i] + Ybx[i];
        vb[i] += sv[i] + Ybv[i];
    }
}

// DP: the parameter-driven base motion (drive terms evaluated per lane, as the forward kernel
// does, and the derivatives of the drive with respect to a, f, g accumulated in FP64).
template <int LAW, int NM, bool MIXED, bool DP = false>
__global__ void __launch_bounds__(64) k_grad(const GradArgs A, const KConst K) {
    using R = typename std::conditional<MIXED, float, double>::type;
    using L = Law<LAW, R>;
    constexpr bool COMP = MIXED;
    constexpr int NS = 4 * NM;      // checkpointed scalars: x, v, cx, cv
    constexpr int NB = 2 * NM + 1;  // segment-buffer scalars: x, v, dJ/du of the next state
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    const L law(p, K);
    const double zc = p[0] * 1e9;
    const int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    const int N = K.N;
    const int64_t W = (int64_t)K.lockin * N;
    const int64_t row = A.target_id ? (int64_t)A.target_id[grp] : 0;
    const int kc = A.kc;
    const int64_t n_lanes = A.n;
    auto fail = [&](int32_t st) {
        A.J[i] = INFINITY;
        for (int j = 0; j < K.n_free; ++j) A.dJ[(int64_t)j * A.ld + i] = NAN;
        A.status[i] = st;
    };
    if (nc < K.lockin || nc > K.n_cycles || row < 0 || row >= A.n_targets) {
        fail(AFM_ST_BAD_INPUT);
        return;
    }
    const double *__restrict__ Urow = A.targets + row * W;
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;
    DriveP<R> dv;
    DriveGrad dgr;
    if constexpr (DP) {
        dv = DriveP<R>(p, K, NM);
        dgr = DriveGrad(p, K, NM);
    }
    // drive terms of global step n at t_n, t_n + h/2, t_n + h: the table's or this lane's own.
    // DP: `edge` carries the term shared with the neighbouring step (t_n + h of step n is t_n of
    // step n + 1), so a sweep up (down) evaluates two new terms per step, the same values.
    // Table: pf holds step n's entries, loaded one step ahead (a lone wave per SIMD has nothing
    // else to hide a load's latency behind); the call loads those of table step sn into pf.
    R pf[3] = {R(0), R(0), R(0)};
    auto tab3 = [&](int s) {
        pf[0] = Dt[2 * s];
        pf[1] = Dt[2 * s + 1];
        pf[2] = Dt[2 * s + 2];
    };
    auto drive3 = [&](int64_t n, int sn, R &d0, R &d1, R &d2, R &edge, bool up) {
        if constexpr (DP) {
            const double j = 2.0 * (double)n;
            d1 = dv.at(j + 1.0);
            if (up) {
                d0 = edge;
                d2 = dv.at(j + 2.0);
                edge = d2;
            } else {
                d2 = edge;
                d0 = dv.at(j);
                edge = d0;
            }
        } else {
            d0 = pf[0];
            d1 = pf[1];
            d2 = pf[2];
            tab3(sn);
        }
    };

    R x[NM], v[NM], cx[NM], cv[NM], om2[NM], cd[NM], gn[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        x[m] = (R)(m == 0 ? zc + K.y0[0] : K.y0[m]);
        v[m] = (R)K.y0[NM + m];
        cx[m] = R(0);
        cv[m] = R(0);
        om2[m] = (R)K.om2[m];
        cd[m] = (R)K.cdamp[m];
        gn[m] = (R)K.gain[m];
    }
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h3 = (R)(K.h / 3.0), h6 = (R)(K.h / 6.0);
    float *__restrict__ ck = A.ckpt;
    float *__restrict__ sg = A.seg;
    auto put = [&](float *base, int64_t slot, int var, int nvar, R val) {
        base[(slot * nvar + var) * n_lanes + i] = (float)val;
    };

    // ---- forward pass with checkpoints
    const int64_t Ntot = (int64_t)nc * N;
    const int64_t first_w = Ntot - W + 1;  // window = states first_w .. Ntot
    double Jn = 0.0, Jd = 0.0;
    int32_t st = 0;
    int64_t n = 0;
    int cdn = 0;  // steps to the next checkpoint
    R edge = R(0);
    if constexpr (DP) edge = dv.at(0.0);
    else tab3(0);
    for (int c = 0; c < nc && !st; ++c) {
        for (int s = 0; s < N; ++s, ++n) {
            if (cdn == 0) {
                const int64_t slot = n / kc;
#pragma unroll
                for (int m = 0; m < NM; ++m) {
                    if constexpr (MIXED) {
                        put(ck, slot, m, NS, x[m]);
                        put(ck, slot, NM + m, NS, v[m]);
                        put(ck, slot, 2 * NM + m, NS, cx[m]);
                        put(ck, slot, 3 * NM + m, NS, cv[m]);
                    }
                }
                if constexpr (!MIXED) {
#pragma unroll
                    for (int m = 0; m < NM; ++m) {  // FP64 state stored as two floats' worth
                        double *ckd = reinterpret_cast<double *>(ck);
                        ckd[(slot * NS + m) * n_lanes + i] = x[m];
                        ckd[(slot * NS + NM + m) * n_lanes + i] = v[m];
                    }
                }
                cdn = kc;
            }
            --cdn;
            R d0, d1, d2;
            drive3(n, s + 1 == N ? 0 : s + 1, d0, d1, d2, edge, true);
            rk4_step<NM, COMP, kFmFree>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, d0, d1, d2);
            if (n + 1 >= first_w) {
                const double u = sample<NM, COMP>(x, cx, zc);
                const double U = Urow[n + 1 - first_w] * 1e9;
                const double e = U - u;
                Jn = __builtin_fma(e, e, Jn);
                Jd = __builtin_fma(U, U, Jd);
            }
        }
        bool fin = true;
#pragma unroll
        for (int m = 0; m < NM; ++m) fin = fin && isfinite(x[m]) && isfinite(v[m]);
        if (!fin) st = AFM_ST_NONFINITE;
        else if (fabs(sample<NM, COMP>(x, cx, zc)) > K.div_nm) st = AFM_ST_DIVERGED;
    }
    const double J = Jn / Jd;
    if (st || !isfinite(J)) {
        fail(st ? st : AFM_ST_NONFINITE);
        return;
    }
    const double coef = -2.0 / Jd;  // dJ/du_n = coef (U_n - u_n)

    // ---- reverse sweep
    R xb[NM], vb[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        xb[m] = R(0);
        vb[m] = R(0);
    }
    double gs[L::NC];
#pragma unroll
    for (int k = 0; k < L::NC; ++k) gs[k] = 0.0;
    double gz = 0.0;
    double gD[3] = {0.0, 0.0, 0.0};  // DP: dJ/d(a, f, g)
    const int64_t nseg = (Ntot + kc - 1) / kc;
    for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
        const int64_t n0 = sgi * kc;
        const int64_t n1 = n0 + kc < Ntot ? n0 + kc : Ntot;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            if constexpr (MIXED) {
                x[m] = ck[(sgi * NS + m) * n_lanes + i];
                v[m] = ck[(sgi * NS + NM + m) * n_lanes + i];
                cx[m] = ck[(sgi * NS + 2 * NM + m) * n_lanes + i];
                cv[m] = ck[(sgi * NS + 3 * NM + m) * n_lanes + i];
            } else {
                const double *ckd = reinterpret_cast<const double *>(ck);
                x[m] = ckd[(sgi * NS + m) * n_lanes + i];
                v[m] = ckd[(sgi * NS + NM + m) * n_lanes + i];
            }
        }
        // recompute the segment, keeping y_n and dJ/du_{n+1}
        int s = (int)(n0 % N);
        if constexpr (DP) edge = dv.at(2.0 * (double)n0);
        else tab3(s);
        for (int64_t q = n0; q < n1; ++q) {
            const int64_t k = q - n0;
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                if constexpr (MIXED) {
                    put(sg, k, m, NB, x[m]);
                    put(sg, k, NM + m, NB, v[m]);
                } else {
                    double *sgd = reinterpret_cast<double *>(sg);
                    sgd[(k * NB + m) * n_lanes + i] = x[m];
                    sgd[(k * NB + NM + m) * n_lanes + i] = v[m];
                }
            }
            R d0, d1, d2;
            drive3(q, s + 1 == N ? 0 : s + 1, d0, d1, d2, edge, true);
            rk4_step<NM, COMP, kFmFree>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, d0, d1, d2);
            if (q + 1 >= first_w) {
                const double u = sample<NM, COMP>(x, cx, zc);
                const double ub = coef * (Urow[q + 1 - first_w] * 1e9 - u);
                if constexpr (MIXED) put(sg, k, 2 * NM, NB, (R)ub);
                else reinterpret_cast<double *>(sg)[(k * NB + 2 * NM) * n_lanes + i] = ub;
            }
            s = s + 1 == N ? 0 : s + 1;
        }
        // walk the segment backwards; a step's four stage contributions are summed in R and
        // flushed to FP64 every step, so the result does not depend on the stride
        s = (int)((n1 - 1) % N);
        double eedge[3] = {0.0, 0.0, 0.0};
        if constexpr (DP) {
            edge = dv.at(2.0 * (double)n1);
            dgr.at(2.0 * (double)n1, eedge);
        } else {
            tab3(s);
        }
        // y_q and dJ/du_{q+1} of step q from the segment buffer, loaded one step ahead
        R pyx[NM], pyv[NM], pub = R(0);
        auto seg_load = [&](int64_t q) {
            const int64_t k = q - n0;
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                if constexpr (MIXED) {
                    pyx[m] = sg[(k * NB + m) * n_lanes + i];
                    pyv[m] = sg[(k * NB + NM + m) * n_lanes + i];
                } else {
                    const double *sgd = reinterpret_cast<const double *>(sg);
                    pyx[m] = sgd[(k * NB + m) * n_lanes + i];
                    pyv[m] = sgd[(k * NB + NM + m) * n_lanes + i];
                }
            }
            if (q + 1 >= first_w) {
                if constexpr (MIXED) pub = sg[(k * NB + 2 * NM) * n_lanes + i];
                else pub = reinterpret_cast<const double *>(sg)[(k * NB + 2 * NM) * n_lanes + i];
            }
        };
        seg_load(n1 - 1);
        for (int64_t q = n1 - 1; q >= n0; --q) {
            R yx[NM], yv[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                yx[m] = pyx[m];
                yv[m] = pyv[m];
            }
            const R ub = pub;
            if (q > n0) seg_load(q - 1);
            if (q + 1 >= first_w) {
#pragma unroll
                for (int m = 0; m < NM; ++m) xb[m] += ub;
            }
            R gsf[L::NC];
#pragma unroll
            for (int k = 0; k < L::NC; ++k) gsf[k] = R(0);
            R gzf = R(0);
            R Db[3] = {R(0), R(0), R(0)};
            R d0, d1, d2;
            drive3(q, s == 0 ? N - 1 : s - 1, d0, d1, d2, edge, false);
            reverse_step<NM, L, DP>(law, yx, yv, xb, vb, om2, cd, gn, h, h2, h3, h6, d0, d1, d2,
                                    gsf, gzf, Db);
#pragma unroll
            for (int k = 0; k < L::NC; ++k) gs[k] += (double)gsf[k];
            gz += (double)gzf;
            if constexpr (DP) {
                double e0[3], e1[3], e2[3];
                const double j = 2.0 * (double)q;
                dgr.at(j, e0);
                dgr.at(j + 1.0, e1);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    e2[k] = eedge[k];
                    eedge[k] = e0[k];
                }
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    gD[k] += (double)Db[0] * e0[k] + (double)Db[1] * e1[k] + (double)Db[2] * e2[k];
            }
            s = s == 0 ? N - 1 : s - 1;
        }
    }
    // the initial state does not depend on the law parameters
    double g[kMaxParams];
#pragma unroll
    for (int q = 0; q < kMaxParams; ++q) g[q] = 0.0;
    L::to_si(p, K, gs, gz, g);
    if constexpr (DP) {
        g[AFM_P_BASE_A] = gD[0];
        g[AFM_P_BASE_F] = gD[1];
        g[AFM_P_BASE_G] = gD[2];
    }
    A.J[i] = J;
    for (int j = 0; j < K.n_free; ++j) {
        double gj = 0.0;
#pragma unroll
        for (int q = 0; q < kMaxParams; ++q)
            if (K.free_index[j] == q) gj = g[q];
        A.dJ[(int64_t)j * A.ld + i] = gj;
    }
    A.status[i] = 0;
}

// ------------------------------------------------------------------------------------------
// Mode-parallel adjoint: G lanes per trajectory (G = 2 for two modes, 4 for three or four, 8 for
// five to eight),
// lane q owning mode q in the forward pass, the checkpoints, the segment buffer and the reverse
// sweep (the transposed stage Jacobians are per mode apart from the force terms, whose sums over
// modes are butterfly sums over the group).  The same operations in the same order as k_grad,
// so the same bits.  A lane without a mode carries an exact zero forward; its adjoint is left
// out of every group sum.

template <int NM, int G, class L, typename R>
__device__ __forceinline__ void stage_eval_mp(const L &law, const ModeLane<R> &ml, R x, R v,
                                              R D, R &a, R &Fd, R &Fdd, R (&dc)[L::NC]) {
    const R d = group_sum<G>(x);
    const R dd = group_sum<G>(v);
    R F = law.grad(d, dd, Fd, Fdd, dc);
    if constexpr (NM < G) F *= ml.w;
    a = Ops<R>::fma(-ml.om2, x - ml.zoff, Ops<R>::fma(-ml.cd, v, Ops<R>::fma(ml.gn, D, F)));
}

template <int NM, int G, class L, typename R>
__device__ __forceinline__ void stage_vjp_mp(const ModeLane<R> &ml, bool real, R kbx, R kbv,
                                             R Fd, R Fdd, const R (&dc)[L::NC], R &Ybx, R &Ybv,
                                             R (&gsf)[L::NC], R &gzf) {
    const R S = group_sum<G>(real ? kbv : R(0));
    Ybx = Ops<R>::fma(-ml.om2, kbv, Fd * S);
    Ybv = Ops<R>::fma(-ml.cd, kbv, Ops<R>::fma(Fdd, S, kbx));
#pragma unroll
    for (int k = 0; k < L::NC; ++k) gsf[k] = Ops<R>::fma(S, dc[k], gsf[k]);
    gzf = Ops<R>::fma(S, Fd, gzf);
}

template <int NM, int G, class L, typename R>
__device__ __forceinline__ void reverse_step_mp(const L &law, const ModeLane<R> &ml, bool real,
                                                R x, R v, R &xb, R &vb, R h, R h2, R h3, R h6,
                                                R D0, R D1, R D2, R (&gsf)[L::NC], R &gzf) {
    R a1, a2, a3, a4, Y, V2, V3, V4;
    R Fd1, Fdd1, Fd2, Fdd2, Fd3, Fdd3, Fd4, Fdd4;
    R dc1[L::NC], dc2[L::NC], dc3[L::NC], dc4[L::NC];
    stage_eval_mp<NM, G>(law, ml, x, v, D0, a1, Fd1, Fdd1, dc1);
    Y = Ops<R>::fma(h2, v, x);
    V2 = Ops<R>::fma(h2, a1, v);
    stage_eval_mp<NM, G>(law, ml, Y, V2, D1, a2, Fd2, Fdd2, dc2);
    Y = Ops<R>::fma(h2, V2, x);
    V3 = Ops<R>::fma(h2, a2, v);
    stage_eval_mp<NM, G>(law, ml, Y, V3, D1, a3, Fd3, Fdd3, dc3);
    Y = Ops<R>::fma(h, V3, x);
    V4 = Ops<R>::fma(h, a3, v);
    stage_eval_mp<NM, G>(law, ml, Y, V4, D2, a4, Fd4, Fdd4, dc4);
    R kbx = h6 * xb, kbv = h6 * vb, Ybx, Ybv, sx, sv;
    stage_vjp_mp<NM, G, L>(ml, real, kbx, kbv, Fd4, Fdd4, dc4, Ybx, Ybv, gsf, gzf);
    sx = Ybx;
    sv = Ybv;
    kbx = Ops<R>::fma(h3, xb, h * Ybx);
    kbv = Ops<R>::fma(h3, vb, h * Ybv);
    stage_vjp_mp<NM, G, L>(ml, real, kbx, kbv, Fd3, Fdd3, dc3, Ybx, Ybv, gsf, gzf);
    sx += Ybx;
    sv += Ybv;
    kbx = Ops<R>::fma(h3, xb, h2 * Ybx);
    kbv = Ops<R>::fma(h3, vb, h2 * Ybv);
    stage_vjp_mp<NM, G, L>(ml, real, kbx, kbv, Fd2, Fdd2, dc2, Ybx, Ybv, gsf, gzf);
    sx += Ybx;
    sv += Ybv;
    kbx = Ops<R>::fma(h6, xb, h2 * Ybx);
    kbv = Ops<R>::fma(h6, vb, h2 * Ybv);
    stage_vjp_mp<NM, G, L>(ml, real, kbx, kbv, Fd1, Fdd1, dc1, Ybx, Ybv, gsf, gzf);
    xb += sx + Ybx;
    vb += sv + Ybv;
}

template <int LAW, int NM, bool MIXED>
__global__ void __launch_bounds__(64) k_grad_mp(const GradArgs A, const KConst K) {
    using R = typename std::conditional<MIXED, float, double>::type;
    using L = Law<LAW, R>;
    constexpr bool COMP = MIXED;
    constexpr int G = NM <= 2 ? 2 : (NM <= 4 ? 4 : 8);
    constexpr int NS = 4 * NM;
    constexpr int NB = 2 * NM + 1;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= A.n) return;  // whole groups (block size a multiple of 8)
    const int q = threadIdx.x & (G - 1);
    const int gbase = (int)(threadIdx.x & 63) & ~(G - 1);
    const bool real = q < NM;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    const L law(p, K);
    const double zc = p[0] * 1e9;
    const int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    const int N = K.N;
    const int64_t W = (int64_t)K.lockin * N;
    const int64_t row = A.target_id ? (int64_t)A.target_id[grp] : 0;
    const int kc = A.kc;
    const int64_t n_lanes = A.n;
    auto fail = [&](int32_t st) {
        if (q != 0) return;
        A.J[i] = INFINITY;
        for (int j = 0; j < K.n_free; ++j) A.dJ[(int64_t)j * A.ld + i] = NAN;
        A.status[i] = st;
    };
    if (nc < K.lockin || nc > K.n_cycles || row < 0 || row >= A.n_targets) {
        fail(AFM_ST_BAD_INPUT);
        return;
    }
    const double *__restrict__ Urow = A.targets + row * W;
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;

    ModeLane<R> ml{R(0), R(0), R(0), R(0), R(0)};
    R x = R(0), v = R(0), cx = R(0), cv = R(0);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        if (q == m) {
            ml.om2 = (R)K.om2[m];
            ml.cd = (R)K.cdamp[m];
            ml.gn = (R)K.gain[m];
            ml.zoff = m == 0 ? law.zc : R(0);
            ml.w = R(1);
            x = (R)(m == 0 ? zc + K.y0[0] : K.y0[m]);
            v = (R)K.y0[NM + m];
        }
    }
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h3 = (R)(K.h / 3.0), h6 = (R)(K.h / 6.0);
    float *__restrict__ ck = A.ckpt;
    float *__restrict__ sg = A.seg;
    // this lane's scalar `var` (own mode's index) of slot `slot` in a [slot][nvar][n] buffer
    auto at = [&](int64_t slot, int var, int nvar) { return (slot * nvar + var) * n_lanes + i; };

    // ---- forward pass with checkpoints
    const int64_t Ntot = (int64_t)nc * N;
    const int64_t first_w = Ntot - W + 1;
    double Jn = 0.0, Jd = 0.0;
    int32_t st = 0;
    int64_t n = 0;
    int cdn = 0;
    for (int c = 0; c < nc && !st; ++c) {
        for (int s = 0; s < N; ++s, ++n) {
            if (cdn == 0) {
                const int64_t slot = n / kc;
                if (real) {
                    if constexpr (MIXED) {
                        ck[at(slot, q, NS)] = x;
                        ck[at(slot, NM + q, NS)] = v;
                        ck[at(slot, 2 * NM + q, NS)] = cx;
                        ck[at(slot, 3 * NM + q, NS)] = cv;
                    } else {
                        double *ckd = reinterpret_cast<double *>(ck);
                        ckd[at(slot, q, NS)] = x;
                        ckd[at(slot, NM + q, NS)] = v;
                    }
                }
                cdn = kc;
            }
            --cdn;
            rk4_step_mp<NM, G, COMP, kFmFree>(law, ml, x, v, cx, cv, h, h2, h6, Dt[2 * s],
                                             Dt[2 * s + 1], Dt[2 * s + 2]);
            if (n + 1 >= first_w) {
                const double u = sample_mp<NM, COMP>(x, cx, zc, gbase);
                const double U = Urow[n + 1 - first_w] * 1e9;
                const double e = U - u;
                Jn = __builtin_fma(e, e, Jn);
                Jd = __builtin_fma(U, U, Jd);
            }
        }
        int nonfinite = !(isfinite(x) && isfinite(v));
        nonfinite |= __shfl_xor(nonfinite, 1, 64);
        if constexpr (G >= 4) nonfinite |= __shfl_xor(nonfinite, 2, 64);
        if constexpr (G == 8) nonfinite |= __shfl_xor(nonfinite, 4, 64);
        if (nonfinite) st = AFM_ST_NONFINITE;
        else if (fabs(sample_mp<NM, COMP>(x, cx, zc, gbase)) > K.div_nm) st = AFM_ST_DIVERGED;
    }
    const double J = Jn / Jd;
    if (st || !isfinite(J)) {
        fail(st ? st : AFM_ST_NONFINITE);
        return;
    }
    const double coef = -2.0 / Jd;

    // ---- reverse sweep
    R xb = R(0), vb = R(0);
    double gs[L::NC];
#pragma unroll
    for (int k = 0; k < L::NC; ++k) gs[k] = 0.0;
    double gz = 0.0;
    const int64_t nseg = (Ntot + kc - 1) / kc;
    for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
        const int64_t n0 = sgi * kc;
        const int64_t n1 = n0 + kc < Ntot ? n0 + kc : Ntot;
        if (real) {
            if constexpr (MIXED) {
                x = ck[at(sgi, q, NS)];
                v = ck[at(sgi, NM + q, NS)];
                cx = ck[at(sgi, 2 * NM + q, NS)];
                cv = ck[at(sgi, 3 * NM + q, NS)];
            } else {
                const double *ckd = reinterpret_cast<const double *>(ck);
                x = ckd[at(sgi, q, NS)];
                v = ckd[at(sgi, NM + q, NS)];
            }
        }
        int s = (int)(n0 % N);
        for (int64_t qq = n0; qq < n1; ++qq) {
            const int64_t k = qq - n0;
            if (real) {
                if constexpr (MIXED) {
                    sg[at(k, q, NB)] = x;
                    sg[at(k, NM + q, NB)] = v;
                } else {
                    double *sgd = reinterpret_cast<double *>(sg);
                    sgd[at(k, q, NB)] = x;
                    sgd[at(k, NM + q, NB)] = v;
                }
            }
            rk4_step_mp<NM, G, COMP, kFmFree>(law, ml, x, v, cx, cv, h, h2, h6, Dt[2 * s],
                                             Dt[2 * s + 1], Dt[2 * s + 2]);
            if (qq + 1 >= first_w) {
                const double u = sample_mp<NM, COMP>(x, cx, zc, gbase);
                const double ub = coef * (Urow[qq + 1 - first_w] * 1e9 - u);
                if (q == 0) {
                    if constexpr (MIXED) sg[at(k, 2 * NM, NB)] = (R)ub;
                    else reinterpret_cast<double *>(sg)[at(k, 2 * NM, NB)] = ub;
                }
            }
            s = s + 1 == N ? 0 : s + 1;
        }
        s = (int)((n1 - 1) % N);
        for (int64_t qq = n1 - 1; qq >= n0; --qq) {
            const int64_t k = qq - n0;
            R yx = R(0), yv = R(0);
            if (qq + 1 >= first_w) {
                R ub;
                if constexpr (MIXED) ub = sg[at(k, 2 * NM, NB)];
                else ub = reinterpret_cast<const double *>(sg)[at(k, 2 * NM, NB)];
                if (real) xb += ub;
            }
            if (real) {
                if constexpr (MIXED) {
                    yx = sg[at(k, q, NB)];
                    yv = sg[at(k, NM + q, NB)];
                } else {
                    const double *sgd = reinterpret_cast<const double *>(sg);
                    yx = sgd[at(k, q, NB)];
                    yv = sgd[at(k, NM + q, NB)];
                }
            }
            R gsf[L::NC];
#pragma unroll
            for (int k2 = 0; k2 < L::NC; ++k2) gsf[k2] = R(0);
            R gzf = R(0);
            reverse_step_mp<NM, G, L>(law, ml, real, yx, yv, xb, vb, h, h2, h3, h6, Dt[2 * s],
                                      Dt[2 * s + 1], Dt[2 * s + 2], gsf, gzf);
#pragma unroll
            for (int k2 = 0; k2 < L::NC; ++k2) gs[k2] += (double)gsf[k2];
            gz += (double)gzf;
            s = s == 0 ? N - 1 : s - 1;
        }
    }
    if (q != 0) return;
    double g[kMaxParams];
#pragma unroll
    for (int qp = 0; qp < kMaxParams; ++qp) g[qp] = 0.0;
    L::to_si(p, K, gs, gz, g);
    A.J[i] = J;
    for (int j = 0; j < K.n_free; ++j) {
        double gj = 0.0;
#pragma unroll
        for (int qp = 0; qp < kMaxParams; ++qp)
            if (K.free_index[j] == qp) gj = g[qp];
        A.dJ[(int64_t)j * A.ld + i] = gj;
    }
    A.status[i] = 0;
}

// ------------------------------------------------------------------------------------------
// Segment-parallel form.  The reverse sweep above is one long dependent chain per trajectory:
// with a few thousand trajectories (one wave per SIMD or less) it is latency-bound.  The adjoint
// recursion is linear in the adjoint state, so the trajectory's checkpoint segments can be
// differentiated independently and combined afterwards:
//   segment s maps the state y_s at its first step to y_{s+1}; let Phi_s = dy_{s+1}/dy_s,
//   S_s = dy_{s+1}/dtheta (theta: the law's constants and z_c, with y_s held fixed), and let
//   c_s = dJ_s/dy_s, p_s = dJ_s/dtheta be the derivatives of the segment's own window terms J_s.
//   Then, from lambda_{n_seg} = 0 backwards, dJ/dtheta = sum_s (p_s + S_s^T lambda_{s+1}) and
//   lambda_s = c_s + Phi_s^T lambda_{s+1}.
// k_grad_ckpt runs the forward pass (checkpoints, J, status, dJ/du scale), k_grad_tan gives every
// (trajectory, segment) pair its own lane, which recomputes the segment from its checkpoint and
// carries the 2 NM + NC + 1 tangent columns of (Phi_s, S_s) forward through the RK4 stages (the
// same stage states and force partials as the reverse sweep), accumulating c_s and p_s from the
// window samples in FP64, k_grad_compose folds each group of B consecutive segments into one
// record of the same form (the recursion over the group applied to a symbolic lambda at the
// group's end: an affine map, composed in FP64 by one lane per (trajectory, group)), and
// k_grad_combine runs the short backward recursion over the groups in FP64, one lane per
// trajectory.  Tangents are in deflection coordinates (mode 1's state is
// the gap g = z_c + u_1, but z_c is a parameter of the map: the z_c column moves the gap at fixed
// deflection), matching the reverse sweep's dJ/dz_c.  The result is the same exact derivative as
// the reverse sweep up to rounding (it depends on the stride only through rounding).

// number of FP64 record entries per segment: Phi (2NM x 2NM), S (2NM x NP), c (2NM), p (NP)
template <int NM, int NP>
constexpr int seg_fields() { return 4 * NM * NM + 2 * NM * NP + 2 * NM + NP; }

template <int LAW, int NM, bool MIXED>
__global__ void __launch_bounds__(64) k_grad_ckpt(const GradArgs A, const KConst K) {
    using R = typename std::conditional<MIXED, float, double>::type;
    using L = Law<LAW, R>;
    constexpr bool COMP = MIXED;
    constexpr int NS = 4 * NM;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    const L law(p, K);
    const double zc = p[0] * 1e9;
    const int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    const int N = K.N;
    const int64_t W = (int64_t)K.lockin * N;
    const int64_t row = A.target_id ? (int64_t)A.target_id[grp] : 0;
    const int kc = A.kc;
    const int64_t n_lanes = A.n;
    double *coef_out = reinterpret_cast<double *>(A.seg);
    auto fail = [&](int32_t st) {
        A.J[i] = INFINITY;
        for (int j = 0; j < K.n_free; ++j) A.dJ[(int64_t)j * A.ld + i] = NAN;
        A.status[i] = st;
        coef_out[i] = 0.0;
    };
    if (nc < K.lockin || nc > K.n_cycles || row < 0 || row >= A.n_targets) {
        fail(AFM_ST_BAD_INPUT);
        return;
    }
    const double *__restrict__ Urow = A.targets + row * W;
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;
    R x[NM], v[NM], cx[NM], cv[NM], om2[NM], cd[NM], gn[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        x[m] = (R)(m == 0 ? zc + K.y0[0] : K.y0[m]);
        v[m] = (R)K.y0[NM + m];
        cx[m] = R(0);
        cv[m] = R(0);
        om2[m] = (R)K.om2[m];
        cd[m] = (R)K.cdamp[m];
        gn[m] = (R)K.gain[m];
    }
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h6 = (R)(K.h / 6.0);
    float *__restrict__ ck = A.ckpt;
    double Jn = 0.0, Jd = 0.0;
    int32_t st = 0;
    int64_t n = 0;
    int cdn = 0;  // steps to the next checkpoint (the state before step n is slot n / kc)
    auto save = [&]() {
        const int64_t slot = n / kc;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            if constexpr (MIXED) {
                ck[(slot * NS + m) * n_lanes + i] = x[m];
                ck[(slot * NS + NM + m) * n_lanes + i] = v[m];
                ck[(slot * NS + 2 * NM + m) * n_lanes + i] = cx[m];
                ck[(slot * NS + 3 * NM + m) * n_lanes + i] = cv[m];
            } else {
                double *ckd = reinterpret_cast<double *>(ck);
                ckd[(slot * NS + m) * n_lanes + i] = x[m];
                ckd[(slot * NS + NM + m) * n_lanes + i] = v[m];
            }
        }
    };
    // with the stride and the period multiples of four, every checkpoint falls on the start of
    // a four-step block: the transient periods then run in blocks whose nine drive entries come
    // in as one group of uniform loads (the same steps and entries as one step at a time, so
    // the same bits)
    const bool blocks = kc % 4 == 0 && N % 4 == 0;
    const int c_win = nc - K.lockin;  // first period of the misfit window
    for (int c = 0; c < nc && !st; ++c) {
        if (c < c_win && blocks) {
            for (int s = 0; s < N; s += 4, n += 4) {
                if (cdn == 0) {
                    save();
                    cdn = kc;
                }
                cdn -= 4;
                // scalar loads: the offset is wave-uniform and the table read-only for the
                // kernel's lifetime (constant address space)
                using CR = const __attribute__((address_space(4))) R;
                CR *dp = (CR *)(Dt + __builtin_amdgcn_readfirstlane(2 * s));
                R e[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) e[k] = dp[k];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    rk4_step<NM, COMP, kFmFree>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6,
                                                e[2 * q], e[2 * q + 1], e[2 * q + 2]);
            }
        } else if (c < c_win) {
            for (int s = 0; s < N; ++s, ++n) {
                if (cdn == 0) {
                    save();
                    cdn = kc;
                }
                --cdn;
                rk4_step<NM, COMP, kFmFree>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, Dt[2 * s],
                                            Dt[2 * s + 1], Dt[2 * s + 2]);
            }
        } else {
            // window period: the state after every step is a sample; step n's target entry is
            // n + 1 - first_w = w0 + s, loaded one step ahead
            const int64_t w0 = (int64_t)(c - c_win) * N;
            double Un = Urow[w0];
            for (int s = 0; s < N; ++s, ++n) {
                if (cdn == 0) {
                    save();
                    cdn = kc;
                }
                --cdn;
                const double Uc = Un;
                Un = Urow[w0 + s + 1 < W ? w0 + s + 1 : w0 + s];
                rk4_step<NM, COMP, kFmFree>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, Dt[2 * s],
                                            Dt[2 * s + 1], Dt[2 * s + 2]);
                const double u = sample<NM, COMP>(x, cx, zc);
                const double U = Uc * 1e9;
                const double e = U - u;
                Jn = __builtin_fma(e, e, Jn);
                Jd = __builtin_fma(U, U, Jd);
            }
        }
        bool fin = true;
#pragma unroll
        for (int m = 0; m < NM; ++m) fin = fin && isfinite(x[m]) && isfinite(v[m]);
        if (!fin) st = AFM_ST_NONFINITE;
        else if (fabs(sample<NM, COMP>(x, cx, zc)) > K.div_nm) st = AFM_ST_DIVERGED;
    }
    const double J = Jn / Jd;
    if (st || !isfinite(J)) {
        fail(st ? st : AFM_ST_NONFINITE);
        return;
    }
    A.J[i] = J;
    A.status[i] = 0;
    coef_out[i] = -2.0 / Jd;  // dJ/du_n = coef (U_n - u_n)
}

// k_grad_ckpt with one lane per mode (the mode-parallel forward of k_grad_mp): G lanes per
// trajectory, lane q integrating mode q with the shared force, the same operations in the same
// order as one lane per trajectory (so the same checkpoints, J and status bit for bit); lanes
// without a mode carry zeros.  For small multi-mode batches, where one lane per trajectory
// leaves most SIMDs idle.
template <int LAW, int NM, bool MIXED>
__global__ void __launch_bounds__(64) k_grad_ckpt_mp(const GradArgs A, const KConst K) {
    using R = typename std::conditional<MIXED, float, double>::type;
    using L = Law<LAW, R>;
    constexpr bool COMP = MIXED;
    constexpr int G = NM <= 2 ? 2 : (NM <= 4 ? 4 : 8);
    constexpr int NS = 4 * NM;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= A.n) return;  // whole groups (block size a multiple of 8)
    const int q = threadIdx.x & (G - 1);
    const int gbase = (int)(threadIdx.x & 63) & ~(G - 1);
    const bool real = q < NM;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    const L law(p, K);
    const double zc = p[0] * 1e9;
    const int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    const int N = K.N;
    const int64_t W = (int64_t)K.lockin * N;
    const int64_t row = A.target_id ? (int64_t)A.target_id[grp] : 0;
    const int kc = A.kc;
    const int64_t n_lanes = A.n;
    double *coef_out = reinterpret_cast<double *>(A.seg);
    auto fail = [&](int32_t st) {
        if (q != 0) return;
        A.J[i] = INFINITY;
        for (int j = 0; j < K.n_free; ++j) A.dJ[(int64_t)j * A.ld + i] = NAN;
        A.status[i] = st;
        coef_out[i] = 0.0;
    };
    if (nc < K.lockin || nc > K.n_cycles || row < 0 || row >= A.n_targets) {
        fail(AFM_ST_BAD_INPUT);
        return;
    }
    const double *__restrict__ Urow = A.targets + row * W;
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;
    ModeLane<R> ml{R(0), R(0), R(0), R(0), R(0)};
    R x = R(0), v = R(0), cx = R(0), cv = R(0);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        if (q == m) {
            ml.om2 = (R)K.om2[m];
            ml.cd = (R)K.cdamp[m];
            ml.gn = (R)K.gain[m];
            ml.zoff = m == 0 ? law.zc : R(0);
            ml.w = R(1);
            x = (R)(m == 0 ? zc + K.y0[0] : K.y0[m]);
            v = (R)K.y0[NM + m];
        }
    }
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h6 = (R)(K.h / 6.0);
    // the forward's block-level contact test (laws with a bound): far blocks without the
    // contact piece, which adds exact zeros there, so the checkpoints keep their bits
    const ModeBound<R> mb(K, NM, q);
    float *__restrict__ ck = A.ckpt;
    double Jn = 0.0, Jd = 0.0;
    int32_t st = 0;
    int64_t n = 0;
    int cdn = 0;  // steps to the next checkpoint (the state before step n is slot n / kc)
    auto save = [&]() {
        if (!real) return;
        const int64_t slot = n / kc;
        if constexpr (MIXED) {
            ck[(slot * NS + q) * n_lanes + i] = x;
            ck[(slot * NS + NM + q) * n_lanes + i] = v;
            ck[(slot * NS + 2 * NM + q) * n_lanes + i] = cx;
            ck[(slot * NS + 3 * NM + q) * n_lanes + i] = cv;
        } else {
            double *ckd = reinterpret_cast<double *>(ck);
            ckd[(slot * NS + q) * n_lanes + i] = x;
            ckd[(slot * NS + NM + q) * n_lanes + i] = v;
        }
    };
    const bool blocks = kc % 4 == 0 && N % 4 == 0;
    const int c_win = nc - K.lockin;
    for (int c = 0; c < nc && !st; ++c) {
        if (c < c_win && blocks) {
            for (int s = 0; s < N; s += 4, n += 4) {
                if (cdn == 0) {
                    save();
                    cdn = kc;
                }
                cdn -= 4;
                using CR = const __attribute__((address_space(4))) R;
                CR *dp = (CR *)(Dt + __builtin_amdgcn_readfirstlane(2 * s));
                R e[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) e[k] = dp[k];
                bool far = false;
                if constexpr (HasBlock<L>::value) far = group_far<G>(law, ml, mb, x, v);
                if (far) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        rk4_step_mp<NM, G, COMP, kFmFar>(law, ml, x, v, cx, cv, h, h2, h6,
                                                        e[2 * k], e[2 * k + 1], e[2 * k + 2]);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        rk4_step_mp<NM, G, COMP, kFmFree>(law, ml, x, v, cx, cv, h, h2, h6,
                                                         e[2 * k], e[2 * k + 1], e[2 * k + 2]);
                }
            }
        } else {
            const bool win = c >= c_win;
            const int64_t w0 = win ? (int64_t)(c - c_win) * N : 0;
            for (int s = 0; s < N; ++s, ++n) {
                if (cdn == 0) {
                    save();
                    cdn = kc;
                }
                --cdn;
                rk4_step_mp<NM, G, COMP, kFmFree>(law, ml, x, v, cx, cv, h, h2, h6, Dt[2 * s],
                                                 Dt[2 * s + 1], Dt[2 * s + 2]);
                if (win) {
                    const double u = sample_mp<NM, COMP>(x, cx, zc, gbase);
                    const double U = Urow[w0 + s] * 1e9;
                    const double e = U - u;
                    Jn = __builtin_fma(e, e, Jn);
                    Jd = __builtin_fma(U, U, Jd);
                }
            }
        }
        int nonfinite = !(isfinite(x) && isfinite(v));
        nonfinite |= __shfl_xor(nonfinite, 1, 64);
        if constexpr (G >= 4) nonfinite |= __shfl_xor(nonfinite, 2, 64);
        if constexpr (G == 8) nonfinite |= __shfl_xor(nonfinite, 4, 64);
        if (nonfinite) st = AFM_ST_NONFINITE;
        else if (fabs(sample_mp<NM, COMP>(x, cx, zc, gbase)) > K.div_nm) st = AFM_ST_DIVERGED;
    }
    const double J = Jn / Jd;
    if (st || !isfinite(J)) {
        fail(st ? st : AFM_ST_NONFINITE);
        return;
    }
    if (q == 0) {
        A.J[i] = J;
        A.status[i] = 0;
        coef_out[i] = -2.0 / Jd;  // dJ/du_n = coef (U_n - u_n)
    }
}

// Tangent of one slope evaluation: (dx, dv) the stage state's tangent, dz the z_c component and
// dcv the constants' components of the column; returns the acceleration tangents.
template <int NM, class L, typename R>
__device__ __forceinline__ void slope_jvp(const R (&dx)[NM], const R (&dv)[NM], R dz,
                                          const R (&dcv)[L::NC], R Fd, R Fdd,
                                          const R (&dc)[L::NC], const R (&om2)[NM],
                                          const R (&cd)[NM], R (&da)[NM]) {
    const R dd = mode_sum<NM>(dx) + dz;
    R dF = Fd * dd;
    if constexpr (L::kRate) dF = Ops<R>::fma(Fdd, mode_sum<NM>(dv), dF);
#pragma unroll
    for (int k = 0; k < L::NC; ++k) dF = Ops<R>::fma(dc[k], dcv[k], dF);
#pragma unroll
    for (int m = 0; m < NM; ++m) da[m] = Ops<R>::fma(-om2[m], dx[m], Ops<R>::fma(-cd[m], dv[m], dF));
}

template <int LAW, int NM, bool MIXED>
__global__ void __launch_bounds__(256) k_grad_tan(const GradArgs A, const KConst K) {
    using R = typename std::conditional<MIXED, float, double>::type;
    using L = Law<LAW, R>;
    constexpr bool COMP = MIXED;
    constexpr int NS = 4 * NM;
    constexpr int NY = 2 * NM;             // state columns
    constexpr int NP = L::NC + 1;          // parameter columns: the constants, then z_c
    constexpr int NF = seg_fields<NM, NP>();
    const int64_t n_lanes = A.n;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = l % n_lanes, sgi = l / n_lanes;
    const int N = K.N, kc = A.kc;
    const int64_t nseg_max = ((int64_t)K.n_cycles * N + kc - 1) / kc;
    if (sgi >= nseg_max) return;
    if (A.status[i] != 0) return;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    const int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    const int64_t Ntot = (int64_t)nc * N;
    const int64_t n0 = sgi * kc;
    if (n0 >= Ntot) return;
    const int64_t n1 = n0 + kc < Ntot ? n0 + kc : Ntot;
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    const L law(p, K);
    const double zc = p[0] * 1e9;
    const int64_t W = (int64_t)K.lockin * N;
    const int64_t row = A.target_id ? (int64_t)A.target_id[grp] : 0;
    const double *__restrict__ Urow = A.targets + row * W;
    const int64_t first_w = Ntot - W + 1;
    const double coef = reinterpret_cast<const double *>(A.seg)[i];
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;
    R x[NM], v[NM], cx[NM], cv[NM], om2[NM], cd[NM], gn[NM];
    const float *__restrict__ ck = A.ckpt;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        om2[m] = (R)K.om2[m];
        cd[m] = (R)K.cdamp[m];
        gn[m] = (R)K.gain[m];
        if constexpr (MIXED) {
            x[m] = ck[(sgi * NS + m) * n_lanes + i];
            v[m] = ck[(sgi * NS + NM + m) * n_lanes + i];
            cx[m] = ck[(sgi * NS + 2 * NM + m) * n_lanes + i];
            cv[m] = ck[(sgi * NS + 3 * NM + m) * n_lanes + i];
        } else {
            const double *ckd = reinterpret_cast<const double *>(ck);
            x[m] = ckd[(sgi * NS + m) * n_lanes + i];
            v[m] = ckd[(sgi * NS + NM + m) * n_lanes + i];
            cx[m] = R(0);
            cv[m] = R(0);
        }
    }
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h6 = (R)(K.h / 6.0);
    // tangent columns: NY state columns (unit start), NP parameter columns (zero start)
    constexpr int NT = NY + NP;
    // (with compensated updates in FP32, as the state: the unit start makes every increment
    // small against the column, and rounding each step against it would bias the segment's
    // map by about the stride times the unit roundoff)
    R tx[NT][NM], tv[NT][NM], ctx[NT][NM], ctv[NT][NM];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            tx[t][m] = (t == m) ? R(1) : R(0);
            tv[t][m] = (t == NM + m) ? R(1) : R(0);
            ctx[t][m] = R(0);
            ctv[t][m] = R(0);
        }
    double acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.0;
    int s = (int)(n0 % N);
    for (int64_t q = n0; q < n1; ++q) {
        const R D0 = Dt[2 * s], D1 = Dt[2 * s + 1], D2 = Dt[2 * s + 2];
        // stage states and force partials at this step, as the reverse sweep forms them
        R a1[NM], a2[NM], a3[NM], a4[NM], Y[NM], V2[NM], V3[NM], V4[NM];
        R Fd1, Fdd1, Fd2, Fdd2, Fd3, Fdd3, Fd4, Fdd4;
        R dc1[L::NC], dc2[L::NC], dc3[L::NC], dc4[L::NC];
        stage_eval<NM>(law, x, v, om2, cd, gn, D0, a1, Fd1, Fdd1, dc1);
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            Y[m] = Ops<R>::fma(h2, v[m], x[m]);
            V2[m] = Ops<R>::fma(h2, a1[m], v[m]);
        }
        stage_eval<NM>(law, Y, V2, om2, cd, gn, D1, a2, Fd2, Fdd2, dc2);
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            Y[m] = Ops<R>::fma(h2, V2[m], x[m]);
            V3[m] = Ops<R>::fma(h2, a2[m], v[m]);
        }
        stage_eval<NM>(law, Y, V3, om2, cd, gn, D1, a3, Fd3, Fdd3, dc3);
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            Y[m] = Ops<R>::fma(h, V3[m], x[m]);
            V4[m] = Ops<R>::fma(h, a3[m], v[m]);
        }
        stage_eval<NM>(law, Y, V4, om2, cd, gn, D2, a4, Fd4, Fdd4, dc4);
        // every tangent column through the four stages and the update
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const R dz = t == NT - 1 ? R(1) : R(0);
            R dcv[L::NC];
#pragma unroll
            for (int k = 0; k < L::NC; ++k) dcv[k] = (t == NY + k) ? R(1) : R(0);
            R e1[NM], e2[NM], e3[NM], e4[NM], X[NM], Vt2[NM], Vt3[NM], Vt4[NM];
            slope_jvp<NM, L>(tx[t], tv[t], dz, dcv, Fd1, Fdd1, dc1, om2, cd, e1);
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                X[m] = Ops<R>::fma(h2, tv[t][m], tx[t][m]);
                Vt2[m] = Ops<R>::fma(h2, e1[m], tv[t][m]);
            }
            slope_jvp<NM, L>(X, Vt2, dz, dcv, Fd2, Fdd2, dc2, om2, cd, e2);
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                X[m] = Ops<R>::fma(h2, Vt2[m], tx[t][m]);
                Vt3[m] = Ops<R>::fma(h2, e2[m], tv[t][m]);
            }
            slope_jvp<NM, L>(X, Vt3, dz, dcv, Fd3, Fdd3, dc3, om2, cd, e3);
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                X[m] = Ops<R>::fma(h, Vt3[m], tx[t][m]);
                Vt4[m] = Ops<R>::fma(h, e3[m], tv[t][m]);
            }
            slope_jvp<NM, L>(X, Vt4, dz, dcv, Fd4, Fdd4, dc4, om2, cd, e4);
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                const R sx = tv[t][m] + R(2) * (Vt2[m] + Vt3[m]) + Vt4[m];
                const R sv = e1[m] + R(2) * (e2[m] + e3[m]) + e4[m];
                if constexpr (COMP) {
                    const R dx = Ops<R>::fma(h6, sx, -ctx[t][m]);
                    const R ux = tx[t][m] + dx;
                    ctx[t][m] = (ux - tx[t][m]) - dx;
                    tx[t][m] = ux;
                    const R dv = Ops<R>::fma(h6, sv, -ctv[t][m]);
                    const R uv = tv[t][m] + dv;
                    ctv[t][m] = (uv - tv[t][m]) - dv;
                    tv[t][m] = uv;
                } else {
                    tx[t][m] = Ops<R>::fma(h6, sx, tx[t][m]);
                    tv[t][m] = Ops<R>::fma(h6, sv, tv[t][m]);
                }
            }
        }
        // the state itself, bit for bit as the forward pass stepped it
        rk4_step<NM, COMP, kFmFree>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, D0, D1, D2);
        if (q + 1 >= first_w) {
            const double u = sample<NM, COMP>(x, cx, zc);
            const double ub = coef * (Urow[q + 1 - first_w] * 1e9 - u);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                double du = 0.0;
#pragma unroll
                for (int m = 0; m < NM; ++m) du += (double)tx[t][m] - (double)ctx[t][m];
                acc[t] = __builtin_fma(ub, du, acc[t]);
            }
        }
        s = s + 1 == N ? 0 : s + 1;
    }
    // record [sgi][field][n]: Phi as [state column j][row r] (rows: x then v), S as
    // [parameter column k][row r], then c (state columns), then p (parameter columns)
    double *rec = reinterpret_cast<double *>(A.seg) + n_lanes + sgi * NF * n_lanes + i;
    int f = 0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int m = 0; m < NM; ++m)
            rec[(int64_t)(f++) * n_lanes] = (double)tx[t][m] - (double)ctx[t][m];
#pragma unroll
        for (int m = 0; m < NM; ++m)
            rec[(int64_t)(f++) * n_lanes] = (double)tv[t][m] - (double)ctv[t][m];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) rec[(int64_t)(f++) * n_lanes] = acc[t];
}

// Fold segments g B .. min((g + 1) B, n_seg) - 1 of a trajectory into one record, written over
// the group's first record: with lambda = alpha + Bm lambda_end carried backwards from the
// identity map at the group's end, each segment gives alpha' = c_s + Phi_s^T alpha,
// Bm' = Phi_s^T Bm (state rows) and adds p_s + S_s^T alpha, S_s^T Bm to the parameter rows; the
// result has the record layout with (Bm, parameter matrix) for (Phi^T, S^T) and (alpha, parameter
// constant) for (c, p).  One lane per (trajectory, group); the lane reads the group's records
// last to first and writes only after reading the first, so groups never overlap.
template <int LAW, int NM, bool MIXED>
__global__ void __launch_bounds__(64) k_grad_compose(const GradArgs A, const KConst K, int B) {
    using R = typename std::conditional<MIXED, float, double>::type;
    using L = Law<LAW, R>;
    constexpr int NY = 2 * NM;
    constexpr int NP = L::NC + 1;
    constexpr int NT = NY + NP;
    constexpr int NF = seg_fields<NM, NP>();
    const int64_t n_lanes = A.n;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = l % n_lanes, gi = l / n_lanes;
    const int64_t nseg_max = ((int64_t)K.n_cycles * K.N + A.kc - 1) / A.kc;
    if (gi >= (nseg_max + B - 1) / B) return;
    if (A.status[i] != 0) return;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    const int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    const int64_t nseg = ((int64_t)nc * K.N + A.kc - 1) / A.kc;
    const int64_t s0 = gi * B;
    if (s0 >= nseg) return;
    const int64_t s1 = s0 + B < nseg ? s0 + B : nseg;
    if (s1 - s0 < 2) return;  // a one-segment group is its own record
    double *recs = reinterpret_cast<double *>(A.seg) + n_lanes;
    double al[NY], bm[NY][NY], ga[NP], gm[NP][NY];
#pragma unroll
    for (int r = 0; r < NY; ++r) {
        al[r] = 0.0;
#pragma unroll
        for (int k = 0; k < NY; ++k) bm[r][k] = r == k ? 1.0 : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        ga[t] = 0.0;
#pragma unroll
        for (int k = 0; k < NY; ++k) gm[t][k] = 0.0;
    }
    for (int64_t sgi = s1 - 1; sgi >= s0; --sgi) {
        const double *rec = recs + sgi * NF * n_lanes + i;
        auto at = [&](int f) { return rec[(int64_t)f * n_lanes]; };
        double na[NY], nb[NY][NY];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            double m[NY];
#pragma unroll
            for (int r = 0; r < NY; ++r) m[r] = at(t * NY + r);
            double d = at(NT * NY + t);
#pragma unroll
            for (int r = 0; r < NY; ++r) d = __builtin_fma(m[r], al[r], d);
            double row[NY];
#pragma unroll
            for (int k = 0; k < NY; ++k) {
                double e = 0.0;
#pragma unroll
                for (int r = 0; r < NY; ++r) e = __builtin_fma(m[r], bm[r][k], e);
                row[k] = e;
            }
            if (t < NY) {
                na[t] = d;
#pragma unroll
                for (int k = 0; k < NY; ++k) nb[t][k] = row[k];
            } else {
                ga[t - NY] += d;
#pragma unroll
                for (int k = 0; k < NY; ++k) gm[t - NY][k] += row[k];
            }
        }
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            al[r] = na[r];
#pragma unroll
            for (int k = 0; k < NY; ++k) bm[r][k] = nb[r][k];
        }
    }
    double *out = recs + s0 * NF * n_lanes + i;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int k = 0; k < NY; ++k)
            out[(int64_t)(t * NY + k) * n_lanes] = t < NY ? bm[t][k] : gm[t - NY][k];
        out[(int64_t)(NT * NY + t) * n_lanes] = t < NY ? al[t] : ga[t - NY];
    }
}

// Backward recursion over the trajectory's records, every B-th (the composed groups).
template <int LAW, int NM, bool MIXED>
__global__ void __launch_bounds__(64) k_grad_combine(const GradArgs A, const KConst K, int B) {
    using R = typename std::conditional<MIXED, float, double>::type;
    using L = Law<LAW, R>;
    constexpr int NY = 2 * NM;
    constexpr int NP = L::NC + 1;
    constexpr int NT = NY + NP;
    constexpr int NF = seg_fields<NM, NP>();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    if (A.status[i] != 0) return;
    const int64_t n_lanes = A.n;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    const int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    const int64_t nseg = ((int64_t)nc * K.N + A.kc - 1) / A.kc;
    const double *recs = reinterpret_cast<const double *>(A.seg) + n_lanes;
    double lam[NY], g[NP];
#pragma unroll
    for (int r = 0; r < NY; ++r) lam[r] = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) g[k] = 0.0;
    for (int64_t sgi = (nseg - 1) / B * B; sgi >= 0; sgi -= B) {
        const double *rec = recs + sgi * NF * n_lanes + i;
        auto at = [&](int f) { return rec[(int64_t)f * n_lanes]; };
        double nl[NY];
        // parameters: p_s + S_s^T lambda_{s+1}; state: c_s + Phi_s^T lambda_{s+1}
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            double d = at(NT * NY + t);
#pragma unroll
            for (int r = 0; r < NY; ++r) d = __builtin_fma(at(t * NY + r), lam[r], d);
            if (t < NY) nl[t] = d;
            else g[t - NY] += d;
        }
#pragma unroll
        for (int r = 0; r < NY; ++r) lam[r] = nl[r];
    }
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    double sc[L::NC];
#pragma unroll
    for (int k = 0; k < L::NC; ++k) sc[k] = g[k];
    double gs[kMaxParams];
#pragma unroll
    for (int q = 0; q < kMaxParams; ++q) gs[q] = 0.0;
    L::to_si(p, K, sc, g[NP - 1], gs);
    for (int j = 0; j < K.n_free; ++j) {
        double gj = 0.0;
#pragma unroll
        for (int q = 0; q < kMaxParams; ++q)
            if (K.free_index[j] == q) gj = gs[q];
        A.dJ[(int64_t)j * A.ld + i] = gj;
    }
}

// whether the segment-parallel form is built for a problem (table drive, at most 4 modes)
constexpr int kSegMaxModes = 4;

template <int LAW, int NM, bool MIXED>
hipError_t launch_t(const GradArgs &a, const KConst &K, hipStream_t s) {
    const int block = 64;
    if constexpr (NM <= kSegMaxModes) {
        if (a.form == kGradSegments && K.drive_mode == AFM_DRIVE_TABLE) {
            const int64_t nseg = ((int64_t)K.n_cycles * K.N + a.kc - 1) / a.kc;
            const int64_t lanes = a.n * nseg;
            if (NM > 1 && a.mp) {  // one lane per mode (see k_grad_ckpt_mp)
                constexpr int G = NM <= 2 ? 2 : (NM <= 4 ? 4 : 8);
                hipLaunchKernelGGL((k_grad_ckpt_mp<LAW, NM, MIXED>),
                                   dim3((unsigned)((a.n * G + 63) / 64)), dim3(64), 0, s, a, K);
            } else {
                hipLaunchKernelGGL((k_grad_ckpt<LAW, NM, MIXED>),
                                   dim3((unsigned)((a.n + 63) / 64)), dim3(64), 0, s, a, K);
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_grad_tan<LAW, NM, MIXED>), dim3((unsigned)((lanes + 255) / 256)),
                               dim3(256), 0, s, a, K);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            // groups of about sqrt(n_seg) segments: n x n_seg / B composing lanes, then B-fold
            // fewer sequential steps per trajectory
            int B = 1;
            if (nseg >= 16) {
                B = (int)std::ceil(std::sqrt((double)nseg));
                const int64_t groups = (nseg + B - 1) / B;
                hipLaunchKernelGGL((k_grad_compose<LAW, NM, MIXED>),
                                   dim3((unsigned)((a.n * groups + 63) / 64)), dim3(64), 0, s, a,
                                   K, B);
                e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL((k_grad_combine<LAW, NM, MIXED>),
                               dim3((unsigned)((a.n + 63) / 64)), dim3(64), 0, s, a, K, B);
            return hipGetLastError();
        }
    }
    if (K.drive_mode != AFM_DRIVE_TABLE) {  // parameter-driven base: one lane per trajectory
        const int64_t grid = (a.n + block - 1) / block;
        hipLaunchKernelGGL((k_grad<LAW, NM, MIXED, true>), dim3((unsigned)grid), dim3(block), 0, s,
                           a, K);
        return hipGetLastError();
    }
    if constexpr (NM > 1) {
        if (a.mp) {
            constexpr int G = NM <= 2 ? 2 : (NM <= 4 ? 4 : 8);
            const int64_t grid = (a.n * G + block - 1) / block;
            hipLaunchKernelGGL((k_grad_mp<LAW, NM, MIXED>), dim3((unsigned)grid), dim3(block), 0,
                               s, a, K);
            return hipGetLastError();
        }
    }
    const int64_t grid = (a.n + block - 1) / block;
    hipLaunchKernelGGL((k_grad<LAW, NM, MIXED>), dim3((unsigned)grid), dim3(block), 0, s, a, K);
    return hipGetLastError();
}

template <int LAW, bool MIXED>
hipError_t launch_modes(const GradArgs &a, const KConst &K, hipStream_t s) {
    switch (K.nm) {
    case 1: return launch_t<LAW, 1, MIXED>(a, K, s);
    case 2: return launch_t<LAW, 2, MIXED>(a, K, s);
    case 3: return launch_t<LAW, 3, MIXED>(a, K, s);
    case 4: return launch_t<LAW, 4, MIXED>(a, K, s);
    case 5: return launch_t<LAW, 5, MIXED>(a, K, s);
    case 6: return launch_t<LAW, 6, MIXED>(a, K, s);
    case 7: return launch_t<LAW, 7, MIXED>(a, K, s);
    case 8: return launch_t<LAW, 8, MIXED>(a, K, s);
    }
    return hipErrorInvalidValue;
}

template <bool MIXED>
hipError_t launch_law(const GradArgs &a, const KConst &K, hipStream_t s) {
    switch (K.law) {
    case AFM_LAW_DMT: return launch_modes<AFM_LAW_DMT, MIXED>(a, K, s);
    case AFM_LAW_LJ: return launch_modes<AFM_LAW_LJ, MIXED>(a, K, s);
    case AFM_LAW_KV: return launch_modes<AFM_LAW_KV, MIXED>(a, K, s);
    case AFM_LAW_HOOKE: return launch_modes<AFM_LAW_HOOKE, MIXED>(a, K, s);
    case AFM_LAW_SD: return launch_modes<AFM_LAW_SD, MIXED>(a, K, s);
    case AFM_LAW_NONE: return launch_modes<AFM_LAW_NONE, MIXED>(a, K, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

size_t grad_ckpt_bytes(const afm_plan *plan, int32_t prec, int64_t n, int32_t kc) {
    const KConst &K = plan->kc;
    const size_t esz = prec == AFM_PREC_MIXED ? sizeof(float) : sizeof(double);
    const int64_t nseg = ((int64_t)K.n_cycles * K.N + kc - 1) / kc;
    return (size_t)nseg * 4 * K.nm * (size_t)n * esz;
}

bool grad_segments_ok(const afm_plan *plan) {
    return plan->kc.nm <= kSegMaxModes && plan->kc.drive_mode == AFM_DRIVE_TABLE;
}

int32_t grad_default_form(const afm_plan *plan) {
    if (plan->grad_form == kGradSweep) return kGradSweep;
    return grad_segments_ok(plan) ? kGradSegments : kGradSweep;
}

size_t grad_seg_bytes(const afm_plan *plan, int32_t prec, int64_t n, int32_t kc, int32_t form) {
    const KConst &K = plan->kc;
    if (form == kGradSegments && grad_segments_ok(plan)) {
        // per trajectory the dJ/du scale, then per segment the FP64 record
        static const int kLawNC[6] = {Law<AFM_LAW_DMT, float>::NC, Law<AFM_LAW_LJ, float>::NC,
                                      Law<AFM_LAW_KV, float>::NC, Law<AFM_LAW_HOOKE, float>::NC,
                                      Law<AFM_LAW_SD, float>::NC, Law<AFM_LAW_NONE, float>::NC};
        const int ny = 2 * K.nm, nt = ny + kLawNC[K.law] + 1;
        const int64_t nseg = ((int64_t)K.n_cycles * K.N + kc - 1) / kc;
        return ((size_t)n + (size_t)nseg * (size_t)(ny * nt + nt) * (size_t)n) * sizeof(double);
    }
    const size_t esz = prec == AFM_PREC_MIXED ? sizeof(float) : sizeof(double);
    return (size_t)kc * (2 * K.nm + 1) * (size_t)n * esz;
}

hipError_t launch_grad_p(const afm_plan *plan, int32_t prec, const GradArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (prec == AFM_PREC_MIXED) return launch_law<true>(a, plan->kc, s);
    return launch_law<false>(a, plan->kc, s);
}

hipError_t launch_grad(const afm_plan *plan, const GradArgs &a, hipStream_t s) {
    return launch_grad_p(plan, plan->precision, a, s);
}

}  // namespace afm
