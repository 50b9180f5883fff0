// forward_impl.hpp -- the forward kernels (one trajectory per lane, several per lane, one lane
// per mode, the persistent work queue) and their launchers, instantiated per force law and
// precision by the small forward_<law>_<precision>.hip units (so that the library builds in
// parallel); forward.hip holds the host-side shape tuner and the dispatch over laws.
//
// cantilever, lock-in projection and window misfit, one trajectory per lane.
//
// The paper integrates the modal equations (Eq. 2) with explicit fourth-order Runge-Kutta
// (Sec. 3.2) and evaluates the cost J_L2 (Eq. 5) for every particle of the swarm (Sec. 3.4).
// Its GPU solver gave each mode its own thread and kept modal coefficients in shared memory;
// here a whole trajectory lives in one lane's registers (state, Kahan compensation and the law's
// constants), so the hot loop touches no memory except the drive and lock-in tables (uniform
// scalar loads) and, inside the lock-in window, the measured trace.
//
// Precision: the mixed variant integrates in FP32 with a compensated (Kahan) state update, and
// accumulates window samples, lock-in sums and misfit in FP64; the plain variant is FP64
// throughout.  The drive phase comes from the integer step index (table lookup), never from an
// accumulated FP32 time.
#pragma once

#include "rk4.hpp"

namespace afm {

namespace {

struct LaneOut {
    double A, phi, J;
    int32_t st;
    int32_t used;  // periods integrated (transient + window, or up to a failure)
};


// Stroboscopic point of the orbit at a period's end (the same drive phase every time): the
// deflection u and its rate u' per unit tau (nm), FP64 with the Kahan residuals.  For a steady
// sinusoid |(u, u')| is its amplitude.
template <int NM, bool COMP, typename R>
__device__ __forceinline__ void strobe(const R (&x)[NM], const R (&v)[NM], const R (&cx)[NM],
                                       const R (&cv)[NM], double zc, double &u, double &ud) {
    u = sample<NM, COMP>(x, cx, zc);
    ud = 0.0;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        ud += (double)v[i];
        if constexpr (COMP) ud -= (double)cv[i];
    }
}

// Adaptive steady-state test at a period's end: the point moved by less than rtol of its size
// since the previous period's end (Pu, Pv, updated here).
template <int NM, bool COMP, typename R>
__device__ __forceinline__ bool steady_exit(const R (&x)[NM], const R (&v)[NM], const R (&cx)[NM],
                                            const R (&cv)[NM], double zc, double rtol, double &Pu,
                                            double &Pv) {
    double u, ud;
    strobe<NM, COMP>(x, v, cx, cv, zc, u, ud);
    const double du = u - Pu, dv = ud - Pv;
    const double d2 = __builtin_fma(du, du, dv * dv), a2 = __builtin_fma(u, u, ud * ud);
    Pu = u;
    Pv = ud;
    return d2 < rtol * rtol * a2;
}

// Integrate T trajectories of nc periods each in one lane and reduce them.  zc: separations in
// nm (FP64).  Urow: measured window traces (m) or nullptr; trow: window trace outputs (m) or
// nullptr.  With T > 1 the trajectories advance step by step side by side (independent
// instruction streams the scheduler interleaves) and share the drive-table loads; a trajectory
// that fails keeps being stepped (its results are discarded) until all have failed.  DP: the
// drive comes from the trajectory's own base-motion parameters (dv) instead of the table (one
// trajectory per lane).  EX: adaptive steady-state exit (one trajectory per lane, steady_exit):
// once a transient period's end point moved by less than K.steady_rtol of its size, the window
// starts with the next period (nc stays the cap).
template <int LAW, int NM, bool MIXED, int FM, int T, bool DP, bool EX>
__device__ __forceinline__ void integrate(
    const Law<LAW, typename std::conditional<MIXED, float, double>::type> (&law)[T],
    const double (&zc)[T], const KConst &K, int nc, const double *const (&Urow)[T],
    double *const (&trow)[T], const DriveP<typename std::conditional<MIXED, float, double>::type> &dv,
    double *const (&mcol)[T], int64_t mld, LaneOut (&o)[T]) {
    using R = typename std::conditional<MIXED, float, double>::type;
    constexpr bool COMP = MIXED;
    // kFmBlock: the four-step blocks of the transient test a bound once per block (point mass
    // with a law that has one); every other loop uses the branch-free form, which adds the same
    // terms
    constexpr bool BLK = FM == kFmBlock && NM == 1 && !DP && HasBlock<Law<LAW, R>>::value;
    constexpr int FS = FM == kFmBlock ? kFmFree : FM;
    static_assert(!DP || T == 1, "a parameter-driven base runs one trajectory per lane");
    static_assert(!EX || (T == 1 && !DP), "the adaptive exit runs one trajectory per lane");
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;
    const double *__restrict__ Lc = K.lock_c;
    const double *__restrict__ Ls = K.lock_s;

    R x[T][NM], v[T][NM], cx[T][NM], cv[T][NM], om2[NM], cd[NM], gn[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        om2[i] = (R)K.om2[i];
        cd[i] = (R)K.cdamp[i];
        gn[i] = (R)K.gain[i];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            x[t][i] = (R)(i == 0 ? zc[t] + K.y0[0] : K.y0[i]);
            v[t][i] = (R)K.y0[NM + i];
            cx[t][i] = R(0);
            cv[t][i] = R(0);
        }
    }
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h6 = (R)(K.h / 6.0);
    const int N = K.N;
    int c_win = nc - K.lockin;  // first window period (EX: moves up once the amplitude settles)
    const double lim = K.div_nm;
    double Sc[T], Ss[T], Jn[T], Jd[T];
    int32_t st[T], used[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        Sc[t] = Ss[t] = Jn[t] = Jd[t] = 0.0;
        st[t] = 0;
        used[t] = 0;
    }
    BlockBound<R> bb{};
    if constexpr (BLK) {
        // coefficients of the block bound (see BlockBound), with 2 % margin; a step too coarse
        // for the bound (denominator below 1/2) disables the skip
        const double hh = K.h, o2 = K.om2[0], c = K.cdamp[0];
        const double den = 1.0 - 16.0 * hh * hh * o2 - 4.0 * hh * c;
        const double q = den >= 0.5 ? 1.02 / den : 0.0;
        bb.c_u = (R)(o2 * q);
        bb.c_v = (R)((4.0 * hh * o2 + c) * q);
        bb.c_f = (R)q;
        bb.c_0 = den >= 0.5 ? (R)(K.dmax * q) : (R)INFINITY;
        bb.h4 = (R)(4.0 * hh * 1.02);
        bb.h16 = (R)(4.0 * hh * 1.02);
    }
    R Dc = R(0);  // DP: drive term at the start of the next step
    if constexpr (DP) Dc = dv.at(0.0);
    // EX: the stroboscopic point (u, u') of the previous period's end (first: the initial state)
    double Pu = 0.0, Pv = 0.0;
    if constexpr (EX) strobe<NM, COMP>(x[0], v[0], cx[0], cv[0], zc[0], Pu, Pv);

    for (int c = 0; c < c_win + K.lockin; ++c) {
        if (DP && c < c_win) {
            const double jb = 2.0 * ((double)c * N);
            for (int s = 0; s < N; ++s) {
                const double j = jb + 2.0 * s;
                const R D1 = dv.at(j + 1.0), D2 = dv.at(j + 2.0);
                rk4_step<NM, COMP, FS>(law[0], x[0], v[0], cx[0], cv[0], om2, cd, gn, h, h2, h6,
                                       Dc, D1, D2);
                Dc = D2;
            }
        } else if (c < c_win) {
            // blocks of four steps, each with its nine drive entries (stage times t, t + h/2,
            // ..., t + 4h: table entries 2s .. 2s + 8 for a block at step s)
            auto run4 = [&](const R (&e)[9]) {
                auto block = [&](auto fm_tag) {
                    constexpr int F = decltype(fm_tag)::value;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
#pragma unroll
                        for (int t = 0; t < T; ++t)
                            rk4_step<NM, COMP, F>(law[t], x[t], v[t], cx[t], cv[t], om2, cd, gn,
                                                  h, h2, h6, e[2 * q], e[2 * q + 1], e[2 * q + 2]);
                    }
                };
                if constexpr (BLK) {
                    bool nr = false;
#pragma unroll
                    for (int t = 0; t < T; ++t) nr = nr || law[t].near(x[t][0], v[t][0], bb);
                    if (__builtin_amdgcn_ballot_w64(nr) == 0)
                        block(std::integral_constant<int, kFmFar>());
                    else
                        block(std::integral_constant<int, FS>());
                } else {
                    block(std::integral_constant<int, FS>());
                }
            };
            int s = 0;
            if constexpr (BLK) {
                // the small-batch kernel, one wave per SIMD, nothing to hide a load behind: the
                // entries are loaded one block ahead into two alternating buffers, issued before
                // the current block's arithmetic and consumed about a thousand cycles later.
                // The compiler barrier after each group keeps the compiler from sinking the
                // loads down to their use; the address is wave-uniform (all lanes read one
                // line).  A prefetch for the block after the last reads at most entry 2N + 8,
                // inside the table's zero padding.
                auto load9 = [&](R (&f)[9], const R *dp) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) f[k] = dp[k];
                    __asm__ volatile("" ::: "memory");
                };
                static_assert(kDrivePad >= 8, "the prefetch reads 8 entries past the table");
                R fa[9], fb[9];
                const R *dp = Dt;
                load9(fa, dp);
                for (; s + 8 <= N; s += 8, dp += 16) {
                    load9(fb, dp + 8);
                    run4(fa);
                    load9(fa, dp + 16);
                    run4(fb);
                }
                if (s + 4 <= N) {  // fa holds block s
                    run4(fa);
                    s += 4;
                }
            } else {
                // many waves per SIMD hide the load: scalar loads at the top of each block (the
                // offset is wave-uniform -- readfirstlane says so where a divergent exit of the
                // enclosing loop hides it -- and the table is read-only for the kernel's
                // lifetime -- the constant address space says so where the compiler cannot
                // prove that no store of this kernel aliases it)
                using CR = const __attribute__((address_space(4))) R;
                for (; s + 4 <= N; s += 4) {
                    CR *dp = (CR *)(Dt + __builtin_amdgcn_readfirstlane(2 * s));
                    R e[9];
#pragma unroll
                    for (int k = 0; k < 9; ++k) e[k] = dp[k];
                    run4(e);
                }
            }
            for (; s < N; ++s) {
#pragma unroll
                for (int t = 0; t < T; ++t)
                    rk4_step<NM, COMP, FS>(law[t], x[t], v[t], cx[t], cv[t], om2, cd, gn, h, h2,
                                           h6, Dt[2 * s], Dt[2 * s + 1], Dt[2 * s + 2]);
            }
        } else {
            const int w0 = (c - c_win) * N;
            const double *__restrict__ Up[T];
            double Un[T];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                Up[t] = Urow[t] ? Urow[t] + w0 : nullptr;
                Un[t] = Up[t] ? Up[t][0] : 0.0;
            }
            const double jb = 2.0 * ((double)c * N);
            // the window loop is instantiated with and without the trace / modal-coordinate
            // stores, so that the common case (misfits only) has no store branches in it
            auto window = [&](auto out_tag) {
                constexpr bool OUT = decltype(out_tag)::value;
                for (int s = 0; s < N; ++s) {
                    const double lc = Lc[s + 1], ls = Ls[s + 1];
                    R D0, D1, D2;
                    if constexpr (DP) {
                        D0 = Dc;
                        D1 = dv.at(jb + 2.0 * s + 1.0);
                        D2 = dv.at(jb + 2.0 * s + 2.0);
                        Dc = D2;
                    } else {
                        D0 = Dt[2 * s];
                        D1 = Dt[2 * s + 1];
                        D2 = Dt[2 * s + 2];
                    }
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        const double Uc = Un[t];
                        if (Up[t]) Un[t] = Up[t][s + 1 < N ? s + 1 : s];
                        rk4_step<NM, COMP, FS>(law[t], x[t], v[t], cx[t], cv[t], om2, cd, gn, h,
                                               h2, h6, D0, D1, D2);
                        // explicit fmas: with contraction left to the compiler, instantiations
                        // that differ only in lanes per trajectory could round differently
                        const double u = sample<NM, COMP>(x[t], cx[t], zc[t]);
                        Sc[t] = __builtin_fma(u, lc, Sc[t]);
                        Ss[t] = __builtin_fma(u, ls, Ss[t]);
                        if (Up[t]) {
                            const double U = Uc * 1e9;
                            const double e = U - u;
                            Jn[t] = __builtin_fma(e, e, Jn[t]);
                            Jd[t] = __builtin_fma(U, U, Jd[t]);
                        }
                        if constexpr (OUT) {
                            if (trow[t]) trow[t][w0 + s] = u * 1e-9;
                            if (mcol[t]) {
                                // modal coordinates (mode 1 from the gap), for deflections
                                // elsewhere
#pragma unroll
                                for (int i = 0; i < NM; ++i) {
                                    double qi = (double)x[t][i];
                                    if constexpr (COMP) qi -= (double)cx[t][i];
                                    if (i == 0) qi -= zc[t];
                                    mcol[t][((int64_t)i * K.lockin * N + w0 + s) * mld] = qi * 1e-9;
                                }
                            }
                        }
                    }
                }
            };
            bool out = false;
#pragma unroll
            for (int t = 0; t < T; ++t) out = out || trow[t] || mcol[t];
            if (out) window(std::true_type{});
            else window(std::false_type{});
        }
        // end-of-period health check: every state entry finite and |u| within the limit
        bool alive = false;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            if (!st[t]) {
                bool fin = true;
#pragma unroll
                for (int i = 0; i < NM; ++i) fin = fin && isfinite(x[t][i]) && isfinite(v[t][i]);
                if (!fin) st[t] = AFM_ST_NONFINITE;
                else if (fabs(sample<NM, COMP>(x[t], cx[t], zc[t])) > lim) st[t] = AFM_ST_DIVERGED;
                if (st[t]) used[t] = c + 1;
            }
            alive = alive || !st[t];
        }
        if (!alive) break;
        if constexpr (EX) {
            // the transient ends after the first period whose end point moved by less than
            // steady_rtol of its size
            if (c < c_win && steady_exit<NM, COMP>(x[0], v[0], cx[0], cv[0], zc[0], K.steady_rtol,
                                                   Pu, Pv))
                c_win = c + 1;
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        o[t].st = st[t];
        o[t].used = st[t] ? used[t] : c_win + K.lockin;
        if (st[t]) {
            o[t].A = NAN;
            o[t].phi = NAN;
            o[t].J = INFINITY;
            if (trow[t])
                for (int w = 0; w < K.lockin * N; ++w) trow[t][w] = NAN;
        } else {
            const double Wn = (double)K.lockin * N;
            const double X = 2.0 * Sc[t] / Wn, Y = 2.0 * Ss[t] / Wn;
            o[t].A = ::sqrt(__builtin_fma(X, X, Y * Y)) * 1e-9;
            o[t].phi = ::atan2(-X, Y);
            const double J = Urow[t] ? Jn[t] / Jd[t] : NAN;
            o[t].J = (Urow[t] && !isfinite(J)) ? INFINITY : J;
        }
    }
}

// One lane's T trajectories ii[t] (those with act[t] false only keep the lane's time loop
// company and write nothing): parameter load, bounds checks, integration, outputs.  All T
// trajectories run nc periods.
template <int LAW, int NM, bool MIXED, int FM, int T, bool DP, bool EX>
__device__ __forceinline__ void lane_forward(const FwdArgs &A, const KConst &K,
                                             const int64_t (&ii)[T], const bool (&act)[T],
                                             int nc) {
    using R = typename std::conditional<MIXED, float, double>::type;
    const int64_t W = (int64_t)K.lockin * K.N;
    DriveP<R> dv;
    Law<LAW, R> law[T];
    double zc[T];
    const double *Urow[T];
    double *trow[T];
    double *mcol[T];
    bool bad[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t i = act[t] ? ii[t] : ii[0];
        const int64_t grp = A.group > 0 ? i / A.group : i;
        double p[kMaxParams];
        load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
        law[t] = Law<LAW, R>(p, K);
        if constexpr (DP) dv = DriveP<R>(p, K, NM);
        zc[t] = p[0] * 1e9;
        Urow[t] = nullptr;
        bad[t] = nc < K.lockin;
        if (A.targets) {
            const int64_t row = A.target_id ? (int64_t)A.target_id[grp]
                                            : (A.row_by_group ? grp : 0);
            bad[t] = bad[t] || row < 0 || row >= A.n_targets;
            Urow[t] = bad[t] ? nullptr : A.targets + row * W;
        }
        trow[t] = (A.trace && act[t]) ? A.trace + i * W : nullptr;
        mcol[t] = (A.mtrace && act[t]) ? A.mtrace + i : nullptr;
    }
    bool all_bad = true;
#pragma unroll
    for (int t = 0; t < T; ++t) all_bad = all_bad && bad[t];
    LaneOut o[T];
    if (!all_bad)
        integrate<LAW, NM, MIXED, FM, T, DP, EX>(law, zc, K, nc, Urow, trow, dv, mcol,
                                                 A.mtrace_ld, o);
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if (!act[t]) continue;
        if (bad[t]) {
            o[t].A = NAN;
            o[t].phi = NAN;
            o[t].J = INFINITY;
            o[t].st = AFM_ST_BAD_INPUT;
            o[t].used = 0;
            if (trow[t])
                for (int64_t w = 0; w < W; ++w) trow[t][w] = NAN;
        }
        const int64_t i = ii[t];
        if (A.periods) A.periods[i] = o[t].used;
        if (A.amp) A.amp[i] = o[t].A;
        if (A.phase) A.phase[i] = o[t].phi;
        if (A.J) A.J[i] = o[t].J;
        if (A.status) A.status[i] = o[t].st;
    }
}

// T trajectories per lane: lane l of block b owns b B T + t B + l, t < T (coalesced per t).
// With T > 1 the period count must be the plan's (no per-trajectory counts).  DP: the
// parameter-driven base motion (T = 1).
template <int LAW, int NM, bool MIXED, int FM, int T, bool DP = false, bool EX = false>
__global__ void __launch_bounds__(256) k_forward(const FwdArgs A, const KConst K) {
    unsigned b = blockIdx.x;
    if (A.xcd_stride > 1) {  // see launch_plain: only workgroups on one XCD do work
        if (b % (unsigned)A.xcd_stride) return;
        b /= (unsigned)A.xcd_stride;
    }
    const int64_t i0 = (int64_t)b * blockDim.x * T + threadIdx.x;
    if (i0 >= A.n) return;
    int64_t ii[T];
    bool act[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        ii[t] = i0 + (int64_t)t * blockDim.x;
        act[t] = ii[t] < A.n;
        if (A.order && act[t]) ii[t] = A.order[ii[t]];  // lane slot -> trajectory
    }
    int nc = K.n_cycles;
    if constexpr (T == 1) {
        const int64_t grp = A.group > 0 ? ii[0] / A.group : ii[0];
        if (A.n_cycles) nc = A.n_cycles[grp];
    }
    lane_forward<LAW, NM, MIXED, FM, T, DP, EX>(A, K, ii, act, nc);
}

// Mode-parallel forward: G lanes per trajectory (G = 2 for two modes, 4 for three or four, 8 for
// five to eight),
// lane q integrating mode q with the shared force (rk4_step_mp).  Same operations in the same
// order as the one-lane kernel, so the same bits; the time loops, health checks and window
// sums are group-uniform (every lane of a group sees the same gap, deflection and flags).  DP:
// the parameter-driven base, every lane of the group evaluating the same drive terms.
template <int LAW, int NM, bool MIXED, int FM, bool DP>
__device__ __forceinline__ LaneOut integrate_mp(
    const Law<LAW, typename std::conditional<MIXED, float, double>::type> &law, double zc,
    const KConst &K, int nc, const double *__restrict__ Urow, double *__restrict__ trow, int q,
    int gbase, const DriveP<typename std::conditional<MIXED, float, double>::type> &dv,
    double *__restrict__ mcol, int64_t mld) {
    using R = typename std::conditional<MIXED, float, double>::type;
    constexpr bool COMP = MIXED;
    constexpr int G = NM <= 2 ? 2 : (NM <= 4 ? 4 : 8);
    // kFmBlock: the four-step blocks of the transient test a bound once per block (a law that
    // has one); every other loop uses the branch-free form, which adds the same terms
    constexpr bool BLK = FM == kFmBlock && !DP && HasBlock<Law<LAW, R>>::value;
    constexpr int FS = FM == kFmBlock ? kFmFree : FM;
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;
    const double *__restrict__ Lc = K.lock_c;
    const double *__restrict__ Ls = K.lock_s;

    ModeLane<R> ml{R(0), R(0), R(0), R(0), R(0)};
    R x = R(0), v = R(0), cx = R(0), cv = R(0);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        if (q == i) {
            ml.om2 = (R)K.om2[i];
            ml.cd = (R)K.cdamp[i];
            ml.gn = (R)K.gain[i];
            ml.zoff = i == 0 ? law.zc : R(0);
            ml.w = R(1);
            x = (R)(i == 0 ? zc + K.y0[0] : K.y0[i]);
            v = (R)K.y0[NM + i];
        }
    }
    const ModeBound<R> mb(K, NM, q);  // this lane's share of the block bound
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h6 = (R)(K.h / 6.0);
    const int N = K.N;
    const int c_win = nc - K.lockin;
    const double lim = K.div_nm;
    double Sc = 0.0, Ss = 0.0, Jn = 0.0, Jd = 0.0;
    int32_t st = 0, used = 0;
    R Dc = R(0);  // DP: drive term at the start of the next step
    if constexpr (DP) Dc = dv.at(0.0);
    // DP: the eight new drive terms of four steps (half-steps j0 .. j0 + 7), evaluated 8 / G per
    // lane -- lane q takes j0 + q + G r -- and gathered over the group (every lane of a group
    // holds the same parameters, so any lane's evaluation is every lane's)
    auto drive8 = [&](double j0, R (&d)[8]) {
        constexpr int PER = 8 / G;
        R mine[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) mine[r] = dv.at(j0 + (double)(q + G * r));
#pragma unroll
        for (int k = 0; k < 8; ++k) d[k] = __shfl(mine[k / G], gbase + k % G, 64);
    };

    for (int c = 0; c < nc; ++c) {
        if (DP && c < c_win) {
            const double jb = 2.0 * ((double)c * N);
            int s = 0;
            for (; s + 4 <= N; s += 4) {
                R d[8];
                drive8(jb + 2.0 * s + 1.0, d);
                rk4_step_mp<NM, G, COMP, FS>(law, ml, x, v, cx, cv, h, h2, h6, Dc, d[0], d[1]);
                rk4_step_mp<NM, G, COMP, FS>(law, ml, x, v, cx, cv, h, h2, h6, d[1], d[2], d[3]);
                rk4_step_mp<NM, G, COMP, FS>(law, ml, x, v, cx, cv, h, h2, h6, d[3], d[4], d[5]);
                rk4_step_mp<NM, G, COMP, FS>(law, ml, x, v, cx, cv, h, h2, h6, d[5], d[6], d[7]);
                Dc = d[7];
            }
            for (; s < N; ++s) {
                const double j = jb + 2.0 * s;
                const R D1 = dv.at(j + 1.0), D2 = dv.at(j + 2.0);
                rk4_step_mp<NM, G, COMP, FS>(law, ml, x, v, cx, cv, h, h2, h6, Dc, D1, D2);
                Dc = D2;
            }
        } else if (c < c_win) {
            int s = 0;
            for (; s + 4 <= N; s += 4) {
                using CR = const __attribute__((address_space(4))) R;
                CR *dp = (CR *)(Dt + __builtin_amdgcn_readfirstlane(2 * s));
                const R e0 = dp[0], e1 = dp[1], e2 = dp[2], e3 = dp[3], e4 = dp[4], e5 = dp[5],
                        e6 = dp[6], e7 = dp[7], e8 = dp[8];
                auto block = [&](auto fm_tag) {
                    constexpr int F = decltype(fm_tag)::value;
                    rk4_step_mp<NM, G, COMP, F>(law, ml, x, v, cx, cv, h, h2, h6, e0, e1, e2);
                    rk4_step_mp<NM, G, COMP, F>(law, ml, x, v, cx, cv, h, h2, h6, e2, e3, e4);
                    rk4_step_mp<NM, G, COMP, F>(law, ml, x, v, cx, cv, h, h2, h6, e4, e5, e6);
                    rk4_step_mp<NM, G, COMP, F>(law, ml, x, v, cx, cv, h, h2, h6, e6, e7, e8);
                };
                bool far = false;
                if constexpr (BLK) far = group_far<G>(law, ml, mb, x, v);
                if (far) block(std::integral_constant<int, kFmFar>());
                else block(std::integral_constant<int, FS>());
            }
            for (; s < N; ++s)
                rk4_step_mp<NM, G, COMP, FS>(law, ml, x, v, cx, cv, h, h2, h6, Dt[2 * s],
                                             Dt[2 * s + 1], Dt[2 * s + 2]);
        } else {
            const int w0 = (c - c_win) * N;
            const double *__restrict__ Up = Urow ? Urow + w0 : nullptr;
            double Un = Up ? Up[0] : 0.0;
            // one window step: RK4, sample, lock-in and misfit sums, and (OUT) the trace and
            // modal-coordinate stores; the loops are instantiated with and without the stores so
            // that the common case (misfits only) has no store branches in them
            auto wstep = [&](auto out_tag, int s, R D0, R D1, R D2) {
                constexpr bool OUT = decltype(out_tag)::value;
                const double Uc = Un;
                if (Up) Un = Up[s + 1 < N ? s + 1 : s];
                rk4_step_mp<NM, G, COMP, FS>(law, ml, x, v, cx, cv, h, h2, h6, D0, D1, D2);
                const double u = sample_mp<NM, COMP>(x, cx, zc, gbase);
                Sc = __builtin_fma(u, Lc[s + 1], Sc);
                Ss = __builtin_fma(u, Ls[s + 1], Ss);
                if (Up) {
                    const double U = Uc * 1e9;
                    const double e = U - u;
                    Jn = __builtin_fma(e, e, Jn);
                    Jd = __builtin_fma(U, U, Jd);
                }
                if constexpr (OUT) {
                    if (trow && q == 0) trow[w0 + s] = u * 1e-9;
                    if (mcol && q < NM) {  // this lane's modal coordinate (mode 1 from the gap)
                        double qi = (double)x;
                        if constexpr (COMP) qi -= (double)cx;
                        if (q == 0) qi -= zc;
                        mcol[((int64_t)q * K.lockin * N + w0 + s) * mld] = qi * 1e-9;
                    }
                }
            };
            auto window = [&](auto out_tag) {
                if constexpr (DP) {
                    const double jb = 2.0 * ((double)c * N);
                    int s = 0;
                    for (; s + 4 <= N; s += 4) {
                        R d[8];
                        drive8(jb + 2.0 * s + 1.0, d);
                        wstep(out_tag, s, Dc, d[0], d[1]);
                        wstep(out_tag, s + 1, d[1], d[2], d[3]);
                        wstep(out_tag, s + 2, d[3], d[4], d[5]);
                        wstep(out_tag, s + 3, d[5], d[6], d[7]);
                        Dc = d[7];
                    }
                    for (; s < N; ++s) {
                        const R D1 = dv.at(jb + 2.0 * s + 1.0), D2 = dv.at(jb + 2.0 * s + 2.0);
                        wstep(out_tag, s, Dc, D1, D2);
                        Dc = D2;
                    }
                } else {
                    for (int s = 0; s < N; ++s)
                        wstep(out_tag, s, Dt[2 * s], Dt[2 * s + 1], Dt[2 * s + 2]);
                }
            };
            if (trow || mcol) window(std::true_type{});
            else window(std::false_type{});
        }
        // end-of-period health check, combined over the group
        int nonfinite = !(isfinite(x) && isfinite(v));
        nonfinite |= __shfl_xor(nonfinite, 1, 64);
        if constexpr (G >= 4) nonfinite |= __shfl_xor(nonfinite, 2, 64);
        if constexpr (G == 8) nonfinite |= __shfl_xor(nonfinite, 4, 64);
        if (nonfinite) {
            st = AFM_ST_NONFINITE;
            used = c + 1;
            break;
        }
        if (fabs(sample_mp<NM, COMP>(x, cx, zc, gbase)) > lim) {
            st = AFM_ST_DIVERGED;
            used = c + 1;
            break;
        }
    }
    LaneOut o;
    o.st = st;
    o.used = st ? used : nc;
    if (st) {
        o.A = NAN;
        o.phi = NAN;
        o.J = INFINITY;
        if (trow && q == 0)
            for (int w = 0; w < K.lockin * N; ++w) trow[w] = NAN;
    } else {
        const double Wn = (double)K.lockin * N;
        const double X = 2.0 * Sc / Wn, Y = 2.0 * Ss / Wn;
        o.A = ::sqrt(__builtin_fma(X, X, Y * Y)) * 1e-9;
        o.phi = ::atan2(-X, Y);
        const double J = Urow ? Jn / Jd : NAN;
        o.J = (Urow && !isfinite(J)) ? INFINITY : J;
    }
    return o;
}

// G lanes per trajectory; the block size is a multiple of 8, so groups never straddle a
// workgroup and every lane of a group exits together.
template <int LAW, int NM, bool MIXED, int FM, bool DP = false>
__global__ void __launch_bounds__(256) k_forward_mp(const FwdArgs A, const KConst K) {
    using R = typename std::conditional<MIXED, float, double>::type;
    constexpr int G = NM <= 2 ? 2 : (NM <= 4 ? 4 : 8);
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= A.n) return;
    const int q = threadIdx.x & (G - 1);
    const int gbase = (int)(threadIdx.x & 63) & ~(G - 1);
    const int64_t grp = A.group > 0 ? i / A.group : i;
    int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    const Law<LAW, R> law(p, K);
    DriveP<R> dv;
    if constexpr (DP) dv = DriveP<R>(p, K, NM);
    const int64_t W = (int64_t)K.lockin * K.N;
    const double *Urow = nullptr;
    bool bad = nc < K.lockin;
    if (A.targets) {
        const int64_t row = A.target_id ? (int64_t)A.target_id[grp] : (A.row_by_group ? grp : 0);
        bad = bad || row < 0 || row >= A.n_targets;
        Urow = bad ? nullptr : A.targets + row * W;
    }
    double *trow = A.trace ? A.trace + i * W : nullptr;
    LaneOut o;
    if (bad) {
        o.A = NAN;
        o.phi = NAN;
        o.J = INFINITY;
        o.st = AFM_ST_BAD_INPUT;
        o.used = 0;
        if (trow && q == 0)
            for (int64_t w = 0; w < W; ++w) trow[w] = NAN;
    } else {
        o = integrate_mp<LAW, NM, MIXED, FM, DP>(law, p[0] * 1e9, K, nc, Urow, trow, q, gbase,
                                                 dv, A.mtrace ? A.mtrace + i : nullptr,
                                                 A.mtrace_ld);
    }
    if (q == 0) {
        if (A.amp) A.amp[i] = o.A;
        if (A.phase) A.phase[i] = o.phi;
        if (A.J) A.J[i] = o.J;
        if (A.status) A.status[i] = o.st;
        if (A.periods) A.periods[i] = o.used;
    }
}

// Persistent work queue for batches of groups with uneven period counts (one pixel's swarm is
// one group).  Each wavefront repeatedly takes the next item -- 64 lanes of one group -- from a
// queue ordered longest first, until the queue is empty; every wave reaches the exit.  The
// group's period count is the same for all lanes of an item, so it is moved to a scalar
// register and the time loops run as uniform scalar loops.
template <int LAW, int NM, bool MIXED, int FM, bool EX = false>
__global__ void __launch_bounds__(256) k_forward_queue(const FwdArgs A, const KConst K) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(A.head, 1);
        item = __shfl(item, 0, 64);
        if (item >= A.n_items) break;
        const int id = A.items[item];
        const int64_t grp = id / A.chunks;
        const int64_t local = (int64_t)(id % A.chunks) * 64 + lane;
        int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
        nc = __builtin_amdgcn_readfirstlane(nc);
        if (local < A.group) {
            int64_t ti = grp * A.group + local;
            if (A.order) ti = A.order[ti];  // lane slot -> trajectory of the same swarm
            const int64_t ii[1] = {ti};
            const bool act[1] = {true};
            lane_forward<LAW, NM, MIXED, FM, 1, false, EX>(A, K, ii, act, nc);
        }
    }
}

// Persistent lane-refill kernel for the adaptive steady-state exit on uneven batches (the
// work-queue batches of afm_invert).  With the exit, trajectories end at their own periods, so a
// wave that kept its 64 trajectories would run until the slowest of them settled.  Here every
// lane owns one trajectory at a time: at each period boundary the lanes whose trajectory has
// finished take the next trajectories of the longest-first order (one atomic per wave, ranks by
// ballot), so the waves stay full until the work runs out, and every wave leaves once no lane has
// work and the order is exhausted.  All lanes of a wave step in period lock-step (same step
// index, so the drive loads stay uniform); a lane's transient periods are plain RK4 steps with
// the steady-state test at their ends, its window periods add the lock-in and misfit terms.
// Per trajectory the arithmetic is that of the one-lane kernel with the exit (k_forward<..., EX>,
// whose branch-free law form adds the same terms as the skip form used here), so the results are
// the same bits.
template <int LAW, int NM, bool MIXED>
__global__ void __launch_bounds__(256) k_forward_lanes(const FwdArgs A, const KConst K) {
    using R = typename std::conditional<MIXED, float, double>::type;
    constexpr bool COMP = MIXED;
    // the wave-uniform contact skip (the lanes of a wave step in period lock-step, so their
    // contacts cluster in the same part of the drive period); it adds the same terms as the
    // branch-free form of the one-lane kernel
    constexpr int FM = Law<LAW, float>::kBranch ? kFmSkip : kFmFree;
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;
    const double *__restrict__ Lc = K.lock_c;
    const double *__restrict__ Ls = K.lock_s;
    const int lane = threadIdx.x & 63;
    const int N = K.N, L = K.lockin;
    const int64_t W = (int64_t)L * N;
    const int64_t total = (int64_t)A.n_items * 64;
    R om2[NM], cd[NM], gn[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        om2[m] = (R)K.om2[m];
        cd[m] = (R)K.cdamp[m];
        gn[m] = (R)K.gain[m];
    }
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h6 = (R)(K.h / 6.0);

    // this lane's trajectory
    int64_t i = -1;      // trajectory index, -1: none
    bool fetch = true;   // the lane needs a trajectory
    bool exhausted = false;
    int c = 0, c_win = 0, nc = 0;
    double zc = 0.0, Pu = 0.0, Pv = 0.0, Pc = 0.0, Ps = 0.0, Jn = 0.0, Jd = 0.0;
    const double *Urow = nullptr;
    Law<LAW, R> law;
    R x[NM], v[NM], cx[NM], cv[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) x[m] = v[m] = cx[m] = cv[m] = R(0);

    auto finish = [&](double Aout, double phi, double J, int32_t st, int32_t used) {
        if (A.amp) A.amp[i] = Aout;
        if (A.phase) A.phase[i] = phi;
        if (A.J) A.J[i] = J;
        if (A.status) A.status[i] = st;
        if (A.periods) A.periods[i] = used;
    };

    for (;;) {
        // refill: lanes without a trajectory take the next ones in order (padding entries of a
        // swarm's last chunk and bad inputs are passed over)
        for (;;) {
            const uint64_t need = __ballot(fetch && !exhausted);
            if (need == 0) break;
            const int first = __ffsll((unsigned long long)need) - 1;
            const int cnt = __popcll(need);
            int base = 0;
            if (lane == first) base = atomicAdd(A.head, cnt);
            base = __shfl(base, first, 64);
            if (fetch && !exhausted) {
                const int64_t t = (int64_t)base + __popcll(need & ((1ull << lane) - 1ull));
                if (t < total) {
                    const int id = A.items[t >> 6];
                    const int64_t grp = id / A.chunks;
                    const int64_t local = (int64_t)(id % A.chunks) * 64 + (t & 63);
                    if (local < A.group) {
                        i = grp * A.group + local;
                        nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
                        const int64_t row = A.target_id ? (int64_t)A.target_id[grp]
                                                        : (A.row_by_group ? grp : 0);
                        if (nc < L || row < 0 || row >= A.n_targets) {
                            finish(NAN, NAN, INFINITY, AFM_ST_BAD_INPUT, 0);
                        } else {
                            double p[kMaxParams];
                            load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
                            law = Law<LAW, R>(p, K);
                            zc = p[0] * 1e9;
                            Urow = A.targets + row * W;
#pragma unroll
                            for (int m = 0; m < NM; ++m) {
                                x[m] = (R)(m == 0 ? zc + K.y0[0] : K.y0[m]);
                                v[m] = (R)K.y0[NM + m];
                                cx[m] = R(0);
                                cv[m] = R(0);
                            }
                            c = 0;
                            c_win = nc - L;
                            strobe<NM, COMP>(x, v, cx, cv, zc, Pu, Pv);
                            Jn = Jd = 0.0;
                            fetch = false;
                        }
                    }
                }
            }
            if ((int64_t)base + cnt >= total) exhausted = true;  // the same for every lane
        }
        const bool act = !fetch;
        if (__ballot(act) == 0) break;  // no lane has work and the order is exhausted

        // one period for every lane with a trajectory
        if (act) {
            const bool inwin = c >= c_win;
            if (c == c_win) Pc = Ps = 0.0;
            const int64_t w0 = inwin ? (int64_t)(c - c_win) * N : 0;
            // the window's lock-in and misfit terms, for the lanes in their window only
            auto book = [&](int s) {
                if (inwin) {
                    const double u = sample<NM, COMP>(x, cx, zc);
                    Pc = __builtin_fma(u, Lc[s + 1], Pc);
                    Ps = __builtin_fma(u, Ls[s + 1], Ps);
                    const double U = Urow[w0 + s] * 1e9;
                    const double e = U - u;
                    Jn = __builtin_fma(e, e, Jn);
                    Jd = __builtin_fma(U, U, Jd);
                }
            };
            int s = 0;
            for (; s + 4 <= N; s += 4) {
                using CR = const __attribute__((address_space(4))) R;
                CR *dp = (CR *)(Dt + __builtin_amdgcn_readfirstlane(2 * s));
                const R e0 = dp[0], e1 = dp[1], e2 = dp[2], e3 = dp[3], e4 = dp[4], e5 = dp[5],
                        e6 = dp[6], e7 = dp[7], e8 = dp[8];
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, e0, e1, e2);
                book(s);
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, e2, e3, e4);
                book(s + 1);
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, e4, e5, e6);
                book(s + 2);
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, e6, e7, e8);
                book(s + 3);
            }
            for (; s < N; ++s) {
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, Dt[2 * s],
                                            Dt[2 * s + 1], Dt[2 * s + 2]);
                book(s);
            }
            // end of the period: health, the exit test, or the window's end
            bool fin = true;
#pragma unroll
            for (int m = 0; m < NM; ++m) fin = fin && isfinite(x[m]) && isfinite(v[m]);
            int32_t st = 0;
            if (!fin) st = AFM_ST_NONFINITE;
            else if (fabs(sample<NM, COMP>(x, cx, zc)) > K.div_nm) st = AFM_ST_DIVERGED;
            if (st) {
                finish(NAN, NAN, INFINITY, st, c + 1);
                fetch = true;
            } else if (!inwin) {
                if (steady_exit<NM, COMP>(x, v, cx, cv, zc, K.steady_rtol, Pu, Pv)) c_win = c + 1;
            } else if (c == c_win + L - 1) {
                const double X = 2.0 * Pc / (double)W, Y = 2.0 * Ps / (double)W;
                const double J = Jn / Jd;
                finish(::sqrt(__builtin_fma(X, X, Y * Y)) * 1e-9, ::atan2(-X, Y),
                       isfinite(J) ? J : INFINITY, 0, c + 1);
                fetch = true;
            }
            ++c;
        }
    }
}

__global__ void k_queue_reset(int32_t *head) {
    if (threadIdx.x == 0) *head = 0;
}

// Force-law form by regime (not tuned: the per-lane branching form rounds the in-contact
// attraction differently, and tuning must never change results).  Small batches (fewer waves
// than SIMDs) are issue-latency bound: the branch-free form (with the block-level test for a
// point mass) needs the fewest issue slots.  Large batches are throughput bound: the per-stage
// skip for FP32 point-mass DMT (the small batches' bits), else the per-lane branch (fewer
// transcendental ops; other waves hide its scalar instructions).

// Workgroups are handed to the 8 XCDs in turn (workgroup b to XCD b mod 8), each XCD with its
// own L2 and 32 CUs.  A launch of at most 32 workgroups is issue-latency bound on as many CUs
// wherever it runs, so it is dispatched as 8x the workgroups of which every 8th works: all the
// working ones then sit on one XCD and read the trajectories' shared data (the target window,
// the drive and lock-in tables) through one L2 instead of eight.
constexpr int kXcds = 8;
constexpr int kCusPerXcd = 32;

// Lane order of a small batch: the law's contact key of every trajectory (NaN ordered last) ...
template <int LAW>
__global__ void __launch_bounds__(256) k_order_keys(const FwdArgs A, const KConst K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    const double k = Law<LAW, double>::contact_key(p);
    A.key_buf[i] = k == k ? k : INFINITY;
}

// ... and its rank: order[rank(i)] = i, ranks by (key, index), so ties (and infinities) keep
// their index order and the ranks are a permutation of 0 .. n - 1.  Keys pass through LDS in
// tiles of the workgroup's size; every lane of a workgroup takes part in every tile.
__global__ void __launch_bounds__(256) k_order_rank(int32_t n, const double *keys, int32_t *order) {
    // the keys compared in FP32 (a coarser key only adds ties, which the index breaks)
    __shared__ float tile[256];
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const float ki = i < n ? (float)keys[i] : 0.0f;
    int32_t r = 0;
    for (int32_t b0 = 0; b0 < n; b0 += 256) {
        const int32_t j = b0 + (int32_t)threadIdx.x;
        tile[threadIdx.x] = j < n ? (float)keys[j] : INFINITY;
        __syncthreads();
        // a full tile of 256: padding entries are +inf at indices >= n, above every lane's
        // index, so no padding entry is ordered before a lane
        const int32_t below = i - b0;  // tile entries k < below have a lower index than lane i
#pragma unroll 16
        for (int32_t k = 0; k < 256; ++k) {
            const float kj = tile[k];
            r += (kj < ki || (kj == ki && k < below)) ? 1 : 0;
        }
        __syncthreads();
    }
    if (i < n) order[r] = i;
}

// Lane order within each swarm of a work-queue batch: order[g seg + rank] = i for the
// trajectories i of swarm g (segment [g seg, (g + 1) seg)), ranked by (key, index) like
// k_order_rank.  The segment's keys are read by every lane of a wave alike.
__global__ void __launch_bounds__(256) k_order_rank_seg(int64_t n, int32_t seg, const double *keys,
                                                       int32_t *order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t g0 = i / seg * seg;
    const int64_t g1 = g0 + seg < n ? g0 + seg : n;
    const double ki = keys[i];
    int32_t r = 0;
    for (int64_t j = g0; j < g1; ++j) {
        const double kj = keys[j];
        r += (kj < ki || (kj == ki && j < i)) ? 1 : 0;
    }
    order[g0 + r] = (int32_t)i;
}

// Plain launch with a given shape: `block` lanes per workgroup, `tpl` trajectories per lane.
template <int LAW, int NM, bool MIXED>
hipError_t launch_plain(const FwdArgs &a0, const KConst &K, FwdShape sh, hipStream_t s) {
    constexpr bool branchy = Law<LAW, float>::kBranch;
    // GPU-filling batches (several waves share each SIMD, which hides a wave's stalls): FP32
    // point-mass DMT skips the contact piece per RK4 stage when no lane of the wave is near
    // contact (the bits of the smaller batches' forms; 257 vs 294 ms for the per-lane branch on
    // 524,288 pixel trajectories of 100-2000 periods, 9.3 vs 9.1 ms on a 40-period batch that
    // is all transient); the other laws with a contact branch, and FP64, branch per lane
    constexpr int kLargeFm = MIXED && NM == 1 && LAW == AFM_LAW_DMT ? kFmSkip : kFmBranch;
    const dim3 blk((unsigned)sh.block);
    const bool large = branchy && a0.n >= kSmallBatch;
    if constexpr (NM > 1) {
        if (sh.tpl == 0) {  // mode-parallel: G lanes per trajectory
            constexpr int G = NM <= 2 ? 2 : (NM <= 4 ? 4 : 8);
            const int64_t per = sh.block / G;
            const dim3 g2((unsigned)((a0.n + per - 1) / per));
            // small batches: the block-level contact test where the law has a bound
            constexpr int kMpFm =
                HasBlock<Law<LAW, typename std::conditional<MIXED, float, double>::type>>::value
                    ? kFmBlock
                    : kFmFree;
            if (large) hipLaunchKernelGGL((k_forward_mp<LAW, NM, MIXED, kFmBranch>), g2, blk, 0, s, a0, K);
            else hipLaunchKernelGGL((k_forward_mp<LAW, NM, MIXED, kMpFm>), g2, blk, 0, s, a0, K);
            return hipGetLastError();
        }
    }
    const int64_t per_block = (int64_t)sh.block * sh.tpl;
    const int64_t nb = (a0.n + per_block - 1) / per_block;
    FwdArgs a = a0;
    a.xcd_stride = nb <= kCusPerXcd ? kXcds : 1;
    if constexpr (NM == 1 &&
                  HasBlock<Law<LAW, typename std::conditional<MIXED, float, double>::type>>::value) {
        // the block-level contact test runs a block without the contact piece only when no lane
        // of the wave can reach contact in it: waves of trajectories ordered by contact key
        // (similar stiffness, similar tapping phase) clear the test in more blocks.  Only the
        // assignment of trajectories to lanes changes, never a result.
        if (!large && a0.order_buf && a0.key_buf && a0.n > 64 && a0.n <= kOrderMax) {
            const dim3 g((unsigned)((a0.n + 255) / 256));
            hipLaunchKernelGGL((k_order_keys<LAW>), g, dim3(256), 0, s, a0, K);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_order_rank, g, dim3(256), 0, s, (int32_t)a0.n,
                               (const double *)a0.key_buf, a0.order_buf);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            a.order = a0.order_buf;
        }
    }
    const dim3 grid((unsigned)(nb * a.xcd_stride));
    if constexpr (NM == 1) {
        if (sh.tpl == 2) {
            if (large) hipLaunchKernelGGL((k_forward<LAW, NM, MIXED, kLargeFm, 2>), grid, blk, 0, s, a, K);
            else hipLaunchKernelGGL((k_forward<LAW, NM, MIXED, kFmBlock, 2>), grid, blk, 0, s, a, K);
            return hipGetLastError();
        }
    }
    if (large) hipLaunchKernelGGL((k_forward<LAW, NM, MIXED, kLargeFm, 1>), grid, blk, 0, s, a, K);
    else hipLaunchKernelGGL((k_forward<LAW, NM, MIXED, kFmBlock, 1>), grid, blk, 0, s, a, K);
    return hipGetLastError();
}

// Parameter-driven base (branch-free law form): `sh.tpl` 0 = one lane per mode, else one
// trajectory per lane.
template <int LAW, int NM, bool MIXED>
hipError_t launch_dp(const FwdArgs &a, const KConst &K, FwdShape sh, hipStream_t s) {
    if constexpr (NM > 1) {
        if (sh.tpl == 0) {
            constexpr int G = NM <= 2 ? 2 : (NM <= 4 ? 4 : 8);
            const int64_t per = sh.block / G;
            hipLaunchKernelGGL((k_forward_mp<LAW, NM, MIXED, kFmFree, true>),
                               dim3((unsigned)((a.n + per - 1) / per)), dim3(sh.block), 0, s, a, K);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_forward<LAW, NM, MIXED, kFmFree, 1, true>),
                       dim3((unsigned)((a.n + sh.block - 1) / sh.block)), dim3(sh.block), 0, s, a,
                       K);
    return hipGetLastError();
}

template <int LAW, int NM, bool MIXED>
hipError_t launch_t(const afm_plan *plan, const FwdArgs &a, const KConst &K, hipStream_t s) {
    constexpr bool branchy = Law<LAW, float>::kBranch;
    if (K.steady_rtol > 0.0) {
        // adaptive steady-state exit: one trajectory per lane (each lane leaves its transient
        // when its own amplitude settles), not tuned; work-queue batches refill lanes as their
        // trajectories finish
        // (the lane kernel keeps no window traces; its order counter stays far from overflow)
        if (a.items && a.targets && !a.trace && !a.mtrace &&
            (int64_t)a.n_items * 64 < ((int64_t)1 << 30)) {
            hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, a.head);
            const unsigned blocks = (unsigned)(plan->n_cu > 0 ? plan->n_cu : 256) * 4;
            hipLaunchKernelGGL((k_forward_lanes<LAW, NM, MIXED>), dim3(blocks), dim3(256), 0, s,
                               a, K);
            return hipGetLastError();
        }
        const int block = a.n < kSmallBatch ? 64 : 256;
        hipLaunchKernelGGL((k_forward<LAW, NM, MIXED, kFmFree, 1, false, true>),
                           dim3((unsigned)((a.n + block - 1) / block)), dim3(block), 0, s, a, K);
        return hipGetLastError();
    }
    if (K.drive_mode != AFM_DRIVE_TABLE) {
        // parameter-driven base: one trajectory per lane or one lane per mode, tuned like the
        // fixed-drive shapes; a work-queue batch runs as a plain grid (per-group period counts
        // are read per lane)
        FwdShape sh;
        hipError_t e = forward_shape(
            plan, MIXED ? AFM_PREC_MIXED : AFM_PREC_FP64, a, NM, s,
            [&](FwdShape c) { return launch_dp<LAW, NM, MIXED>(a, K, c, s); }, &sh);
        if (e != hipSuccess) return e;
        return launch_dp<LAW, NM, MIXED>(a, K, sh, s);
    }
    if (a.items) {
        // persistent grid: 4 waves per SIMD on every CU.  All lanes of a wave belong to one
        // swarm (one separation), so they enter contact together: the wave-uniform skip form,
        // tested per stage (measured 11 % faster here than the per-lane branching form, 19 %
        // faster than the four-step block test, whose bound is conservative, and 8 % faster
        // than the block test with per-stage skips inside the blocks near contact; with four
        // waves per SIMD the other waves hide each stage test's branch)
        FwdArgs aq = a;
        if constexpr (NM == 1 && HasBlock<Law<LAW, float>>::value) {
            // the skip form leaves the contact piece out of a stage only when no lane of the
            // wave is near contact: within each swarm, the particles go to lanes in
            // contact-key order, so that a wave holds particles of similar stiffness
            if (a.order_buf && a.key_buf && a.group > 64) {
                const dim3 g((unsigned)((a.n + 255) / 256));
                hipLaunchKernelGGL((k_order_keys<LAW>), g, dim3(256), 0, s, a, K);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(k_order_rank_seg, g, dim3(256), 0, s, a.n, a.group,
                                   (const double *)a.key_buf, a.order_buf);
                e = hipGetLastError();
                if (e != hipSuccess) return e;
                aq.order = a.order_buf;
            }
        }
        hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, a.head);
        const int n_cu = plan->n_cu > 0 ? plan->n_cu : 256;
        const unsigned blocks = (unsigned)n_cu * 4;
        if constexpr (NM == 1 && HasBlock<Law<LAW, float>>::value) {
            // no more items than SIMDs: a wave per SIMD at most, where the per-stage branch
            // stalls a lone wave and the block-level test runs far blocks without it (the same
            // bits; see launch_plain)
            if ((int64_t)a.n_items <= (int64_t)n_cu * 4) {
                hipLaunchKernelGGL((k_forward_queue<LAW, NM, MIXED, kFmBlock>), dim3(blocks),
                                   dim3(256), 0, s, aq, K);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_forward_queue<LAW, NM, MIXED, branchy ? kFmSkip : kFmFree>),
                           dim3(blocks), dim3(256), 0, s, aq, K);
        return hipGetLastError();
    }
    FwdArgs ao = a;  // the plan's lane-order buffers for small batches
    ao.order_buf = plan->d_order;
    ao.key_buf = plan->d_order_keys;
    FwdShape sh;
    hipError_t e = forward_shape(plan, MIXED ? AFM_PREC_MIXED : AFM_PREC_FP64, ao, NM, s,
                                 [&](FwdShape c) { return launch_plain<LAW, NM, MIXED>(ao, K, c, s); },
                                 &sh);
    if (e != hipSuccess) return e;
    return launch_plain<LAW, NM, MIXED>(ao, K, sh, s);
}

template <int LAW, bool MIXED>
hipError_t launch_modes(const afm_plan *plan, const FwdArgs &a, const KConst &K, hipStream_t s) {
    switch (K.nm) {
    case 1: return launch_t<LAW, 1, MIXED>(plan, a, K, s);
    case 2: return launch_t<LAW, 2, MIXED>(plan, a, K, s);
    case 3: return launch_t<LAW, 3, MIXED>(plan, a, K, s);
    case 4: return launch_t<LAW, 4, MIXED>(plan, a, K, s);
    case 5: return launch_t<LAW, 5, MIXED>(plan, a, K, s);
    case 6: return launch_t<LAW, 6, MIXED>(plan, a, K, s);
    case 7: return launch_t<LAW, 7, MIXED>(plan, a, K, s);
    case 8: return launch_t<LAW, 8, MIXED>(plan, a, K, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// Launch of the forward kernel for one force law and precision (explicitly instantiated in the
// forward_<law>_<precision>.hip units).
template <int LAW, bool MIXED>
hipError_t launch_fwd_law(const afm_plan *plan, const FwdArgs &a, const KConst &K, hipStream_t s) {
    return launch_modes<LAW, MIXED>(plan, a, K, s);
}

}  // namespace afm
