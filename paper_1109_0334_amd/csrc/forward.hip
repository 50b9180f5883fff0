// forward.hip -- batched forward solve: RK4 time integration of the base-driven modal
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
#include "rk4.hpp"

namespace afm {

namespace {

struct LaneOut {
    double A, phi, J;
    int32_t st;
};

// Integrate one trajectory of nc periods and reduce it.  zc: separation in nm (FP64).
// Urow: measured window trace (m) or nullptr; trow: window trace output (m) or nullptr.
template <int LAW, int NM, bool MIXED, int FM>
__device__ __forceinline__ LaneOut integrate(
    const Law<LAW, typename std::conditional<MIXED, float, double>::type> &law, double zc,
    const KConst &K, int nc, const double *__restrict__ Urow, double *__restrict__ trow) {
    using R = typename std::conditional<MIXED, float, double>::type;
    constexpr bool COMP = MIXED;
    const R *__restrict__ Dt;
    if constexpr (MIXED) Dt = K.drive_f;
    else Dt = K.drive_d;
    const double *__restrict__ Lc = K.lock_c;
    const double *__restrict__ Ls = K.lock_s;

    R x[NM], v[NM], cx[NM], cv[NM], om2[NM], cd[NM], gn[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        x[i] = (R)(i == 0 ? zc + K.y0[0] : K.y0[i]);
        v[i] = (R)K.y0[NM + i];
        cx[i] = R(0);
        cv[i] = R(0);
        om2[i] = (R)K.om2[i];
        cd[i] = (R)K.cdamp[i];
        gn[i] = (R)K.gain[i];
    }
    const R h = (R)K.h, h2 = (R)(0.5 * K.h), h6 = (R)(K.h / 6.0);
    const int N = K.N;
    const int c_win = nc - K.lockin;
    const double lim = K.div_nm;
    double Sc = 0.0, Ss = 0.0, Jn = 0.0, Jd = 0.0;
    int32_t st = 0;

    for (int c = 0; c < nc; ++c) {
        if (c < c_win) {
            // four steps per pass: their nine drive entries (stage times t, t + h/2, ..., t + 4h)
            // come in as one block of uniform loads
            int s = 0;
            for (; s + 4 <= N; s += 4) {
                // scalar loads: s is wave-uniform (readfirstlane says so where a divergent exit
                // of the enclosing loop hides it) and the table is read-only for the kernel's
                // lifetime (the constant address space says so where the compiler cannot prove
                // that no store of this kernel aliases it)
                using CR = const __attribute__((address_space(4))) R;
                CR *dp = (CR *)(Dt + __builtin_amdgcn_readfirstlane(2 * s));
                const R e0 = dp[0], e1 = dp[1], e2 = dp[2], e3 = dp[3], e4 = dp[4], e5 = dp[5],
                        e6 = dp[6], e7 = dp[7], e8 = dp[8];
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, e0, e1, e2);
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, e2, e3, e4);
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, e4, e5, e6);
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, e6, e7, e8);
            }
            for (; s < N; ++s)
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, Dt[2 * s],
                                       Dt[2 * s + 1], Dt[2 * s + 2]);
        } else {
            const int w0 = (c - c_win) * N;
            const double *__restrict__ Up = Urow ? Urow + w0 : nullptr;
            double Un = Up ? Up[0] : 0.0;
            for (int s = 0; s < N; ++s) {
                const double Uc = Un;
                if (Up) Un = Up[s + 1 < N ? s + 1 : s];
                rk4_step<NM, COMP, FM>(law, x, v, cx, cv, om2, cd, gn, h, h2, h6, Dt[2 * s],
                                       Dt[2 * s + 1], Dt[2 * s + 2]);
                const double u = sample<NM, COMP>(x, cx, zc);
                Sc += u * Lc[s + 1];
                Ss += u * Ls[s + 1];
                if (Up) {
                    const double U = Uc * 1e9;
                    const double e = U - u;
                    Jn += e * e;
                    Jd += U * U;
                }
                if (trow) trow[w0 + s] = u * 1e-9;
            }
        }
        // end-of-period health check: every state entry finite and |u| within the limit
        bool fin = true;
#pragma unroll
        for (int i = 0; i < NM; ++i) fin = fin && isfinite(x[i]) && isfinite(v[i]);
        if (!fin) {
            st = AFM_ST_NONFINITE;
            break;
        }
        if (fabs(sample<NM, COMP>(x, cx, zc)) > lim) {
            st = AFM_ST_DIVERGED;
            break;
        }
    }
    LaneOut o;
    o.st = st;
    if (st) {
        o.A = NAN;
        o.phi = NAN;
        o.J = INFINITY;
        if (trow)
            for (int w = 0; w < K.lockin * N; ++w) trow[w] = NAN;
    } else {
        const double Wn = (double)K.lockin * N;
        const double X = 2.0 * Sc / Wn, Y = 2.0 * Ss / Wn;
        o.A = ::sqrt(X * X + Y * Y) * 1e-9;
        o.phi = ::atan2(-X, Y);
        const double J = Urow ? Jn / Jd : NAN;
        o.J = (Urow && !isfinite(J)) ? INFINITY : J;
    }
    return o;
}

// One lane's trajectory i (group grp): parameter load, bounds checks, integration, outputs.
template <int LAW, int NM, bool MIXED, int FM>
__device__ __forceinline__ void lane_forward(const FwdArgs &A, const KConst &K, int64_t i,
                                             int64_t grp, int nc) {
    using R = typename std::conditional<MIXED, float, double>::type;
    double p[kMaxParams];
    load_params(p, K, A.base, A.base_ld, grp, A.theta, A.ld, i);
    const Law<LAW, R> law(p, K);
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
        if (trow)
            for (int64_t w = 0; w < W; ++w) trow[w] = NAN;
    } else {
        o = integrate<LAW, NM, MIXED, FM>(law, p[0] * 1e9, K, nc, Urow, trow);
    }
    if (A.amp) A.amp[i] = o.A;
    if (A.phase) A.phase[i] = o.phi;
    if (A.J) A.J[i] = o.J;
    if (A.status) A.status[i] = o.st;
}

template <int LAW, int NM, bool MIXED, int FM>
__global__ void __launch_bounds__(256) k_forward(const FwdArgs A, const KConst K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int64_t grp = A.group > 0 ? i / A.group : i;
    const int nc = A.n_cycles ? A.n_cycles[grp] : K.n_cycles;
    lane_forward<LAW, NM, MIXED, FM>(A, K, i, grp, nc);
}

// Persistent work queue for batches of groups with uneven period counts (one pixel's swarm is
// one group).  Each wavefront repeatedly takes the next item -- 64 lanes of one group -- from a
// queue ordered longest first, until the queue is empty; every wave reaches the exit.  The
// group's period count is the same for all lanes of an item, so it is moved to a scalar
// register and the time loops run as uniform scalar loops.
template <int LAW, int NM, bool MIXED, int FM>
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
        if (local < A.group) lane_forward<LAW, NM, MIXED, FM>(A, K, grp * A.group + local, grp, nc);
    }
}

__global__ void k_queue_reset(int32_t *head) {
    if (threadIdx.x == 0) *head = 0;
}

// Small batches (fewer waves than SIMDs) are issue-latency bound: one-wave blocks spread over
// the CUs and the branch-free law minimises issue slots.  Large batches are throughput bound:
// 4-wave blocks and the branching law (fewer transcendental ops).
constexpr int64_t kSmallBatch = 65536;

template <int LAW, int NM, bool MIXED>
hipError_t launch_t(const FwdArgs &a, const KConst &K, int32_t n_cu, hipStream_t s) {
    constexpr bool branchy = Law<LAW, float>::kBranch;
    if (a.items) {
        // persistent grid: 4 waves per SIMD on every CU.  All lanes of a wave belong to one
        // swarm (one separation), so they enter contact together: the wave-uniform skip form
        // (measured 11 % faster here than the per-lane branching form)
        hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, a.head);
        const unsigned blocks = (unsigned)(n_cu > 0 ? n_cu : 256) * 4;
        hipLaunchKernelGGL((k_forward_queue<LAW, NM, MIXED, branchy ? kFmSkip : kFmFree>),
                           dim3(blocks), dim3(256), 0, s, a, K);
        return hipGetLastError();
    }
    const int block = a.n < kSmallBatch ? 64 : 256;
    const int64_t grid = (a.n + block - 1) / block;
    if constexpr (branchy) {
        if (a.n >= kSmallBatch) {
            hipLaunchKernelGGL((k_forward<LAW, NM, MIXED, kFmBranch>), dim3((unsigned)grid),
                               dim3(block), 0, s, a, K);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_forward<LAW, NM, MIXED, kFmFree>), dim3((unsigned)grid), dim3(block), 0,
                       s, a, K);
    return hipGetLastError();
}

template <int LAW, bool MIXED>
hipError_t launch_modes(const FwdArgs &a, const KConst &K, int32_t cu, hipStream_t s) {
    switch (K.nm) {
    case 1: return launch_t<LAW, 1, MIXED>(a, K, cu, s);
    case 2: return launch_t<LAW, 2, MIXED>(a, K, cu, s);
    case 3: return launch_t<LAW, 3, MIXED>(a, K, cu, s);
    case 4: return launch_t<LAW, 4, MIXED>(a, K, cu, s);
    }
    return hipErrorInvalidValue;
}

template <bool MIXED>
hipError_t launch_law(const FwdArgs &a, const KConst &K, int32_t cu, hipStream_t s) {
    switch (K.law) {
    case AFM_LAW_DMT: return launch_modes<AFM_LAW_DMT, MIXED>(a, K, cu, s);
    case AFM_LAW_LJ: return launch_modes<AFM_LAW_LJ, MIXED>(a, K, cu, s);
    case AFM_LAW_KV: return launch_modes<AFM_LAW_KV, MIXED>(a, K, cu, s);
    case AFM_LAW_HOOKE: return launch_modes<AFM_LAW_HOOKE, MIXED>(a, K, cu, s);
    case AFM_LAW_SD: return launch_modes<AFM_LAW_SD, MIXED>(a, K, cu, s);
    case AFM_LAW_NONE: return launch_modes<AFM_LAW_NONE, MIXED>(a, K, cu, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_forward_p(const afm_plan *plan, int32_t prec, const FwdArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (prec == AFM_PREC_MIXED) return launch_law<true>(a, plan->kc, plan->n_cu, s);
    return launch_law<false>(a, plan->kc, plan->n_cu, s);
}

hipError_t launch_forward(const afm_plan *plan, const FwdArgs &a, hipStream_t s) {
    return launch_forward_p(plan, plan->precision, a, s);
}

}  // namespace afm
