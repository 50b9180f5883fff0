// points.hip -- deflection at points along the beam (the paper's deflection points, n_dp,
// Sec. 3.2): u(x_k, t) = sum_i w[k][i] q_i(t) over the tip-normalised modal coordinates q_i
// (App. B, Eq. 13 with w[k][i] = Phi_i(x_k) / Phi_i(L)).  The forward kernels write the modal
// coordinates of the lock-in window into a plan-owned workspace (trajectory fastest); one thread
// per trajectory then forms every point's deflection and lock-in amplitude and phase in FP64.
#include <algorithm>
#include <cmath>

#include "afm_internal.hpp"

namespace afm {

namespace {

constexpr int kMaxPoints = 16;
constexpr size_t kPointsChunkBytes = size_t(1) << 30;  // modal-trace workspace per chunk

struct PointArgs {
    int64_t n;                  // trajectories in this chunk
    int64_t n_all, off;         // output leading dimension and this chunk's first trajectory
    int32_t nm, np, N, W;
    const double *mt;           // [nm][W][n] modal coordinates, m
    const double *lock_c, *lock_s;
    const int32_t *status;      // [n] (chunk-relative)
    double *amp, *phase;        // [np][n_all]
    double *trace;              // [np][n_all][W] or nullptr
    double w[kMaxPoints * kMaxModes];
};

__global__ void __launch_bounds__(256) k_points(const PointArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n) return;
    const bool ok = a.status[t] == 0;
    const int64_t g = a.off + t;
    for (int k = 0; k < a.np; ++k) {
        double *tr = a.trace ? a.trace + ((int64_t)k * a.n_all + g) * a.W : nullptr;
        if (!ok) {
            a.amp[(int64_t)k * a.n_all + g] = NAN;
            a.phase[(int64_t)k * a.n_all + g] = NAN;
            if (tr)
                for (int s = 0; s < a.W; ++s) tr[s] = NAN;
            continue;
        }
        const double *wk = a.w + k * kMaxModes;
        double Sc = 0.0, Ss = 0.0;
        for (int s = 0; s < a.W; ++s) {
            double u = 0.0;
            for (int i = 0; i < a.nm; ++i)
                u = __builtin_fma(wk[i], a.mt[((int64_t)i * a.W + s) * a.n + t], u);
            // window sample s has drive-phase index (s + 1) mod N (the table's entry N is entry 0)
            const int p = s % a.N + 1;
            Sc = __builtin_fma(u, a.lock_c[p], Sc);
            Ss = __builtin_fma(u, a.lock_s[p], Ss);
            if (tr) tr[s] = u;
        }
        const double X = 2.0 * Sc / a.W, Y = 2.0 * Ss / a.W;
        a.amp[(int64_t)k * a.n_all + g] = ::sqrt(__builtin_fma(X, X, Y * Y));
        a.phase[(int64_t)k * a.n_all + g] = ::atan2(-X, Y);
    }
}

}  // namespace

}  // namespace afm

extern "C" {

afm_status afm_forward_points(afm_plan *plan, int64_t n, const double *theta,
                              const int32_t *n_cycles, int32_t n_points, const double *weights,
                              double *amp, double *phase, double *trace, int32_t *status,
                              afm_stream_t stream) {
    using namespace afm;
    afm_status st = check_forward_args(plan, n, theta);
    if (st != AFM_OK) return st;
    if (n_points < 1 || n_points > kMaxPoints)
        return fail(AFM_ERR_INVALID, "afm_forward_points: n_points must be in [1, 16]");
    if (!weights) return fail(AFM_ERR_INVALID, "afm_forward_points: weights are required");
    const int nm = plan->kc.nm;
    PointArgs pa{};
    for (int k = 0; k < n_points; ++k)
        for (int i = 0; i < nm; ++i) {
            const double w = weights[k * nm + i];
            if (!std::isfinite(w)) return fail(AFM_ERR_INVALID, "afm_forward_points: non-finite weight");
            pa.w[k * kMaxModes + i] = w;
        }
    if (n == 0) return AFM_OK;
    if (!amp || !phase || !status)
        return fail(AFM_ERR_INVALID, "afm_forward_points: amp, phase and status are required");
    const int32_t N = plan->kc.N, W = plan->kc.lockin * N;
    const size_t per = (size_t)nm * W * sizeof(double);
    const int64_t chunk = std::min<int64_t>(n, std::max<int64_t>(64, kPointsChunkBytes / per));
    const size_t bytes = per * (size_t)chunk;
    if (plan->mws_bytes < bytes) {
        if (plan->mws) (void)hipFree(plan->mws);
        plan->mws = nullptr;
        plan->mws_bytes = 0;
        if (hipMalloc(&plan->mws, bytes) != hipSuccess)
            return fail(AFM_ERR_NOMEM, "afm_forward_points: workspace allocation failed");
        plan->mws_bytes = bytes;
    }
    hipStream_t s = (hipStream_t)stream;
    pa.n_all = n;
    pa.nm = nm;
    pa.np = n_points;
    pa.N = N;
    pa.W = W;
    pa.mt = (const double *)plan->mws;
    pa.lock_c = plan->kc.lock_c;
    pa.lock_s = plan->kc.lock_s;
    pa.amp = amp;
    pa.phase = phase;
    pa.trace = trace;
    for (int64_t off = 0; off < n; off += chunk) {
        const int64_t cn = std::min(chunk, n - off);
        FwdArgs a{};
        a.n = cn;
        a.ld = n;
        a.theta = theta ? theta + off : nullptr;
        a.n_cycles = n_cycles ? n_cycles + off : nullptr;
        a.status = status + off;
        a.mtrace = (double *)plan->mws;
        a.mtrace_ld = cn;
        hipError_t e = launch_forward(plan, a, s);
        if (e != hipSuccess) return hip_fail(e, "afm_forward_points forward launch");
        pa.n = cn;
        pa.off = off;
        pa.status = status + off;
        hipLaunchKernelGGL(k_points, dim3((unsigned)((cn + 255) / 256)), dim3(256), 0, s, pa);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "afm_forward_points launch");
    }
    return AFM_OK;
}

}  // extern "C"
