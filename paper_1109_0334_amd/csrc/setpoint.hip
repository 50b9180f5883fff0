// setpoint.hip -- afm_separations: the tip-sample separation at which each pixel's steady
// amplitude equals its set-point.
//
// Dynamic AFM holds the oscillation amplitude at a set-point by feedback on the separation
// (Sec. 1).  Reading: the separation z_c of a pixel is where the steady amplitude (plain FP64
// forward solve over many periods, lock-in over the last few) crosses s A0 when the tip
// approaches from A0 + 2 nm in fixed steps -- the first crossing, as an approach curve meets it
// -- narrowed by rounds of 16-point sections of the bracket.  Every amplitude is a forward solve
// of the library; a round's trial separations of all pixels go in one launch, and the bracket
// logic runs in small kernels between the launches, so the host only enqueues.
#include "afm_internal.hpp"

namespace afm {

namespace {

constexpr int kSections = 16;

// theta[s * K + k] = z_top - k * step: the approach grid (m), the same for every pixel
__global__ void k_sep_grid(int64_t n, int32_t K, double z_top, double step, double *theta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    theta[i] = z_top - (double)(i % K) * step;
}

// First grid point (from the top) whose amplitude is below the set-point (a failed solve counts
// as below): the bracket is [that point, the one before it].  No such point, or the very first
// one: NaN (no crossing found).
__global__ void k_sep_bracket(int32_t S, int32_t K, double z_top, double step, const double *amp,
                              const int32_t *status, const double *setpoint, double A0,
                              double *lo, double *hi) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double target = setpoint[s] * A0;
    int first = -1;
    for (int k = 0; k < K; ++k) {
        const int64_t i = (int64_t)s * K + k;
        const double A = status[i] == 0 ? amp[i] : -INFINITY;
        if (A < target) {
            first = k;
            break;
        }
    }
    if (first > 0) {
        lo[s] = z_top - (double)first * step;
        hi[s] = z_top - (double)(first - 1) * step;
    } else {
        lo[s] = NAN;
        hi[s] = NAN;
    }
}

// Trial separations of one round: lo + (hi - lo) j / (M + 1), j = 1 .. M (0 where there is no
// bracket, so that the launch stays well defined).
__global__ void k_sep_trials(int32_t S, const double *lo, const double *hi, double *theta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * kSections) return;
    const int s = (int)(i / kSections), j = (int)(i % kSections) + 1;
    const double l = lo[s], h = hi[s];
    theta[i] = isfinite(l) && isfinite(h) ? l + (h - l) * ((double)j / (kSections + 1)) : 0.0;
}

// Narrow the bracket to the first trial at or above the set-point and the trial before it (or
// lo); with no trial above it, to [the last trial, hi].
__global__ void k_sep_update(int32_t S, const double *theta, const double *amp,
                             const int32_t *status, const double *setpoint, double A0, double *lo,
                             double *hi) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    if (!isfinite(lo[s]) || !isfinite(hi[s])) return;
    const double target = setpoint[s] * A0;
    const int64_t b = (int64_t)s * kSections;
    int idx = -1;
    for (int j = 0; j < kSections; ++j) {
        const double A = status[b + j] == 0 ? amp[b + j] : -INFINITY;
        if (A >= target) {
            idx = j;
            break;
        }
    }
    if (idx >= 0) {
        if (idx > 0) lo[s] = theta[b + idx - 1];
        hi[s] = theta[b + idx];
    } else {
        lo[s] = theta[b + kSections - 1];
    }
}

__global__ void k_sep_final(int32_t S, const double *lo, const double *hi, double *zc) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    zc[s] = 0.5 * (lo[s] + hi[s]);
}

unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

}  // namespace afm

using namespace afm;

extern "C" afm_status afm_separations(afm_plan *plan, int32_t n_pixels, const double *params,
                                      const double *setpoint, int32_t periods,
                                      int32_t lockin_periods, double step, int32_t rounds,
                                      double *zc, afm_stream_t stream) {
    if (!plan) return fail(AFM_ERR_INVALID, "plan is NULL");
    if (n_pixels < 0) return fail(AFM_ERR_INVALID, "afm_separations: n_pixels < 0");
    if (n_pixels == 0) return AFM_OK;
    if (!setpoint || !zc) return fail(AFM_ERR_INVALID, "afm_separations: setpoint and zc are required");
    if (lockin_periods < 1 || periods < lockin_periods)
        return fail(AFM_ERR_INVALID, "afm_separations: need 1 <= lockin_periods <= periods");
    if (rounds < 0 || rounds > 64) return fail(AFM_ERR_INVALID, "afm_separations: rounds out of [0, 64]");
    if (!(step >= 0.0) || !std::isfinite(step))
        return fail(AFM_ERR_INVALID, "afm_separations: step must be finite and >= 0");
    if (plan->kc.drive_mode != AFM_DRIVE_TABLE)
        return fail(AFM_ERR_INVALID, "afm_separations: needs the fixed drive table");
    const double A0 = plan->prob.free_amplitude;
    const double dz = step > 0.0 ? step : 0.25e-9;
    const double z_top = A0 + 2e-9;
    const int32_t K = (int32_t)(z_top / dz);
    if (K < 2 || K > 100000) return fail(AFM_ERR_INVALID, "afm_separations: step gives too few or too many grid points");
    const int64_t S = n_pixels;
    const int64_t n_grid = S * K, n_max = std::max<int64_t>(n_grid, S * kSections);
    if (n_max > INT32_MAX) return fail(AFM_ERR_INVALID, "afm_separations: too many pixels");

    // the amplitude solves: the plan's problem in FP64 over `periods` periods, z_c the one free
    // parameter, every other parameter from the pixel's vector
    afm_problem pr = plan->prob;
    pr.n_cycles = periods;
    pr.lockin_cycles = lockin_periods;
    pr.steady_rtol = 0.0;
    pr.n_free = 1;
    pr.free_index[0] = 0;
    pr.lo[0] = 0.0;
    pr.hi[0] = 1.0;
    pr.log_scale[0] = 0;
    afm_plan *sub = nullptr;
    afm_status st = afm_plan_create(&pr, AFM_PREC_FP64, &sub);
    if (st != AFM_OK) return st;
    // each launch is long and of a new size: take GPU-filling four-wave workgroups, untimed
    (void)afm_set_launch_shape(sub, 256, 1);
    hipStream_t s = (hipStream_t)stream;
    char *mem = nullptr;
    const size_t bytes = (size_t)n_max * (3 * sizeof(double) + sizeof(int32_t)) + 2 * S * sizeof(double);
    hipError_t e = hipMalloc(&mem, bytes);
    if (e != hipSuccess) {
        afm_plan_destroy(sub);
        return fail(AFM_ERR_NOMEM, "afm_separations: workspace allocation failed");
    }
    double *theta = (double *)mem, *amp = theta + n_max, *phase = amp + n_max;
    double *lo = phase + n_max, *hi = lo + S;
    int32_t *status = (int32_t *)(hi + S);
    FwdArgs a{};
    a.theta = theta;
    a.amp = amp;
    a.phase = phase;
    a.status = status;
    a.base = params;
    a.base_ld = S;
    // approach grid
    a.n = a.ld = n_grid;
    a.group = K;
    hipLaunchKernelGGL(k_sep_grid, dim3(blocks(n_grid, 256)), dim3(256), 0, s, n_grid, K, z_top,
                       dz, theta);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_forward(sub, a, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sep_bracket, dim3(blocks(S, 64)), dim3(64), 0, s, (int32_t)S, K,
                           z_top, dz, amp, status, setpoint, A0, lo, hi);
        e = hipGetLastError();
    }
    // sections
    a.n = a.ld = S * kSections;
    a.group = kSections;
    for (int r = 0; r < rounds && e == hipSuccess; ++r) {
        hipLaunchKernelGGL(k_sep_trials, dim3(blocks(S * kSections, 256)), dim3(256), 0, s,
                           (int32_t)S, lo, hi, theta);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_forward(sub, a, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_sep_update, dim3(blocks(S, 64)), dim3(64), 0, s, (int32_t)S,
                               theta, amp, status, setpoint, A0, lo, hi);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sep_final, dim3(blocks(S, 64)), dim3(64), 0, s, (int32_t)S, lo, hi, zc);
        e = hipGetLastError();
    }
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    (void)hipFree(mem);
    afm_plan_destroy(sub);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_separations");
}
