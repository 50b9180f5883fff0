// api.hip -- the extern "C" entry points of libafm: plan set-up (non-dimensionalisation, base
// amplitude, initial state, drive and lock-in tables), argument validation, and dispatch to
// the forward and swarm kernels.  Host code only.
#include <algorithm>
#include <complex>
#include <cstring>
#include <new>
#include <vector>

#include "afm_internal.hpp"

namespace afm {

namespace {
thread_local std::string g_err;
const int kLawParams[6] = {5, 5, 6, 2, 3, 1};
}  // namespace

void set_error(const std::string &msg) { g_err = msg; }

afm_status fail(afm_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

afm_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return AFM_ERR_HIP;
}

afm_status check_forward_args(const afm_plan *plan, int64_t n, const double *theta) {
    if (!plan) return fail(AFM_ERR_INVALID, "plan is NULL");
    if (n < 0) return fail(AFM_ERR_INVALID, "n < 0");
    if (n > 0 && plan->prob.n_free > 0 && !theta) return fail(AFM_ERR_INVALID, "theta is NULL");
    if (n > (int64_t)1 << 40) return fail(AFM_ERR_INVALID, "n too large");
    return AFM_OK;
}

// Validate a problem and fill the plan's constants.  The base amplitude follows from the free
// linear response H_i = gamma_i / (Om_i^2 - 1 + i Om_i / Q_i) (per unit base amplitude, in units
// of wd): a = A0 / |sum_i H_i|.  The free steady state at t = 0 is x_i = Im(a H_i),
// x_i' = Re(a H_i) (per unit tau).
static afm_status build_constants(const afm_problem &pr, int32_t precision, afm_plan *plan,
                                  std::vector<float> &drive_f, std::vector<double> &drive_d,
                                  std::vector<double> &lock) {
    if (precision != AFM_PREC_MIXED && precision != AFM_PREC_FP64)
        return fail(AFM_ERR_INVALID, "precision must be AFM_PREC_MIXED or AFM_PREC_FP64");
    if (pr.n_modes < 1 || pr.n_modes > kMaxModes) return fail(AFM_ERR_INVALID, "n_modes out of range");
    if (pr.law < 0 || pr.law > AFM_LAW_NONE) return fail(AFM_ERR_INVALID, "unknown law");
    if (pr.steps_per_cycle < 4 || pr.steps_per_cycle > kMaxSteps)
        return fail(AFM_ERR_INVALID, "steps_per_cycle must be in [4, 4096]");
    if (pr.lockin_cycles < 1) return fail(AFM_ERR_INVALID, "lockin_cycles must be >= 1");
    if (pr.n_cycles < pr.lockin_cycles) return fail(AFM_ERR_INVALID, "n_cycles < lockin_cycles");
    if ((int64_t)pr.lockin_cycles * pr.steps_per_cycle > (int64_t)1 << 30)
        return fail(AFM_ERR_INVALID, "lock-in window too long");
    if (!(pr.k > 0) || !(pr.f0 > 0) || !(pr.drive_freq > 0) || !(pr.free_amplitude > 0))
        return fail(AFM_ERR_INVALID, "k, f0, drive_freq and free_amplitude must be positive");
    if (pr.ic != AFM_IC_FREE_STEADY && pr.ic != AFM_IC_REST) return fail(AFM_ERR_INVALID, "unknown ic");
    if (pr.polish_precision < AFM_POLISH_PLAN || pr.polish_precision > AFM_POLISH_FP64)
        return fail(AFM_ERR_INVALID, "unknown polish_precision");
    for (int i = 0; i < pr.n_modes; ++i)
        if (!(pr.q[i] > 0) || !(pr.ratio[i] > 0) || !std::isfinite(pr.gain[i]))
            return fail(AFM_ERR_INVALID, "mode quality factors and ratios must be positive");
    if (pr.drive_mode != AFM_DRIVE_TABLE && pr.drive_mode != AFM_DRIVE_PARAMS)
        return fail(AFM_ERR_INVALID, "unknown drive_mode");
    const bool dparams = pr.drive_mode == AFM_DRIVE_PARAMS;
    if (dparams && pr.ic != AFM_IC_REST)
        return fail(AFM_ERR_INVALID, "a parameter-driven base motion needs ic = AFM_IC_REST");
    if (!(pr.steady_rtol >= 0.0) || !std::isfinite(pr.steady_rtol))
        return fail(AFM_ERR_INVALID, "steady_rtol must be finite and >= 0");
    if (pr.steady_rtol > 0.0 && dparams)
        return fail(AFM_ERR_INVALID, "the steady-state exit needs the periodic drive table");
    const int np = kLawParams[pr.law];
    // a slot a trajectory reads: the law's, and with PARAMS the base motion's (8 .. 10)
    auto used = [&](int q) { return (q >= 0 && q < np) || (dparams && q >= AFM_P_BASE_A && q <= AFM_P_BASE_G); };
    if (pr.n_free < 0 || pr.n_free > np + (dparams ? 3 : 0))
        return fail(AFM_ERR_INVALID, "n_free out of range for the law");
    for (int j = 0; j < pr.n_free; ++j) {
        if (!used(pr.free_index[j]))
            return fail(AFM_ERR_INVALID, "free_index out of range for the law");
        for (int l = 0; l < j; ++l)
            if (pr.free_index[l] == pr.free_index[j]) return fail(AFM_ERR_INVALID, "free_index repeated");
        if (!(pr.lo[j] < pr.hi[j])) return fail(AFM_ERR_INVALID, "search box needs lo < hi");
        if (pr.log_scale[j] && !(pr.lo[j] > 0)) return fail(AFM_ERR_INVALID, "log-scaled box needs lo > 0");
    }

    KConst &K = plan->kc;
    std::memset(&K, 0, sizeof(K));
    K.nm = pr.n_modes;
    K.law = pr.law;
    K.N = pr.steps_per_cycle;
    K.n_cycles = pr.n_cycles;
    K.lockin = pr.lockin_cycles;
    K.n_free = pr.n_free;
    K.drive_mode = pr.drive_mode;
    K.steady_rtol = pr.steady_rtol;
    K.fref = pr.drive_freq;
    for (int j = 0; j < kMaxParams; ++j) {
        K.free_index[j] = j < pr.n_free ? pr.free_index[j] : -1;
        K.params[j] = used(j) ? pr.params[j] : 0.0;
    }
    K.k = pr.k;
    K.wd = 2.0 * M_PI * pr.drive_freq;
    const double fr = pr.f0 / pr.drive_freq;
    K.G = fr * fr;
    K.h = 2.0 * M_PI / pr.steps_per_cycle;
    std::complex<double> Hs(0.0, 0.0);
    std::complex<double> H[kMaxModes];
    for (int i = 0; i < pr.n_modes; ++i) {
        const double Om = pr.ratio[i] * fr;
        K.om2[i] = Om * Om;
        K.cdamp[i] = Om / pr.q[i];
        K.gain[i] = pr.gain[i];
        H[i] = pr.gain[i] / std::complex<double>(Om * Om - 1.0, Om / pr.q[i]);
        Hs += H[i];
    }
    if (!(std::abs(Hs) > 0)) return fail(AFM_ERR_INVALID, "free response vanishes (zero drive gains)");
    const double a_nm = pr.free_amplitude * 1e9 / std::abs(Hs);
    for (int i = 0; i < pr.n_modes; ++i) {
        if (pr.ic == AFM_IC_FREE_STEADY) {
            K.y0[i] = (a_nm * H[i]).imag();
            K.y0[pr.n_modes + i] = (a_nm * H[i]).real();
        }
    }
    K.div_nm = (pr.div_limit > 0 ? pr.div_limit : 100.0) * pr.free_amplitude * 1e9;
    const int N = pr.steps_per_cycle;
    // 2N + 1 entries (stage times 0, h/2, ..., 2 pi) and 8 zeros that only the time loop's
    // one-block-ahead prefetch reads (never used in arithmetic)
    drive_f.resize(2 * N + 1 + kDrivePad);
    drive_d.resize(2 * N + 1 + kDrivePad);
    // a point mass takes its gain into the table (the kernel then adds the entry directly)
    const double tab_gain = pr.n_modes == 1 ? pr.gain[0] : 1.0;
    for (int j = 0; j <= 2 * N + kDrivePad; ++j) {
        const double d = j >= 2 * N ? 0.0 : tab_gain * a_nm * std::sin(M_PI * (double)j / (double)N);
        drive_d[j] = d;
        drive_f[j] = (float)d;
    }
    K.dmax = 0.0;
    for (const double d : drive_d) K.dmax = std::max(K.dmax, std::fabs(d));
    lock.resize(2 * (N + 1));
    for (int p = 0; p <= N; ++p) {
        const int q = p == N ? 0 : p;
        lock[p] = std::cos(2.0 * M_PI * (double)q / (double)N);
        lock[N + 1 + p] = std::sin(2.0 * M_PI * (double)q / (double)N);
    }
    plan->pso_w = pr.pso_w != 0 ? pr.pso_w : 0.7298;
    plan->pso_c1 = pr.pso_c1 != 0 ? pr.pso_c1 : 1.49618;
    plan->pso_c2 = pr.pso_c2 != 0 ? pr.pso_c2 : 1.49618;
    plan->pso_vmax = pr.pso_vmax != 0 ? pr.pso_vmax : 1.0;
    return AFM_OK;
}

void release_graph(afm_plan *plan);  // invert.hip

int32_t polish_prec(const afm_plan *plan) {
    switch (plan->prob.polish_precision) {
    case AFM_POLISH_MIXED: return AFM_PREC_MIXED;
    case AFM_POLISH_FP64: return AFM_PREC_FP64;
    default: return plan->precision;
    }
}

}  // namespace afm

using namespace afm;

extern "C" {

const char *afm_last_error(void) { return g_err.c_str(); }

const char *afm_version(void) { return "afm-mi355x 0.1 (gfx950)"; }

afm_status afm_plan_create(const afm_problem *problem, int32_t precision, afm_plan **out) {
    if (!out) return fail(AFM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!problem) return fail(AFM_ERR_INVALID, "problem is NULL");
    afm_plan *plan = new (std::nothrow) afm_plan();
    if (!plan) return fail(AFM_ERR_NOMEM, "host allocation failed");
    plan->prob = *problem;
    plan->precision = precision;
    std::vector<float> df;
    std::vector<double> dd, lk;
    afm_status st = build_constants(*problem, precision, plan, df, dd, lk);
    if (st != AFM_OK) {
        delete plan;
        return st;
    }
    hipError_t e = hipGetDevice(&plan->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&plan->n_cu, hipDeviceAttributeMultiprocessorCount, plan->device);
    if (e == hipSuccess) e = hipMalloc(&plan->d_drive_f, df.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&plan->d_drive_d, dd.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&plan->d_lock, lk.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&plan->d_order, kOrderMax * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&plan->d_order_keys, kOrderMax * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(plan->d_drive_f, df.data(), df.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(plan->d_drive_d, dd.data(), dd.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(plan->d_lock, lk.data(), lk.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&plan->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        afm_status r = hip_fail(e, "afm_plan_create");
        afm_plan_destroy(plan);
        return r;
    }
    plan->kc.drive_f = plan->d_drive_f;
    plan->kc.drive_d = plan->d_drive_d;
    plan->kc.lock_c = plan->d_lock;
    plan->kc.lock_s = plan->d_lock + problem->steps_per_cycle + 1;
    *out = plan;
    return AFM_OK;
}

afm_status afm_set_launch_shape(afm_plan *plan, int32_t block, int32_t tpl) {
    if (!plan) return fail(AFM_ERR_INVALID, "afm_set_launch_shape: plan is NULL");
    if (block == 0) {
        plan->pinned_shape = afm::FwdShape{0, 0};
        return AFM_OK;
    }
    if (!(block == 64 || block == 128 || block == 256) || !(tpl == 0 || tpl == 1 || tpl == 2))
        return fail(AFM_ERR_INVALID, "afm_set_launch_shape: block must be 0, 64, 128 or 256 and "
                                     "tpl 0, 1 or 2");
    plan->pinned_shape = afm::FwdShape{block, tpl};
    return AFM_OK;
}

afm_status afm_set_grad_form(afm_plan *plan, int32_t form) {
    if (!plan) return fail(AFM_ERR_INVALID, "afm_set_grad_form: plan is NULL");
    if (form != AFM_GRAD_AUTO && form != AFM_GRAD_SWEEP && form != AFM_GRAD_SEGMENTS)
        return fail(AFM_ERR_INVALID, "afm_set_grad_form: unknown form");
    if (form == AFM_GRAD_SEGMENTS && !grad_segments_ok(plan))
        return fail(AFM_ERR_UNSUPPORTED,
                    "afm_set_grad_form: the segment form needs the drive table and at most 4 modes");
    plan->grad_form = form;
    plan->tuned_n = -1;  // tune again under the new setting
    return AFM_OK;
}

afm_status afm_plan_destroy(afm_plan *plan) {
    if (!plan) return AFM_OK;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    release_graph(plan);
    if (plan->ws) (void)hipFree(plan->ws);
    if (plan->gws) (void)hipFree(plan->gws);
    if (plan->pws) (void)hipFree(plan->pws);
    if (plan->mws) (void)hipFree(plan->mws);
    if (plan->qws) (void)hipFree(plan->qws);
    if (plan->d_drive_f) (void)hipFree(plan->d_drive_f);
    if (plan->d_drive_d) (void)hipFree(plan->d_drive_d);
    if (plan->d_lock) (void)hipFree(plan->d_lock);
    if (plan->d_order) (void)hipFree(plan->d_order);
    if (plan->d_order_keys) (void)hipFree(plan->d_order_keys);
    if (plan->ev_in) (void)hipEventDestroy(plan->ev_in);
    if (plan->ev_out) (void)hipEventDestroy(plan->ev_out);
    if (plan->stream) (void)hipStreamDestroy(plan->stream);
    delete plan;
    return AFM_OK;
}

afm_status afm_forward_batch(afm_plan *plan, int64_t n, const double *theta,
                             const int32_t *n_cycles, double *amp, double *phase, double *trace,
                             int32_t *status, afm_stream_t stream) {
    afm_status st = check_forward_args(plan, n, theta);
    if (st != AFM_OK) return st;
    if (n > 0 && (!amp || !phase || !status)) return fail(AFM_ERR_INVALID, "amp, phase and status are required");
    FwdArgs a{};
    a.n = n;
    a.ld = n;
    a.theta = theta;
    a.n_cycles = n_cycles;
    a.amp = amp;
    a.phase = phase;
    a.trace = trace;
    a.status = status;
    hipError_t e = launch_forward(plan, a, (hipStream_t)stream);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_forward_batch launch");
}

afm_status afm_forward_steady(afm_plan *plan, int64_t n, const double *theta,
                              const int32_t *n_cycles, double *amp, double *phase, double *trace,
                              int32_t *status, int32_t *periods, afm_stream_t stream) {
    afm_status st = check_forward_args(plan, n, theta);
    if (st != AFM_OK) return st;
    if (n > 0 && (!amp || !phase || !status || !periods))
        return fail(AFM_ERR_INVALID, "amp, phase, status and periods are required");
    FwdArgs a{};
    a.n = n;
    a.ld = n;
    a.theta = theta;
    a.n_cycles = n_cycles;
    a.amp = amp;
    a.phase = phase;
    a.trace = trace;
    a.status = status;
    a.periods = periods;
    hipError_t e = launch_forward(plan, a, (hipStream_t)stream);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_forward_steady launch");
}

afm_status afm_misfit(afm_plan *plan, int64_t n, const double *theta, const int32_t *n_cycles,
                      const int32_t *target_id, const double *targets, int32_t n_targets,
                      double *J, int32_t *status, afm_stream_t stream) {
    afm_status st = check_forward_args(plan, n, theta);
    if (st != AFM_OK) return st;
    if (n > 0 && (!targets || !J || !status)) return fail(AFM_ERR_INVALID, "targets, J and status are required");
    if (n > 0 && n_targets < 1) return fail(AFM_ERR_INVALID, "n_targets < 1");
    FwdArgs a{};
    a.n = n;
    a.ld = n;
    a.theta = theta;
    a.n_cycles = n_cycles;
    a.target_id = target_id;
    a.targets = targets;
    a.n_targets = n_targets;
    a.J = J;
    a.status = status;
    hipError_t e = launch_forward(plan, a, (hipStream_t)stream);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_misfit launch");
}

static afm_status ensure_grad_ws(afm_plan *plan, size_t bytes) {
    if (plan->gws_bytes >= bytes) return AFM_OK;
    if (plan->gws) (void)hipFree(plan->gws);  // hipFree waits for work still using it
    plan->gws = nullptr;
    plan->gws_bytes = 0;
    if (hipMalloc(&plan->gws, bytes) != hipSuccess)
        return fail(AFM_ERR_NOMEM, "afm_grad_batch: workspace allocation failed");
    plan->gws_bytes = bytes;
    return AFM_OK;
}


static afm_status run_grad(afm_plan *plan, GradArgs a, int32_t kc, int32_t mp, int32_t form,
                           hipStream_t s) {
    const size_t cb = grad_ckpt_bytes(plan, plan->precision, a.n, kc);
    const size_t sb = grad_seg_bytes(plan, plan->precision, a.n, kc, form);
    afm_status st = ensure_grad_ws(plan, cb + ((sb + 255) & ~(size_t)255) + 256);
    if (st != AFM_OK) return st;
    a.kc = kc;
    a.mp = plan->kc.nm > 1 ? mp : 0;
    a.form = form;
    a.seg = (float *)plan->gws;
    a.ckpt = (float *)((char *)plan->gws + ((sb + 255) & ~(size_t)255));
    hipError_t e = launch_grad(plan, a, s);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_grad_batch launch");
}

static afm_status check_swarm(const afm_plan *plan, const afm_swarm *sw) {
    if (!plan) return fail(AFM_ERR_INVALID, "plan is NULL");
    if (!sw) return fail(AFM_ERR_INVALID, "swarm is NULL");
    if (sw->n_dim != plan->prob.n_free || sw->n_dim < 1)
        return fail(AFM_ERR_INVALID, "swarm n_dim must equal the problem's n_free (>= 1)");
    if (sw->particles < 1 || sw->swarms < 1) return fail(AFM_ERR_INVALID, "particles and swarms must be >= 1");
    if ((int64_t)sw->particles * sw->swarms > INT32_MAX)
        return fail(AFM_ERR_INVALID, "swarm too large");
    if (!sw->z || !sw->v || !sw->pbest_z || !sw->pbest_J || !sw->gbest_z || !sw->gbest_J ||
        !sw->gen_to_cutoff || !sw->theta)
        return fail(AFM_ERR_INVALID, "swarm array is NULL");
    return AFM_OK;
}

afm_status afm_grad_batch(afm_plan *plan, int64_t n, const double *theta, const int32_t *n_cycles,
                          const int32_t *target_id, const double *targets, int32_t n_targets,
                          double *J, double *dJ, int32_t ckpt_stride, int32_t *status,
                          afm_stream_t stream) {
    afm_status st = check_forward_args(plan, n, theta);
    if (st != AFM_OK) return st;
    if (n > 0 && (!targets || !J || !status || (plan->prob.n_free > 0 && !dJ)))
        return fail(AFM_ERR_INVALID, "targets, J, dJ and status are required");
    if (n > 0 && n_targets < 1) return fail(AFM_ERR_INVALID, "n_targets < 1");
    if (ckpt_stride < 0) return fail(AFM_ERR_INVALID, "ckpt_stride < 0");
    if (plan->kc.steady_rtol > 0.0)
        return fail(AFM_ERR_UNSUPPORTED, "the adjoint of the adaptive steady-state exit is not built");
    if (n == 0) return AFM_OK;
    GradArgs a{};
    a.n = n;
    a.ld = n;
    a.theta = theta;
    a.n_cycles = n_cycles;
    a.target_id = target_id;
    a.targets = targets;
    a.n_targets = n_targets;
    a.J = J;
    a.dJ = dJ;
    a.status = status;
    hipStream_t s = (hipStream_t)stream;
    const bool tuned = plan->tuned_n == n && plan->tuned_kc > 0;
    // mode-parallel (several modes) unless tuning found otherwise; both compute the same bits
    const int32_t mp_default = tuned ? plan->tuned_mp : (n * 4 <= 65536 ? 1 : 0);
    const int32_t form_default = tuned ? plan->tuned_form : grad_default_form(plan);
    if (ckpt_stride > 0) return run_grad(plan, a, ckpt_stride, mp_default, form_default, s);
    if (tuned) return run_grad(plan, a, plan->tuned_kc, plan->tuned_mp, plan->tuned_form, s);
    // autotune: time each candidate stride and form (the reverse sweep and the segment-parallel
    // form, with several modes each with one lane per trajectory or one lane per mode for the
    // passes along the trajectory) on this call's inputs, keep the fastest; candidates needing
    // more than 8 GiB of workspace are left out
    struct Cand { int32_t kc, mp, form; };
    std::vector<Cand> cand;
    for (int32_t kc : {16, 64, 256}) {
        if (plan->grad_form != kGradSegments || !grad_segments_ok(plan)) {
            cand.push_back({kc, 0, kGradSweep});
            if (plan->kc.nm > 1) cand.push_back({kc, 1, kGradSweep});
        }
        if (plan->grad_form != kGradSweep && grad_segments_ok(plan) &&
            grad_seg_bytes(plan, plan->precision, n, kc, kGradSegments) +
                    grad_ckpt_bytes(plan, plan->precision, n, kc) <= ((size_t)8 << 30))
        {
            cand.push_back({kc, 0, kGradSegments});
            if (plan->kc.nm > 1) cand.push_back({kc, 1, kGradSegments});
        }
    }
    if (cand.empty()) cand.push_back({256, 0, kGradSweep});
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(AFM_ERR_HIP, "afm_grad_batch: event creation failed");
    float best_ms = 0;
    Cand best = cand[0];
    for (size_t c = 0; c < cand.size(); ++c) {
        (void)hipEventRecord(e0, s);
        st = run_grad(plan, a, cand[c].kc, cand[c].mp, cand[c].form, s);
        if (st != AFM_OK) break;
        (void)hipEventRecord(e1, s);
        float ms = 0;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = fail(AFM_ERR_HIP, "afm_grad_batch: timing failed");
            break;
        }
        if (c == 0 || ms < best_ms) {
            best_ms = ms;
            best = cand[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != AFM_OK) return st;
    plan->tuned_n = n;
    plan->tuned_kc = best.kc;
    plan->tuned_mp = best.mp;
    plan->tuned_form = best.form;
    // the outputs must be the chosen configuration's: the forms agree only to rounding
    const Cand &last = cand.back();
    if (last.kc == best.kc && last.mp == best.mp && last.form == best.form) return AFM_OK;
    return run_grad(plan, a, best.kc, best.mp, best.form, s);
}

afm_status afm_polish(afm_plan *plan, int64_t n, double *z, const double *params,
                      const int32_t *n_cycles, const int32_t *target_id, const double *targets,
                      int32_t n_targets, int32_t steps, double *J, afm_stream_t stream) {
    if (!plan) return fail(AFM_ERR_INVALID, "plan is NULL");
    if (n < 0 || steps < 0) return fail(AFM_ERR_INVALID, "n and steps must be >= 0");
    if (plan->prob.n_free < 1) return fail(AFM_ERR_INVALID, "the problem has no free parameters");
    if (plan->kc.steady_rtol > 0.0)
        return fail(AFM_ERR_UNSUPPORTED, "the adjoint of the adaptive steady-state exit is not built");
    if (n == 0) return AFM_OK;
    if (!z || !targets || !J) return fail(AFM_ERR_INVALID, "z, targets and J are required");
    if (n_targets < 1) return fail(AFM_ERR_INVALID, "n_targets < 1");
    const size_t bytes = polish_total_bytes(plan, n, kPolishStride);
    if (plan->pws_bytes < bytes) {
        if (plan->pws) (void)hipFree(plan->pws);
        plan->pws = nullptr;
        plan->pws_bytes = 0;
        if (hipMalloc(&plan->pws, bytes) != hipSuccess)
            return fail(AFM_ERR_NOMEM, "afm_polish: workspace allocation failed");
        plan->pws_bytes = bytes;
    }
    hipError_t e = enqueue_polish(plan, plan->pws, n, z, target_id, targets, n_targets, n_cycles,
                                  params, steps, kPolishStride, J, (hipStream_t)stream);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_polish launch");
}

afm_status afm_swarm_init(afm_plan *plan, afm_swarm *swarm, uint64_t seed, afm_stream_t stream) {
    afm_status st = check_swarm(plan, swarm);
    if (st != AFM_OK) return st;
    hipError_t e = launch_swarm_init(plan, *swarm, seed, (hipStream_t)stream);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_swarm_init launch");
}

afm_status afm_pso_step(afm_plan *plan, afm_swarm *swarm, const double *J, uint64_t seed,
                        int32_t iter, int32_t is_last, double cutoff, afm_stream_t stream) {
    afm_status st = check_swarm(plan, swarm);
    if (st != AFM_OK) return st;
    if (!J) return fail(AFM_ERR_INVALID, "J is NULL");
    if (iter < 0) return fail(AFM_ERR_INVALID, "iter < 0");
    hipError_t e = launch_pso_step(plan, *swarm, J, seed, iter, is_last, cutoff, (hipStream_t)stream);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_pso_step launch");
}

}  // extern "C"
