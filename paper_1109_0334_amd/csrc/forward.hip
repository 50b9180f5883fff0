// forward.hip -- host side of the batched forward solve: the launch-shape tuner and the
// dispatch over force laws and precisions.  The kernels (RK4 time integration of the
// base-driven modal cantilever, lock-in projection and window misfit) are in forward_impl.hpp,
// compiled once per law and precision by the forward_<law>_<precision>.hip units.
#include "afm_internal.hpp"

namespace afm {

namespace {

template <bool MIXED>
hipError_t launch_law(const afm_plan *plan, const FwdArgs &a, const KConst &K, hipStream_t s) {
    switch (K.law) {
    case AFM_LAW_DMT: return launch_fwd_law<AFM_LAW_DMT, MIXED>(plan, a, K, s);
    case AFM_LAW_LJ: return launch_fwd_law<AFM_LAW_LJ, MIXED>(plan, a, K, s);
    case AFM_LAW_KV: return launch_fwd_law<AFM_LAW_KV, MIXED>(plan, a, K, s);
    case AFM_LAW_HOOKE: return launch_fwd_law<AFM_LAW_HOOKE, MIXED>(plan, a, K, s);
    case AFM_LAW_SD: return launch_fwd_law<AFM_LAW_SD, MIXED>(plan, a, K, s);
    case AFM_LAW_NONE: return launch_fwd_law<AFM_LAW_NONE, MIXED>(plan, a, K, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// Launch shape of a plain forward launch: the plan's tuned choice for this precision, batch
// size and period-count mode; tuned on first use (every candidate timed once on the real
// arguments, after one warm-up launch) unless the stream is being captured, in which case the
// default shape is used (one-wave blocks for small batches, four-wave blocks for large ones,
// one trajectory per lane).  Every candidate computes bit-identical results, so tuning never
// changes an output.
hipError_t forward_shape(const afm_plan *plan, int32_t prec, const FwdArgs &a, int nm,
                         hipStream_t s, const std::function<hipError_t(FwdShape)> &launch,
                         FwdShape *out) {
    const int32_t has_nc = a.n_cycles != nullptr;
    const bool pair_ok = nm == 1 && !has_nc && plan->kc.drive_mode == AFM_DRIVE_TABLE;
    if (plan->pinned_shape.block > 0) {
        *out = plan->pinned_shape;
        if ((out->tpl == 2 && !pair_ok) || (out->tpl == 0 && nm == 1)) out->tpl = 1;
        return hipSuccess;
    }
    for (const FwdTune &t : plan->fwd_tune)
        if (t.n == a.n && t.prec == prec && t.has_nc == has_nc) {
            *out = t.shape;
            return hipSuccess;
        }
    // default: one lane per mode while the groups still fit one wave per SIMD (there it
    // shortens every wave's instruction stream); otherwise one lane per trajectory
    FwdShape def{a.n < kSmallBatch ? 64 : 256, (nm > 1 && a.n * 4 <= kSmallBatch) ? 0 : 1};
    *out = def;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusNone) return hipSuccess;
    std::vector<FwdShape> cand;
    for (int b : {64, 128, 256}) {
        cand.push_back({b, 1});
        if (pair_ok) cand.push_back({b, 2});
        if (nm > 1) cand.push_back({b, 0});
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch(def);  // warm-up (code load, caches)
    // time every candidate; keep the default unless another is at least 2 % faster (shapes
    // within timing noise of each other would otherwise flip from run to run)
    std::vector<float> ms(cand.size(), 0.0f);
    for (size_t k = 0; k < cand.size() && e == hipSuccess; ++k) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch(cand[k]);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms[k], e0, e1);
    }
    float best = 0.0f;
    if (e == hipSuccess) {
        size_t kd = 0, kb = 0;
        for (size_t k = 0; k < cand.size(); ++k) {
            if (cand[k].block == def.block && cand[k].tpl == def.tpl) kd = k;
            if (ms[k] < ms[kb]) kb = k;
        }
        const size_t pick = ms[kb] < 0.98f * ms[kd] ? kb : kd;
        *out = cand[pick];
        best = ms[pick];
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    plan->fwd_tune.push_back({a.n, prec, has_nc, *out, best});
    return hipSuccess;
}

bool forward_shape_known(const afm_plan *plan, int32_t prec, const FwdArgs &a) {
    if (plan->pinned_shape.block > 0) return true;
    const int32_t has_nc = a.n_cycles != nullptr;
    for (const FwdTune &t : plan->fwd_tune)
        if (t.n == a.n && t.prec == prec && t.has_nc == has_nc) return true;
    return false;
}

hipError_t launch_forward_p(const afm_plan *plan, int32_t prec, const FwdArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (prec == AFM_PREC_MIXED) return launch_law<true>(plan, a, plan->kc, s);
    return launch_law<false>(plan, a, plan->kc, s);
}

hipError_t launch_forward(const afm_plan *plan, const FwdArgs &a, hipStream_t s) {
    return launch_forward_p(plan, plan->precision, a, s);
}

}  // namespace afm
