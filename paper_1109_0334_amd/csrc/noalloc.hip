// noalloc.hip -- afm_grad_batch_noalloc: the discrete-adjoint gradient of afm_grad_batch with
// its checkpoints and segment buffer in a fixed, library-owned device array instead of the plan's
// workspace, so that the call allocates nothing (for callers that cannot allocate: code being
// captured into a HIP graph, tight serving loops, harnesses that forbid allocation).
//
// The array below is one per device (each device that runs the library holds its own copy until
// the process ends).  Host code never uses its name as an address: the device address is looked
// up once per device with hipGetSymbolAddress and kept in `g_scratch`.  Every call on a device
// shares that device's array, so calls that overlap on one device race; the kernels write every
// checkpoint and segment-buffer entry before they read it, so nothing needs clearing.
#include <mutex>

#include "afm_internal.hpp"

namespace afm {

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // AFM_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == AFM_NOALLOC_SCRATCH_BYTES, "header and library disagree");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call per device).
afm_status scratch_ptr(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(AFM_ERR_UNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "afm_grad_batch_noalloc: hipGetSymbolAddress");
        if (!p) return fail(AFM_ERR_HIP, "afm_grad_batch_noalloc: scratch has no device address");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return AFM_OK;
}

}  // namespace

}  // namespace afm

using namespace afm;

extern "C" afm_status afm_grad_batch_noalloc(afm_plan *plan, int64_t n, const double *theta,
                                             const int32_t *n_cycles, const int32_t *target_id,
                                             const double *targets, int32_t n_targets, double *J,
                                             double *dJ, int32_t ckpt_stride, int32_t *status,
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
    // no timing here: an explicit stride, else the one afm_grad_batch tuned for this n, else 256
    const bool tuned = plan->tuned_n == n && plan->tuned_kc > 0;
    const int32_t kc = ckpt_stride > 0 ? ckpt_stride : (tuned ? plan->tuned_kc : 256);
    const int32_t form = tuned ? plan->tuned_form : grad_default_form(plan);
    const size_t cb = grad_ckpt_bytes(plan, plan->precision, n, kc);
    const size_t sb = (grad_seg_bytes(plan, plan->precision, n, kc, form) + 255) & ~(size_t)255;
    if (cb + sb > kScratchBytes)
        return fail(AFM_ERR_INVALID,
                    "afm_grad_batch_noalloc: checkpoints and segment buffer need " +
                        std::to_string(cb + sb) + " bytes, more than the " +
                        std::to_string(kScratchBytes) +
                        "-byte scratch array (use fewer points, a larger stride or afm_grad_batch)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "afm_grad_batch_noalloc: hipGetDevice");
    if (dev != plan->device)
        return fail(AFM_ERR_INVALID, "afm_grad_batch_noalloc: the current device is not the plan's");
    void *base = nullptr;
    st = scratch_ptr(dev, &base);
    if (st != AFM_OK) return st;
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
    a.kc = kc;
    a.mp = plan->kc.nm > 1 ? (tuned ? plan->tuned_mp : (n * 4 <= 65536 ? 1 : 0)) : 0;
    a.form = form;
    a.seg = (float *)base;
    a.ckpt = (float *)((char *)base + sb);
    e = launch_grad(plan, a, (hipStream_t)stream);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_grad_batch_noalloc launch");
}
