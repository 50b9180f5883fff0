// Forward kernels for the spring-damper contact law, FP32 state with FP64 sums.
#include "forward_impl.hpp"

template hipError_t afm::launch_fwd_law<AFM_LAW_SD, true>(
    const afm_plan *, const afm::FwdArgs &, const afm::KConst &, hipStream_t);
