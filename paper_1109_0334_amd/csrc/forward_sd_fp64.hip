// Forward kernels for the spring-damper contact law, plain FP64.
#include "forward_impl.hpp"

template hipError_t afm::launch_fwd_law<AFM_LAW_SD, false>(
    const afm_plan *, const afm::FwdArgs &, const afm::KConst &, hipStream_t);
