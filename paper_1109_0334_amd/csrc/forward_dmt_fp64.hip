// Forward kernels for the DMT law, plain FP64.
#include "forward_impl.hpp"

template hipError_t afm::launch_fwd_law<AFM_LAW_DMT, false>(
    const afm_plan *, const afm::FwdArgs &, const afm::KConst &, hipStream_t);
