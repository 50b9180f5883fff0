// Forward kernels for the Lennard-Jones type law, plain FP64.
#include "forward_impl.hpp"

template hipError_t afm::launch_fwd_law<AFM_LAW_LJ, false>(
    const afm_plan *, const afm::FwdArgs &, const afm::KConst &, hipStream_t);
