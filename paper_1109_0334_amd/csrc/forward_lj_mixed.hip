// Forward kernels for the Lennard-Jones type law, FP32 state with FP64 sums.
#include "forward_impl.hpp"

template hipError_t afm::launch_fwd_law<AFM_LAW_LJ, true>(
    const afm_plan *, const afm::FwdArgs &, const afm::KConst &, hipStream_t);
