// stepwise.hip -- one kernel per Euler-Maruyama step, state in device memory.
#include "internal.hpp"

namespace oim {

int launch_stepwise_sparse(Problem*, const oim_run_cfg*, const float*, const float*, const float*,
                           const uint64_t*, int64_t, float*, uint32_t*, const oim_readout*,
                           hipStream_t) {
    return set_error(OIM_E_UNSUPPORTED, "replica too large for the LDS-resident kernel");
}

}  // namespace oim
