// sparse_persistent_uw.hip -- the LDS-resident kernel's instantiations for
// problems whose couplings all share one weight, +1 or -1 (unit-weight
// max-cut, antiferromagnetic colouring): their sliced-ELL image holds the
// neighbours' LDS offsets alone, half the bytes of the general image, with
// the same results bit for bit.  A translation unit of its own so the two
// sets of instantiations compile in parallel.
#include "persistent_kernel.hpp"

namespace oim {
namespace persist {

#define OIM_UNIFORM_ENTRY(TB, MS, RPL)                                                   \
    {persistent_sparse_kernel<TB, MS, 0, RPL, true>,                                     \
     persistent_sparse_kernel<TB, MS, 2, RPL, true>,                                     \
     persistent_sparse_kernel<TB, MS, 3, RPL, true>},

const KernelFn kUniformKernels[kVariantCount][3] = {OIM_PERSIST_VARIANTS(OIM_UNIFORM_ENTRY)};

}  // namespace persist
}  // namespace oim
