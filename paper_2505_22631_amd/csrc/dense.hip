// dense.hip -- dense (all-to-all) coupling path.
#include "internal.hpp"

namespace oim {

int dense_prepare(Problem* p, const float* J) {
    const size_t bytes = (size_t)p->n * p->n * sizeof(float);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->d_Jdense), bytes);
    if (e != hipSuccess) {
        p->d_Jdense = nullptr;
        return e == hipErrorOutOfMemory ? set_error(OIM_E_NOMEM, "dense J: out of device memory")
                                        : hip_error(e, "hipMalloc dense J");
    }
    e = hipMemcpy(p->d_Jdense, J, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "upload dense J");
    return OIM_OK;
}

void dense_release(Problem* p) {
    hipFree(p->d_Jdense);
    hipFree(p->d_Jhi);
    hipFree(p->d_Jlo);
    p->d_Jdense = nullptr;
    p->d_Jhi = p->d_Jlo = nullptr;
}

int launch_dense(Problem*, const oim_run_cfg*, const float*, const float*, const float*,
                 const uint64_t*, int64_t, float*, uint32_t*, const oim_readout*,
                 hipStream_t) {
    return set_error(OIM_E_UNSUPPORTED, "dense run not available yet");
}

}  // namespace oim
