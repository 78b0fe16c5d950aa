// noalloc.hip -- oim_run_noalloc: oim_run for callers that cannot allocate
// device memory (code under hipGraph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The stepwise and dense loops need a workspace (phase words, the (sin, cos)
// or split-X ping-pong buffers, readout partials and per-call arguments).
// oim_run allocates it on first use and caches it in the problem; this entry
// point takes it from a fixed device array, `scratch`, of kScratchBytes that
// the library's code object carries, so the call allocates nothing.  Each
// device holds its own copy of the array at its own address, looked up once
// per device with hipGetSymbolAddress on the first call made with that device
// current; host code passes that address, never the array's name (which on
// the host is only a stand-in for the symbol).  Every call on a device shares
// the array: calls that overlap on one device (concurrent streams or threads)
// race on it.  Nothing in it needs to start at zero: each run writes every
// part it later reads (the init kernel fills the state and both buffers, the
// first readout of a call resets the best-so-far, the per-call argument block
// is written by the call's first kernel).
#include <mutex>

#include "internal.hpp"

namespace oim {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device).
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(OIM_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return set_error(OIM_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return OIM_OK;
}

}  // namespace

}  // namespace oim

extern "C" {

__attribute__((visibility("default"))) size_t oim_noalloc_scratch_bytes(void) {
    return oim::kScratchBytes;
}

__attribute__((visibility("default"))) int oim_run_noalloc(oim_problem h, const oim_run_cfg* cfg,
                                                           const float* K, const float* Ks,
                                                           const float* sigma,
                                                           const uint64_t* seeds, int64_t step0,
                                                           float* theta, uint32_t* phase,
                                                           const oim_readout* ro,
                                                           hipStream_t stream) {
    using namespace oim;
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    int st = run_common_checks(p, cfg, K, Ks, sigma, seeds, step0, theta, ro);
    if (st) return st;
    if (cfg->steps == 0) return OIM_OK;
    const uint32_t loop = cfg->flags & OIM_LOOP_MASK;
    const bool persistent =
        !p->dense && (loop == OIM_LOOP_PERSISTENT || (loop == OIM_LOOP_AUTO && persistent_sparse_fits(p)));
    // the LDS-resident loop keeps its state on chip: no workspace at all
    if (persistent)
        return launch_persistent_sparse(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro,
                                        stream);
    const size_t need =
        p->dense ? dense_workspace_bytes(p, cfg) : stepwise_workspace_bytes(p, cfg);
    if (need > kScratchBytes)
        return set_error(OIM_E_UNSUPPORTED,
                         "run needs " + std::to_string(need) + " bytes of workspace; the "
                         "allocation-free entry point holds " + std::to_string(kScratchBytes));
    void* work = nullptr;
    if ((st = scratch_address(p->device, &work))) return st;
    if (p->dense)
        return launch_dense_ws(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream, work);
    return launch_stepwise_sparse_ws(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream,
                                     work);
}

}  // extern "C"
