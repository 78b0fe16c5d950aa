// api.cpp -- the extern "C" entry points of include/oim.h.
// Host-side validation always runs before the first HIP call of an entry
// point; device memory of a problem is owned by its oim_problem handle.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

namespace oim {
const char* last_error_cstr();
}  // namespace oim

using namespace oim;

namespace {

// count elements from the host, followed by `pad` zero elements.
template <typename T>
int dev_upload(T** dst, const T* src, size_t count, const char* what, size_t pad = 0) {
    *dst = nullptr;
    if (count + pad == 0) return OIM_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), (count + pad) * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        if (e == hipErrorOutOfMemory) return set_error(OIM_E_NOMEM, std::string(what) + ": out of device memory");
        return hip_error(e, what);
    }
    if (count) e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e == hipSuccess && pad) e = hipMemset(*dst + count, 0, pad * sizeof(T));
    if (e != hipSuccess) return hip_error(e, what);
    return OIM_OK;
}

void release(Problem* p) {
    if (!p) return;
    hipFree(p->d_row_ptr);
    hipFree(p->d_col);
    hipFree(p->d_J);
    hipFree(p->d_ell_col);
    hipFree(p->d_ell_J);
    hipFree(p->d_sell_desc);
    hipFree(p->d_sell);
    hipFree(p->d_sell_uw);
    hipFree(p->d_row_split);
    hipFree(p->d_inst);
    hipFree(p->d_order);
    stepwise_release(p);
    hipFree(p->d_work);
    adjoint_release(p);
    hipFree(p->d_adj);
    dense_release(p);
    unregister_problem(p);
    delete p;
}

void weight_stats(Problem* p, int32_t n, const int64_t* row_ptr, const int32_t* col,
                  const float* J) {
    bool integer = true;
    double mx = 0.0, upper = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double row = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const double w = J[e];
            row += std::fabs(w);
            if (col[e] > i) upper += w;
            if (w != std::nearbyint(w) || std::fabs(w) >= 16777216.0) integer = false;
        }
        if (row > mx) mx = row;
    }
    p->integer_weights = integer;
    p->max_abs_row_sum = mx;
    p->sum_J_upper = upper;
}

int current_device(int* dev) {
    const hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    return OIM_OK;
}

int check_device(const Problem* p) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return set_error(OIM_E_STATE, "problem belongs to another device");
    return OIM_OK;
}

}  // namespace

extern "C" {

__attribute__((visibility("default"))) int oim_abi_version(void) { return OIM_ABI_VERSION; }

__attribute__((visibility("default"))) const char* oim_status_str(int s) {
    switch (s) {
        case OIM_OK: return "OIM_OK";
        case OIM_E_ARG: return "OIM_E_ARG";
        case OIM_E_CSR: return "OIM_E_CSR";
        case OIM_E_ASYM: return "OIM_E_ASYM";
        case OIM_E_NONFINITE: return "OIM_E_NONFINITE";
        case OIM_E_UNSUPPORTED: return "OIM_E_UNSUPPORTED";
        case OIM_E_NOMEM: return "OIM_E_NOMEM";
        case OIM_E_HIP: return "OIM_E_HIP";
        case OIM_E_STATE: return "OIM_E_STATE";
        default: return "OIM_E_UNKNOWN";
    }
}

__attribute__((visibility("default"))) const char* oim_last_error(void) {
    return last_error_cstr();
}

__attribute__((visibility("default"))) int oim_problem_from_csr_blocks(
    int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx, const float* J,
    int32_t n_inst, const int32_t* inst_off, uint32_t flags, oim_problem* out) {
    clear_error();
    if (!out) return set_error(OIM_E_ARG, "out is NULL");
    *out = nullptr;
    if (flags != 0) return set_error(OIM_E_ARG, "flags must be 0");
    int st = validate_csr(n, nnz, row_ptr, col_idx, J);
    if (st) return st;
    if ((st = validate_blocks(n, row_ptr, col_idx, n_inst, inst_off))) return st;
    Problem* p = new (std::nothrow) Problem();
    if (!p) return set_error(OIM_E_NOMEM, "host allocation failed");
    p->n = n;
    p->nnz = nnz;
    p->n_inst = n_inst;
    p->max_inst_n = n;
    p->max_inst_nnz = nnz;
    if (n_inst > 1) {
        p->max_inst_n = 0;
        p->max_inst_nnz = 0;
        for (int32_t b = 0; b < n_inst; ++b) {
            p->max_inst_n = std::max(p->max_inst_n, inst_off[b + 1] - inst_off[b]);
            p->max_inst_nnz = std::max<int64_t>(p->max_inst_nnz,
                                                row_ptr[inst_off[b + 1]] - row_ptr[inst_off[b]]);
        }
    }
    p->unit_weights = true;
    for (int64_t e = 0; e < nnz && p->unit_weights; ++e)
        if (std::fabs(J[e]) != 1.0f) p->unit_weights = false;
    p->max_inst_ell = 0;
    for (int32_t b = 0; b < n_inst; ++b) {
        const int32_t r0 = n_inst > 1 ? inst_off[b] : 0, r1 = n_inst > 1 ? inst_off[b + 1] : n;
        int64_t ell = 0;
        for (int32_t s0 = r0; s0 < r1; s0 += 256) {
            int64_t dmax = 0;
            for (int32_t i = s0; i < std::min(r1, s0 + 256); ++i)
                dmax = std::max<int64_t>(dmax, row_ptr[i + 1] - row_ptr[i]);
            ell += 256 * ((dmax + 3) & ~int64_t(3));
        }
        p->max_inst_ell = std::max(p->max_inst_ell, ell);
    }
    weight_stats(p, n, row_ptr, col_idx, J);
    SellImage img;
    // one weight of +1 or -1 on every entry: the kernel reads a half-size
    // image of offsets alone (OIM_UNIFORM_WEIGHT_IMAGE=0 keeps the general one)
    float w0 = nnz > 0 ? J[0] : 0.f;
    if (!(w0 == 1.0f || w0 == -1.0f)) w0 = 0.f;
    for (int64_t e = 1; e < nnz && w0 != 0.f; ++e)
        if (J[e] != w0) w0 = 0.f;
    if (const char* env = getenv("OIM_UNIFORM_WEIGHT_IMAGE"))
        if (atoi(env) == 0) w0 = 0.f;
    build_sell(n, row_ptr, col_idx, J, n_inst, n_inst > 1 ? inst_off : nullptr, img, w0);
    p->uniform_w = w0;
    p->sell_slices = img.slices;
    p->max_slices = img.max_slices;
    p->sell_entries = (int64_t)img.entries.size();
    // row_ptr with kCsrPad more copies of nnz: rows past n are empty
    std::vector<int64_t> row_ptr_padded(row_ptr, row_ptr + (size_t)n + 1);
    row_ptr_padded.resize((size_t)n + 1 + kCsrPad, nnz);
    if ((st = current_device(&p->device)) ||
        (st = dev_upload(&p->d_row_ptr, row_ptr_padded.data(), row_ptr_padded.size(),
                         "upload row_ptr")) ||
        (st = dev_upload(&p->d_col, col_idx, (size_t)nnz, "upload col_idx", kCsrPad)) ||
        (st = dev_upload(&p->d_J, J, (size_t)nnz, "upload J", kCsrPad)) ||
        (st = dev_upload(&p->d_sell_desc, img.desc.data(), img.desc.size(), "upload slices")) ||
        (st = dev_upload(&p->d_sell, img.entries.data(), img.entries.size(), "upload sell")) ||
        (st = dev_upload(&p->d_sell_uw, img.entries_uw.data(), img.entries_uw.size(),
                         "upload unit-weight sell")) ||
        (st = dev_upload(&p->d_row_split, img.row_split.data(), img.row_split.size(),
                         "upload row split")) ||
        (st = dev_upload(&p->d_inst, img.inst.data(), img.inst.size(), "upload instances")) ||
        (st = dev_upload(&p->d_order, img.order.data(), img.order.size(), "upload order"))) {
        release(p);
        return st;
    }
    // the padded row image of the stepwise loop (OIM_STEPWISE_ELL=0 never
    // builds it, =1 builds it for any single graph)
    int ell_mode = 2;
    if (const char* env = getenv("OIM_STEPWISE_ELL")) ell_mode = atoi(env) == 0 ? 0 : 1;
    if (n_inst == 1 && ell_wanted(n, row_ptr, ell_mode)) {
        EllImage ell;
        build_ell(n, row_ptr, col_idx, J, ell);
        p->ell_D = ell.D;
        if ((st = dev_upload(&p->d_ell_col, ell.col.data(), ell.col.size(), "upload ell col")) ||
            (st = dev_upload(&p->d_ell_J, ell.J.data(), ell.J.size(), "upload ell J"))) {
            release(p);
            return st;
        }
    }
    *out = register_problem(p);
    return OIM_OK;
}

__attribute__((visibility("default"))) int oim_problem_from_csr(
    int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx, const float* J,
    uint32_t flags, oim_problem* out) {
    return oim_problem_from_csr_blocks(n, nnz, row_ptr, col_idx, J, 1, nullptr, flags, out);
}

__attribute__((visibility("default"))) int oim_problem_from_dense(int32_t n, const float* J,
                                                                  uint32_t flags,
                                                                  oim_problem* out) {
    clear_error();
    if (!out) return set_error(OIM_E_ARG, "out is NULL");
    *out = nullptr;
    if (flags != 0) return set_error(OIM_E_ARG, "flags must be 0");
    int st = validate_dense(n, J);
    if (st) return st;
    Problem* p = new (std::nothrow) Problem();
    if (!p) return set_error(OIM_E_NOMEM, "host allocation failed");
    p->n = n;
    p->dense = true;
    // statistics over the off-diagonal entries
    bool integer = true;
    double mx = 0.0, upper = 0.0;
    int64_t nz = 0;
    for (int32_t i = 0; i < n; ++i) {
        double row = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double w = J[(int64_t)i * n + j];
            if (w != 0.0) ++nz;
            row += std::fabs(w);
            if (j > i) upper += w;
            if (w != std::nearbyint(w) || std::fabs(w) >= 16777216.0) integer = false;
        }
        if (row > mx) mx = row;
    }
    p->nnz = nz;
    p->integer_weights = integer;
    p->max_abs_row_sum = mx;
    p->sum_J_upper = upper;
    if ((st = current_device(&p->device)) || (st = dense_prepare(p, J))) {
        release(p);
        return st;
    }
    *out = register_problem(p);
    return OIM_OK;
}

__attribute__((visibility("default"))) void oim_problem_destroy(oim_problem h) {
    Problem* p = checked(h);
    if (!p) return;
    hipDeviceSynchronize();
    release(p);
}

__attribute__((visibility("default"))) int oim_problem_info_get(oim_problem h,
                                                                oim_problem_info* info) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    if (!info) return set_error(OIM_E_ARG, "info is NULL");
    std::memset(info, 0, sizeof *info);
    info->n = p->n;
    info->is_dense = p->dense ? 1 : 0;
    info->nnz = p->nnz;
    info->integer_weights = p->integer_weights ? 1 : 0;
    info->n_instances = p->n_inst;
    info->max_abs_row_sum = p->max_abs_row_sum;
    info->sum_J_upper = p->sum_J_upper;
    info->max_instance_n = p->dense ? p->n : p->max_inst_n;
    info->uniform_weight = p->d_sell_uw ? p->uniform_w : 0.f;
    info->stepwise_row_length = p->d_ell_col ? p->ell_D : 0;
    return OIM_OK;
}

}  // extern "C"

namespace oim {

// Argument checks of oim_run and of its allocation-free variant, before any
// device work.
int run_common_checks(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                      const float* sigma, const uint64_t* seeds, int64_t step0,
                      const float* theta, const oim_readout* ro) {
    int st = validate_cfg(p, cfg);
    if (st) return st;
    if (!theta || !seeds) return set_error(OIM_E_ARG, "theta or seeds is NULL");
    if (cfg->steps > 0 && (!K || !Ks || !sigma))
        return set_error(OIM_E_ARG, "schedule pointer is NULL");
    if (step0 < 0 || step0 + (int64_t)cfg->steps > ((int64_t)1 << 32))
        return set_error(OIM_E_ARG, "global step index must stay below 2^32");
    if (ro && cfg->readout_every == 0 && (ro->trace || ro->best_h || ro->best_step || ro->best_colour))
        return set_error(OIM_E_ARG, "readout buffers given with readout_every = 0");
    const uint32_t loop = cfg->flags & OIM_LOOP_MASK;
    if (p->dense && loop == OIM_LOOP_PERSISTENT)
        return set_error(OIM_E_UNSUPPORTED, "dense problems run stepwise");
    if (!p->dense && p->n_inst > 1 && (loop == OIM_LOOP_STEPWISE || !persistent_sparse_fits(p)))
        return set_error(OIM_E_UNSUPPORTED, "block-diagonal batches run on the LDS-resident loop only");
    if (!p->dense && loop == OIM_LOOP_PERSISTENT && !persistent_sparse_fits(p))
        return set_error(OIM_E_UNSUPPORTED, "replica does not fit the LDS-resident kernel");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return set_error(OIM_E_STATE, "problem belongs to another device");
    return OIM_OK;
}

}  // namespace oim

extern "C" {

__attribute__((visibility("default"))) int oim_run(oim_problem h, const oim_run_cfg* cfg,
                                                   const float* K, const float* Ks,
                                                   const float* sigma, const uint64_t* seeds,
                                                   int64_t step0, float* theta, uint32_t* phase,
                                                   const oim_readout* ro, hipStream_t stream) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    int st = run_common_checks(p, cfg, K, Ks, sigma, seeds, step0, theta, ro);
    if (st) return st;
    if (cfg->steps == 0) return OIM_OK;  // nothing to integrate; theta untouched
    const uint32_t loop = cfg->flags & OIM_LOOP_MASK;
    if (p->dense) return launch_dense(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream);
    if (loop == OIM_LOOP_PERSISTENT || (loop == OIM_LOOP_AUTO && persistent_sparse_fits(p)))
        return launch_persistent_sparse(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro,
                                        stream);
    return launch_stepwise_sparse(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream);
}

__attribute__((visibility("default"))) int oim_autotune(oim_problem h, const oim_run_cfg* cfg,
                                                        const float* K, const float* Ks,
                                                        const float* sigma,
                                                        const uint64_t* seeds, const float* theta,
                                                        int32_t trial_steps,
                                                        oim_tune_report* report,
                                                        hipStream_t stream) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    int st = validate_cfg(p, cfg);
    if (st) return st;
    if (p->dense) return set_error(OIM_E_UNSUPPORTED, "autotuning applies to sparse problems");
    if (trial_steps < 1 || trial_steps > cfg->steps)
        return set_error(OIM_E_ARG, "trial_steps must be in [1, cfg->steps]");
    if (!K || !Ks || !sigma || !seeds || !theta) return set_error(OIM_E_ARG, "NULL array");
    if ((st = check_device(p))) return st;
    return tune_persistent(p, cfg, K, Ks, sigma, seeds, theta, trial_steps, report, stream);
}

__attribute__((visibility("default"))) int oim_set_tuning(oim_problem h, int32_t q, int32_t block,
                                                          int32_t slices_per_wave,
                                                          int32_t rows_per_lane) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    if (q < 2 || q > kMaxQ) return set_error(OIM_E_ARG, "q must be in [2, 16]");
    if (p->dense) return set_error(OIM_E_UNSUPPORTED, "tuning applies to sparse problems");
    const int qc = q == 2 ? 1 : q == 3 ? 2 : 0;
    if (block == 0) {
        p->tuned_tb[qc] = p->tuned_ms[qc] = 0;
        p->tuned_rpl[qc] = 4;
        return OIM_OK;
    }
    if (!persistent_variant_fits(p, block, slices_per_wave, rows_per_lane))
        return set_error(OIM_E_ARG, "no launch variant (" + std::to_string(block) + ", " +
                                        std::to_string(slices_per_wave) + ", " +
                                        std::to_string(rows_per_lane) +
                                        ") covering the largest instance");
    p->tuned_tb[qc] = (int16_t)block;
    p->tuned_ms[qc] = (int16_t)slices_per_wave;
    p->tuned_rpl[qc] = (int16_t)rows_per_lane;
    return OIM_OK;
}

__attribute__((visibility("default"))) int oim_adjoint_checkpoint_words(oim_problem h,
                                                                        const oim_adjoint_cfg* cfg,
                                                                        int64_t* words) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    if (!words) return set_error(OIM_E_ARG, "words is NULL");
    const int st = validate_adjoint_cfg(p, cfg);
    if (st) return st;
    *words = adjoint_checkpoint_words(p, cfg);
    return OIM_OK;
}

namespace {
int adjoint_common(Problem* p, const oim_adjoint_cfg* cfg, const float* K, const float* Ks,
                   const float* sigma, const uint64_t* seeds, int64_t step0) {
    int st = validate_adjoint_cfg(p, cfg);
    if (st) return st;
    if (!seeds) return set_error(OIM_E_ARG, "seeds is NULL");
    if (cfg->steps > 0 && (!K || !Ks || !sigma))
        return set_error(OIM_E_ARG, "schedule pointer is NULL");
    if (step0 < 0 || step0 + (int64_t)cfg->steps > ((int64_t)1 << 32))
        return set_error(OIM_E_ARG, "global step index must stay below 2^32");
    return check_device(p);
}
}  // namespace

__attribute__((visibility("default"))) int oim_adjoint_forward(
    oim_problem h, const oim_adjoint_cfg* cfg, const float* K, const float* Ks, const float* sigma,
    const uint64_t* seeds, int64_t step0, const float* theta0, uint32_t* ckpt, float* theta_T,
    double* loss, hipStream_t stream) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    int st = adjoint_common(p, cfg, K, Ks, sigma, seeds, step0);
    if (st) return st;
    if (!theta0) return set_error(OIM_E_ARG, "theta0 is NULL");
    if (cfg->steps > 0 && !ckpt) return set_error(OIM_E_ARG, "ckpt is NULL");
    return launch_adjoint_forward(p, cfg, K, Ks, sigma, seeds, step0, theta0, ckpt, theta_T, loss,
                                  stream);
}

__attribute__((visibility("default"))) int oim_adjoint_backward(
    oim_problem h, const oim_adjoint_cfg* cfg, const float* K, const float* Ks, const float* sigma,
    const uint64_t* seeds, int64_t step0, const uint32_t* ckpt, double* gK, double* gKs,
    double* gsigma, hipStream_t stream) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    int st = adjoint_common(p, cfg, K, Ks, sigma, seeds, step0);
    if (st) return st;
    if (cfg->steps == 0) return OIM_OK;
    if (!ckpt || !gK || !gKs || !gsigma) return set_error(OIM_E_ARG, "NULL array");
    return launch_adjoint_backward(p, cfg, K, Ks, sigma, seeds, step0, ckpt, gK, gKs, gsigma,
                                   stream);
}

__attribute__((visibility("default"))) int oim_phase_from_theta(int64_t count,
                                                                const float* theta,
                                                                uint32_t* phase,
                                                                hipStream_t stream) {
    clear_error();
    if (count < 0) return set_error(OIM_E_ARG, "count must be >= 0");
    if (count > 0 && (!theta || !phase)) return set_error(OIM_E_ARG, "NULL array");
    return launch_phase_convert(count, theta, phase, nullptr, nullptr, stream);
}

__attribute__((visibility("default"))) int oim_theta_from_phase(int64_t count,
                                                                const uint32_t* phase,
                                                                float* theta,
                                                                hipStream_t stream) {
    clear_error();
    if (count < 0) return set_error(OIM_E_ARG, "count must be >= 0");
    if (count > 0 && (!theta || !phase)) return set_error(OIM_E_ARG, "NULL array");
    return launch_phase_convert(count, nullptr, nullptr, phase, theta, stream);
}

__attribute__((visibility("default"))) int oim_round(int32_t q, int64_t count, const float* theta,
                                                     int8_t* colour, hipStream_t stream) {
    clear_error();
    if (q < 2 || q > kMaxQ) return set_error(OIM_E_ARG, "q must be in [2, 16]");
    if (count < 0) return set_error(OIM_E_ARG, "count must be >= 0");
    if (count > 0 && (!theta || !colour)) return set_error(OIM_E_ARG, "NULL array");
    return launch_round(q, count, theta, colour, stream);
}

__attribute__((visibility("default"))) int oim_cut(oim_problem h, int32_t R, const int8_t* colour,
                                                   int64_t* cut_i64, double* cut_f64,
                                                   hipStream_t stream) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    if (R < 1) return set_error(OIM_E_ARG, "R must be >= 1");
    if (!colour) return set_error(OIM_E_ARG, "colour is NULL");
    if (cut_i64 && !p->integer_weights)
        return set_error(OIM_E_UNSUPPORTED, "exact int64 cut needs integer weights");
    if (!cut_i64 && !cut_f64) return OIM_OK;
    int st = check_device(p);
    if (st) return st;
    return launch_cut(p, R, colour, cut_i64, cut_f64, stream);
}

__attribute__((visibility("default"))) int oim_conflicts(oim_problem h, int32_t R,
                                                         const int8_t* colour, int64_t* conflicts,
                                                         hipStream_t stream) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    if (R < 1) return set_error(OIM_E_ARG, "R must be >= 1");
    if (!colour || !conflicts) return set_error(OIM_E_ARG, "NULL array");
    int st = check_device(p);
    if (st) return st;
    return launch_conflicts(p, R, colour, conflicts, stream);
}

__attribute__((visibility("default"))) int oim_energy(oim_problem h, int32_t q, int32_t R,
                                                      const float* theta, const int8_t* colour,
                                                      double* h_model, double* h_eq6,
                                                      hipStream_t stream) {
    clear_error();
    Problem* p = checked(h);
    if (!p) return set_error(OIM_E_STATE, "invalid or destroyed problem");
    if (q < 2 || q > kMaxQ) return set_error(OIM_E_ARG, "q must be in [2, 16]");
    if (R < 1) return set_error(OIM_E_ARG, "R must be >= 1");
    if (h_model && !colour) return set_error(OIM_E_ARG, "colour is NULL");
    if (h_eq6 && !theta) return set_error(OIM_E_ARG, "theta is NULL");
    if (!h_model && !h_eq6) return OIM_OK;
    int st = check_device(p);
    if (st) return st;
    return launch_energy(p, q, R, theta, colour, h_model, h_eq6, stream);
}

}  // extern "C"
