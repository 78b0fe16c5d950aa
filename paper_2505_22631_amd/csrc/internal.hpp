// internal.hpp -- host-side structures shared by the library's translation
// units (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "oim.h"

namespace oim {

constexpr int kMaxQ = 16;
constexpr int kSliceQuads = 64;  // quads (4 oscillators) per slice = one wave's lanes
constexpr int kAdjMaxN = 4096;   // largest instance the adjoint kernels hold in LDS

// Sliced-ELL image of a symmetric CSR, laid out for the LDS-resident kernel:
// slice s covers quads 64s..64s+63 (oscillators 4*quad + j, j = 0..3).  All
// 256 rows of a slice are padded to one degree deg_s (a multiple of 4).  Entry
// e of row j of lane l is the int2 (LDS byte offset of the neighbour's
// (sin, cos) pair, bits of J); entries e and e+1 (e even) of a lane are
// adjacent so one 16-byte load fetches both:
//   int4 index = (base_s + j * deg_s / 2 + e / 2) * 64 + l,  half = e % 2.
// Padding entries carry J = 0 and point at a valid row.  Oscillator i lives
// at LDS slot (i % 4) * (64 * slices) + i / 4 (four planes, one per quad
// member) so the lanes of a wave touch consecutive (sin, cos) pairs.
// A block-diagonal batch gets one image per instance, concatenated: each
// instance starts on a slice boundary and its LDS offsets are local.
struct SellImage {
    int32_t slices = 0;
    std::vector<int2> desc;      // [slices]: (base_s in int4 rows, deg_s)
    std::vector<int2> entries;   // [sum_s 4 * deg_s * 64]
    // With one weight w0 = +-1 on every entry, the same rows as LDS byte
    // offsets alone, four consecutive entries of a row per 16 bytes:
    //   uint4 index = (base_s / 2 + j * deg_s / 4 + e / 4) * 64 + l, word e % 4;
    // padding entries point at the zero entry after the table and the
    // readout colours (byte offset 36 * 64 * slices of the instance).  Empty
    // otherwise.
    std::vector<uint32_t> entries_uw;
    // Per slice s (of the whole batch), row j, lane l, at (s * 4 + j) * 64 + l:
    // (index of the row's first entry with column > the row's own index,
    // row length); rows past an instance's end are (0, 0).  The readouts sum
    // a row's entries from the first to the second.
    std::vector<int2> row_split;
    std::vector<int4> inst;      // [instances]: (first slice, slices, first oscillator, n_b)
    std::vector<int32_t> order;  // instances, most slices first
    int32_t max_slices = 0;
};

constexpr size_t kCsrPad = 4;

struct Problem {
    uint64_t handle = 0;  // registry key, the value callers hold as oim_problem
    int device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    bool dense = false;
    bool integer_weights = false;
    double max_abs_row_sum = 0.0;
    double sum_J_upper = 0.0;

    // device: original CSR (sparse problems), for the readouts and the
    // stepwise loop.  row_ptr is followed by kCsrPad copies of nnz (rows
    // n .. n + 3 are empty, so the bounds of any quad's rows are in bounds),
    // col and J by kCsrPad zero entries (a group of 4 consecutive entries
    // starting at any index <= nnz is in bounds)
    int64_t* d_row_ptr = nullptr;
    int32_t* d_col = nullptr;
    float* d_J = nullptr;

    // device: the CSR padded to ell_D entries per row (EllImage), for the
    // stepwise step kernel, or null (single graphs whose rows are of similar
    // length)
    int32_t* d_ell_col = nullptr;
    float* d_ell_J = nullptr;
    int32_t ell_D = 0;

    // instances of a block-diagonal batch (1 for a single graph)
    int32_t n_inst = 1;
    int32_t max_inst_n = 0;  // largest instance (oscillators)
    int64_t max_inst_nnz = 0;  // most stored entries of one instance
    int64_t max_inst_ell = 0;  // most entries of one instance's padded row image (slices of
                               // 256 rows, each padded to its longest row rounded up to 4)
    bool unit_weights = false; // every |J| is 1
    int4* d_inst = nullptr;
    int32_t* d_order = nullptr;
    int32_t max_slices = 0;

    // device: sliced-ELL image for the LDS-resident step kernel
    int32_t sell_slices = 0;
    int64_t sell_entries = 0;
    int2* d_sell_desc = nullptr;
    int2* d_sell = nullptr;
    uint32_t* d_sell_uw = nullptr;  // unit-weight image, or null
    int2* d_row_split = nullptr;    // SellImage::row_split
    float uniform_w = 0.f;          // the weight every entry shares (+1 or -1), or 0

    // device: dense coupling (dense problems), FP32 and the BF16 split
    float* d_Jdense = nullptr;
    unsigned char* d_Jtiled = nullptr;  // J_hi / J_lo in per-stage tiles
    unsigned char* d_Jtiled32 = nullptr;  // FP32 J in per-stage tiles (made on first FP32 run)

    // cached workspace for the stepwise / dense loops
    void* d_work = nullptr;
    size_t work_bytes = 0;
    // captured step loops of the stepwise form (stepwise.hip), by launch shape
    void* step_plans = nullptr;

    // launch variant of the LDS-resident kernel chosen by the autotuner, per
    // SHIL order class (generic, q = 2, q = 3); 0 = not tuned
    int16_t tuned_tb[3] = {0, 0, 0};
    int16_t tuned_ms[3] = {0, 0, 0};
    int16_t tuned_rpl[3] = {4, 4, 4};

    // cached scratch of the adjoint backward pass, and its second stream and
    // events (start, recomputed[2], adjoint done[2])
    void* d_adj = nullptr;
    size_t adj_bytes = 0;
    hipStream_t adj_stream = nullptr;
    hipEvent_t adj_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

// error plumbing (errors.cpp)
int set_error(int status, const std::string& msg);
int hip_error(hipError_t e, const char* what);
void clear_error();

// validation helpers (validate.cpp): host only, no HIP calls
int validate_csr(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                 const float* J);
int validate_dense(int32_t n, const float* J);
int validate_cfg(const Problem* p, const oim_run_cfg* cfg);
// Handle registry: a problem is known by a number that is never reused, so a
// handle used after oim_problem_destroy is detected without touching freed
// memory.  register_problem fills p->handle; checked() returns the live
// problem of a handle or null; unregister_problem forgets it.
oim_problem register_problem(Problem* p);
Problem* checked(oim_problem h);
void unregister_problem(Problem* p);
int validate_blocks(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t n_inst,
                    const int32_t* inst_off);
// uniform_w: the weight every entry shares (+1 or -1) to build the
// unit-weight image too, or 0.
void build_sell(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const float* J,
                int32_t n_inst, const int32_t* inst_off, SellImage& out, float uniform_w = 0.f);

// Every row padded to the same length D (the longest row rounded up to 4,
// at least 4), quads of rows padded to 4 rows, stored quad by quad in
// groups of 4 entries: entry e = 4t + h of row i = 4m + j at
// m * 4D + 16t + 4j + h, so the group t of a quad's four rows is 16
// consecutive words; each row keeps its CSR order.  A padding entry has
// weight 0 and the row's own column (row n - 1 for rows past n), so a
// gather over it reads a valid word and adds nothing.  With an entry's
// position computed from its quad index alone, the stepwise step kernel
// needs no row bounds before its entry loads.
struct EllImage {
    int32_t D = 0;
    std::vector<int32_t> col;
    std::vector<float> J;
};

// Whether a graph takes the padded image: `mode` 0 never, 1 always,
// otherwise when its rows are of similar length (quads x D / 4 groups of 4
// entries at most 5/4 of what the CSR loop walks, each quad to its longest
// row, one group at least).
bool ell_wanted(int32_t n, const int64_t* row_ptr, int mode);
void build_ell(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const float* J,
               EllImage& out);

// kernels' host launchers
int launch_persistent_sparse(const Problem* p, const oim_run_cfg* cfg, const float* K,
                             const float* Ks, const float* sigma, const uint64_t* seeds,
                             int64_t step0, float* theta, uint32_t* phase,
                             const oim_readout* ro, hipStream_t stream);
int launch_stepwise_sparse(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                           const float* sigma, const uint64_t* seeds, int64_t step0,
                           float* theta, uint32_t* phase, const oim_readout* ro,
                           hipStream_t stream);
void stepwise_release(Problem* p);
size_t stepwise_workspace_bytes(const Problem* p, const oim_run_cfg* cfg);
int launch_stepwise_sparse_ws(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                              const float* sigma, const uint64_t* seeds, int64_t step0,
                              float* theta, uint32_t* phase, const oim_readout* ro,
                              hipStream_t stream, void* work);
size_t dense_workspace_bytes(const Problem* p, const oim_run_cfg* cfg);
int launch_dense_ws(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                    const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
                    uint32_t* phase, const oim_readout* ro, hipStream_t stream, void* work);
// checks of oim_run shared with its allocation-free variant (api.cpp)
int run_common_checks(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                      const float* sigma, const uint64_t* seeds, int64_t step0,
                      const float* theta, const oim_readout* ro);
int launch_dense(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                 const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
                 uint32_t* phase, const oim_readout* ro, hipStream_t stream);
int dense_prepare(Problem* p, const float* J);
void dense_release(Problem* p);
int launch_phase_convert(int64_t count, const float* theta_in, uint32_t* phase_out,
                         const uint32_t* phase_in, float* theta_out, hipStream_t s);
bool persistent_sparse_fits(const Problem* p);
bool persistent_variant_fits(const Problem* p, int tb, int ms, int rpl);
int tune_persistent(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                    const float* sigma, const uint64_t* seeds, const float* theta,
                    int32_t trial_steps, oim_tune_report* rep, hipStream_t stream);
int validate_adjoint_cfg(const Problem* p, const oim_adjoint_cfg* cfg);
int64_t adjoint_checkpoint_words(const Problem* p, const oim_adjoint_cfg* cfg);
constexpr int kAdjEvents = 5;
void adjoint_release(Problem* p);
int launch_adjoint_forward(Problem* p, const oim_adjoint_cfg* cfg, const float* K, const float* Ks,
                           const float* sigma, const uint64_t* seeds, int64_t step0,
                           const float* theta0, uint32_t* ckpt, float* thetaT, double* loss,
                           hipStream_t stream);
int launch_adjoint_backward(Problem* p, const oim_adjoint_cfg* cfg, const float* K, const float* Ks,
                            const float* sigma, const uint64_t* seeds, int64_t step0,
                            const uint32_t* ckpt, double* gK, double* gKs, double* gS,
                            hipStream_t stream);
int launch_round(int32_t q, int64_t count, const float* theta, int8_t* colour, hipStream_t s);
int launch_cut(const Problem* p, int32_t R, const int8_t* colour, int64_t* cut_i64,
               double* cut_f64, hipStream_t s);
int launch_conflicts(const Problem* p, int32_t R, const int8_t* colour, int64_t* conflicts,
                     hipStream_t s);
int launch_energy(const Problem* p, int32_t q, int32_t R, const float* theta,
                  const int8_t* colour, double* h_model, double* h_eq6, hipStream_t s);

}  // namespace oim
