/*
 * oim.h -- C ABI of the MI355X simulated oscillator Ising/Potts machine.
 *
 * The library integrates the noisy Kuramoto network with sub-harmonic
 * injection locking of arXiv 2505.22631 (Sec. II-D Eq. 4, Sec. II-E Eq. 5,
 * Algorithm 1) on a gfx950 GPU and reads the result out as spins/colours,
 * cut values, colouring conflicts and energies (Sec. II-A Eq. 1 and 2,
 * Sec. II-E Eq. 6).
 *
 * Conventions (every entry point):
 *   - Phases are radians.  theta is a caller-owned FP32 device array laid out
 *     [R][n] (replica-major).  The library keeps phases in one period.
 *   - On the device a phase is a 32-bit fixed-point fraction of a turn,
 *     u = theta / 2pi * 2^32 mod 2^32 (the "phase word"): the wrap into one
 *     period is exact and the state resolution is 2^-32 turn.  Runs read and
 *     write FP32 radians; callers that need the exact state (checkpoints,
 *     bit-exact resume) also pass the phase words.
 *   - J is the Ising/Potts coupling of Eq. 1 / Eq. 2 (H = -sum_{i<j} J_ij s_i s_j).
 *     Max-cut with edge weights w maps to J = -w, graph colouring to J = -1 on
 *     every edge (Sec. II-C).  J must be symmetric; the diagonal is ignored.
 *   - The integrated drift, per oscillator i and step t, is
 *         f_i = -K_t * sum_j J_ij sin(theta_i - theta_j) - Ks_t * sin(q theta_i)
 *     and the Euler-Maruyama step is
 *         theta_i <- wrap(theta_i + dt f_i + sigma_t sqrt(dt) xi_{i,t}),
 *     all oscillators updated from the phases of step t (Algorithm 1).
 *   - xi_{i,t} for replica r comes from Philox4x32-10 (Salmon et al., SC'11)
 *     with key (seed_r low word, seed_r high word) and counter (i/4, t, b, 0),
 *     t the global step index, i the oscillator's index within its instance
 *     and b the instance (0 unless the problem is a block-diagonal batch,
 *     oim_problem_from_csr_blocks); words (x0,x1) feed oscillators i%4 = 0,1 and
 *     (x2,x3) feed i%4 = 2,3 through Box-Muller on 24-bit uniforms
 *     u1 = ((xa>>8)+1)/2^24, u2 = (xb>>8)/2^24: the even oscillator of a pair
 *     takes sqrt(-2 ln u1) cos(2 pi u2), the odd one the sine.
 *   - Device pointers must be on the device that was current when the problem
 *     was created.  Work is enqueued on `stream` (NULL = the null stream) and
 *     is asynchronous unless stated otherwise.
 *   - Every function returns an oim_status and never aborts.  All argument
 *     checks run on the host before any device work, so a rejected call leaves
 *     device memory untouched.  oim_last_error() holds a per-thread detail
 *     string for the last failure.
 *   - A problem may be used by one stream at a time.
 *   - A handle is a number that is never reused: using it after
 *     oim_problem_destroy returns OIM_E_STATE.
 */
#ifndef OIM_H
#define OIM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OIM_ABI_VERSION 4

typedef enum {
    OIM_OK = 0,
    OIM_E_ARG = 1,          /* bad argument: NULL pointer, size or range     */
    OIM_E_CSR = 2,          /* malformed CSR (order, range, loops, repeats)  */
    OIM_E_ASYM = 3,         /* J is not exactly symmetric                    */
    OIM_E_NONFINITE = 4,    /* NaN or Inf in J                               */
    OIM_E_UNSUPPORTED = 5,  /* valid request the library cannot serve        */
    OIM_E_NOMEM = 6,        /* device or host allocation failed              */
    OIM_E_HIP = 7,          /* a HIP runtime call failed (see last_error)    */
    OIM_E_STATE = 8         /* object used after destroy / wrong device      */
} oim_status;

typedef struct oim_problem_s* oim_problem;

/* Version of this ABI (OIM_ABI_VERSION). */
int oim_abi_version(void);

/* Static name of a status code ("OIM_E_CSR", ...). */
const char* oim_status_str(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char* oim_last_error(void);

/* ------------------------------------------------------------------------
 * Problem upload (Sec. III-B: the coupling matrix is stored on the device).
 * Inputs are HOST pointers and are copied; the caller may free them after the
 * call returns.  The call is synchronous.
 * ---------------------------------------------------------------------- */

/* Sparse coupling in CSR form: row_ptr[n+1] (row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = nnz), col_idx[nnz] strictly increasing within each row, in
 * [0, n), no diagonal entries; J[nnz] finite and symmetric (the entry (j,i)
 * exists and has bit-identical value for every stored (i,j)).
 * Errors: OIM_E_ARG (n < 1, n > 2^24, nnz < 0, NULL pointer), OIM_E_CSR,
 * OIM_E_ASYM, OIM_E_NONFINITE, OIM_E_NOMEM, OIM_E_HIP.  flags must be 0. */
int oim_problem_from_csr(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                         const float* J, uint32_t flags, oim_problem* out);

/* A batch of independent instances as one block-diagonal CSR: instance b
 * holds oscillators inst_off[b] .. inst_off[b+1]-1 (inst_off[0] = 0,
 * strictly increasing, inst_off[n_inst] = n) and no entry couples two
 * instances (else OIM_E_CSR).  Each (instance, replica) runs as an independent
 * solve; in-run readouts are per (replica, instance), laid out r * n_inst + b
 * (NEXT: the ragged multi-instance batch of the colouring benchmark).  Such
 * problems run on the LDS-resident loop only.  Other arguments and errors as
 * for oim_problem_from_csr.  oim_problem_from_csr is the n_inst = 1 case. */
int oim_problem_from_csr_blocks(int32_t n, int64_t nnz, const int64_t* row_ptr,
                                const int32_t* col_idx, const float* J, int32_t n_inst,
                                const int32_t* inst_off, uint32_t flags, oim_problem* out);

/* Dense coupling J[n][n] row-major (Sec. III-B: flattened coupling matrix).
 * J must be finite and symmetric off the diagonal; the diagonal is ignored.
 * Errors as for oim_problem_from_csr.  1 <= n <= 65536.  flags must be 0. */
int oim_problem_from_dense(int32_t n, const float* J, uint32_t flags, oim_problem* out);

/* Frees every device and host resource of p.  NULL is a no-op.  Waits for the
 * device work already enqueued on p to finish. */
void oim_problem_destroy(oim_problem p);

typedef struct {
    int32_t n;                 /* oscillators                                       */
    int32_t is_dense;          /* 1 for oim_problem_from_dense                      */
    int64_t nnz;               /* stored off-diagonal nonzeros (both triangles)     */
    int32_t integer_weights;   /* 1 if every J is an integer of magnitude < 2^24    */
    int32_t n_instances;       /* instances of a block-diagonal batch (else 1)      */
    double max_abs_row_sum;    /* max_i sum_j |J_ij| (Gershgorin bound of J)         */
    double sum_J_upper;        /* sum_{i<j} J_ij; max-cut total weight W = -this     */
    int32_t max_instance_n;    /* oscillators of the largest instance (n if one)    */
    float uniform_weight;      /* +1 or -1 when every stored J equals it (the      */
                               /* LDS-resident loop then reads a half-size image   */
                               /* of neighbour offsets alone, same results bit for */
                               /* bit), else 0                                     */
    int32_t stepwise_row_length; /* entries per row of the padded row image the   */
                               /* stepwise loop reads (a single graph whose rows   */
                               /* are of similar length; same results bit for bit  */
                               /* as the CSR), else 0 (the CSR)                    */
} oim_problem_info;

/* Fills *info (host memory).  Synchronous, no device work. */
int oim_problem_info_get(oim_problem p, oim_problem_info* info);

/* ------------------------------------------------------------------------
 * Run: steps of Algorithm 1 on R independent replicas.
 * ---------------------------------------------------------------------- */

/* cfg.flags: loop form and precision (one of each; 0 = AUTO / FP32). */
#define OIM_LOOP_AUTO        0x0u
#define OIM_LOOP_PERSISTENT  0x1u  /* one launch, replica state resident in LDS      */
#define OIM_LOOP_STEPWISE    0x2u  /* one kernel per step, state in device memory    */
#define OIM_LOOP_MASK        0x3u
#define OIM_PREC_FP32        0x0u  /* FP32 coupling sum (dense: FP32 products on MFMA) */
#define OIM_PREC_BF16X3      0x10u /* dense only: BF16 three-term split on MFMA       */
#define OIM_PREC_MASK        0x30u
#define OIM_SCHED_PER_REPLICA 0x100u /* K, Ks, sigma are [R][steps]: one schedule per  */
                                     /* replica (shared by its instances); default     */
                                     /* [steps] for every replica                      */

typedef struct {
    int32_t q;              /* stable phases per oscillator: 2 = Ising, 3.. = Potts (<= 16) */
    int32_t R;              /* replicas (independent copies, own seeds), >= 1              */
    int32_t steps;          /* Euler-Maruyama steps, >= 0                                 */
    float dt;               /* time step h of Algorithm 1, finite and > 0                  */
    int32_t readout_every;  /* M > 0: threshold + energy every M steps and after the last  */
                            /* step; 0: no in-run readout                                  */
    uint32_t flags;         /* OIM_LOOP_* | OIM_PREC_* | OIM_SCHED_PER_REPLICA               */
} oim_run_cfg;

/* Optional in-run readout buffers (device memory, any may be NULL).
 * With M = readout_every > 0 there are ceil(steps / M) readouts, after local
 * steps M, 2M, ... and after the last step.  At each readout every replica's
 * phases are thresholded to colours k = floor(q * u / 2^32 + 1/2) mod q from
 * the exact phase words u, and H is evaluated: Eq. 1 (q = 2, spin s = 1 - 2k)
 * or Eq. 2 (q >= 3).
 *   trace[ceil(steps/M)][R*I]  H at every readout (I = instances, entry r*I+b)
 *   best_h[R*I]                lowest H seen in this call (first occurrence)
 *   best_step[R*I]             global step index after which best_h was seen
 *   best_colour[R][n]          colours at that readout (per instance range)    */
typedef struct {
    double* trace;
    double* best_h;
    int32_t* best_step;
    int8_t* best_colour;
} oim_readout;

/* K, Ks, sigma: device FP32 [steps], indexed by the LOCAL step s = 0..steps-1
 * (coupling strength, SHIL strength, noise amplitude per step); with
 * OIM_SCHED_PER_REPLICA they are [R][steps], row r driving replica r (a
 * batched sweep of annealing schedules, as in Sec. III-D / Fig. 3b).
 * seeds: device uint64 [R].  step0: global index of the first step (noise
 * counter).  theta: device FP32 [R][n], overwritten with the final phases in
 * [0, 2pi); an input phase that is NaN or infinite is taken as 0.  phase: NULL, or device uint32 [R][n] phase words; when given,
 * the initial state is read from phase (theta's input is ignored) and the
 * final state is written to both.  Resuming with the phase words of a
 * previous call, step0 = its end and the schedule suffix reproduces an
 * uninterrupted run bit for bit.  steps = 0 does no device work.
 * readout may be NULL.  The call only enqueues work on `stream` (every loop
 * form); the stepwise form captures its step loop into a hipGraph on the
 * first call for a launch shape (q, R, readout period) and replays the cached
 * graph on later calls, and its workspace is cached in p (both freed by
 * oim_problem_destroy).  Errors: OIM_E_ARG, OIM_E_UNSUPPORTED (e.g. BF16X3 on
 * a sparse problem, PERSISTENT when a replica does not fit in LDS),
 * OIM_E_NOMEM, OIM_E_HIP. */
int oim_run(oim_problem p, const oim_run_cfg* cfg, const float* K, const float* Ks,
            const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
            uint32_t* phase, const oim_readout* readout, hipStream_t stream);

/* oim_run for callers that cannot allocate device memory: code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, checks, results (bit for bit) and asynchrony as oim_run,
 * but no allocation of any kind: the LDS-resident loop needs no workspace;
 * the stepwise and dense loops take theirs from a fixed device array of
 * oim_noalloc_scratch_bytes() (64 MiB) inside the library, one per device,
 * held until the process ends, and launch their per-step kernels directly
 * (no hipGraph is instantiated).  A run whose workspace exceeds the array is
 * rejected with OIM_E_UNSUPPORTED (the stepwise loop needs about
 * 8 * n * ceil(R / 64) * 64 bytes, the dense loop
 * 20 * ceil(n / 128) * 128 * ceil(R / 64) * 64 bytes); so is an FP32 run on
 * a dense problem whose FP32 image of J has not been made by an earlier
 * oim_run with OIM_PREC_FP32.  Every call on one device shares that device's
 * array: calls that overlap on one device (other streams or threads) race
 * and must not be issued.  Errors: as oim_run, without OIM_E_NOMEM. */
int oim_run_noalloc(oim_problem p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                    const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
                    uint32_t* phase, const oim_readout* readout, hipStream_t stream);

/* Size in bytes of the per-device array oim_run_noalloc takes its
 * workspace from. */
size_t oim_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------
 * Launch-shape autotuning of the LDS-resident loop (the per-thread batch of
 * oscillators of Sec. III-C, chosen by measurement).  A launch variant is a
 * workgroup size (64 ... 1024 threads), a number of 64-quad slices per wave
 * group and a number of rows of each quad of 4 oscillators per lane: 4 (a
 * lane owns whole quads) or 2 or 1 (the waves of a group split each quad's
 * rows, which keeps every wave busy on instances of few slices with long
 * rows).  Any variant gives bit-identical results, only the speed differs.
 * ---------------------------------------------------------------------- */
#define OIM_TUNE_MAX 64
typedef struct {
    int32_t n_tried;                          /* variants timed (<= OIM_TUNE_MAX listed) */
    int32_t chosen_block;                     /* threads per workgroup of the winner */
    int32_t chosen_slices_per_wave;
    int32_t chosen_rows_per_lane;
    float chosen_ms;                          /* its median time in the final pass */
    int32_t block[OIM_TUNE_MAX];              /* every variant tried, in order */
    int32_t slices_per_wave[OIM_TUNE_MAX];
    int32_t rows_per_lane[OIM_TUNE_MAX];
    float ms[OIM_TUNE_MAX];                   /* best of two timings, milliseconds */
} oim_tune_report;

/* Times every launch variant that covers the problem's largest instance on
 * the first trial_steps steps of the given schedules (device arrays of at
 * least cfg->steps entries; seeds [R]; theta [R][n] device, read only: the
 * trials run on a scratch copy, without readout; with OIM_SCHED_PER_REPLICA
 * the schedules are [R][cfg->steps] and each replica runs the first steps of
 * its own row), then the four fastest again three times on
 * min(cfg->steps, 2 trial_steps) steps, and keeps the one with the smallest
 * median for later oim_run calls on p with the same SHIL order class (q = 2,
 * q = 3, other).  cfg gives q, R, dt; its steps must be >= trial_steps >= 1.
 * report may be NULL.  Synchronous (waits for the trials on stream).
 * Allocates and frees a scratch copy of theta.  Errors: OIM_E_ARG,
 * OIM_E_UNSUPPORTED (dense problem, or a replica that does not fit the
 * LDS-resident loop), OIM_E_NOMEM, OIM_E_HIP. */
int oim_autotune(oim_problem p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                 const float* sigma, const uint64_t* seeds, const float* theta,
                 int32_t trial_steps, oim_tune_report* report, hipStream_t stream);

/* Sets the launch variant for SHIL order q's class directly (a choice cached
 * from an earlier oim_autotune on a problem of the same shape); block = 0
 * returns to the default choice.  Errors: OIM_E_ARG (q out of range, no
 * such variant, or one whose waves do not cover the largest instance or
 * whose LDS does not fit), OIM_E_UNSUPPORTED (dense problem). */
int oim_set_tuning(oim_problem p, int32_t q, int32_t block, int32_t slices_per_wave,
                   int32_t rows_per_lane);

/* Phase words <-> radians for count elements (device arrays):
 * phase = rint(frac(theta / 2pi) * 2^32) mod 2^32 (FP64), and
 * theta = nearest FP32 to phase * 2pi / 2^32, kept below 2pi.
 * Non-finite theta gives phase 0. */
int oim_phase_from_theta(int64_t count, const float* theta, uint32_t* phase, hipStream_t stream);
int oim_theta_from_phase(int64_t count, const uint32_t* phase, float* theta, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Readout (Sec. III-B phase threshold kernel; Eq. 1, 2, 6).
 *
 * Every FP64 sum of these readouts, and of the in-run readouts of oim_run,
 * follows one fixed order: each row i sums its terms over the upper triangle
 * j > i in ascending column order, starting from +0; the row sums are
 * combined by the pairwise tree over rows (zero-padded to a power of two,
 * adjacent pairs first, lower rows on the left).  The values are therefore
 * reproducible bit for bit from identical colours, on any loop form, and for
 * integer weights (exact in any order) they equal the exact sums.
 * ---------------------------------------------------------------------- */

/* colour[k] = floor(fmaf(theta[k], (float)(q / 2pi), 0.5f)) mod q for
 * count elements (FP32 decision), -1 where theta is NaN, Inf or
 * |theta| >= 2^20.  Device arrays; 2 <= q <= 16; count >= 0. */
int oim_round(int32_t q, int64_t count, const float* theta, int8_t* colour, hipStream_t stream);

/* Max-cut value per replica: cut[r] = sum_{i<j} (-J_ij) [colour_ri != colour_rj]
 * over colour[R][n].  cut_i64 (exact) requires integer_weights; cut_f64 is the
 * same sum in FP64 (exact for integer weights).  Either may be NULL. */
int oim_cut(oim_problem p, int32_t R, const int8_t* colour, int64_t* cut_i64, double* cut_f64,
            hipStream_t stream);

/* Colouring conflicts per replica: #{i<j : J_ij != 0, colour_ri == colour_rj}. */
int oim_conflicts(oim_problem p, int32_t R, const int8_t* colour, int64_t* conflicts,
                  hipStream_t stream);

/* Energies per replica, FP64: h_model[r] = Eq. 1 (q = 2) or Eq. 2 (q >= 3) at
 * colour[R][n]; h_eq6[r] = sum_{i<j} (-J_ij) cos(theta_ri - theta_rj), Eq. 6
 * with the edge weights w = -J, at the continuous phases theta[R][n].
 * Either output may be NULL (then its input may be NULL too). */
int oim_energy(oim_problem p, int32_t q, int32_t R, const float* theta, const int8_t* colour,
               double* h_model, double* h_eq6, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Schedule gradients: adjoint of the fixed-noise trajectory (the annealing
 * schedules K(t), Ks(t) and the noise amplitude of Sec. II-D / Eq. 5 as
 * tunable parameters; sparse problems, every instance of at most 4096
 * oscillators).
 *
 * Loss, per replica r and instance b, at the phases after the last step:
 *     L_rb = sum_{i<j in b} w_ij (1 - cos(theta_i - theta_j)) / 2,  w = -J
 * (the relaxed cut: the cut value when every phase sits at 0 or pi).  The
 * gradients are those of L = sum_rb L_rb with respect to K[s], Ks[s] and
 * sigma[s] of the trajectory oim_run integrates with the same arguments
 * (same noise stream; the wrap of the phase has derivative 1).
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t q;                /* SHIL order, 2..16 */
    int32_t R;                /* replicas per instance */
    int32_t steps;            /* Euler-Maruyama steps, >= 0 */
    float dt;                 /* step, > 0 */
    int32_t checkpoint_every; /* C >= 1: phase words kept every C steps */
    uint32_t flags;           /* must be 0 */
} oim_adjoint_cfg;

/* Size of the checkpoint buffer in uint32 words:
 * ceil(steps / C) * R * (instance slots of the problem). */
int oim_adjoint_checkpoint_words(oim_problem p, const oim_adjoint_cfg* cfg, int64_t* words);

/* Forward pass.  theta0: device FP32 [R][n] initial phases (radians);
 * ckpt: device uint32 [words], caller-owned, written with the phase words of
 * steps 0, C, 2C, ...; theta_T: NULL or device FP32 [R][n], the final
 * phases; loss: NULL or device FP64 [R * I], entry r * I + b.  The other
 * arguments are those of oim_run (schedules [steps], seeds [R], step0).
 * Errors: OIM_E_ARG, OIM_E_UNSUPPORTED (dense problem or an instance above
 * 4096 oscillators), OIM_E_HIP. */
int oim_adjoint_forward(oim_problem p, const oim_adjoint_cfg* cfg, const float* K,
                        const float* Ks, const float* sigma, const uint64_t* seeds,
                        int64_t step0, const float* theta0, uint32_t* ckpt, float* theta_T,
                        double* loss, hipStream_t stream);

/* Backward pass from the checkpoints of a forward pass with the same
 * arguments: recomputes every C-step segment from its checkpoint, runs the
 * adjoint recurrence back through it, and writes dL/dK, dL/dKs, dL/dsigma as
 * device FP64 [steps] (sums over replicas and instances in a fixed order).
 * The recomputation of a segment runs on a second stream owned by p, made on
 * the first backward call (default priority), overlapping the adjoint of the
 * later segment on `stream`; the work forks from and joins back into
 * `stream`, so the call stays asynchronous and later work on `stream` sees
 * the gradients.  Uses a workspace cached in p (2 (C + 1) R slots words,
 * R slots floats, plus 128 bytes per step and workgroup); one stream at a
 * time per problem.  Errors as the forward pass, plus OIM_E_NOMEM. */
int oim_adjoint_backward(oim_problem p, const oim_adjoint_cfg* cfg, const float* K,
                         const float* Ks, const float* sigma, const uint64_t* seeds,
                         int64_t step0, const uint32_t* ckpt, double* gK, double* gKs,
                         double* gsigma, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* OIM_H */
