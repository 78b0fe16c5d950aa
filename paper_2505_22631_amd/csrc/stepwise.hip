// stepwise.hip -- Algorithm 1 with the replica state in device memory, one
// kernel per Euler-Maruyama step, for replicas too large for the
// LDS-resident kernel.
//
// Layout: replica index fastest, [n][Rp] (Rp = R rounded up to 64), two
// buffers of phase words (ping-pong: step s reads buffer s % 2 and writes
// buffer (s + 1) % 2, which keeps the synchronous update of Algorithm 1).
// The state is the phase word alone (4 bytes per oscillator and replica):
// the (sin, cos) of a neighbour is recomputed from its word where it is
// gathered, the same function of the same word as anywhere else, so the
// results equal the LDS-resident loop's bit for bit.  A wave owns one quad
// (4 consecutive oscillators) and 64 replicas: CSR entries are wave-uniform
// (scalar loads) and each neighbour gather is one coalesced 256-byte load.
// Lane r draws the quad's four normals with one Philox call keyed by replica
// r's seed.
//
// The step loop is a hipGraph of `chunk` step kernels plus a node that
// advances a device-resident step base; the executable graph is replayed
// ceil(steps / chunk) times (step kernels past the last step return at
// once).  In-run readouts are graph nodes too (chunk is a multiple of the
// readout period), with the final partial readout launched after the
// replays.  Everything a call changes (schedule, seed and readout pointers,
// first step, step count) lives in a small device block that the captured
// kernels read, written by a one-thread kernel at the start of each call, so
// a graph is captured once per problem and launch shape (q, R, readout
// period, chunk) and kept in the problem's plan cache; a call enqueues work
// and returns without waiting for it.
#include <float.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <new>
#include <type_traits>

#include "internal.hpp"
#include "noise.hpp"
#include "phase.hpp"
#include "tree.hpp"

namespace oim {

namespace {

constexpr int kQuadsPerBlock = 4;  // one per wave, 256 threads

// Per-call arguments, in device memory (see the header comment).
struct CallArgs {
    const float* K;
    const float* Ks;
    const float* sigma;
    const uint64_t* seeds;
    double* trace;        // [ceil(steps/M)][R] or null
    int8_t* best_colour;  // [R][n] or null
    int64_t step0;        // global index of local step 0
    int32_t steps;
    int32_t sched_stride; // 0: one schedule for all replicas; steps: [R][steps]
    float dt;
    int32_t base;         // local index of node 0 of the current chunk
};

struct StepArgs {
    const int64_t* row_ptr;  // n + 1 entries and 4 copies of nnz
    const int32_t* col;   // nnz entries and 4 zero entries of padding, or the padded image
    const float* J;       // the same
    int64_t nnz;
    int ell_D;            // entries per row of the padded image (ELL kernels)
    uint32_t state_bytes; // bytes of one [np][Rp] buffer of phase words (BUF kernels: < 2^32)
    const uint32_t* Uin;  // [np][Rp] phase words of step s
    uint32_t* Uout;       // [np][Rp] phase words of step s + 1
    const CallArgs* call;
    int k;                // position of this node in the chunk
    int n, R, Rp, q;
    int gx;               // quad blocks (workgroups per replica block)
};

// Workgroup id -> (quad block, replica block).  Consecutive workgroup ids go
// to the 8 XCDs in turn; each XCD is given a contiguous range of quad
// blocks (all of one replica block before the next), so the neighbour rows
// a workgroup gathers (the quads around its own) were mostly fetched into
// the same XCD's L2 by its neighbours.  A bijection on [0, nb): the blocks
// past the last multiple of 8 keep their index.
__device__ __forceinline__ void step_block(int b, int nb, int gx, int& qb, int& rb) {
    constexpr int kXcds = 8;
    const int full = nb / kXcds * kXcds;
    int t = b;
    if (b < full) t = (b % kXcds) * (full / kXcds) + b / kXcds;
    rb = t / gx;
    qb = t - rb * gx;
}

// A pointer read from the per-call block, as a global-memory pointer (such a
// pointer is generic to the compiler, which would otherwise load through it
// with flat instructions).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_ptr(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

// One Euler-Maruyama step of one quad for 64 replicas per wave.  ELL: the
// entries come from the padded row image (every row ell_D entries, padding
// of weight 0), so their positions follow from the quad index and their
// loads go out with the per-call block's: two batches of dependent loads per
// step instead of three.  BUF: the state words are addressed as buffer
// offsets (state buffers below 4 GiB), else at 64-bit global addresses.
template <int QM, bool ELL, bool BUF>
__global__ __launch_bounds__(256) void stepwise_step_kernel(StepArgs a) {
    const int lane = threadIdx.x & 63;
    int qb, rb;
    step_block(blockIdx.x, gridDim.x, a.gx, qb, rb);
    const int m = qb * kQuadsPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (4 * m >= a.n) return;
    const int r = rb * 64 + lane;
    const int Rp = a.Rp, q = QM ? QM : a.q;
    const int rs = r < a.R ? r : a.R - 1;  // padding lanes borrow a replica's entries
    // Lane r's word of a row of the [np][Rp] state.  BUF: a buffer access
    // with the row's byte offset in a scalar register (scalar arithmetic on
    // the wave-uniform row) and the lane's in a vector register shared by
    // every load and store of the step, so no 64-bit address arithmetic per
    // lane and access; this needs a state buffer below 4 GiB.  Otherwise a
    // global access at a 64-bit address.
    const int roff = r * 4;
    const uint32_t row_bytes = (uint32_t)Rp * 4u;
    const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a.Uin, (short)0, (int)a.state_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a.Uout, (short)0, (int)a.state_bytes, 0x00020000);
    auto lane_word = [&](int row) -> uint32_t {
        if constexpr (BUF)
            return __builtin_amdgcn_raw_buffer_load_b32(rin, roff, (int)((uint32_t)row * row_bytes), 0);
        else
            return a.Uin[(size_t)row * Rp + r];
    };
    auto store_word = [&](int row, uint32_t v) {
        if constexpr (BUF)
            __builtin_amdgcn_raw_buffer_store_b32(v, rout, roff, (int)((uint32_t)row * row_bytes), 0);
        else
            a.Uout[(size_t)row * Rp + r] = v;
    };
    // Every load of a step is issued up front, in batches with one wait
    // each: the per-call block, the quad's row bounds and its own words;
    // then the schedule entries, the seed and the first group of each row's
    // entries; then the neighbours' words (with the padded image the first
    // two batches are one).  Nothing before the store depends on whether
    // this node's step is still part of the run (a node past the last step
    // computes on local step 0's entries and writes nothing), and no select
    // or branch depends on a loaded value, so the compiler keeps the loads
    // together.
    const CallArgs& c = *a.call;
    int base = c.base, steps = c.steps, stride = c.sched_stride;
    int64_t step0 = c.step0;
    float dt = c.dt;
    const float* Kp = c.K;
    const float* Ksp = c.Ks;
    const float* sgp = c.sigma;
    const uint64_t* seedp = c.seeds;
    int64_t eb[4];
    int len[4];
    int lmax = 0;
    if constexpr (ELL) {
        // group g / 4 of row j of the quad at m * 4D + 4g + 4j (in steps
        // of 4 entries: g advances the base by 16)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            eb[j] = (int64_t)m * 4 * a.ell_D + 4 * j;
            len[j] = a.ell_D;
        }
        lmax = a.ell_D;
    } else {
        int64_t rp[5];  // row_ptr carries 4 entries of padding (empty rows)
#pragma unroll
        for (int j = 0; j < 5; ++j) rp[j] = a.row_ptr[4 * m + j];
        // one wait for the per-call block and the row bounds together: every
        // use of them goes through this statement
        asm(""
            : "+s"(base), "+s"(steps), "+s"(stride), "+s"(step0), "+s"(dt), "+s"(Kp),
                       "+s"(Ksp), "+s"(sgp), "+s"(seedp), "+s"(rp[0]), "+s"(rp[1]), "+s"(rp[2]),
                       "+s"(rp[3]), "+s"(rp[4]));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            eb[j] = rp[j];
            len[j] = (int)(rp[j + 1] - rp[j]);
            lmax = len[j] > lmax ? len[j] : lmax;
        }
    }
    // The quad's four rows are walked in lock-step, four entries of each
    // per group, so sixteen neighbour loads are in flight together.  Row
    // lengths are wave-uniform (every lane is a replica of the same quad), so
    // a row shorter than the longest costs only its idle slots.  Group t of
    // row j is the 4 entries from eb + t, clamped to nnz (the arrays carry 4
    // zero entries past the end, so a group is always in bounds and its
    // column indexes valid); a slot past the row's end gets weight 0 by
    // masking its bits, which leaves the sums unchanged (the words are
    // finite).  The padded image needs neither: its groups are in bounds
    // and its padding weighs 0.  Each row keeps its order: entries at even
    // offsets into one partial sum, odd ones into the other.
    int ci[4][4];
    uint32_t wb[4][4];
    auto load_cols = [&](int g) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int64_t base = eb[j] + (ELL ? 4 * g : g);
            if constexpr (!ELL) base = base < a.nnz ? base : a.nnz;
#pragma unroll
            for (int h = 0; h < 4; ++h) ci[j][h] = a.col[base + h];
        }
    };
    auto load_weights = [&](int g) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int64_t base = eb[j] + (ELL ? 4 * g : g);
            if constexpr (!ELL) base = base < a.nnz ? base : a.nnz;
#pragma unroll
            for (int h = 0; h < 4; ++h) wb[j][h] = __float_as_uint(a.J[base + h]);
        }
    };
    auto load_entries = [&](int g) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int64_t base = eb[j] + (ELL ? 4 * g : g);
            if constexpr (!ELL) base = base < a.nnz ? base : a.nnz;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                wb[j][h] = __float_as_uint(a.J[base + h]);
                ci[j][h] = a.col[base + h];
            }
        }
    };
    // The first group's four rows' entry loads (scalar loads) are all issued
    // before the first use: the loaded values pass through empty asm
    // statements that no load may cross, so nothing that uses them is
    // scheduled between the loads (each use of a scalar load waits for all
    // of them).  Later groups are read with vector loads, which complete in
    // order, and need no such help.
    auto pin_entries = [&]() {
        asm(""
            : "+s"(ci[0][0]), "+s"(ci[0][1]), "+s"(ci[0][2]), "+s"(ci[0][3]),
              "+s"(ci[1][0]), "+s"(ci[1][1]), "+s"(ci[1][2]), "+s"(ci[1][3]),
              "+s"(ci[2][0]), "+s"(ci[2][1]), "+s"(ci[2][2]), "+s"(ci[2][3]),
              "+s"(ci[3][0]), "+s"(ci[3][1]), "+s"(ci[3][2]), "+s"(ci[3][3]),
              "+s"(wb[0][0]), "+s"(wb[0][1]), "+s"(wb[0][2]), "+s"(wb[0][3]),
              "+s"(wb[1][0]), "+s"(wb[1][1]), "+s"(wb[1][2]), "+s"(wb[1][3]),
              "+s"(wb[2][0]), "+s"(wb[2][1]), "+s"(wb[2][2]), "+s"(wb[2][3]),
              "+s"(wb[3][0]), "+s"(wb[3][1]), "+s"(wb[3][2]), "+s"(wb[3][3]));
    };
    uint32_t p[4][4];
    float w[4][4];
    auto load_words = [&](int g) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                // the column is wave-uniform (every lane is a replica of the
                // same quad); later groups' columns arrive in vector
                // registers, so say so
                p[j][h] = lane_word(__builtin_amdgcn_readfirstlane(ci[j][h]));
                if constexpr (ELL) {
                    w[j][h] = __uint_as_float(wb[j][h]);
                } else {
                    const uint32_t keep = 0u - (uint32_t)(g + h < len[j]);
                    w[j][h] = __uint_as_float(wb[j][h] & keep);
                }
            }
    };
    uint32_t u0[4];
    if constexpr (ELL) {
        // the first group's columns (the weights are not needed before the
        // neighbours' words arrive: they go out with them)
        load_cols(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) u0[j] = lane_word(4 * m + j);
        // one wait for the per-call block and the columns together
        asm(""
            : "+s"(base), "+s"(steps), "+s"(stride), "+s"(step0), "+s"(dt), "+s"(Kp),
              "+s"(Ksp), "+s"(sgp), "+s"(seedp),
              "+s"(ci[0][0]), "+s"(ci[0][1]), "+s"(ci[0][2]), "+s"(ci[0][3]),
              "+s"(ci[1][0]), "+s"(ci[1][1]), "+s"(ci[1][2]), "+s"(ci[1][3]),
              "+s"(ci[2][0]), "+s"(ci[2][1]), "+s"(ci[2][2]), "+s"(ci[2][3]),
              "+s"(ci[3][0]), "+s"(ci[3][1]), "+s"(ci[3][2]), "+s"(ci[3][3]));
        load_weights(0);
    }
    const int s_node = base + a.k;
    const bool live = s_node < steps;
    const int s = live ? s_node : 0;
    const uint32_t t = (uint32_t)(step0 + s);
    const int64_t so = (int64_t)rs * stride + s;
    const float Kv = global_ptr(Kp)[so];
    const float Ksv = global_ptr(Ksp)[so];
    const float sgv = global_ptr(sgp)[so];
    const uint64_t seed = global_ptr(seedp)[rs];
    if constexpr (!ELL) {
#pragma unroll
        for (int j = 0; j < 4; ++j) u0[j] = lane_word(4 * m + j);
        load_entries(0);
        pin_entries();
    }
    auto gather = [&](int g) {
        load_entries(g);
        load_words(g);
    };
    float A0[4], B0[4], A1[4], B1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) A0[j] = B0[j] = A1[j] = B1[j] = 0.f;
    auto accumulate = [&]() {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int h = 0; h < 4; h += 2) {
                const float s0 = sin_turn(p[j][h]), c0 = cos_turn(p[j][h]);
                const float s1 = sin_turn(p[j][h + 1]), c1 = cos_turn(p[j][h + 1]);
                A0[j] = __builtin_fmaf(w[j][h], c0, A0[j]);
                B0[j] = __builtin_fmaf(w[j][h], s0, B0[j]);
                A1[j] = __builtin_fmaf(w[j][h + 1], c1, A1[j]);
                B1[j] = __builtin_fmaf(w[j][h + 1], s1, B1[j]);
            }
    };
    load_words(0);
    // the quad's normals while the neighbour loads are in flight
    float z[4];
    normals4((uint32_t)m, t, 0u, (uint32_t)seed, (uint32_t)(seed >> 32), z);
    // pin the normals here (left alone, the compiler sinks them to the
    // update, after the last neighbour load has returned)
    asm volatile("" ::"v"(z[0]), "v"(z[1]), "v"(z[2]), "v"(z[3]) : "memory");
    accumulate();
    for (int g = 4; g < lmax; g += 4) {
        gather(g);
        accumulate();
    }
    if (!live) return;
    const float kc = -dt * Kv * kTurnScale;
    const float ks = -dt * Ksv * kTurnScale;
    const float ns = sgv * __builtin_sqrtf(dt) * kTurnScale;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int i = 4 * m + j;
        if (i >= a.n) break;
        const float os = sin_turn(u0[j]), oc = cos_turn(u0[j]);
        const float A = A0[j] + A1[j], B = B0[j] + B1[j];
        const float coup = os * A - oc * B;
        const float drift = kc * coup + ks * sin_q<QM>(os, oc, u0[j], q);
        store_word(i, advance(u0[j], __builtin_fmaf(ns, z[j], drift)));
    }
}

__global__ void advance_base_kernel(CallArgs* call, int chunk) { call->base += chunk; }

__global__ void set_call_kernel(CallArgs* call, CallArgs v) { *call = v; }

// [R][n] theta or phase words -> [np][Rp] phase words (both buffers, so the
// padding rows and replicas hold defined words everywhere).
__global__ __launch_bounds__(256) void stepwise_init_kernel(const float* theta, const uint32_t* phase,
                                                            uint32_t* U0, uint32_t* U1,
                                                            int n, int R, int np, int Rp) {
    const size_t total = (size_t)np * Rp;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / Rp), r = (int)(e % Rp);
        uint32_t u = 0;
        if (i < n && r < R) {
            const size_t src = (size_t)r * n + i;
            u = phase ? phase[src] : phase_from_theta(theta[src]);
        }
        U0[e] = u;
        U1[e] = u;
    }
}

__global__ __launch_bounds__(256) void stepwise_final_kernel(const uint32_t* U, float* theta,
                                                             uint32_t* phase, int n, int R, int Rp) {
    const size_t total = (size_t)R * n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / n), i = (int)(e % n);
        const uint32_t u = U[(size_t)i * Rp + r];
        theta[e] = theta_from_phase(u);
        if (phase) phase[e] = u;
    }
}

struct ReadArgs {
    const int64_t* row_ptr;
    const int32_t* col;
    const float* J;
    const uint32_t* U;
    double* part;  // [gridDim.x][Rp]
    const CallArgs* call;
    int k;         // node position in the chunk, or -1: after the last step
    int n, Rp, q;
};

// Partial sums of sum_{i<j} J_ij term(k_i, k_j) per block of 16 rows (four
// quads, one per wave) and replica (term = s_i s_j for q = 2, delta(k_i, k_j)
// for q >= 3), in the library's fixed FP64 order: each row over j > i in
// column order, a quad's rows as (r0 + r1) + (r2 + r3), the block's quads as
// (w0 + w1) + (w2 + w3) -- the pairwise tree over the block's rows.
__global__ __launch_bounds__(256) void stepwise_readout_kernel(ReadArgs a) {
    __shared__ double red[kQuadsPerBlock][64];
    const int steps = a.call->steps;
    const int s = a.k < 0 ? steps - 1 : a.call->base + a.k;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = blockIdx.y * 64 + lane;
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
    if (s < steps) {
        const int m = blockIdx.x * kQuadsPerBlock + wave;
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * m + j;
            if (i >= a.n) break;
            const int ci = nearest_state(a.U[(size_t)i * a.Rp + r], a.q);
            double acc = 0.0;
            for (int64_t e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
                const int c = a.col[e];
                if (c <= i) continue;
                const int cj = nearest_state(a.U[(size_t)c * a.Rp + r], a.q);
                const double w = (double)a.J[e];
                acc += (a.q == 2) ? (ci == cj ? w : -w) : (ci == cj ? w : 0.0);
            }
            rs[j] = acc;
        }
    }
    red[wave][lane] = (rs[0] + rs[1]) + (rs[2] + rs[3]);
    __syncthreads();
    if (wave == 0 && s < steps)
        a.part[(size_t)blockIdx.x * a.Rp + r] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

struct BestArgs {
    const double* part;
    int nblocks;
    const uint32_t* U;
    double* best;     // running best (workspace)
    int32_t* best_at; // running best step (workspace)
    const CallArgs* call;
    int k;            // node position in the chunk, or -1: after the last step
    int M, n, R, Rp, q;
};

// One workgroup per replica: H = -(the pairwise tree over the blocks'
// partials), trace entry, best-so-far and the colours of a new best.  The
// partials, zero-padded to a power of two P, are taken in rounds of
// CH = min(P, 4096) values; in a round each of the 256 threads folds an
// aligned chunk of CH / 256 (at most 16) values by the pairwise tree in
// registers, the 256 chunk sums are folded pairwise in LDS, and thread 0
// pushes the round's sum into a tree over rounds.  This is the pairwise tree
// over the padded sequence (padding zeros add exactly).
__global__ __launch_bounds__(256) void stepwise_best_kernel(BestArgs a) {
    __shared__ int improved;
    __shared__ double sums[256];
    __shared__ double stack[TreeAcc::kLevels];
    const CallArgs& c = *a.call;
    const int s = a.k < 0 ? c.steps - 1 : c.base + a.k;
    if (s >= c.steps) return;
    const int r = blockIdx.x;
    int64_t P = 1;
    while (P < a.nblocks) P <<= 1;
    const int CH = P < 4096 ? (int)P : 4096;
    const int B = CH >= 256 ? CH / 256 : 1;
    const int64_t rounds = P / CH;
    TreeAcc outer(stack);
    for (int64_t rd = 0; rd < rounds; ++rd) {
        const int64_t first = rd * CH + (int64_t)threadIdx.x * B;
        double v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            v[i] = (i < B && first + i < a.nblocks) ? a.part[(size_t)(first + i) * a.Rp + r] : 0.0;
        // the tree over 16 slots; slots past B hold +0, so the result is the
        // tree over the chunk's B values
#pragma unroll
        for (int len = 16; len > 1; len >>= 1)
#pragma unroll
            for (int i = 0; i < len / 2; ++i) v[i] = v[2 * i] + v[2 * i + 1];
        sums[threadIdx.x] = v[0];
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            if ((threadIdx.x & (2 * d - 1)) == 0) sums[threadIdx.x] = sums[threadIdx.x] + sums[threadIdx.x + d];
            __syncthreads();
        }
        if (threadIdx.x == 0) outer.push(sums[0]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double H = -outer.finish();
        const int kread = (s + a.M) / a.M - 1;
        if (c.trace) c.trace[(size_t)kread * a.R + r] = H;
        improved = (kread == 0 || H < a.best[r]) ? 1 : 0;
        if (improved) {
            a.best[r] = H;
            a.best_at[r] = (int32_t)(c.step0 + s + 1);
        }
    }
    __syncthreads();
    if (improved && c.best_colour)
        for (int i = threadIdx.x; i < a.n; i += blockDim.x)
            c.best_colour[(size_t)r * a.n + i] = (int8_t)nearest_state(a.U[(size_t)i * a.Rp + r], a.q);
}

int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? OIM_OK : hip_error(e, what);
}

// One captured step loop: the executable graphs of a chunk (two when the
// chunk is odd: the table parity then flips from replay to replay), the
// workspace they were captured on, and an event recorded after their last
// use so they can be destroyed safely.
struct Plan {
    int q = 0, R = 0, M = 0, chunk = 0;
    const void* work = nullptr;
    hipGraph_t g[2] = {nullptr, nullptr};
    hipGraphExec_t x[2] = {nullptr, nullptr};
    hipEvent_t done = nullptr;
    uint64_t last_use = 0;
};

struct PlanCache {
    static constexpr int kMax = 4;
    Plan plans[kMax];
    int count = 0;
    uint64_t clock = 0;
};

void destroy_plan(Plan& pl) {
    if (pl.done) {
        (void)hipEventSynchronize(pl.done);
        (void)hipEventDestroy(pl.done);
    }
    for (int i = 0; i < 2; ++i) {
        if (pl.x[i]) (void)hipGraphExecDestroy(pl.x[i]);
        if (pl.g[i]) (void)hipGraphDestroy(pl.g[i]);
    }
    pl = Plan{};
}

void clear_plans(Problem* p) {
    PlanCache* c = static_cast<PlanCache*>(p->step_plans);
    if (!c) return;
    for (int i = 0; i < c->count; ++i) destroy_plan(c->plans[i]);
    c->count = 0;
}

}  // namespace

void stepwise_release(Problem* p) {
    clear_plans(p);
    delete static_cast<PlanCache*>(p->step_plans);
    p->step_plans = nullptr;
}

namespace {

struct Shape {
    int n, R, steps, M, Rp, quads, np, gx, chunk;
    size_t cells, args_off, bytes;
};

Shape shape_of(const Problem* p, const oim_run_cfg* cfg) {
    Shape sh{};
    sh.n = p->n;
    sh.R = cfg->R;
    sh.steps = cfg->steps;
    sh.M = cfg->readout_every;
    sh.Rp = (sh.R + 63) / 64 * 64;
    sh.quads = (sh.n + 3) / 4;
    sh.np = sh.quads * 4;
    sh.gx = (sh.quads + kQuadsPerBlock - 1) / kQuadsPerBlock;
    sh.cells = (size_t)sh.np * sh.Rp;
    // chunk: a multiple of the readout period, about 64 steps
    int chunk = std::min(sh.steps, 64);
    if (sh.M > 0) chunk = std::max(1, (std::min(sh.steps, std::max(64, sh.M)) / sh.M)) * sh.M;
    sh.chunk = std::max(1, std::min(chunk, sh.steps));
    sh.args_off = (sh.cells * (4 + 4) + (size_t)sh.gx * sh.Rp * 8 + (size_t)sh.R * 12 + 255) &
                  ~(size_t)255;
    sh.bytes = sh.args_off + 256;
    return sh;
}

// The stepwise loop on a workspace of at least stepwise_workspace_bytes:
// with `graph`, the chunk of steps comes from the problem's plan cache
// (captured on first use) and is replayed; without, the same kernels are
// launched one by one on the stream (no capture, no allocation).
int run_stepwise(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                 const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
                 uint32_t* phase, const oim_readout* ro, hipStream_t stream, void* work,
                 bool graph) {
    const Shape sh = shape_of(p, cfg);
    const int n = sh.n, R = sh.R, steps = sh.steps, M = sh.M, Rp = sh.Rp, np = sh.np, gx = sh.gx;
    const int chunk = sh.chunk;
    const size_t cells = sh.cells, args_off = sh.args_off;
    if (graph && !p->step_plans) {
        p->step_plans = new (std::nothrow) PlanCache();
        if (!p->step_plans) return set_error(OIM_E_NOMEM, "plan cache");
    }
    unsigned char* w = static_cast<unsigned char*>(work);
    uint32_t* U0 = reinterpret_cast<uint32_t*>(w);
    uint32_t* U1 = U0 + cells;
    double* part = reinterpret_cast<double*>(U1 + cells);
    double* best = part + (size_t)gx * Rp;
    int32_t* best_at = reinterpret_cast<int32_t*>(best + R);
    CallArgs* call = reinterpret_cast<CallArgs*>(w + args_off);

    // this call's arguments, for every kernel below (stream order)
    CallArgs ca{};
    ca.K = K;
    ca.Ks = Ks;
    ca.sigma = sigma;
    ca.seeds = seeds;
    ca.trace = ro ? ro->trace : nullptr;
    ca.best_colour = ro ? ro->best_colour : nullptr;
    ca.step0 = step0;
    ca.steps = steps;
    ca.sched_stride = (cfg->flags & OIM_SCHED_PER_REPLICA) ? cfg->steps : 0;
    ca.dt = cfg->dt;
    ca.base = 0;
    hipLaunchKernelGGL(set_call_kernel, dim3(1), dim3(1), 0, stream, call, ca);
    int st = check_launch("set_call_kernel");
    if (st) return st;
    hipLaunchKernelGGL(stepwise_init_kernel, dim3(2048), dim3(256), 0, stream, theta, phase, U0, U1,
                       n, R, np, Rp);
    if ((st = check_launch("stepwise_init_kernel"))) return st;

    using StepFn = void (*)(StepArgs);
    const bool ell = p->d_ell_col != nullptr;
    // buffer addressing for states below 4 GiB (OIM_STEPWISE_GLOBAL_ADDR=1
    // takes the 64-bit global addressing of larger states for any size)
    bool buf = cells * 4 < ((size_t)1 << 32);
    if (const char* env = getenv("OIM_STEPWISE_GLOBAL_ADDR"))
        if (atoi(env) != 0) buf = false;
    static const StepFn kStep[2][2][3] = {
        {{stepwise_step_kernel<0, false, false>, stepwise_step_kernel<2, false, false>,
          stepwise_step_kernel<3, false, false>},
         {stepwise_step_kernel<0, false, true>, stepwise_step_kernel<2, false, true>,
          stepwise_step_kernel<3, false, true>}},
        {{stepwise_step_kernel<0, true, false>, stepwise_step_kernel<2, true, false>,
          stepwise_step_kernel<3, true, false>},
         {stepwise_step_kernel<0, true, true>, stepwise_step_kernel<2, true, true>,
          stepwise_step_kernel<3, true, true>}}};
    StepFn fn = kStep[ell][buf][cfg->q == 2 ? 1 : cfg->q == 3 ? 2 : 0];
    StepArgs sa{};
    sa.row_ptr = p->d_row_ptr;
    sa.col = ell ? p->d_ell_col : p->d_col;
    sa.J = ell ? p->d_ell_J : p->d_J;
    sa.nnz = p->nnz;
    sa.ell_D = p->ell_D;
    sa.state_bytes = buf ? (uint32_t)(cells * 4) : 0u;
    sa.call = call;
    sa.n = n;
    sa.R = R;
    sa.Rp = Rp;
    sa.q = cfg->q;
    sa.gx = gx;
    // the state after local step s is in buffer (s + 1) % 2; after the run,
    // in buffer steps % 2
    uint32_t* const Ufinal = (steps & 1) ? U1 : U0;
    ReadArgs ra{p->d_row_ptr, p->d_col, p->d_J, Ufinal, part, call, 0, n, Rp, cfg->q};
    BestArgs ba{};
    ba.part = part;
    ba.nblocks = gx;
    ba.U = Ufinal;
    ba.best = best;
    ba.best_at = best_at;
    ba.call = call;
    ba.M = M;
    ba.n = n;
    ba.R = R;
    ba.Rp = Rp;
    ba.q = cfg->q;

    // Record one chunk: step kernels (with readouts where due) and the base
    // advance.  Buffer parity alternates per step (step s reads buffer s % 2);
    // an odd chunk flips it from one replay to the next, so it has a graph
    // for each parity.
    auto record_chunk = [&](hipStream_t s, bool parity) -> int {
        for (int k = 0; k < chunk; ++k) {
            const bool odd = ((k & 1) != 0) != parity;
            sa.Uin = odd ? U1 : U0;
            sa.Uout = odd ? U0 : U1;
            ra.U = sa.Uout;
            ba.U = sa.Uout;
            sa.k = k;
            hipLaunchKernelGGL(fn, dim3(gx * (Rp / 64)), dim3(256), 0, s, sa);
            int rc = check_launch("stepwise_step_kernel");
            if (rc) return rc;
            if (M > 0 && (k + 1) % M == 0) {
                ra.k = k;
                hipLaunchKernelGGL(stepwise_readout_kernel, dim3(gx, Rp / 64), dim3(256), 0, s, ra);
                if ((rc = check_launch("stepwise_readout_kernel"))) return rc;
                ba.k = k;
                hipLaunchKernelGGL(stepwise_best_kernel, dim3(R), dim3(256), 0, s, ba);
                if ((rc = check_launch("stepwise_best_kernel"))) return rc;
            }
        }
        hipLaunchKernelGGL(advance_base_kernel, dim3(1), dim3(1), 0, s, call, chunk);
        return check_launch("advance_base_kernel");
    };

    const bool flip = (chunk & 1) != 0;
    const int replays = (steps + chunk - 1) / chunk;
    hipError_t e = hipSuccess;
    if (!graph) {
        for (int c = 0; c < replays; ++c)
            if ((st = record_chunk(stream, flip && (c & 1)))) return st;
    } else {
        PlanCache& cache = *static_cast<PlanCache*>(p->step_plans);
        Plan* plan = nullptr;
        for (int i = 0; i < cache.count; ++i) {
            Plan& c = cache.plans[i];
            if (c.q == cfg->q && c.R == R && c.M == M && c.chunk == chunk && c.work == work) {
                plan = &c;
                break;
            }
        }
        if (!plan) {
            // capture a new plan, evicting the least recently used one if full
            int slot = cache.count;
            if (cache.count == PlanCache::kMax) {
                slot = 0;
                for (int i = 1; i < cache.count; ++i)
                    if (cache.plans[i].last_use < cache.plans[slot].last_use) slot = i;
                destroy_plan(cache.plans[slot]);
            } else {
                ++cache.count;
            }
            Plan& pl = cache.plans[slot];
            pl = Plan{};
            hipStream_t cap = nullptr;
            e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
            if (e != hipSuccess) st = hip_error(e, "capture stream");
            for (int par = 0; par < (flip ? 2 : 1) && !st; ++par) {
                e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) {
                    st = hip_error(e, "hipStreamBeginCapture");
                    break;
                }
                st = record_chunk(cap, par == 1);
                e = hipStreamEndCapture(cap, &pl.g[par]);
                if (!st && e != hipSuccess) st = hip_error(e, "hipStreamEndCapture");
                if (!st && (e = hipGraphInstantiate(&pl.x[par], pl.g[par], nullptr, nullptr, 0)) != hipSuccess)
                    st = hip_error(e, "hipGraphInstantiate");
            }
            if (cap) (void)hipStreamDestroy(cap);
            if (!st && (e = hipEventCreateWithFlags(&pl.done, hipEventDisableTiming)) != hipSuccess)
                st = hip_error(e, "plan event");
            if (st) {
                destroy_plan(pl);
                // keep the cache dense: move the last plan into the freed slot
                if (slot != cache.count - 1) {
                    pl = cache.plans[cache.count - 1];
                    cache.plans[cache.count - 1] = Plan{};
                }
                --cache.count;
                return st;
            }
            pl.q = cfg->q;
            pl.R = R;
            pl.M = M;
            pl.chunk = chunk;
            pl.work = work;
            plan = &pl;
        }
        plan->last_use = ++cache.clock;
        for (int c = 0; c < replays; ++c) {
            e = hipGraphLaunch(plan->x[flip ? (c & 1) : 0], stream);
            if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
        }
        e = hipEventRecord(plan->done, stream);
        if (e != hipSuccess) return hip_error(e, "plan event record");
    }
    // readout after the last step when steps is not a multiple of M
    if (M > 0 && steps % M != 0) {
        ReadArgs rl = ra;
        rl.k = -1;
        rl.U = Ufinal;
        BestArgs bl = ba;
        bl.k = -1;
        bl.U = Ufinal;
        hipLaunchKernelGGL(stepwise_readout_kernel, dim3(gx, Rp / 64), dim3(256), 0, stream, rl);
        if ((st = check_launch("stepwise_readout_kernel"))) return st;
        hipLaunchKernelGGL(stepwise_best_kernel, dim3(R), dim3(256), 0, stream, bl);
        if ((st = check_launch("stepwise_best_kernel"))) return st;
    }
    if (ro && M > 0 && steps > 0) {
        if (ro->best_h) {
            e = hipMemcpyAsync(ro->best_h, best, sizeof(double) * R, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return hip_error(e, "best_h copy");
        }
        if (ro->best_step) {
            e = hipMemcpyAsync(ro->best_step, best_at, sizeof(int32_t) * R, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return hip_error(e, "best_step copy");
        }
    }
    hipLaunchKernelGGL(stepwise_final_kernel, dim3(2048), dim3(256), 0, stream, Ufinal, theta, phase,
                       n, R, Rp);
    return check_launch("stepwise_final_kernel");
}

}  // namespace

size_t stepwise_workspace_bytes(const Problem* p, const oim_run_cfg* cfg) {
    return shape_of(p, cfg).bytes;
}

int launch_stepwise_sparse(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                           const float* sigma, const uint64_t* seeds, int64_t step0,
                           float* theta, uint32_t* phase, const oim_readout* ro,
                           hipStream_t stream) {
    const size_t need = stepwise_workspace_bytes(p, cfg);
    if (p->work_bytes < need) {
        clear_plans(p);  // they were captured on the old workspace
        (void)hipFree(p->d_work);
        p->d_work = nullptr;
        p->work_bytes = 0;
        hipError_t e = hipMalloc(&p->d_work, need);
        if (e != hipSuccess) {
            p->d_work = nullptr;
            return e == hipErrorOutOfMemory ? set_error(OIM_E_NOMEM, "stepwise workspace")
                                            : hip_error(e, "hipMalloc stepwise workspace");
        }
        p->work_bytes = need;
    }
    return run_stepwise(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream, p->d_work,
                        true);
}

int launch_stepwise_sparse_ws(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                              const float* sigma, const uint64_t* seeds, int64_t step0,
                              float* theta, uint32_t* phase, const oim_readout* ro,
                              hipStream_t stream, void* work) {
    return run_stepwise(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream, work,
                        false);
}

}  // namespace oim
