// persistent_kernel.hpp -- the whole Euler-Maruyama loop of Algorithm 1 for
// a sparse coupling in ONE launch, one workgroup per replica, the replica's
// state resident in LDS.  The kernel template is instantiated for its launch
// variants by sparse_persistent.hip (general weights) and
// sparse_persistent_uw.hip (uniform unit weights).
//
// Per step t (Sec. II-E Eq. 5 with the descent sign, Algorithm 1):
//   phase A  every oscillator's coupling sum from the phases of step t,
//            c_i = sum_j J_ij sin(th_i - th_j) = s_i sum_j J_ij c_j - c_i sum_j J_ij s_j,
//            gathered over the sliced-ELL rows from the (sin, cos) table in LDS,
//            folded with the SHIL term and the Philox noise into the step's
//            increment drift_i (registers)
//   barrier
//   phase B  Euler-Maruyama update, wrap, and the (sin, cos) table refreshed
//            for step t+1
//   barrier
// The state is a 32-bit fixed-point phase per oscillator (phase.hpp), held
// in registers; the step in 2^-32-turn units is
//   u <- u + rint(kc c_i + ks sin(q th_i) + ns xi),
//   kc = -dt K_t 2^32/2pi, ks = -dt Ks_t 2^32/2pi, ns = sigma_t sqrt(dt) 2^32/2pi,
// and the wrap is the integer overflow.
//
// Work split: slice = 64 quads; wave w of the workgroup owns slices
// w, w + W, w + 2W, ... (W waves); lane l of a slice owns quad 64*slice + l,
// i.e. oscillators 4*quad + j, j = 0..3, whose phases stay in registers for
// the whole run.  One Philox call per lane per step yields the quad's four
// normals.
#pragma once
#include <float.h>

#include "internal.hpp"
#include "noise.hpp"
#include "phase.hpp"
#include "tree.hpp"

// Every multiply-add of the step is written out (fmaf) and the compiler may
// not contract the others, so all launch variants round identically whatever
// their register allocation and scheduling.
#pragma clang fp contract(off)

namespace oim {

namespace persist {

struct PersistArgs {
    const int4* sell;   // sliced-ELL entries, two per int4 (see SellImage)
    const int4* sell_uw;  // uniform unit weights: LDS offsets alone, four per int4, or null
    const int2* row_split;  // per slice, row j, lane: (first entry of the upper triangle, length)
    uint32_t sell_uw_bytes;
    float w0;           // the uniform weight (+1 or -1) when sell_uw is set
    const int2* desc;   // per slice: (base in int4 rows, padded degree)
    const int4* inst;   // per instance: (first slice, slices, first oscillator, oscillators)
    const int32_t* order;  // instances, most slices first
    int32_t I;          // instances
    int32_t n_total;    // oscillators of all instances (row length of theta)
    uint32_t sell_bytes;
    int32_t q;
    int32_t steps;
    int32_t M;          // readout period (0 = none)
    int64_t step0;
    float dt;
    const float* K;
    const float* Ks;
    const float* sigma;
    const uint64_t* seeds;
    float* theta;       // [R][n_total]
    uint32_t* phase;    // [R][n_total] or null
    double* trace;      // [ceil(steps/M)][R][I]
    double* best_h;     // [R][I]
    int32_t* best_step; // [R][I]
    int8_t* best_colour;  // [R][n_total]
    int32_t R;
    int32_t sched_stride;  // 0: one schedule for all replicas; steps: [R][steps]
    int32_t slice_sums;    // 1: the readout keeps every slice's sum in LDS (room for it)
};

// Tree levels of the in-run readout's sum over slices (2^8 slices at most).
constexpr int kSliceTreeLevels = 8;

// Index within the instance of the oscillator at LDS slot `slot`
// (slot = (i % 4) * plane + i / 4).
__device__ __forceinline__ int slot_index(int slot, int plane) {
    const int p = (slot >= plane) + (slot >= 2 * plane) + (slot >= 3 * plane);
    return 4 * (slot - p * plane) + p;
}

__device__ __forceinline__ int4 load_pair(__amdgpu_buffer_rsrc_t rsrc, int voff, int soff) {
    return __builtin_bit_cast(int4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, soff, 0));
}

// (sin, cos) of the oscillator at an LDS byte offset.  The dynamic LDS of
// this kernel is its only LDS and starts at address 0, so the offset is the
// address itself (no per-edge base add).
__device__ __forceinline__ float2 sc_at(const unsigned char*, int byte_off) {
    typedef __attribute__((address_space(3))) const uint64_t lds_u64;
    const uint64_t v = *reinterpret_cast<lds_u64*>((uint32_t)byte_off);
    return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}

// Launch shape: TB threads (W = TB / 64 waves), MS slices per wave group,
// RPL rows of every quad per lane.  RPL = 4: a lane owns whole quads (one
// wave per slice).  RPL = 2 or 1 (rows split): G = 4 / RPL waves share a
// slice, wave w owning rows g * RPL .. g * RPL + RPL - 1 of each quad of its
// slices (g = w % G), so instances with few slices and long rows keep every
// wave busy.  Every oscillator's arithmetic -- its row's multiply-adds in
// entry order, its Philox normal, its update -- is the same in all shapes,
// so they give identical results.
template <int TB, int MS, int QM, int RPL, bool UWT>
__global__ __launch_bounds__(TB) void persistent_sparse_kernel(PersistArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    // workgroup -> (instance, replica).  Consecutive workgroup ids go to the
    // 8 XCDs in turn, each with its own L2; the replicas of one instance are
    // kept on one XCD (they read the same edge image every step) and the
    // instances, largest first, are dealt to the XCDs in turn: XCD c takes
    // instances c, c + 8, c + 16, ... of the order, all replicas of each
    // before the next.  Instances past the last multiple of 8 follow in
    // plain order.
    int grp, r;
    {
        const int b = blockIdx.x;
        const int I8 = a.I / 8 * 8;
        const int head = a.R * I8;
        if (b < head) {
            const int c = b & 7, k = b >> 3;
            grp = c + 8 * (k / a.R);
            r = k % a.R;
        } else {
            grp = I8 + (b - head) / a.R;
            r = (b - head) % a.R;
        }
    }
    const int inst_id = a.order[grp];
    const int4 idesc = a.inst[inst_id];
    const int slice0 = idesc.x, S = idesc.y, off = idesc.z, n = idesc.w;
    const int plane = S * 64;
    constexpr int W = TB / 64;
    constexpr int G = 4 / RPL;     // waves per slice
    constexpr int WS = W / G;      // wave groups (slices in flight)
    constexpr int U = 8 / RPL;     // 16-byte entry loads per row per iteration
    float2* sc = reinterpret_cast<float2*>(smem);                   // [4 * plane]
    unsigned char* col8 = smem + (size_t)8 * 4 * plane;            // [4 * plane] (readout)
    // (0, 0) at byte 36 * plane, what padding entries of the unit-weight image read
    float2* zero_entry = reinterpret_cast<float2*>(col8 + 4 * plane);
    double* red = reinterpret_cast<double*>(col8 + 4 * plane + 16);  // [W]
    double* tstack = red + W;                                                   // tree levels
    // readout state of thread 0: [0] improved flag, [1] best step, [2..3] best H
    int* flag = reinterpret_cast<int*>(tstack + kSliceTreeLevels);
    double* best_lds = reinterpret_cast<double*>(flag + 2);
    double* part = reinterpret_cast<double*>(flag + 8);             // [WS][G][64], RPL < 4
    double* ssum = part + (RPL < 4 ? TB : 0);                        // [MS * WS], slice_sums

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = wave % G, ws = wave / G;
    const int j0 = g * RPL;        // first row of the quad this wave owns
    const int q = QM ? QM : a.q;
    const uint64_t seed = a.seeds[r];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    float* th = a.theta + (int64_t)r * a.n_total + off;
    uint32_t* pw = a.phase ? a.phase + (int64_t)r * a.n_total + off : nullptr;
    const int out_id = r * a.I + inst_id;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.sell, (short)0, (int)a.sell_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsrc_uw =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.sell_uw, (short)0, (int)a.sell_uw_bytes, 0x00020000);
    const int voff = lane * 16;

    uint32_t ph[MS][RPL];
    float drift[MS][RPL];
    int sbase[MS], sdeg[MS];

#pragma unroll
    for (int k = 0; k < MS; ++k) {
        const int slice = ws + k * WS;
        const int2 d = slice < S ? a.desc[slice0 + slice] : make_int2(0, 0);
        sbase[k] = __builtin_amdgcn_readfirstlane(d.x);
        sdeg[k] = __builtin_amdgcn_readfirstlane(d.y);
        const int m = slice * 64 + lane;
#pragma unroll
        for (int jj = 0; jj < RPL; ++jj) {
            const int j = j0 + jj;
            const int i = 4 * m + j;
            const bool valid = slice < S && i < n;
            const uint32_t u = valid ? (pw ? pw[i] : phase_from_theta(th[i])) : 0u;
            ph[k][jj] = u;
            drift[k][jj] = 0.0f;
            if (slice < S) sc[j * plane + m] = make_float2(sin_turn(u), cos_turn(u));
        }
    }
    if (threadIdx.x == 0) {
        *best_lds = DBL_MAX;
        *zero_entry = make_float2(0.f, 0.f);
        flag[1] = -1;
    }
    __syncthreads();

    const float sqrt_dt = __builtin_sqrtf(a.dt);

    // Schedules arrive 64 steps at a time, one step per lane, with the next
    // chunk's vector loads in flight while the current chunk is used; each
    // step reads its three values with v_readlane, so no step waits on a
    // scalar load.
    const int64_t sched_off = (int64_t)r * a.sched_stride;
    auto sched = [&](const float* v, int c) {
        const int i = c * 64 + lane;
        return i < a.steps ? v[sched_off + i] : 0.0f;
    };
    float cK = sched(a.K, 0), cKs = sched(a.Ks, 0), cS = sched(a.sigma, 0);
    float nK = sched(a.K, 1), nKs = sched(a.Ks, 1), nS = sched(a.sigma, 1);

    for (int s = 0; s < a.steps; ++s) {
        const uint32_t t = (uint32_t)(a.step0 + s);
        if (s > 0 && (s & 63) == 0) {
            cK = nK;
            cKs = nKs;
            cS = nS;
            const int c = (s >> 6) + 1;
            nK = sched(a.K, c);
            nKs = sched(a.Ks, c);
            nS = sched(a.sigma, c);
        }
        const int sl = s & 63;
        const float Kt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cK), sl));
        const float Kst = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cKs), sl));
        const float St = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cS), sl));
        const float kc = -a.dt * Kt * kTurnScale;
        const float ks = -a.dt * Kst * kTurnScale;
        const float ns = St * sqrt_dt * kTurnScale;

        // ---- phase A: noise, and coupling sums over the sliced-ELL rows ----
        // The first edge loads of a slice are issued, then its Philox noise
        // is computed while they are in flight (the noise depends only on
        // the replica, the quad and the step); per iteration 16-byte buffer
        // loads (scalar offsets, no per-lane address math) over the lane's
        // rows -- with general weights 8 loads of 2 edges, with uniform unit
        // weights 4 loads of 4 edges -- and 16 LDS reads.  drift then holds
        // the whole increment of the step, noise included.
#pragma unroll
        for (int k = 0; k < MS; ++k) {
            if (ws + k * WS < S) {
                const int m = (ws + k * WS) * 64 + lane;
                // the normals wait in drift, whose registers are free until
                // the sums below are complete; the empty asm keeps their
                // computation here, in the shadow of the loads, instead of
                // letting it sink to its use after the sums.  The quad index
                // and the key are re-materialised every step (empty asm) so
                // partial Philox rounds are not precomputed and kept live in
                // registers across the whole run.
                auto noise = [&]() __attribute__((always_inline)) {
                    uint32_t mm = (uint32_t)m, kk0 = k0, kk1 = k1;
                    asm volatile("" : "+v"(mm), "+s"(kk0), "+s"(kk1));
                    if constexpr (RPL == 4) {
                        normals4(mm, t, (uint32_t)inst_id, kk0, kk1, drift[k]);
                        asm volatile("" : "+v"(drift[k][0]), "+v"(drift[k][1]), "+v"(drift[k][2]),
                                     "+v"(drift[k][3]));
                    } else if constexpr (RPL == 2) {
                        normals2(mm, t, (uint32_t)inst_id, kk0, kk1, g, drift[k]);
                        asm volatile("" : "+v"(drift[k][0]), "+v"(drift[k][1]));
                    } else {
                        float z2[2];
                        normals2(mm, t, (uint32_t)inst_id, kk0, kk1, g >> 1, z2);
                        drift[k][0] = (g & 1) ? z2[1] : z2[0];
                        asm volatile("" : "+v"(drift[k][0]));
                    }
                };
                float A[RPL], B[RPL];
                if constexpr (UWT) {
                    // Uniform weight w0 = +-1: each entry is a neighbour's LDS
                    // byte offset alone (padding points at the zero entry), the
                    // row sums its (cos, sin) in entry order and the sum is
                    // scaled by w0 at the end: (-1) x (a chain of roundings)
                    // equals the chain of roundings of the negated terms, so
                    // the result is the multiply-add chain's up to the sign
                    // of a zero sum, which no phase update can tell apart.
                    constexpr int U4 = U / 2;  // 16-byte loads (4 edges) per row per iteration
                    const int D4 = sdeg[k] >> 2;
                    int4 v[RPL][U4];
                    auto load_iter = [&](int e4) __attribute__((always_inline)) {
#pragma unroll
                        for (int jj = 0; jj < RPL; ++jj) {
                            const int soff = ((sbase[k] >> 1) + (j0 + jj) * D4 + e4) * 1024;
#pragma unroll
                            for (int h = 0; h < U4; ++h)
                                if (h == 0 || e4 + h < D4) v[jj][h] = load_pair(rsrc_uw, voff + h * 1024, soff);
                        }
                    };
                    if (D4 > 0) load_iter(0);
                    noise();
#pragma unroll
                    for (int jj = 0; jj < RPL; ++jj) A[jj] = B[jj] = 0.f;
                    for (int e4 = 0; e4 < D4; e4 += U4) {
                        if (RPL == 4 && e4 > 0) load_iter(e4);
                        float2 p[U4][RPL][4];
#pragma unroll
                        for (int h = 0; h < U4; ++h)
#pragma unroll
                            for (int jj = 0; jj < RPL; ++jj) {
                                if (h == 0 || e4 + h < D4) {
                                    p[h][jj][0] = sc_at(smem, v[jj][h].x);
                                    p[h][jj][1] = sc_at(smem, v[jj][h].y);
                                    p[h][jj][2] = sc_at(smem, v[jj][h].z);
                                    p[h][jj][3] = sc_at(smem, v[jj][h].w);
                                }
                            }
                        // split rows (long rows, several iterations): the next
                        // iteration's offsets are loaded now, their L2 round
                        // trip under this iteration's LDS reads and sums (the
                        // reads above have taken their addresses); whole-quad
                        // shapes keep their registers for occupancy
                        if (RPL < 4 && e4 + U4 < D4) load_iter(e4 + U4);
#pragma unroll
                        for (int h = 0; h < U4; ++h) {
                            if (h == 0 || e4 + h < D4) {
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj)
#pragma unroll
                                    for (int x = 0; x < 4; ++x) {
                                        A[jj] = A[jj] + p[h][jj][x].y;
                                        B[jj] = B[jj] + p[h][jj][x].x;
                                    }
                            }
                        }
                    }
#pragma unroll
                    for (int jj = 0; jj < RPL; ++jj) {
                        A[jj] = a.w0 * A[jj];
                        B[jj] = a.w0 * B[jj];
                    }
                } else {
                    const int D2 = sdeg[k] >> 1;
                    int4 v[RPL][U];
                    // loads past the row end (possible only when U > 2, since
                    // rows hold an even number of 16-byte pairs) are skipped
                    auto load_iter = [&](int e2) __attribute__((always_inline)) {
#pragma unroll
                        for (int jj = 0; jj < RPL; ++jj) {
                            const int soff = (sbase[k] + (j0 + jj) * D2 + e2) * 1024;
#pragma unroll
                            for (int h = 0; h < U; ++h)
                                if (h < 2 || e2 + h < D2) v[jj][h] = load_pair(rsrc, voff + h * 1024, soff);
                        }
                    };
                    if (D2 > 0) load_iter(0);
                    noise();
#pragma unroll
                    for (int jj = 0; jj < RPL; ++jj) A[jj] = B[jj] = 0.f;
                    for (int e2 = 0; e2 < D2; e2 += U) {
                        if (e2 > 0) load_iter(e2);
                        // all neighbour reads of the iteration are in flight
                        // before the first multiply-add consumes one
                        float2 p[U][RPL][2];
#pragma unroll
                        for (int h = 0; h < U; ++h)
#pragma unroll
                            for (int jj = 0; jj < RPL; ++jj) {
                                if (h < 2 || e2 + h < D2) {
                                    p[h][jj][0] = sc_at(smem, v[jj][h].x);
                                    p[h][jj][1] = sc_at(smem, v[jj][h].z);
                                }
                            }
#pragma unroll
                        for (int h = 0; h < U; ++h) {
                            if (h < 2 || e2 + h < D2) {
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj) {
                                    A[jj] = __builtin_fmaf(__int_as_float(v[jj][h].y), p[h][jj][0].y, A[jj]);
                                    B[jj] = __builtin_fmaf(__int_as_float(v[jj][h].y), p[h][jj][0].x, B[jj]);
                                    A[jj] = __builtin_fmaf(__int_as_float(v[jj][h].w), p[h][jj][1].y, A[jj]);
                                    B[jj] = __builtin_fmaf(__int_as_float(v[jj][h].w), p[h][jj][1].x, B[jj]);
                                }
                            }
                        }
                    }
                }
#pragma unroll
                for (int jj = 0; jj < RPL; ++jj) {
                    const float2 own = sc[(j0 + jj) * plane + m];
                    const float coup = __builtin_fmaf(own.x, A[jj], -(own.y * B[jj]));
                    // sin(3 theta) = s (3 - 4 s^2) with its multiply-add fused
                    const float sq = QM == 3 ? own.x * __builtin_fmaf(-4.0f * own.x, own.x, 3.0f)
                                             : sin_q<QM>(own.x, own.y, ph[k][jj], q);
                    // the deterministic part of the increment; which of its two
                    // products is fused keeps the rounding this kernel has
                    // always had (the SHIL term for q = 2, the coupling term
                    // otherwise), so results are unchanged bit for bit
                    const float det = QM == 2 ? __builtin_fmaf(ks, sq, kc * coup)
                                              : __builtin_fmaf(kc, coup, ks * sq);
                    drift[k][jj] = __builtin_fmaf(ns, drift[k][jj], det);
                }
            }
        }
        __syncthreads();

        // ---- phase B: Euler-Maruyama update, wrap, table refresh ----
#pragma unroll
        for (int k = 0; k < MS; ++k) {
            const int slice = ws + k * WS;
            const int m = slice * 64 + lane;
            // Rows past n are padding: they are advanced and stored like the
            // others (their slots exist in every plane) but no edge reads them,
            // which keeps per-lane masks out of the loop.
            if (slice < S) {
#pragma unroll
                for (int jj = 0; jj < RPL; ++jj) {
                    const uint32_t u = advance(ph[k][jj], drift[k][jj]);
                    ph[k][jj] = u;
                    sc[(j0 + jj) * plane + m] = make_float2(sin_turn(u), cos_turn(u));
                }
            }
        }
        __syncthreads();

        // ---- optional readout: threshold, Eq. 1 / Eq. 2, best-so-far ----
        if (a.M > 0 && ((s + 1) % a.M == 0 || s + 1 == a.steps)) {
#pragma unroll
            for (int k = 0; k < MS; ++k) {
                const int slice = ws + k * WS;
                const int m = slice * 64 + lane;
                if (slice < S) {
#pragma unroll
                    for (int jj = 0; jj < RPL; ++jj)
                        col8[(j0 + jj) * plane + m] = (unsigned char)nearest_state(ph[k][jj], q);
                }
            }
            __syncthreads();
            // Eq. 1 / Eq. 2 in the library's fixed FP64 order: each row sums
            // its terms over j > i in column order (the ELL row is the CSR row;
            // its entries from the row's split point to its length are the
            // upper triangle); a quad's rows fold as (r0 + r1) +
            // (r2 + r3) and the lanes by the xor butterfly (partner distance
            // 1, 2, ..., 32), which is the pairwise tree over the slice's 256
            // rows.  The tree over slices: with room in LDS every slice's sum
            // is stored and wave 0 folds them (two per lane, then the lanes by
            // distance 1, 2, ..., 32, lower index first); otherwise thread 0
            // folds them, in order, into the same tree, one round of WS
            // slices at a time.
            // The loops below are kept rolled (the slice's descriptor is
            // re-read) so the readout, which runs only every M steps, adds no
            // registers to the step loop.
            TreeAccN<kSliceTreeLevels> tree(tstack);
#pragma unroll 1
            for (int k = 0; k < MS; ++k) {
                if (k * WS >= S) break;  // uniform over the workgroup
                const int slice = ws + k * WS;
                double v = 0.0;
                if (slice < S) {
                    const int2 d = a.desc[slice0 + slice];
                    const int sb = __builtin_amdgcn_readfirstlane(d.x);
                    const int D2 = __builtin_amdgcn_readfirstlane(d.y) >> 1;
                    const int m = slice * 64 + lane;
                    double rs[RPL];
                    int ci[RPL];
                    // Whole quads (the common shapes) find a neighbour's index from
                    // its LDS slot; split-row shapes, whose rows are long, read each
                    // row's split point instead (fewer operations per entry, more
                    // registers, which the whole-quad shapes cannot spare).
                    if constexpr (RPL == 4) {
#pragma unroll
                        for (int jj = 0; jj < RPL; ++jj) {
                            rs[jj] = 0.0;
                            ci[jj] = col8[(j0 + jj) * plane + m];
                        }
                        if constexpr (UWT) {
                            // the unit-weight image: four offsets per load, the
                            // padding (the zero entry's offset) skipped; the terms
                            // are those of the general image in the same order
                            const int D4 = D2 >> 1;
                            const int zoff = 36 * plane;
                            const float wu = a.w0;
                            constexpr int UR4 = RPL == 1 ? 2 : 1;
                            for (int e4 = 0; e4 < D4; e4 += UR4) {
                                int4 e[RPL][UR4];
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj)
#pragma unroll
                                    for (int h = 0; h < UR4; ++h)
                                        if (h == 0 || e4 + h < D4)
                                            e[jj][h] = load_pair(rsrc_uw, voff + h * 1024,
                                                                 ((sb >> 1) + (j0 + jj) * D4 + e4) * 1024);
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj) {
                                    const int own = 4 * m + j0 + jj;
#pragma unroll
                                    for (int h = 0; h < UR4; ++h) {
                                        if (h >= 1 && e4 + h >= D4) break;
                                        const int o4[4] = {e[jj][h].x, e[jj][h].y, e[jj][h].z, e[jj][h].w};
#pragma unroll
                                        for (int x = 0; x < 4; ++x) {
                                            if (o4[x] == zoff) continue;
                                            const int c = col8[o4[x] >> 3];
                                            const bool up = slot_index(o4[x] >> 3, plane) > own;
                                            const float tt = (q == 2) ? (ci[jj] == c ? wu : -wu)
                                                                      : (ci[jj] == c ? wu : 0.f);
                                            rs[jj] += up ? (double)tt : 0.0;
                                        }
                                    }
                                }
                            }
                        } else {
                            // UR entry pairs of every row per iteration (8 loads in
                            // all for whole quads, 4 for split rows, which have fewer
                            // registers to spare), issued before the first is used;
                            // each row still adds its terms in entry order
                            constexpr int UR = RPL == 4 ? 2 : 4 / RPL;
                            for (int e2 = 0; e2 < D2; e2 += UR) {
                                int4 e[RPL][UR];
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj)
#pragma unroll
                                    for (int h = 0; h < UR; ++h)
                                        if (h < 2 || e2 + h < D2)
                                            e[jj][h] = load_pair(rsrc, voff + h * 1024, (sb + (j0 + jj) * D2 + e2) * 1024);
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj) {
                                    const int own = 4 * m + j0 + jj;
#pragma unroll
                                    for (int h = 0; h < UR; ++h) {
                                        if (h >= 2 && e2 + h >= D2) break;
                                        const int4 x = e[jj][h];
                                        const int c0 = col8[x.x >> 3], c1 = col8[x.z >> 3];
                                        const float w0 = __int_as_float(x.y), w1 = __int_as_float(x.w);
                                        // upper triangle only: the neighbour's index from its slot
                                        const bool up0 = slot_index(x.x >> 3, plane) > own;
                                        const bool up1 = slot_index(x.z >> 3, plane) > own;
                                        const float t0 = (q == 2) ? (ci[jj] == c0 ? w0 : -w0) : (ci[jj] == c0 ? w0 : 0.f);
                                        const float t1 = (q == 2) ? (ci[jj] == c1 ? w1 : -w1) : (ci[jj] == c1 ? w1 : 0.f);
                                        rs[jj] += up0 ? (double)t0 : 0.0;
                                        rs[jj] += up1 ? (double)t1 : 0.0;
                                    }
                                }
                            }
                        }
                    } else {
                        // the row's upper triangle j > i: its entries from p on
                        // (columns ascend along a row), before its length
                        int up0[RPL], rlen[RPL];
#pragma unroll
                        for (int jj = 0; jj < RPL; ++jj) {
                            rs[jj] = 0.0;
                            ci[jj] = col8[(j0 + jj) * plane + m];
                            const int2 sp = a.row_split[((slice0 + slice) * 4 + j0 + jj) * 64 + lane];
                            up0[jj] = sp.x;
                            rlen[jj] = sp.y;
                        }
                        if constexpr (UWT) {
                            // the unit-weight image: four offsets per load; every
                            // term is +-w0 (or 0), so the row counts them in an
                            // integer, whose product with w0 is the sum of the
                            // terms in any order, exactly
                            const int D4 = D2 >> 1;
                            constexpr int UR4 = RPL == 1 ? 2 : 1;
                            int cnt[RPL];
#pragma unroll
                            for (int jj = 0; jj < RPL; ++jj) cnt[jj] = 0;
                            for (int e4 = 0; e4 < D4; e4 += UR4) {
                                int4 e[RPL][UR4];
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj)
#pragma unroll
                                    for (int h = 0; h < UR4; ++h)
                                        if (h == 0 || e4 + h < D4)
                                            e[jj][h] = load_pair(rsrc_uw, voff + h * 1024,
                                                                 ((sb >> 1) + (j0 + jj) * D4 + e4) * 1024);
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj) {
#pragma unroll
                                    for (int h = 0; h < UR4; ++h) {
                                        if (h >= 1 && e4 + h >= D4) break;
                                        const int o4[4] = {e[jj][h].x, e[jj][h].y, e[jj][h].z, e[jj][h].w};
#pragma unroll
                                        for (int x = 0; x < 4; ++x) {
                                            const int idx = 4 * (e4 + h) + x;
                                            const bool up = idx >= up0[jj] && idx < rlen[jj];
                                            // (padding, never counted, points past the colours)
                                            const bool eq = ci[jj] == col8[up ? o4[x] >> 3 : 0];
                                            const int tt = eq ? 1 : (q == 2 ? -1 : 0);
                                            cnt[jj] += up ? tt : 0;
                                        }
                                    }
                                }
                            }
#pragma unroll
                            for (int jj = 0; jj < RPL; ++jj) rs[jj] = (double)a.w0 * (double)cnt[jj];
                        } else {
                            // UR entry pairs of every row per iteration (8 loads in
                            // all for whole quads, 4 for split rows, which have fewer
                            // registers to spare), issued before the first is used;
                            // each row adds its terms in entry order
                            constexpr int UR = RPL == 4 ? 2 : 4 / RPL;
                            for (int e2 = 0; e2 < D2; e2 += UR) {
                                int4 e[RPL][UR];
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj)
#pragma unroll
                                    for (int h = 0; h < UR; ++h)
                                        if (h < 2 || e2 + h < D2)
                                            e[jj][h] = load_pair(rsrc, voff + h * 1024, (sb + (j0 + jj) * D2 + e2) * 1024);
#pragma unroll
                                for (int jj = 0; jj < RPL; ++jj) {
#pragma unroll
                                    for (int h = 0; h < UR; ++h) {
                                        if (h >= 2 && e2 + h >= D2) break;
                                        const int4 x = e[jj][h];
                                        const int i0 = 2 * (e2 + h);
                                        const bool u0 = i0 >= up0[jj] && i0 < rlen[jj];
                                        const bool u1 = i0 + 1 >= up0[jj] && i0 + 1 < rlen[jj];
                                        const int c0 = col8[x.x >> 3], c1 = col8[x.z >> 3];
                                        const float w0 = __int_as_float(x.y), w1 = __int_as_float(x.w);
                                        const float t0 = (q == 2) ? (ci[jj] == c0 ? w0 : -w0) : (ci[jj] == c0 ? w0 : 0.f);
                                        const float t1 = (q == 2) ? (ci[jj] == c1 ? w1 : -w1) : (ci[jj] == c1 ? w1 : 0.f);
                                        rs[jj] += u0 ? (double)t0 : 0.0;
                                        rs[jj] += u1 ? (double)t1 : 0.0;
                                    }
                                }
                            }
                        }
                    }
                    if constexpr (RPL == 4) v = (rs[0] + rs[1]) + (rs[2] + rs[3]);
                    else if constexpr (RPL == 2) v = rs[0] + rs[1];
                    else v = rs[0];
                }
                if constexpr (RPL < 4) {
                    // the quad's partial sums meet in LDS; wave g = 0 folds them
                    part[(ws * G + g) * 64 + lane] = v;
                    __syncthreads();
                    if (g == 0 && slice < S) {
                        const double* pp = part + ws * G * 64 + lane;
                        if constexpr (RPL == 2) v = pp[0] + pp[64];
                        else v = (pp[0] + pp[64]) + (pp[128] + pp[192]);
                    }
                }
                if (g == 0 && slice < S) {
                    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
                    if (lane == 0) {
                        if (a.slice_sums) ssum[slice] = v;
                        else red[ws] = v;
                    }
                }
                if (a.slice_sums) {
                    // part is reused by the next slice
                    if constexpr (RPL < 4) __syncthreads();
                    continue;
                }
                __syncthreads();
                if (threadIdx.x == 0)
                    for (int w = 0; w < WS && k * WS + w < S; ++w) tree.push(red[w]);
                __syncthreads();
            }
            double total = 0.0;
            if (a.slice_sums) {
                __syncthreads();
                if (wave == 0) {
                    // S <= 128 slices: two per lane, zero-padded
                    const double v0 = 2 * lane < S ? ssum[2 * lane] : 0.0;
                    const double v1 = 2 * lane + 1 < S ? ssum[2 * lane + 1] : 0.0;
                    double v = v0 + v1;
                    for (int o = 1; o < 64; o <<= 1) v = v + __shfl_down(v, o, 64);
                    total = v;
                }
            } else if (threadIdx.x == 0) {
                total = tree.finish();
            }
            if (threadIdx.x == 0) {
                const double H = -total;
                const int kread = (s + a.M) / a.M - 1;
                if (a.trace) a.trace[(int64_t)kread * a.R * a.I + out_id] = H;
                int improved = 0;
                if (H < *best_lds) {
                    *best_lds = H;
                    flag[1] = (int32_t)(a.step0 + s + 1);
                    improved = 1;
                }
                flag[0] = improved;
            }
            __syncthreads();
            if (flag[0] && a.best_colour) {
                int8_t* bc = a.best_colour + (int64_t)r * a.n_total + off;
#pragma unroll 1
                for (int k = 0; k < MS; ++k) {
                    const int slice = ws + k * WS;
                    const int m = slice * 64 + lane;
#pragma unroll
                    for (int jj = 0; jj < RPL; ++jj) {
                        const int i = 4 * m + j0 + jj;
                        if (slice < S && i < n) bc[i] = (int8_t)col8[(j0 + jj) * plane + m];
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- final phases ----
#pragma unroll
    for (int k = 0; k < MS; ++k) {
        const int slice = ws + k * WS;
        const int m = slice * 64 + lane;
#pragma unroll
        for (int jj = 0; jj < RPL; ++jj) {
            const int i = 4 * m + j0 + jj;
            if (slice < S && i < n) {
                th[i] = theta_from_phase(ph[k][jj]);
                if (pw) pw[i] = ph[k][jj];
            }
        }
    }
    if (threadIdx.x == 0) {
        const int32_t best_at = flag[1];
        if (a.best_h) a.best_h[out_id] = best_at >= 0 ? *best_lds : __builtin_inf();
        if (a.best_step) a.best_step[out_id] = best_at;
    }
}

using KernelFn = void (*)(PersistArgs);

// Launch variants (threads per workgroup, slices per wave group, rows of a
// quad per lane), in the order the autotuner tries them: block sizes from
// one wave up -- the small ones suit batches of small instances (fewer idle
// lanes, cheap barriers) -- then the split-row shapes, which suit instances
// of a few slices with long rows.
#define OIM_PERSIST_VARIANTS(X)                                                          \
    X(64, 1, 4) X(64, 2, 4) X(64, 3, 4) X(64, 4, 4) X(64, 6, 4) X(64, 8, 4)               \
    X(128, 1, 4) X(128, 2, 4) X(128, 3, 4) X(128, 4, 4) X(128, 6, 4) X(128, 8, 4)         \
    X(256, 1, 4) X(256, 2, 4) X(256, 3, 4) X(256, 4, 4) X(256, 6, 4) X(256, 8, 4)         \
    X(256, 10, 4) X(256, 12, 4)                                                          \
    X(512, 1, 4) X(512, 2, 4) X(512, 3, 4) X(512, 4, 4) X(512, 5, 4) X(512, 6, 4)         \
    X(512, 8, 4) X(512, 10, 4)                                                           \
    X(640, 4, 4) X(768, 3, 4) X(768, 4, 4)                                               \
    X(1024, 1, 4) X(1024, 2, 4) X(1024, 3, 4) X(1024, 4, 4) X(1024, 5, 4)               \
    X(256, 1, 1) X(256, 1, 2) X(512, 1, 1) X(512, 1, 2) X(512, 2, 2) X(1024, 1, 1)       \
    X(1024, 2, 1) X(1024, 1, 2) X(1024, 2, 2)

#define OIM_PERSIST_COUNT_ONE(TB, MS, RPL) +1
constexpr int kVariantCount = 0 OIM_PERSIST_VARIANTS(OIM_PERSIST_COUNT_ONE);

// The unit-weight instantiations (q classes generic, 2, 3) of every variant,
// in list order; defined in sparse_persistent_uw.hip.
extern const KernelFn kUniformKernels[kVariantCount][3];

}  // namespace persist
}  // namespace oim
