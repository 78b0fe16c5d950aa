// dense.hip -- all-to-all coupling (Sec. III-B: flattened dense J; the
// paper's O(n^2) derivative loop) as a GEMM on the matrix cores.
//
// With S = sin(Theta), C = cos(Theta) stored replica-major ([R][n]), the
// coupling sum of Eq. 5 for all oscillators and replicas is
//     c_ir = sum_j J_ij sin(th_ir - th_jr) = s_ir (J C)_ir - c_ir (J S)_ir,
// so one step is Y = J [S | C] (M = n rows, N = 2R columns, K = n) plus an
// elementwise epilogue.  J and X = [S | C] are split into BF16 pairs
// (x = x_hi + x_lo, x_hi = bf16(x), x_lo = bf16(x - x_hi)) and
//     J X ~ J_hi X_hi + J_hi X_lo + J_lo X_hi
// is accumulated in FP32 on v_mfma_f32_16x16x32_bf16 (the dropped J_lo X_lo
// term is ~2^-16 relative).  With OIM_PREC_FP32 the product runs instead with
// FP32 operands on v_mfma_f32_16x16x4_f32 (dense_step32_kernel below).  J's
// diagonal is zeroed at upload.
//
// One kernel per Euler-Maruyama step: workgroup tile = 128 rows x 64
// replicas (S and C columns of the same replicas), 4 waves of 64 rows x 32
// replicas, K in stages of 32 moved into a ring of 4 LDS buffers.  The
// epilogue owns, per lane, quads of 4 consecutive rows of one replica -- the
// MFMA accumulator layout -- so it draws one Philox call per quad, advances
// the phase words and writes the next step's split [S | C] (ping-pong).
#include <float.h>

#include <cmath>

#include "internal.hpp"
#include "noise.hpp"
#include "phase.hpp"
#include "tree.hpp"

namespace oim {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 128;  // rows per workgroup
constexpr int kTR = 64;   // replicas per workgroup
constexpr int kTK = 32;   // K per stage (one MFMA K-step)
constexpr int kDepth = 4; // LDS stage buffers (kDepth - 1 stages of loads in flight)
constexpr int kSegs = kTK / 8;                            // 16-byte segments per LDS row
constexpr int kStageBytes = (2 * kTM + 4 * kTR) * kTK * 2;  // A hi/lo + B 4 comps
constexpr int kTB = 256;  // threads

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_val(hi));
}

// Byte offset of 16-byte segment `seg` of LDS row `row` (rows of kTK bf16 =
// 64 bytes), XOR-swizzled by row so that the 8 consecutive rows a group of
// lanes reads at one logical segment cover all banks once.
__device__ __forceinline__ int swz(int row, int seg) {
    return row * (kTK * 2) + ((seg ^ ((row >> 1) & (kSegs - 1))) << 4);
}

// Operands live in HBM as tiled images of what one stage puts in LDS, so that
// every DMA instruction of a wave moves 1 KiB of contiguous memory:
//   J: block (row tile ti, stage kc) of 16 KiB at (ti * nk + kc) * 16 KiB,
//      J_hi rows then J_lo rows (kA bytes each);
//   X: block (replica tile tr, stage kc) of 16 KiB at (tr * nk + kc) * 16 KiB,
//      components S_hi, S_lo, C_hi, C_lo (kB bytes each).
// Inside a block a row of kTK = 32 elements is 64 bytes, segments swizzled
// exactly as in LDS.  Byte offset of element (row rr, column kk) of a region:
__device__ __forceinline__ int tile_off(int rr, int kk) {
    return swz(rr, kk >> 3) + (kk & 7) * 2;
}

struct DenseArgs {
    const unsigned char* Jt;   // tiled J_hi / J_lo, np x np each
    const unsigned char* Xin;  // tiled X = [S | C] split, Rp x np x 4 components
    unsigned char* Xout;
    uint32_t* U;           // [Rp][np] phase words
    const uint64_t* seeds;
    int np, Rp, n, R, q, nk;
    const float* K;        // schedules, [steps] or [R][steps] (sched_stride = steps)
    const float* Ks;
    const float* sigma;
    int sched_stride;
    int s;                 // local step index
    uint32_t t;            // global step index
    float dt, sqrt_dt;
};

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

constexpr int kRow = kTK * 2;              // bytes per LDS row
constexpr int kA = kTM * kRow;             // one A matrix per stage
constexpr int kB = kTR * kRow;             // one B component per stage
constexpr int kWaveChunks = kStageBytes / 1024 / (kTB / 64);  // 1 KiB DMA chunks per wave per stage
constexpr int kBlock = kStageBytes / 2;    // bytes of one tiled J or X block (one stage)

// s_waitcnt immediate that waits until at most `n` vector-memory operations
// of this wave are outstanding (lgkm and exp counters left at their maxima).
__device__ __forceinline__ constexpr int vmcnt_imm(int n) {
    return (n & 0xf) | ((n >> 4) << 14) | (0x7 << 4) | (0xf << 8);
}

// Barrier that completes this wave's LDS reads and nothing else: the DMA
// loads of later stages stay in flight (a workgroup fence, as in
// __syncthreads, would wait for every outstanding vector-memory operation).
// The wait is a builtin so the compiler's own counter bookkeeping sees it; the
// empty asm statements keep memory accesses from moving across the barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt and expcnt at their maxima
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Workgroup -> (row tile, replica tile).  The grid is one-dimensional and
// consecutive workgroups go to the 8 XCDs in turn, each XCD with its own L2;
// the tiles are numbered so that XCD c runs a contiguous range of them, row
// tile major: the replica tiles that share a row tile of J (and read the
// same J blocks at the same stage) sit on one XCD, in consecutive slots.
__device__ __forceinline__ void block_tiles(int ntr, int& ti, int& tr) {
    const int N = (int)gridDim.x, L = (int)blockIdx.x;
    const int c = L & 7, slot = L >> 3;
    const int f = c * (N >> 3) + (c < (N & 7) ? c : (N & 7)) + slot;
    ti = f / ntr;
    tr = f - ti * ntr;
}

// One 256-thread workgroup per CU (one wave per SIMD).  Stages move from
// global memory to LDS with direct DMA loads (global_load_lds_dwordx4: lane
// l of a wave writes bytes 16l..16l+15 of a 1 KiB LDS chunk), so no staging
// registers are needed and kDepth - 1 stages are in flight while one is
// multiplied.  The XOR swizzle of the LDS rows is applied on the source
// side: lane l fetches the segment that belongs at its fixed LDS slot.
template <int QM>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(1, 1)))
void dense_step_kernel(DenseArgs a) {
    __shared__ __align__(1024) unsigned char lds[kDepth][kStageBytes];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    int ti, tr;
    block_tiles(a.Rp / kTR, ti, tr);
    const int i0 = ti * kTM, r0 = tr * kTR;
    const int np = a.np, Rp = a.Rp;
    const size_t plane = (size_t)Rp * np;

    // Chunk c of a stage (1 KiB) sits at LDS bytes 1024c: chunks 0-15 are the
    // J block of the stage, 16-31 the X block.  Wave w moves chunks
    // 8w..8w+7, lane l the 16 bytes at 16l of each.
    const unsigned char* src = wave < 2
        ? a.Jt + (size_t)ti * a.nk * kBlock + wave * kWaveChunks * 1024 + lane * 16
        : a.Xin + (size_t)tr * a.nk * kBlock + (wave - 2) * kWaveChunks * 1024 + lane * 16;
    auto issue = [&](int kc, int buf) __attribute__((always_inline)) {
        unsigned char* dst = lds[buf] + wave * kWaveChunks * 1024;
        const unsigned char* sp = src + (size_t)kc * kBlock;
#pragma unroll
        for (int x = 0; x < kWaveChunks; ++x)
            __builtin_amdgcn_global_load_lds((glb_void_t*)(sp + x * 1024),
                                             (lds_void_t*)(dst + x * 1024), 16, 0, 0);
    };

    f32x4 acc[4][2][2];  // [row block][replica block][S, C]
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[b][c][0] = acc[b][c][1] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int nk = np / kTK;  // a multiple of 4 (np is a multiple of 128)
    const int frow = lane & 15, fseg = lane >> 4;

    // MFMA operand fragments of one stage: lane l holds row l%16 of each
    // 16-row block at K offsets 8(l/16)..8(l/16)+7.
    struct Frags {
        bf16x8 ah[4], al[4];          // J_hi, J_lo of the wave's 4 row blocks
        bf16x8 bh[2][2], bl[2][2];    // X_hi, X_lo [replica block][S, C]
    };
    auto read_frags = [&](const unsigned char* base, Frags& f) __attribute__((always_inline)) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int row = wn * 32 + cb * 16 + frow;
#pragma unroll
            for (int sc = 0; sc < 2; ++sc) {
                const unsigned char* bb = base + 2 * kA + (2 * sc) * kB;
                f.bh[cb][sc] = *reinterpret_cast<const bf16x8*>(bb + swz(row, fseg));
                f.bl[cb][sc] = *reinterpret_cast<const bf16x8*>(bb + kB + swz(row, fseg));
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = wm * 64 + b * 16 + frow;
            f.ah[b] = *reinterpret_cast<const bf16x8*>(base + swz(row, fseg));
            f.al[b] = *reinterpret_cast<const bf16x8*>(base + kA + swz(row, fseg));
        }
    };
    // the three split products of one accumulator are 16 MFMAs apart, so no
    // MFMA waits for the result of the one before it
    auto mfmas = [&](const Frags& f) __attribute__((always_inline)) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int sc = 0; sc < 2; ++sc)
                        acc[b][cb][sc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            p == 2 ? f.al[b] : f.ah[b], p == 1 ? f.bl[cb][sc] : f.bh[cb][sc],
                            acc[b][cb][sc], 0, 0, 0);
    };
    // One stage kc < nk - 1: its fragments were requested a stage earlier
    // (cur).  After the barrier stage kc + 1 is readable and the buffer of
    // stage kc - 1 is free: the DMA of stage kc + kDepth - 1 (clamped to the
    // last stage near the end, which only refills a buffer nobody reads
    // again), the fragment reads of stage kc + 1 and the MFMAs of stage kc are
    // interleaved so that neither the DMA queue nor LDS holds up the matrix
    // cores.
    auto stage = [&](int kc, Frags& cur, Frags& nxt) __attribute__((always_inline)) {
        // stages 0 .. kc + kDepth - 2 are issued; stage kc + 1 has landed
        // when only the kDepth - 3 stages after it are outstanding
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((kDepth - 3) * kWaveChunks));
        lds_barrier();
        // the reads come first in program order: the compiler cannot tell the
        // DMA's LDS target from the buffer being read and keeps that order
        read_frags(lds[(kc + 1) % kDepth], nxt);
        issue(kc + kDepth - 1 < nk ? kc + kDepth - 1 : nk - 1, (kc + kDepth - 1) % kDepth);
        mfmas(cur);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // DS read
            __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);  // MFMA
        }
#pragma unroll
        for (int i = 0; i < kWaveChunks; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM (DMA)
            __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);  // MFMA
        }
    };

#pragma unroll
    for (int d = 0; d < kDepth - 1; ++d) issue(d, d);
    __builtin_amdgcn_s_waitcnt(vmcnt_imm((kDepth - 2) * kWaveChunks));
    lds_barrier();
    Frags F0, F1;
    read_frags(lds[0], F0);
    for (int kc = 0; kc < nk - 2; kc += 2) {
        stage(kc, F0, F1);
        stage(kc + 1, F1, F0);
    }
    stage(nk - 2, F0, F1);
    // The epilogue's phase words and keys are requested in one batch before
    // the last stage's MFMAs, so their latency overlaps them (U is padded to
    // Rp x np, so every quad's load is in bounds).
    const int qi0 = i0 + wm * 64 + 4 * (lane >> 4);  // first row of the quads of block b = 0
    uint4 uq[2][4];
    uint64_t seedv[2];
    float sK[2], sKs[2], sS[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int r = r0 + wn * 32 + cb * 16 + (lane & 15);
        seedv[cb] = r < a.R ? a.seeds[r] : 0ull;
        const int64_t so = (int64_t)(r < a.R ? r : 0) * a.sched_stride + a.s;
        sK[cb] = a.K[so];
        sKs[cb] = a.Ks[so];
        sS[cb] = a.sigma[so];
#pragma unroll
        for (int b = 0; b < 4; ++b)
            uq[cb][b] = *reinterpret_cast<const uint4*>(a.U + (size_t)r * np + qi0 + b * 16);
    }
    mfmas(F1);
    // the refills issued by the last stages land before the LDS is released
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));

    // ---- epilogue: SHIL, noise, Euler-Maruyama update, next split X ----
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int r = r0 + wn * 32 + cb * 16 + (lane & 15);
        const bool rvalid = r < a.R;
        // step coefficients in 2^-32-turn units
        const float kcoef = -a.dt * sK[cb] * kTurnScale;
        const float kscoef = -a.dt * sKs[cb] * kTurnScale;
        const float nscoef = sS[cb] * a.sqrt_dt * kTurnScale;
        const uint32_t k0 = (uint32_t)seedv[cb], k1 = (uint32_t)(seedv[cb] >> 32);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = qi0 + b * 16;  // first row of the quad
            if (!rvalid || i >= a.n) continue;
            uint32_t u[4] = {uq[cb][b].x, uq[cb][b].y, uq[cb][b].z, uq[cb][b].w};
            float z[4];
            normals4((uint32_t)(i >> 2), a.t, 0u, k0, k1, z);
            uint16_t shi[4], slo[4], chi[4], clo[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const float s0 = sin_turn(u[x]), c0 = cos_turn(u[x]);
                const float coup = s0 * acc[b][cb][1][x] - c0 * acc[b][cb][0][x];
                const float drift = kcoef * coup + kscoef * sin_q<QM>(s0, c0, u[x], a.q);
                if (i + x < a.n) u[x] = advance(u[x], __builtin_fmaf(nscoef, z[x], drift));
                const float s1 = i + x < a.n ? sin_turn(u[x]) : 0.f;
                const float c1 = i + x < a.n ? cos_turn(u[x]) : 0.f;
                split_bf16(s1, shi[x], slo[x]);
                split_bf16(c1, chi[x], clo[x]);
            }
            *reinterpret_cast<uint4*>(a.U + (size_t)r * np + i) = uint4{u[0], u[1], u[2], u[3]};
            unsigned char* xo = a.Xout + ((size_t)(r >> 6) * a.nk + (i >> 5)) * kBlock +
                                tile_off(r & 63, i & 31);
            *reinterpret_cast<uint2*>(xo + 0 * kB) =
                uint2{shi[0] | ((uint32_t)shi[1] << 16), shi[2] | ((uint32_t)shi[3] << 16)};
            *reinterpret_cast<uint2*>(xo + 1 * kB) =
                uint2{slo[0] | ((uint32_t)slo[1] << 16), slo[2] | ((uint32_t)slo[3] << 16)};
            *reinterpret_cast<uint2*>(xo + 2 * kB) =
                uint2{chi[0] | ((uint32_t)chi[1] << 16), chi[2] | ((uint32_t)chi[3] << 16)};
            *reinterpret_cast<uint2*>(xo + 3 * kB) =
                uint2{clo[0] | ((uint32_t)clo[1] << 16), clo[2] | ((uint32_t)clo[3] << 16)};
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 coupling (OIM_PREC_FP32): the same product Y = J [S | C] with FP32
// operands on v_mfma_f32_16x16x4_f32 (FP32 products, FP32 accumulation: the
// paper's own precision), same workgroup tile, same stage size (32 K values of
// FP32 = 32 KiB of J and X per stage), same DMA ring and barriers.
//
// Image layout: a row of one stage block holds 32 FP32 values (128 bytes).
// MFMA K-step kk (0..7) of a stage takes K index 4 kk + g in lane group
// g = lane / 16, so the values are stored K-permuted, position 8 g + kk holding
// K index 4 kk + g: each lane group's 8 values of a stage are 32 contiguous
// bytes (two 16-byte reads).  The permutation is the same for J's columns and
// X's rows, so the product is the same sum over K.  The eight 16-byte
// segments of a row are XOR-swizzled by (row / 2) % 8, which spreads the 16
// rows one lane group reads over all banks.
//   J: block (row tile ti, stage kc) at (ti * nk + kc) * 16 KiB, 128 rows;
//   X: block (replica tile tr, stage kc) at (tr * nk + kc) * 16 KiB, S rows
//      (64) then C rows (64).
constexpr int kRow32 = kTK * 4;  // bytes per FP32 row

__device__ __forceinline__ int swz32(int row, int seg) {
    return row * kRow32 + ((seg ^ ((row >> 1) & 7)) << 4);
}
// byte offset of (row rr, K index kk) inside a block region
__device__ __forceinline__ int tile_off32(int rr, int kk) {
    const int pos = (kk & 3) * 8 + (kk >> 2);
    return swz32(rr, pos >> 2) + (pos & 3) * 4;
}

template <int QM>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(1, 1)))
void dense_step32_kernel(DenseArgs a) {
    __shared__ __align__(1024) unsigned char lds[kDepth][kStageBytes];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    int ti, tr;
    block_tiles(a.Rp / kTR, ti, tr);
    const int i0 = ti * kTM, r0 = tr * kTR;
    const int np = a.np;

    const unsigned char* src = wave < 2
        ? a.Jt + (size_t)ti * a.nk * kBlock + wave * kWaveChunks * 1024 + lane * 16
        : a.Xin + (size_t)tr * a.nk * kBlock + (wave - 2) * kWaveChunks * 1024 + lane * 16;
    auto issue = [&](int kc, int buf) __attribute__((always_inline)) {
        unsigned char* dst = lds[buf] + wave * kWaveChunks * 1024;
        const unsigned char* sp = src + (size_t)kc * kBlock;
#pragma unroll
        for (int x = 0; x < kWaveChunks; ++x)
            __builtin_amdgcn_global_load_lds((glb_void_t*)(sp + x * 1024),
                                             (lds_void_t*)(dst + x * 1024), 16, 0, 0);
    };

    f32x4 acc[4][2][2];  // [row block][replica block][S, C]
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[b][c][0] = acc[b][c][1] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int nk = a.nk;
    const int frow = lane & 15, g = lane >> 4;
    // lane group g's 8 values of a row: segments 2g and 2g + 1
    struct Frags32 {
        f32x4 a[4][2];      // J, 4 row blocks
        f32x4 b[2][2][2];   // X [replica block][S, C]
    };
    auto read_frags = [&](const unsigned char* base, Frags32& f) __attribute__((always_inline)) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int row = wn * 32 + cb * 16 + frow;
#pragma unroll
            for (int sc = 0; sc < 2; ++sc) {
                const unsigned char* bb = base + kTM * kRow32 + sc * kTR * kRow32;
                f.b[cb][sc][0] = *reinterpret_cast<const f32x4*>(bb + swz32(row, 2 * g));
                f.b[cb][sc][1] = *reinterpret_cast<const f32x4*>(bb + swz32(row, 2 * g + 1));
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = wm * 64 + b * 16 + frow;
            f.a[b][0] = *reinterpret_cast<const f32x4*>(base + swz32(row, 2 * g));
            f.a[b][1] = *reinterpret_cast<const f32x4*>(base + swz32(row, 2 * g + 1));
        }
    };
    auto mfmas = [&](const Frags32& f) __attribute__((always_inline)) {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int sc = 0; sc < 2; ++sc)
                        acc[b][cb][sc] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            f.a[b][kk >> 2][kk & 3], f.b[cb][sc][kk >> 2][kk & 3], acc[b][cb][sc],
                            0, 0, 0);
    };
    auto stage = [&](int kc, Frags32& cur, Frags32& nxt) __attribute__((always_inline)) {
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((kDepth - 3) * kWaveChunks));
        lds_barrier();
        read_frags(lds[(kc + 1) % kDepth], nxt);
        issue(kc + kDepth - 1 < nk ? kc + kDepth - 1 : nk - 1, (kc + kDepth - 1) % kDepth);
        mfmas(cur);
    };

#pragma unroll
    for (int d = 0; d < kDepth - 1; ++d) issue(d, d);
    __builtin_amdgcn_s_waitcnt(vmcnt_imm((kDepth - 2) * kWaveChunks));
    lds_barrier();
    Frags32 F0, F1;
    read_frags(lds[0], F0);
    for (int kc = 0; kc < nk - 2; kc += 2) {
        stage(kc, F0, F1);
        stage(kc + 1, F1, F0);
    }
    stage(nk - 2, F0, F1);
    const int qi0 = i0 + wm * 64 + 4 * (lane >> 4);
    uint4 uq[2][4];
    uint64_t seedv[2];
    float sK[2], sKs[2], sS[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int r = r0 + wn * 32 + cb * 16 + (lane & 15);
        seedv[cb] = r < a.R ? a.seeds[r] : 0ull;
        const int64_t so = (int64_t)(r < a.R ? r : 0) * a.sched_stride + a.s;
        sK[cb] = a.K[so];
        sKs[cb] = a.Ks[so];
        sS[cb] = a.sigma[so];
#pragma unroll
        for (int b = 0; b < 4; ++b)
            uq[cb][b] = *reinterpret_cast<const uint4*>(a.U + (size_t)r * np + qi0 + b * 16);
    }
    mfmas(F1);
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));

    // ---- epilogue: SHIL, noise, Euler-Maruyama update, next [S | C] ----
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int r = r0 + wn * 32 + cb * 16 + (lane & 15);
        const bool rvalid = r < a.R;
        const float kcoef = -a.dt * sK[cb] * kTurnScale;
        const float kscoef = -a.dt * sKs[cb] * kTurnScale;
        const float nscoef = sS[cb] * a.sqrt_dt * kTurnScale;
        const uint32_t k0 = (uint32_t)seedv[cb], k1 = (uint32_t)(seedv[cb] >> 32);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = qi0 + b * 16;
            if (!rvalid || i >= a.n) continue;
            uint32_t u[4] = {uq[cb][b].x, uq[cb][b].y, uq[cb][b].z, uq[cb][b].w};
            float z[4];
            normals4((uint32_t)(i >> 2), a.t, 0u, k0, k1, z);
            float s1[4], c1[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const float s0 = sin_turn(u[x]), c0 = cos_turn(u[x]);
                const float coup = s0 * acc[b][cb][1][x] - c0 * acc[b][cb][0][x];
                const float drift = kcoef * coup + kscoef * sin_q<QM>(s0, c0, u[x], a.q);
                if (i + x < a.n) u[x] = advance(u[x], __builtin_fmaf(nscoef, z[x], drift));
                s1[x] = i + x < a.n ? sin_turn(u[x]) : 0.f;
                c1[x] = i + x < a.n ? cos_turn(u[x]) : 0.f;
            }
            *reinterpret_cast<uint4*>(a.U + (size_t)r * np + i) = uint4{u[0], u[1], u[2], u[3]};
            unsigned char* xo = a.Xout + ((size_t)(r >> 6) * a.nk + (i >> 5)) * kBlock;
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int off = tile_off32(r & 63, (i & 31) + x);
                *reinterpret_cast<float*>(xo + off) = s1[x];
                *reinterpret_cast<float*>(xo + kTR * kRow32 + off) = c1[x];
            }
        }
    }
}

// Phase words and FP32 [S | C] of the initial state in the FP32 image layout.
__global__ __launch_bounds__(256) void dense_init32_kernel(const float* theta, const uint32_t* phase,
                                                           uint32_t* U, unsigned char* X,
                                                           unsigned char* X2, int n, int R, int np,
                                                           int Rp) {
    const size_t plane = (size_t)Rp * np;
    const int nk = np / kTK;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < plane;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / np), i = (int)(e % np);
        uint32_t u = 0;
        float s = 0.f, c = 0.f;
        if (r < R && i < n) {
            const size_t src = (size_t)r * n + i;
            u = phase ? phase[src] : phase_from_theta(theta[src]);
            s = sin_turn(u);
            c = cos_turn(u);
        }
        U[e] = u;
        const size_t o = ((size_t)(r >> 6) * nk + (i >> 5)) * kBlock + tile_off32(r & 63, i & 31);
        *reinterpret_cast<float*>(X + o) = s;
        *reinterpret_cast<float*>(X + o + kTR * kRow32) = c;
        *reinterpret_cast<float*>(X2 + o) = s;
        *reinterpret_cast<float*>(X2 + o + kTR * kRow32) = c;
    }
}

// J -> FP32 image with the diagonal and the padding zeroed.
__global__ __launch_bounds__(256) void dense_tile32_kernel(const float* J, unsigned char* Jt, int n,
                                                           int np) {
    const size_t total = (size_t)np * np;
    const int nk = np / kTK;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / np), j = (int)(e % np);
        const float v = (i < n && j < n && i != j) ? J[(size_t)i * n + j] : 0.f;
        const size_t o = ((size_t)(i / kTM) * nk + j / kTK) * kBlock + tile_off32(i % kTM, j % kTK);
        *reinterpret_cast<float*>(Jt + o) = v;
    }
}

// Phase words and split [S | C] of the initial state, written to both
// ping-pong sets; padding rows and replicas get X = 0 in both (they add
// nothing to any coupling sum and the step kernel never writes them).
__global__ __launch_bounds__(256) void dense_init_kernel(const float* theta, const uint32_t* phase,
                                                         uint32_t* U, unsigned char* X,
                                                         unsigned char* X2, int n, int R, int np,
                                                         int Rp) {
    const size_t plane = (size_t)Rp * np;
    const int nk = np / kTK;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < plane;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / np), i = (int)(e % np);
        uint32_t u = 0;
        float s = 0.f, c = 0.f;
        if (r < R && i < n) {
            const size_t src = (size_t)r * n + i;
            u = phase ? phase[src] : phase_from_theta(theta[src]);
            s = sin_turn(u);
            c = cos_turn(u);
        }
        U[e] = u;
        uint16_t sh, sl, ch, cl;
        split_bf16(s, sh, sl);
        split_bf16(c, ch, cl);
        const size_t o = ((size_t)(r >> 6) * nk + (i >> 5)) * kBlock + tile_off(r & 63, i & 31);
        const uint16_t v[4] = {sh, sl, ch, cl};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            *reinterpret_cast<uint16_t*>(X + o + k * kB) = v[k];
            *reinterpret_cast<uint16_t*>(X2 + o + k * kB) = v[k];
        }
    }
}

__global__ __launch_bounds__(256) void dense_final_kernel(const uint32_t* U, float* theta,
                                                          uint32_t* phase, int n, int R, int np) {
    const size_t total = (size_t)R * n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / n), i = (int)(e % n);
        const uint32_t u = U[(size_t)r * np + i];
        theta[e] = theta_from_phase(u);
        if (phase) phase[e] = u;
    }
}

// J -> tiled (J_hi, J_lo) with the diagonal and the padding zeroed.
__global__ __launch_bounds__(256) void dense_split_kernel(const float* J, unsigned char* Jt, int n,
                                                          int np) {
    const size_t total = (size_t)np * np;
    const int nk = np / kTK;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / np), j = (int)(e % np);
        const float v = (i < n && j < n && i != j) ? J[(size_t)i * n + j] : 0.f;
        uint16_t h, l;
        split_bf16(v, h, l);
        const size_t o = ((size_t)(i / kTM) * nk + j / kTK) * kBlock + tile_off(i % kTM, j % kTK);
        *reinterpret_cast<uint16_t*>(Jt + o) = h;
        *reinterpret_cast<uint16_t*>(Jt + o + kA) = l;
    }
}

// Thresholded energy per replica from the phase words (in-run readout):
// one workgroup per replica, H = Eq. 1 (q = 2) or Eq. 2 (q >= 3) in the
// library's fixed FP64 order: thread t owns row 256 b + t of block b and
// sums its terms over j > i in column order; a block's rows are folded by
// the pairwise tree (lanes by the xor butterfly, partner distance 1, ..., 32,
// then the four waves), and the blocks by the same tree, in order, in
// thread 0.
__global__ __launch_bounds__(256) void dense_readout_kernel(const float* J, const uint32_t* U,
                                                            int n, int np, int q, double* Hout) {
    __shared__ double red[4];
    __shared__ double stack[TreeAcc::kLevels];
    const int r = blockIdx.x;
    const uint32_t* ur = U + (size_t)r * np;
    TreeAcc tree(stack);
    for (int i0 = 0; i0 < n; i0 += 256) {
        const int i = i0 + (int)threadIdx.x;
        double part = 0.0;
        if (i < n) {
            const int ci = nearest_state(ur[i], q);
            const float* row = J + (size_t)i * n;
            for (int j = i + 1; j < n; ++j) {
                const int cj = nearest_state(ur[j], q);
                const double w = (double)row[j];
                part += (q == 2) ? (ci == cj ? w : -w) : (ci == cj ? w : 0.0);
            }
        }
        for (int o = 1; o < 64; o <<= 1) part += __shfl_xor(part, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
        __syncthreads();
        if (threadIdx.x == 0) tree.push((red[0] + red[1]) + (red[2] + red[3]));
        __syncthreads();
    }
    if (threadIdx.x == 0) Hout[r] = -tree.finish();
}

// Trace / best-so-far bookkeeping after a readout (one thread per replica).
__global__ void dense_best_kernel(const double* H, int R, int kread, int32_t gstep, double* trace,
                                  double* best_h, int32_t* best_step, double* best_tmp,
                                  int32_t* best_tmp_step, int8_t* best_colour,
                                  const uint32_t* U, int n, int np, int q, int first) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double h = H[r];
    if (trace) trace[(size_t)kread * R + r] = h;
    if (first || h < best_tmp[r]) {
        best_tmp[r] = h;
        best_tmp_step[r] = gstep;
        if (best_colour)
            for (int i = 0; i < n; ++i) best_colour[(size_t)r * n + i] = (int8_t)nearest_state(U[(size_t)r * np + i], q);
    }
    (void)best_h;
    (void)best_step;
}

using StepFn = void (*)(DenseArgs);

int alloc_or_fail(void** p, size_t bytes, const char* what) {
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) return OIM_OK;
    *p = nullptr;
    return e == hipErrorOutOfMemory ? set_error(OIM_E_NOMEM, std::string(what) + ": out of device memory")
                                    : hip_error(e, what);
}

int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? OIM_OK : hip_error(e, what);
}

}  // namespace

int dense_prepare(Problem* p, const float* J) {
    const int n = p->n;
    const int np = (n + kTM - 1) / kTM * kTM;  // also a multiple of kTK
    const size_t bytes = (size_t)n * n * sizeof(float);
    int st;
    if ((st = alloc_or_fail(reinterpret_cast<void**>(&p->d_Jdense), bytes, "dense J"))) return st;
    hipError_t e = hipMemcpy(p->d_Jdense, J, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "upload dense J");
    const size_t pb = (size_t)np * np * 2 * sizeof(uint16_t);
    if ((st = alloc_or_fail(reinterpret_cast<void**>(&p->d_Jtiled), pb, "tiled J")))
        return st;
    hipLaunchKernelGGL(dense_split_kernel, dim3(4096), dim3(256), 0, 0, p->d_Jdense, p->d_Jtiled,
                       n, np);
    if ((st = check_launch("dense_split_kernel"))) return st;
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_error(e, "dense split");
    return OIM_OK;
}

void dense_release(Problem* p) {
    hipFree(p->d_Jdense);
    hipFree(p->d_Jtiled);
    hipFree(p->d_Jtiled32);
    p->d_Jdense = nullptr;
    p->d_Jtiled = nullptr;
    p->d_Jtiled32 = nullptr;
}

namespace {

// Workspace of one run: U (4 B) + two X sets (8 B each: 4 x BF16 or 2 x FP32)
// per (replica, row) slot, then the readout scratch H[R], best tmp [R]
// (FP64) and best step [R].
size_t dense_need(int n, int R) {
    const int np = (n + kTM - 1) / kTM * kTM;
    const int Rp = (R + kTR - 1) / kTR * kTR;
    const size_t plane = (size_t)Rp * np;
    return plane * 4 + 2 * 4 * plane * 2 + (size_t)R * 8 * 2 + (size_t)R * 4 + 256;
}

int run_dense(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
              const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
              uint32_t* phase, const oim_readout* ro, hipStream_t stream, void* work) {
    const bool fp32 = (cfg->flags & OIM_PREC_MASK) == OIM_PREC_FP32;
    const int n = p->n, R = cfg->R;
    const int np = (n + kTM - 1) / kTM * kTM;
    const int Rp = (R + kTR - 1) / kTR * kTR;
    const size_t plane = (size_t)Rp * np;
    const int M = cfg->readout_every;
    unsigned char* w = static_cast<unsigned char*>(work);
    uint32_t* U = reinterpret_cast<uint32_t*>(w);
    unsigned char* X0 = w + plane * 4;
    unsigned char* X1 = X0 + 4 * plane * 2;
    double* H = reinterpret_cast<double*>(w + plane * 4 + 2 * 4 * plane * 2);
    double* btmp = H + R;
    int32_t* bstep = reinterpret_cast<int32_t*>(btmp + R);

    if (fp32)
        hipLaunchKernelGGL(dense_init32_kernel, dim3(2048), dim3(256), 0, stream, theta, phase, U,
                           X0, X1, n, R, np, Rp);
    else
        hipLaunchKernelGGL(dense_init_kernel, dim3(2048), dim3(256), 0, stream, theta, phase, U, X0,
                           X1, n, R, np, Rp);
    int st = check_launch("dense_init_kernel");
    if (st) return st;
    StepFn fn;
    if (fp32)
        fn = cfg->q == 2 ? dense_step32_kernel<2> : cfg->q == 3 ? dense_step32_kernel<3>
                                                                : dense_step32_kernel<0>;
    else
        fn = cfg->q == 2 ? dense_step_kernel<2> : cfg->q == 3 ? dense_step_kernel<3>
                                                              : dense_step_kernel<0>;
    DenseArgs a{};
    a.Jt = fp32 ? p->d_Jtiled32 : p->d_Jtiled;
    a.nk = np / kTK;
    a.U = U;
    a.seeds = seeds;
    a.np = np;
    a.Rp = Rp;
    a.n = n;
    a.R = R;
    a.q = cfg->q;
    // the step kernels read their schedule entries from device memory
    a.K = K;
    a.Ks = Ks;
    a.sigma = sigma;
    a.sched_stride = (cfg->flags & OIM_SCHED_PER_REPLICA) ? cfg->steps : 0;
    a.dt = cfg->dt;
    a.sqrt_dt = std::sqrt(cfg->dt);
    hipError_t e = hipSuccess;
    dim3 grid((np / kTM) * (Rp / kTR));
    for (int s = 0; s < cfg->steps; ++s) {
        a.Xin = (s & 1) ? X1 : X0;
        a.Xout = (s & 1) ? X0 : X1;
        a.t = (uint32_t)(step0 + s);
        a.s = s;
        hipLaunchKernelGGL(fn, grid, dim3(kTB), 0, stream, a);
        if ((st = check_launch("dense_step_kernel"))) return st;
        if (M > 0 && ((s + 1) % M == 0 || s + 1 == cfg->steps)) {
            const int kread = (s + M) / M - 1;
            hipLaunchKernelGGL(dense_readout_kernel, dim3(R), dim3(256), 0, stream, p->d_Jdense, U,
                               n, np, cfg->q, H);
            if ((st = check_launch("dense_readout_kernel"))) return st;
            hipLaunchKernelGGL(dense_best_kernel, dim3((R + 63) / 64), dim3(64), 0, stream, H, R,
                               kread, (int32_t)(step0 + s + 1), ro ? ro->trace : nullptr, nullptr,
                               nullptr, btmp, bstep, ro ? ro->best_colour : nullptr, U, n, np,
                               cfg->q, kread == 0 ? 1 : 0);
            if ((st = check_launch("dense_best_kernel"))) return st;
        }
    }

    if (ro && M > 0 && cfg->steps > 0) {
        if (ro->best_h) {
            e = hipMemcpyAsync(ro->best_h, btmp, sizeof(double) * R, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return hip_error(e, "best_h copy");
        }
        if (ro->best_step) {
            e = hipMemcpyAsync(ro->best_step, bstep, sizeof(int32_t) * R, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return hip_error(e, "best_step copy");
        }
    }
    hipLaunchKernelGGL(dense_final_kernel, dim3(2048), dim3(256), 0, stream, U, theta, phase, n, R, np);
    return check_launch("dense_final_kernel");
}

}  // namespace

size_t dense_workspace_bytes(const Problem* p, const oim_run_cfg* cfg) {
    return dense_need(p->n, cfg->R);
}

int launch_dense(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                 const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
                 uint32_t* phase, const oim_readout* ro, hipStream_t stream) {
    const bool fp32 = (cfg->flags & OIM_PREC_MASK) == OIM_PREC_FP32;
    const int n = p->n;
    const int np = (n + kTM - 1) / kTM * kTM;
    if (fp32 && !p->d_Jtiled32) {
        // the FP32 image of J, made once per problem on the caller's stream
        int st = alloc_or_fail(reinterpret_cast<void**>(&p->d_Jtiled32),
                               (size_t)np * np * sizeof(float), "FP32 tiled J");
        if (st) return st;
        hipLaunchKernelGGL(dense_tile32_kernel, dim3(4096), dim3(256), 0, stream, p->d_Jdense,
                           p->d_Jtiled32, n, np);
        if ((st = check_launch("dense_tile32_kernel"))) return st;
    }
    const size_t need = dense_workspace_bytes(p, cfg);
    if (p->work_bytes < need) {
        (void)hipFree(p->d_work);
        p->d_work = nullptr;
        p->work_bytes = 0;
        int st = alloc_or_fail(&p->d_work, need, "dense workspace");
        if (st) return st;
        p->work_bytes = need;
    }
    return run_dense(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream, p->d_work);
}

int launch_dense_ws(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                    const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
                    uint32_t* phase, const oim_readout* ro, hipStream_t stream, void* work) {
    const bool fp32 = (cfg->flags & OIM_PREC_MASK) == OIM_PREC_FP32;
    if (fp32 && !p->d_Jtiled32)
        return set_error(OIM_E_UNSUPPORTED,
                         "the FP32 image of J is made by a first oim_run with OIM_PREC_FP32");
    return run_dense(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream, work);
}

}  // namespace oim
