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
// term is ~2^-16 relative).  J's diagonal is zeroed at upload.
//
// One kernel per Euler-Maruyama step: workgroup tile = 128 rows x 64
// replicas (S and C columns of the same replicas), 4 waves of 64 rows x 32
// replicas, K in chunks of 32 staged through LDS (double buffered).  The
// epilogue owns, per lane, quads of 4 consecutive rows of one replica -- the
// MFMA accumulator layout -- so it draws one Philox call per quad, advances
// the phase words and writes the next step's split [S | C] (ping-pong).
#include <float.h>

#include <cmath>

#include "internal.hpp"
#include "noise.hpp"
#include "phase.hpp"

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

struct DenseArgs {
    const uint16_t* Jhi;   // [np][np]
    const uint16_t* Jlo;
    const uint16_t* Xin;   // [4][Rp][np]: S_hi, S_lo, C_hi, C_lo
    uint16_t* Xout;
    uint32_t* U;           // [Rp][np] phase words
    const uint64_t* seeds;
    int np, Rp, n, R, q;
    float kc, ks, ns;      // step coefficients in 2^-32-turn units (unused for init)
    const float* K;
    const float* Ks;
    const float* sigma;
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

// s_waitcnt immediate that waits until at most `n` vector-memory operations
// of this wave are outstanding (lgkm and exp counters left at their maxima).
__device__ __forceinline__ constexpr int vmcnt_imm(int n) {
    return (n & 0xf) | ((n >> 4) << 14) | (0x7 << 4) | (0xf << 8);
}

// Barrier that completes this wave's LDS reads and nothing else: the DMA
// loads of later stages stay in flight (a workgroup fence, as in
// __syncthreads, would wait for every outstanding vector-memory operation).
// The memory clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
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
    const int i0 = blockIdx.x * kTM, r0 = blockIdx.y * kTR;
    const int np = a.np, Rp = a.Rp;
    const size_t plane = (size_t)Rp * np;

    // Chunk c of a stage (16 rows x 64 bytes) sits at LDS bytes 1024c: chunks
    // 0-7 are J_hi rows, 8-15 J_lo rows, 16-31 the four X components (4 chunks
    // each).  Wave w moves chunks 8w..8w+7; lane l lands on row l/4 of the
    // chunk, slot l%4, which holds logical segment (l%4) ^ ((row>>1)&3).
    const int lrow = lane >> 2, lseg = (lane & 3) ^ ((lrow >> 1) & (kSegs - 1));
    const uint16_t* src[kWaveChunks];
#pragma unroll
    for (int x = 0; x < kWaveChunks; ++x) {
        const int c = wave * kWaveChunks + x;
        if (c < 16) {
            const int row = (c & 7) * 16 + lrow;
            src[x] = (c < 8 ? a.Jhi : a.Jlo) + (size_t)(i0 + row) * np + lseg * 8;
        } else {
            const int comp = (c - 16) >> 2, row = ((c - 16) & 3) * 16 + lrow;
            src[x] = a.Xin + comp * plane + (size_t)(r0 + row) * np + lseg * 8;
        }
    }
    auto issue = [&](int kc) __attribute__((always_inline)) {
        unsigned char* dst = lds[kc % kDepth] + wave * kWaveChunks * 1024;
#pragma unroll
        for (int x = 0; x < kWaveChunks; ++x)
            __builtin_amdgcn_global_load_lds((glb_void_t*)(src[x] + (size_t)kc * kTK),
                                             (lds_void_t*)(dst + x * 1024), 16, 0, 0);
    };

    f32x4 acc[4][2][2];  // [row block][replica block][S, C]
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[b][c][0] = acc[b][c][1] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int nk = np / kTK;  // at least kDepth (np is a multiple of 128)
    const int frow = lane & 15, fseg = lane >> 4;
#pragma unroll
    for (int d = 0; d < kDepth - 1; ++d) issue(d);
    for (int kc = 0; kc < nk; ++kc) {
        // stage kc has landed once at most (stages issued after it) x chunks
        // of this wave's DMA loads are outstanding
        const int ahead = nk - 1 - kc < kDepth - 2 ? nk - 1 - kc : kDepth - 2;
        if (ahead == kDepth - 2) __builtin_amdgcn_s_waitcnt(vmcnt_imm((kDepth - 2) * kWaveChunks));
        else if (ahead == 1) __builtin_amdgcn_s_waitcnt(vmcnt_imm(kWaveChunks));
        else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        // all waves' chunks of stage kc are in LDS, and every wave is done
        // reading the buffer that stage kc + kDepth - 1 overwrites
        lds_barrier();
        if (kc + kDepth - 1 < nk) issue(kc + kDepth - 1);
        const unsigned char* base = lds[kc % kDepth];
        bf16x8 bh[2][2], bl[2][2];  // [replica block][S, C]
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int row = wn * 32 + cb * 16 + frow;
#pragma unroll
            for (int sc = 0; sc < 2; ++sc) {
                const unsigned char* bb = base + 2 * kA + (2 * sc) * kB;
                bh[cb][sc] = *reinterpret_cast<const bf16x8*>(bb + swz(row, fseg));
                bl[cb][sc] = *reinterpret_cast<const bf16x8*>(bb + kB + swz(row, fseg));
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = wm * 64 + b * 16 + frow;
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(base + swz(row, fseg));
            const bf16x8 al = *reinterpret_cast<const bf16x8*>(base + kA + swz(row, fseg));
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
                for (int sc = 0; sc < 2; ++sc) {
                    f32x4 c = acc[b][cb][sc];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cb][sc], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cb][sc], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cb][sc], c, 0, 0, 0);
                    acc[b][cb][sc] = c;
                }
            }
        }
    }

    // ---- epilogue: SHIL, noise, Euler-Maruyama update, next split X ----
    const float kcoef = a.kc, kscoef = a.ks, nscoef = a.ns;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int r = r0 + wn * 32 + cb * 16 + (lane & 15);
        const bool rvalid = r < a.R;
        const uint64_t seed = rvalid ? a.seeds[r] : 0ull;
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + wm * 64 + b * 16 + 4 * (lane >> 4);  // first row of the quad
            if (!rvalid || i >= a.n) continue;
            uint4 u4 = *reinterpret_cast<const uint4*>(a.U + (size_t)r * np + i);
            uint32_t u[4] = {u4.x, u4.y, u4.z, u4.w};
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
            const size_t off = (size_t)r * np + i;
            *reinterpret_cast<uint2*>(a.Xout + 0 * plane + off) =
                uint2{shi[0] | ((uint32_t)shi[1] << 16), shi[2] | ((uint32_t)shi[3] << 16)};
            *reinterpret_cast<uint2*>(a.Xout + 1 * plane + off) =
                uint2{slo[0] | ((uint32_t)slo[1] << 16), slo[2] | ((uint32_t)slo[3] << 16)};
            *reinterpret_cast<uint2*>(a.Xout + 2 * plane + off) =
                uint2{chi[0] | ((uint32_t)chi[1] << 16), chi[2] | ((uint32_t)chi[3] << 16)};
            *reinterpret_cast<uint2*>(a.Xout + 3 * plane + off) =
                uint2{clo[0] | ((uint32_t)clo[1] << 16), clo[2] | ((uint32_t)clo[3] << 16)};
        }
    }
}

// Phase words and split [S | C] of the initial state, written to both
// ping-pong sets; padding rows and replicas get X = 0 in both (they add
// nothing to any coupling sum and the step kernel never writes them).
__global__ __launch_bounds__(256) void dense_init_kernel(const float* theta, const uint32_t* phase,
                                                         uint32_t* U, uint16_t* X, uint16_t* X2,
                                                         int n, int R, int np, int Rp) {
    const size_t plane = (size_t)Rp * np;
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
        X[e] = X2[e] = sh;
        X[plane + e] = X2[plane + e] = sl;
        X[2 * plane + e] = X2[2 * plane + e] = ch;
        X[3 * plane + e] = X2[3 * plane + e] = cl;
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

// J -> (J_hi, J_lo) with the diagonal and the padding zeroed.
__global__ __launch_bounds__(256) void dense_split_kernel(const float* J, uint16_t* hi, uint16_t* lo,
                                                          int n, int np) {
    const size_t total = (size_t)np * np;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / np), j = (int)(e % np);
        const float v = (i < n && j < n && i != j) ? J[(size_t)i * n + j] : 0.f;
        uint16_t h, l;
        split_bf16(v, h, l);
        hi[e] = h;
        lo[e] = l;
    }
}

// Thresholded energy per replica from the phase words (in-run readout):
// one workgroup per replica, rows strided over threads, FP64 sums in a
// fixed order.  H = Eq. 1 (q = 2) or Eq. 2 (q >= 3).
__global__ __launch_bounds__(256) void dense_readout_kernel(const float* J, const uint32_t* U,
                                                            int n, int np, int q, double* Hout) {
    __shared__ double red[4];
    const int r = blockIdx.x;
    const uint32_t* ur = U + (size_t)r * np;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ci = nearest_state(ur[i], q);
        const float* row = J + (size_t)i * n;
        double part = 0.0;
        for (int j = i + 1; j < n; ++j) {
            const int cj = nearest_state(ur[j], q);
            const double w = (double)row[j];
            part += (q == 2) ? (ci == cj ? w : -w) : (ci == cj ? w : 0.0);
        }
        acc += part;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) Hout[r] = -(red[0] + red[1] + red[2] + red[3]);
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
    const size_t pb = (size_t)np * np * sizeof(uint16_t);
    if ((st = alloc_or_fail(reinterpret_cast<void**>(&p->d_Jhi), pb, "J_hi")) ||
        (st = alloc_or_fail(reinterpret_cast<void**>(&p->d_Jlo), pb, "J_lo")))
        return st;
    hipLaunchKernelGGL(dense_split_kernel, dim3(4096), dim3(256), 0, 0, p->d_Jdense, p->d_Jhi,
                       p->d_Jlo, n, np);
    if ((st = check_launch("dense_split_kernel"))) return st;
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_error(e, "dense split");
    return OIM_OK;
}

void dense_release(Problem* p) {
    hipFree(p->d_Jdense);
    hipFree(p->d_Jhi);
    hipFree(p->d_Jlo);
    p->d_Jdense = nullptr;
    p->d_Jhi = p->d_Jlo = nullptr;
}

int launch_dense(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                 const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
                 uint32_t* phase, const oim_readout* ro, hipStream_t stream) {
    if ((cfg->flags & OIM_PREC_MASK) != OIM_PREC_BF16X3)
        return set_error(OIM_E_UNSUPPORTED, "dense problems run with OIM_PREC_BF16X3");
    const int n = p->n, R = cfg->R;
    const int np = (n + kTM - 1) / kTM * kTM;
    const int Rp = (R + kTR - 1) / kTR * kTR;
    const size_t plane = (size_t)Rp * np;
    const int M = cfg->readout_every;
    const int nread = M > 0 ? (cfg->steps + M - 1) / M : 0;
    // workspace: U (4 B) + two X sets (4 x 2 B each) per slot, then readout
    // scratch: H[R], best tmp [R] (f64), best step [R]
    const size_t need = plane * 4 + 2 * 4 * plane * 2 + (size_t)R * 8 * 2 + (size_t)R * 4 + 256;
    if (p->work_bytes < need) {
        hipFree(p->d_work);
        p->d_work = nullptr;
        p->work_bytes = 0;
        int st = alloc_or_fail(&p->d_work, need, "dense workspace");
        if (st) return st;
        p->work_bytes = need;
    }
    unsigned char* w = static_cast<unsigned char*>(p->d_work);
    uint32_t* U = reinterpret_cast<uint32_t*>(w);
    uint16_t* X0 = reinterpret_cast<uint16_t*>(w + plane * 4);
    uint16_t* X1 = X0 + 4 * plane;
    double* H = reinterpret_cast<double*>(w + plane * 4 + 2 * 4 * plane * 2);
    double* btmp = H + R;
    int32_t* bstep = reinterpret_cast<int32_t*>(btmp + R);

    hipLaunchKernelGGL(dense_init_kernel, dim3(2048), dim3(256), 0, stream, theta, phase, U, X0, X1,
                       n, R, np, Rp);
    int st = check_launch("dense_init_kernel");
    if (st) return st;
    StepFn fn = cfg->q == 2 ? dense_step_kernel<2> : cfg->q == 3 ? dense_step_kernel<3>
                                                                   : dense_step_kernel<0>;
    DenseArgs a{};
    a.Jhi = p->d_Jhi;
    a.Jlo = p->d_Jlo;
    a.U = U;
    a.seeds = seeds;
    a.np = np;
    a.Rp = Rp;
    a.n = n;
    a.R = R;
    a.q = cfg->q;
    // schedule values are read on the host side of each launch from device
    // memory only through the coefficients below; copy the schedule once.
    std::vector<float> hK(cfg->steps), hKs(cfg->steps), hS(cfg->steps);
    hipError_t e = hipMemcpyAsync(hK.data(), K, sizeof(float) * cfg->steps, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hKs.data(), Ks, sizeof(float) * cfg->steps, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hS.data(), sigma, sizeof(float) * cfg->steps, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_error(e, "copy schedules");
    const float dt = cfg->dt;
    const float sqrt_dt = std::sqrt(dt);
    const float scale = 683565275.57643158978045f;
    dim3 grid(np / kTM, Rp / kTR);
    for (int s = 0; s < cfg->steps; ++s) {
        a.Xin = (s & 1) ? X1 : X0;
        a.Xout = (s & 1) ? X0 : X1;
        a.t = (uint32_t)(step0 + s);
        a.kc = -dt * hK[s] * scale;
        a.ks = -dt * hKs[s] * scale;
        a.ns = hS[s] * sqrt_dt * scale;
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
    (void)nread;
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

}  // namespace oim
