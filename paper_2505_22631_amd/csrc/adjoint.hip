// adjoint.hip -- gradient of the relaxed cut at the last step with respect to
// the per-step schedules K_t, Ks_t and sigma_t of a fixed-noise
// Euler-Maruyama trajectory (Sec. II-E Eq. 5 integrated as in Algorithm 1;
// the schedules are the annealing knobs of Sec. II-D / Fig. 3b).
//
// Loss (sum over replicas and instances), w = -J:
//     L = sum_{i<j} w_ij (1 - cos(th_T,i - th_T,j)) / 2
// Adjoint of th_{t+1} = th_t + dt f(th_t) + sigma_t sqrt(dt) xi_t with
// f_i = -K_t sum_j J_ij sin(th_i - th_j) - Ks_t sin(q th_i), J symmetric:
//     lam_T,i  = 1/2 sum_j w_ij sin(th_i - th_j)
//     lam_t,k  = lam_{t+1,k} + dt [ K_t sum_j J_kj cos(th_k - th_j) (lam_j - lam_k)
//                                   - q Ks_t cos(q th_k) lam_k ]      (lam at t+1)
//     dL/dK_t  = -dt sum_i lam_{t+1,i} sum_j J_ij sin(th_t,i - th_t,j)
//     dL/dKs_t = -dt sum_i lam_{t+1,i} sin(q th_t,i)
//     dL/dsig_t = sqrt(dt) sum_i lam_{t+1,i} xi_t,i
// The wrap of the phase has derivative 1 almost everywhere.  With the
// identities cos(a-b) = ca cb + sa sb and sin(a-b) = sa cb - ca sb every sum
// above is a CSR gather of four per-node values (s, c, s lam, c lam).
//
// Forward kernel: one workgroup per (instance, replica), phases in registers
// (one quad of 4 consecutive oscillators per thread slot), neighbour (s, c)
// in an LDS ping-pong table; the phase words are checkpointed every C steps
// into caller memory.  Backward kernel: per segment of C steps (last first) it
// recomputes the states from the checkpoint (the Philox noise is a pure
// function of (seed, oscillator, step, instance), so the recomputation is
// exact), keeps them in device scratch, and runs the adjoint recurrence back
// through the segment.  Per-step gradient partials are reduced over each wave
// and summed over waves and workgroups in FP64 in a fixed order.
#include <float.h>

#include <cmath>

#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "internal.hpp"
#include "noise.hpp"
#include "phase.hpp"

// The forward kernel and the backward kernel's recomputation must round every
// step identically, so no multiply-add is fused unless written as fmaf.
#pragma clang fp contract(off)

namespace oim {

namespace {

constexpr int kAdjTB = 512;
constexpr int kAdjWaves = kAdjTB / 64;
constexpr int kAdjQPT = kAdjMaxN / 4 / kAdjTB;  // quads per thread at the size limit
constexpr int kCsrGlobal = 0, kCsrLdsUnit = 1, kCsrLds = 2, kEllUnit = 3;
constexpr int kEllSlices = kAdjMaxN / 4 / 64;  // slices of 64 quads at the size limit

struct AdjArgs {
    const int64_t* row_ptr;
    const int32_t* col;
    const float* J;
    int tabN;              // table length in LDS (largest instance, rounded up to 4)
    int64_t max_nnz;       // most stored entries of one instance
    int64_t max_ell;       // most padded row-image entries of one instance (kEllUnit)
    const int4* inst;      // per instance: first slice, slices, first oscillator, size
    int I, n_total, P;     // instances, oscillators, padded words per replica
    int R, q, steps, C, nseg;
    int64_t step0;
    float dt;
    const float* K;
    const float* Ks;
    const float* sigma;
    const uint64_t* seeds;
    const float* theta0;   // [R][n_total] radians
    uint32_t* ckpt;        // [nseg][R][P] phase words
    float* thetaT;         // [R][n_total] or null
    double* loss;          // [R * I] or null
    uint32_t* seg;         // [C + 1][R][P] states of one segment (backward)
    float4* gpart;         // [steps][R * I][kAdjWaves] (backward)
    float* lam;            // [R][P] adjoint state between segments (backward)
    int cur_seg;           // segment of this launch (backward)
};

template <int QM>
__device__ __forceinline__ float cos_q(float s, float c, uint32_t u, int q) {
    if constexpr (QM == 2) {
        return __builtin_fmaf(-2.0f * s, s, 1.0f);
    } else if constexpr (QM == 3) {
        return c * __builtin_fmaf(4.0f * c, c, -3.0f);
    } else {
        return cos_turn((uint32_t)q * u);
    }
}

// Per-workgroup view of its instance and replica.
struct Ctx {
    int wg, b, r, off, nb, nq, base;
    uint32_t k0, k1;
};

__device__ __forceinline__ Ctx make_ctx(const AdjArgs& a) {
    Ctx x;
    x.wg = blockIdx.x;
    x.b = x.wg % a.I;
    x.r = x.wg / a.I;
    const int4 in = a.inst[x.b];
    x.off = in.z;
    x.nb = in.w;
    x.nq = (in.w + 3) / 4;
    x.base = in.x * (4 * kSliceQuads);
    const uint64_t seed = a.seeds[x.r];
    x.k0 = (uint32_t)seed;
    x.k1 = (uint32_t)(seed >> 32);
    return x;
}

// Offset of (slot, replica, local oscillator) in a [slots][R][P] phase array.
__device__ __forceinline__ size_t slot_index(const AdjArgs& a, const Ctx& x, int slot, int i) {
    return ((size_t)slot * a.R + x.r) * a.P + x.base + i;
}

// Where a workgroup reads its instance's CSR rows.  CSR_LDS: copies in LDS
// made at kernel start (row offsets relative to the instance, 16-bit local
// column indices, and either FP32 weights or, with UNIT, the sign of a
// unit weight in the index's top bit); otherwise the global CSR through L2.
// ELL_UNIT (unit weights, forward kernel): the step loop reads a padded row
// image in LDS (gather_quad_ell); the whole-row sums of the loss use the
// global CSR.
template <int MODE>
struct Rows {
    static constexpr bool kGlobal = MODE == kCsrGlobal || MODE == kEllUnit;
    // entry positions: 64-bit in the global CSR, 32-bit in the LDS copy (no
    // 64-bit compares and adds in the gathers' loops)
    using Idx = std::conditional_t<kGlobal, int64_t, int32_t>;
    const AdjArgs* a;
    int off;
    const int32_t* rp;    // LDS row offsets [nb + 1]
    const uint16_t* col;  // LDS column indices
    const float* w;       // LDS weights (MODE == kCsrLds)
    // ELL_UNIT: the row image and, per slice of the thread's quads, the
    // padded row length and the slice's offset in the image (wave-uniform)
    const uint16_t* ell;
    int ellD[kAdjQPT], ellBase[kAdjQPT];
    __device__ __forceinline__ Idx begin(int i) const {
        if constexpr (kGlobal) return a->row_ptr[off + i];
        else return rp[i];
    }
    __device__ __forceinline__ Idx end(int i) const {
        if constexpr (kGlobal) return a->row_ptr[off + i + 1];
        else return rp[i + 1];
    }
    __device__ __forceinline__ void edge(Idx e, int& j, float& wt) const {
        if constexpr (kGlobal) {
            j = a->col[e] - off;
            wt = a->J[e];
        } else if constexpr (MODE == kCsrLdsUnit) {
            const uint32_t c = col[e];
            j = (int)(c & 0x7fffu);
            wt = (c & 0x8000u) ? -1.0f : 1.0f;
        } else {
            j = col[e];
            wt = w[e];
        }
    }
};

// Gather over the CSR row of local oscillator i from an LDS table of
// (s, c, s lam, c lam): A = sum J c_j, B = sum J s_j and, if LAM,
// Cl = sum J c_j lam_j, Dl = sum J s_j lam_j.
template <bool LAM, int MODE>
__device__ __forceinline__ void gather(const Rows<MODE>& g,
                                       const std::conditional_t<LAM, float4, float2>* tab, int i,
                                       float& A, float& B, float& Cl, float& Dl) {
    using Idx = typename Rows<MODE>::Idx;
    const Idx e0 = g.begin(i), e1 = g.end(i);
    float A0 = 0.f, B0 = 0.f, C0 = 0.f, D0 = 0.f, A1 = 0.f, B1 = 0.f, C1 = 0.f, D1 = 0.f;
    Idx e = e0;
    // eight edges at a time: eight index reads, then eight table reads, in
    // flight together; edges at even offsets from e0 go to the first partial
    // sums and odd ones to the second, in order, exactly as in the pairwise
    // loop below, so the sums do not depend on the unrolling
    for (; e + 8 <= e1; e += 8) {
        int jj[8];
        float ww[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) g.edge(e + k, jj[k], ww[k]);
        if constexpr (LAM) {
            float4 pv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) pv[k] = tab[jj[k]];
#pragma unroll
            for (int k = 0; k < 8; k += 2) {
                A0 = __builtin_fmaf(ww[k], pv[k].y, A0);
                B0 = __builtin_fmaf(ww[k], pv[k].x, B0);
                C0 = __builtin_fmaf(ww[k], pv[k].w, C0);
                D0 = __builtin_fmaf(ww[k], pv[k].z, D0);
                A1 = __builtin_fmaf(ww[k + 1], pv[k + 1].y, A1);
                B1 = __builtin_fmaf(ww[k + 1], pv[k + 1].x, B1);
                C1 = __builtin_fmaf(ww[k + 1], pv[k + 1].w, C1);
                D1 = __builtin_fmaf(ww[k + 1], pv[k + 1].z, D1);
            }
        } else {
            float2 pv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) pv[k] = tab[jj[k]];
#pragma unroll
            for (int k = 0; k < 8; k += 2) {
                A0 = __builtin_fmaf(ww[k], pv[k].y, A0);
                B0 = __builtin_fmaf(ww[k], pv[k].x, B0);
                A1 = __builtin_fmaf(ww[k + 1], pv[k + 1].y, A1);
                B1 = __builtin_fmaf(ww[k + 1], pv[k + 1].x, B1);
            }
        }
    }
    for (; e + 2 <= e1; e += 2) {
        int j0, j1;
        float w0, w1;
        g.edge(e, j0, w0);
        g.edge(e + 1, j1, w1);
        if constexpr (LAM) {
            const float4 p0 = tab[j0], p1 = tab[j1];
            A0 = __builtin_fmaf(w0, p0.y, A0);
            B0 = __builtin_fmaf(w0, p0.x, B0);
            C0 = __builtin_fmaf(w0, p0.w, C0);
            D0 = __builtin_fmaf(w0, p0.z, D0);
            A1 = __builtin_fmaf(w1, p1.y, A1);
            B1 = __builtin_fmaf(w1, p1.x, B1);
            C1 = __builtin_fmaf(w1, p1.w, C1);
            D1 = __builtin_fmaf(w1, p1.z, D1);
        } else {
            const float2 p0 = tab[j0];
            const float2 p1 = tab[j1];
            A0 = __builtin_fmaf(w0, p0.y, A0);
            B0 = __builtin_fmaf(w0, p0.x, B0);
            A1 = __builtin_fmaf(w1, p1.y, A1);
            B1 = __builtin_fmaf(w1, p1.x, B1);
        }
    }
    if (e < e1) {
        int j0;
        float w0;
        g.edge(e, j0, w0);
        if constexpr (LAM) {
            const float4 p0 = tab[j0];
            A0 = __builtin_fmaf(w0, p0.y, A0);
            B0 = __builtin_fmaf(w0, p0.x, B0);
            C0 = __builtin_fmaf(w0, p0.w, C0);
            D0 = __builtin_fmaf(w0, p0.z, D0);
        } else {
            const float2 p0 = tab[j0];
            A0 = __builtin_fmaf(w0, p0.y, A0);
            B0 = __builtin_fmaf(w0, p0.x, B0);
        }
    }
    A = A0 + A1;
    B = B0 + B1;
    Cl = C0 + C1;
    Dl = D0 + D1;
}

// Forward sums (A, B of gather) for the four rows of quad k of the thread from
// the ELL row image: the slice's rows are padded to one length D (a multiple
// of 4; pads point at the tables' zero entry), entry e of row j of the lane's
// quad at u16 offset base + ((j D/4 + e/4) 64 + lane) 4 + e % 4, so each
// 8-byte read brings four consecutive entries of one row and the loop length
// is the same for the whole wave.  Per row the partial sums take the even and
// the odd entries in order, exactly as gather does, and a pad adds +-0 to a
// partial sum that is never -0: the results are the same bits.
__device__ __forceinline__ void gather_quad_ell(const Rows<kEllUnit>& g, const float2* tab, int k,
                                                int lane, float (&A)[4], float (&B)[4]) {
    const int D4 = g.ellD[k] >> 2;
    const uint2* img = reinterpret_cast<const uint2*>(g.ell + g.ellBase[k]) + lane;
    float a0[4], b0[4], a1[4], b1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) a0[j] = b0[j] = a1[j] = b1[j] = 0.f;
    for (int gi = 0; gi < D4; ++gi) {
        uint2 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = img[(j * D4 + gi) * 64];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t word = t < 2 ? v[j].x : v[j].y;
                const uint32_t c = (t & 1) ? word >> 16 : word & 0xffffu;
                const float wt = (c & 0x8000u) ? -1.0f : 1.0f;
                const float2 p = tab[c & 0x7fffu];
                if (t & 1) {
                    a1[j] = __builtin_fmaf(wt, p.y, a1[j]);
                    b1[j] = __builtin_fmaf(wt, p.x, b1[j]);
                } else {
                    a0[j] = __builtin_fmaf(wt, p.y, a0[j]);
                    b0[j] = __builtin_fmaf(wt, p.x, b0[j]);
                }
            }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        A[j] = a0[j] + a1[j];
        B[j] = b0[j] + b1[j];
    }
}

// Writes (s, c) of the thread's oscillators into a table.
__device__ __forceinline__ void put_sc(const Ctx& x, float2* tab, const uint32_t (&u)[kAdjQPT][4]) {
#pragma unroll
    for (int k = 0; k < kAdjQPT; ++k) {
        const int m = threadIdx.x + k * kAdjTB;
        if (m >= x.nq) break;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            tab[4 * m + j] = make_float2(sin_turn(u[k][j]), cos_turn(u[k][j]));
    }
}

// One synchronous Euler-Maruyama step of the thread's oscillators reading
// neighbour (s, c) from tin and writing the new (s, c) into tout.
template <int QM, int MODE>
__device__ __forceinline__ void fwd_step(const AdjArgs& a, const Ctx& x, const Rows<MODE>& g, int s,
                                         const float2* tin, float2* tout,
                                         uint32_t (&u)[kAdjQPT][4]) {
    const int q = QM ? QM : a.q;
    const uint32_t t = (uint32_t)(a.step0 + s);
    const float kc = -a.dt * a.K[s] * kTurnScale;
    const float ks = -a.dt * a.Ks[s] * kTurnScale;
    const float ns = a.sigma[s] * __builtin_sqrtf(a.dt) * kTurnScale;
#pragma unroll
    for (int k = 0; k < kAdjQPT; ++k) {
        const int m = threadIdx.x + k * kAdjTB;
        if (m >= x.nq) break;
        float z[4];
        normals4((uint32_t)m, t, (uint32_t)x.b, x.k0, x.k1, z);
        float Aq[4], Bq[4];
        if constexpr (MODE == kEllUnit) gather_quad_ell(g, tin, k, threadIdx.x & 63, Aq, Bq);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * m + j;
            if (i >= x.nb) break;
            float A, B, Cl, Dl;
            if constexpr (MODE == kEllUnit) {
                A = Aq[j];
                B = Bq[j];
            } else {
                gather<false>(g, tin, i, A, B, Cl, Dl);
            }
            const float si = sin_turn(u[k][j]), ci = cos_turn(u[k][j]);
            const float coup = __builtin_fmaf(si, A, -(ci * B));
            const float drift = __builtin_fmaf(kc, coup, ks * sin_q<QM>(si, ci, u[k][j], q));
            u[k][j] = advance(u[k][j], __builtin_fmaf(ns, z[j], drift));
        }
    }
    put_sc(x, tout, u);
}

__device__ __forceinline__ void load_words(const AdjArgs& a, const Ctx& x, const uint32_t* src,
                                           int slot, uint32_t (&u)[kAdjQPT][4]) {
#pragma unroll
    for (int k = 0; k < kAdjQPT; ++k) {
        const int m = threadIdx.x + k * kAdjTB;
        if (m >= x.nq) break;
        const uint4 v = *reinterpret_cast<const uint4*>(src + slot_index(a, x, slot, 4 * m));
        u[k][0] = v.x;
        u[k][1] = v.y;
        u[k][2] = v.z;
        u[k][3] = v.w;
    }
}

__device__ __forceinline__ void store_words(const AdjArgs& a, const Ctx& x, uint32_t* dst, int slot,
                                            const uint32_t (&u)[kAdjQPT][4]) {
#pragma unroll
    for (int k = 0; k < kAdjQPT; ++k) {
        const int m = threadIdx.x + k * kAdjTB;
        if (m >= x.nq) break;
        *reinterpret_cast<uint4*>(dst + slot_index(a, x, slot, 4 * m)) =
            uint4{u[k][0], u[k][1], u[k][2], u[k][3]};
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The same two tables as (s, c) alone, 8 bytes per oscillator from the start
// of each table's space: the forward steps read only (s, c), and at an
// 8-byte stride a gather's random reads spread over all LDS banks (at the
// 16-byte stride of the full entries, over half of them).  Entry tabN of
// each stays zero (padding of the row image points there); the full entries
// it overlaps are written before the backward reads them.
__device__ __forceinline__ float2* tab2_of(unsigned char* smem, int tabN, int k) {
    return reinterpret_cast<float2*>(smem) + (size_t)k * 2 * (tabN + 1);
}

// Dynamic LDS: two tables of tabN + 1 float4 (entry tabN of each stays zero),
// then (CSR in LDS) the instance's row offsets, 16-bit column indices and FP32
// weights, or (ELL_UNIT) per-slice lengths and the padded row image.  Fills
// the row copy; the caller's first barrier publishes it.
template <int MODE>
__device__ __forceinline__ Rows<MODE> setup_rows(const AdjArgs& a, const Ctx& x, unsigned char* smem) {
    Rows<MODE> g;
    g.a = &a;
    g.off = x.off;
    float4* tabs = reinterpret_cast<float4*>(smem);
    if (threadIdx.x < 2) {
        tabs[(size_t)threadIdx.x * (a.tabN + 1) + a.tabN] = make_float4(0.f, 0.f, 0.f, 0.f);
        tab2_of(smem, a.tabN, threadIdx.x)[a.tabN] = make_float2(0.f, 0.f);
    }
    unsigned char* p = smem + (size_t)32 * (a.tabN + 1);
    if constexpr (MODE == kEllUnit) {
        // slice s holds quads 64 s .. 64 s + 63, i.e. the quads of wave
        // s % 8 for k = s / 8 (thread t owns quad t + k kAdjTB)
        int* lenD = reinterpret_cast<int*>(p);
        g.ell = reinterpret_cast<const uint16_t*>(p + 16 * kEllSlices);
        uint16_t* img = reinterpret_cast<uint16_t*>(p + 16 * kEllSlices);
        const int lane = threadIdx.x & 63;
        int deg[kAdjQPT][4];
        int64_t rb[kAdjQPT][4];
#pragma unroll
        for (int k = 0; k < kAdjQPT; ++k) {
            const int m = threadIdx.x + k * kAdjTB;
            int dmax = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * m + j;
                rb[k][j] = i < x.nb ? a.row_ptr[x.off + i] : 0;
                deg[k][j] = i < x.nb ? (int)(a.row_ptr[x.off + i + 1] - rb[k][j]) : 0;
                dmax = deg[k][j] > dmax ? deg[k][j] : dmax;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const int other = __shfl_xor(dmax, o, 64);
                dmax = other > dmax ? other : dmax;
            }
            const int s = m >> 6;
            if (lane == 0 && s < kEllSlices) lenD[s] = (dmax + 3) & ~3;
        }
        __syncthreads();
        const int nsl = (x.nq + 63) >> 6;
#pragma unroll
        for (int k = 0; k < kAdjQPT; ++k) {
            const int s = (int)((threadIdx.x + k * kAdjTB) >> 6);
            int base = 0;
            for (int s2 = 0; s2 < s && s2 < nsl; ++s2) base += 256 * lenD[s2];
            const int D = s < nsl ? lenD[s] : 0;
            g.ellD[k] = __builtin_amdgcn_readfirstlane(D);
            g.ellBase[k] = __builtin_amdgcn_readfirstlane(base);
            const int m = threadIdx.x + k * kAdjTB;
            if (m >= x.nq) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                for (int e = 0; e < D; ++e) {
                    uint16_t v = (uint16_t)a.tabN;  // pad: the zero entry
                    if (e < deg[k][j]) {
                        const int64_t ge = rb[k][j] + e;
                        const uint32_t c = (uint32_t)(a.col[ge] - x.off);
                        v = (uint16_t)(c | (a.J[ge] < 0.0f ? 0x8000u : 0u));
                    }
                    img[base + ((j * (D >> 2) + (e >> 2)) * 64 + lane) * 4 + (e & 3)] = v;
                }
        }
        return g;
    }
    g.rp = reinterpret_cast<const int32_t*>(p);
    int32_t* rp = reinterpret_cast<int32_t*>(p);
    p += ((size_t)4 * (a.tabN + 1) + 15) & ~(size_t)15;
    uint16_t* col = reinterpret_cast<uint16_t*>(p);
    g.col = col;
    p += ((size_t)2 * a.max_nnz + 15) & ~(size_t)15;
    float* w = reinterpret_cast<float*>(p);
    g.w = w;
    if constexpr (MODE != kCsrGlobal) {
        const int64_t e0 = a.row_ptr[x.off];
        const int64_t ne = a.row_ptr[x.off + x.nb] - e0;
        for (int i = threadIdx.x; i <= x.nb; i += kAdjTB)
            rp[i] = (int32_t)(a.row_ptr[x.off + i] - e0);
        for (int64_t e = threadIdx.x; e < ne; e += kAdjTB) {
            const uint32_t c = (uint32_t)(a.col[e0 + e] - x.off);
            const float wt = a.J[e0 + e];
            if constexpr (MODE == kCsrLdsUnit) {
                col[e] = (uint16_t)(c | (wt < 0.0f ? 0x8000u : 0u));
            } else {
                col[e] = (uint16_t)c;
                w[e] = wt;
            }
        }
    }
    return g;
}

template <int QM, int MODE>
__global__ __launch_bounds__(kAdjTB) void adjoint_forward_kernel(AdjArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kAdjWaves];
    const Ctx x = make_ctx(a);
    const Rows<MODE> g = setup_rows<MODE>(a, x, smem);
    auto tab = [&](int k) { return tab2_of(smem, a.tabN, k); };
    uint32_t u[kAdjQPT][4];
#pragma unroll
    for (int k = 0; k < kAdjQPT; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * (threadIdx.x + k * kAdjTB) + j;
            u[k][j] = i < x.nb ? phase_from_theta(a.theta0[(size_t)x.r * a.n_total + x.off + i]) : 0u;
        }
    put_sc(x, tab(0), u);
    __syncthreads();
    for (int s = 0; s < a.steps; ++s) {
        if (s % a.C == 0) store_words(a, x, a.ckpt, s / a.C, u);
        fwd_step<QM>(a, x, g, s, tab(s & 1), tab((s + 1) & 1), u);
        __syncthreads();
    }
    // relaxed cut of the final phases: sum_i (c_i A_i + s_i B_i - sum_j J_ij) / 4
    const float2* fin = tab(a.steps & 1);
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < kAdjQPT; ++k) {
        const int m = threadIdx.x + k * kAdjTB;
        if (m >= x.nq) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * m + j;
            if (i >= x.nb) break;
            float A, B, Cl, Dl;
            gather<false>(g, fin, i, A, B, Cl, Dl);
            double rs = 0.0;
            for (int64_t e = g.begin(i); e < g.end(i); ++e) {
                int j;
                float wt;
                g.edge(e, j, wt);
                rs += (double)wt;
            }
            const float si = sin_turn(u[k][j]), ci = cos_turn(u[k][j]);
            part += 0.25 * ((double)ci * A + (double)si * B - rs);
            if (a.thetaT) a.thetaT[(size_t)x.r * a.n_total + x.off + i] = theta_from_phase(u[k][j]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0 && a.loss) {
        double tot = 0.0;
        for (int w = 0; w < kAdjWaves; ++w) tot += red[w];
        a.loss[x.wg] = tot;
    }
}

// Backward pass, segment a.cur_seg (steps t0 .. t1 - 1), in two kernels that
// run on two streams so that the recomputation of one segment overlaps the
// adjoint of the next (later) one, each kernel on its own half of the CUs.
//
// Recompute: the segment's states from its checkpoint, written to a.seg
// (slot s - t0 holds the state at step s; the last segment also computes its
// final step and stores the state at t1 in slot t1 - t0).  The Philox noise is
// a pure function of (seed, oscillator, step, instance) and every placement
// of the rows gives the same bits, so these are the forward pass's states.
template <int QM, int MODE>
__global__ __launch_bounds__(kAdjTB) void adjoint_recompute_kernel(AdjArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Ctx x = make_ctx(a);
    const Rows<MODE> g = setup_rows<MODE>(a, x, smem);
    auto tab = [&](int k) { return tab2_of(smem, a.tabN, k); };
    const int sg = a.cur_seg;
    const int t0 = sg * a.C;
    const int t1 = t0 + a.C < a.steps ? t0 + a.C : a.steps;
    const bool last = sg == a.nseg - 1;
    uint32_t u[kAdjQPT][4];
    load_words(a, x, a.ckpt, sg, u);
    put_sc(x, tab(0), u);
    __syncthreads();
    int p = 0;
    for (int s = t0; s < t1; ++s) {
        store_words(a, x, a.seg, s - t0, u);
        if (s + 1 < t1 || last) {
            fwd_step<QM>(a, x, g, s, tab(p), tab(p ^ 1), u);
            p ^= 1;
            __syncthreads();
        }
    }
    if (last) store_words(a, x, a.seg, t1 - t0, u);
}

// Adjoint: the recurrence back through the segment's stored states, from the
// adjoint state left by the later segment in a.lam (or, for the last
// segment, lam_T from the final phases); the adjoint state at t0 goes back
// to a.lam.  Per-step gradient partials per wave go to a.gpart.
template <int QM, int MODE>
__global__ __launch_bounds__(kAdjTB) void adjoint_segment_kernel(AdjArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Ctx x = make_ctx(a);
    const Rows<MODE> g = setup_rows<MODE>(a, x, smem);
    float4* const tabs = reinterpret_cast<float4*>(smem);
    auto tab = [&](int k) { return tabs + (size_t)k * (a.tabN + 1); };
    const int q = QM ? QM : a.q;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwg = a.R * a.I;
    const float sqrt_dt = __builtin_sqrtf(a.dt);
    const int sg = a.cur_seg;
    const int t0 = sg * a.C;
    const int t1 = t0 + a.C < a.steps ? t0 + a.C : a.steps;
    uint32_t u[kAdjQPT][4];
    float lam[kAdjQPT][4];
    int p = 0;  // table written next
    if (sg == a.nseg - 1) {
        // lam_T from the final phases
        load_words(a, x, a.seg, t1 - t0, u);
        put_sc(x, tab2_of(smem, a.tabN, p), u);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kAdjQPT; ++k) {
            const int m = threadIdx.x + k * kAdjTB;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * m + j;
                lam[k][j] = 0.f;
                if (m >= x.nq || i >= x.nb) continue;
                float A, B, Cl, Dl;
                gather<false>(g, tab2_of(smem, a.tabN, p), i, A, B, Cl, Dl);
                const float si = sin_turn(u[k][j]), ci = cos_turn(u[k][j]);
                lam[k][j] = -0.5f * (si * A - ci * B);
            }
        }
        p ^= 1;
    } else {
#pragma unroll
        for (int k = 0; k < kAdjQPT; ++k) {
            const int m = threadIdx.x + k * kAdjTB;
#pragma unroll
            for (int j = 0; j < 4; ++j) lam[k][j] = 0.f;
            if (m >= x.nq) continue;
            const float4 v = *reinterpret_cast<const float4*>(a.lam + slot_index(a, x, 0, 4 * m));
            lam[k][0] = v.x;
            lam[k][1] = v.y;
            lam[k][2] = v.z;
            lam[k][3] = v.w;
        }
    }
    for (int s = t1 - 1; s >= t0; --s) {
        load_words(a, x, a.seg, s - t0, u);
        const uint32_t t = (uint32_t)(a.step0 + s);
#pragma unroll
        for (int k = 0; k < kAdjQPT; ++k) {
            const int m = threadIdx.x + k * kAdjTB;
            if (m >= x.nq) break;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float si = sin_turn(u[k][j]), ci = cos_turn(u[k][j]);
                tab(p)[4 * m + j] = make_float4(si, ci, si * lam[k][j], ci * lam[k][j]);
            }
        }
        __syncthreads();
        const float Kt = a.K[s], Kst = a.Ks[s];
        float gk = 0.f, gks = 0.f, gs = 0.f;
#pragma unroll
        for (int k = 0; k < kAdjQPT; ++k) {
            const int m = threadIdx.x + k * kAdjTB;
            if (m >= x.nq) break;
            float z[4];
            normals4((uint32_t)m, t, (uint32_t)x.b, x.k0, x.k1, z);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * m + j;
                if (i >= x.nb) break;
                float A, B, Cl, Dl;
                gather<true>(g, tab(p), i, A, B, Cl, Dl);
                const float si = sin_turn(u[k][j]), ci = cos_turn(u[k][j]);
                const float l = lam[k][j];
                const float csin = si * A - ci * B;
                const float ccos = ci * Cl + si * Dl - l * (ci * A + si * B);
                gk = __builtin_fmaf(l, csin, gk);
                gks = __builtin_fmaf(l, sin_q<QM>(si, ci, u[k][j], q), gks);
                gs = __builtin_fmaf(l, z[j], gs);
                lam[k][j] = l + a.dt * (Kt * ccos - (float)q * Kst * cos_q<QM>(si, ci, u[k][j], q) * l);
            }
        }
        gk = wave_sum(gk);
        gks = wave_sum(gks);
        gs = wave_sum(gs);
        if (lane == 0)
            a.gpart[((size_t)s * nwg + x.wg) * kAdjWaves + wave] =
                make_float4(-a.dt * gk, -a.dt * gks, sqrt_dt * gs, 0.f);
        p ^= 1;
    }
#pragma unroll
    for (int k = 0; k < kAdjQPT; ++k) {
        const int m = threadIdx.x + k * kAdjTB;
        if (m >= x.nq) break;
        *reinterpret_cast<float4*>(a.lam + slot_index(a, x, 0, 4 * m)) =
            make_float4(lam[k][0], lam[k][1], lam[k][2], lam[k][3]);
    }
}

// gK[s] etc. = sum over workgroups and waves of the partials, FP64, fixed order.
__global__ __launch_bounds__(256) void adjoint_reduce_kernel(const float4* gpart, int steps, int nparts,
                                                             double* gK, double* gKs, double* gS) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= steps) return;
    const float4* p = gpart + (size_t)s * nparts;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = 0; k < nparts; ++k) {
        const float4 v = p[k];
        a += (double)v.x;
        b += (double)v.y;
        c += (double)v.z;
    }
    gK[s] = a;
    gKs[s] = b;
    gS[s] = c;
}

using AdjFn = void (*)(AdjArgs);

// LDS bytes of the two tables, and of the CSR copy in each mode.
size_t tab_bytes(int tabN) { return (size_t)32 * (tabN + 1); }
size_t ell_bytes(int64_t entries) { return 16 * kEllSlices + (((size_t)2 * entries + 15) & ~(size_t)15); }
size_t csr_bytes(int tabN, int64_t nnz, bool weights) {
    size_t b = ((size_t)4 * (tabN + 1) + 15) & ~(size_t)15;
    b += ((size_t)2 * nnz + 15) & ~(size_t)15;
    if (weights) b += (size_t)4 * nnz;
    return b;
}
constexpr size_t kAdjLdsLimit = 160 * 1024 - 256;  // dynamic LDS next to the static reduction slots

// Row placement for a problem: the padded row image in LDS for unit weights
// when it fits (forward kernel only), else the CSR in LDS (unit weights need
// no weight array), else the global CSR.  The backward kernel keeps the CSR:
// its adjoint gathers read 16-byte table entries, and the padded slots cost
// more there than the shorter dependency chains save (measured).
// OIM_ADJ_ROWS=csr or =global skips the earlier choices (a switch for
// comparing the placements; all give the same bits).
int csr_mode(const Problem* p, int tabN, size_t* lds, bool allow_ell) {
    const size_t t = tab_bytes(tabN);
    const bool small_idx = p->max_inst_n <= 0x7fff;
    const char* env = getenv("OIM_ADJ_ROWS");
    const int skip = env && !strcmp(env, "global") ? 2 : env && !strcmp(env, "csr") ? 1 : 0;
    if (skip >= 2) {
        *lds = t;
        return kCsrGlobal;
    }
    if (skip < 1 && allow_ell && small_idx && p->unit_weights && p->max_inst_ell > 0 &&
        t + ell_bytes(p->max_inst_ell) <= kAdjLdsLimit) {
        *lds = t + ell_bytes(p->max_inst_ell);
        return kEllUnit;
    }
    if (small_idx && p->unit_weights && t + csr_bytes(tabN, p->max_inst_nnz, false) <= kAdjLdsLimit) {
        *lds = t + csr_bytes(tabN, p->max_inst_nnz, false);
        return kCsrLdsUnit;
    }
    if (small_idx && t + csr_bytes(tabN, p->max_inst_nnz, true) <= kAdjLdsLimit) {
        *lds = t + csr_bytes(tabN, p->max_inst_nnz, true);
        return kCsrLds;
    }
    *lds = t;
    return kCsrGlobal;
}

AdjFn forward_fn(int q, int mode) {
    const int qc = q == 2 ? 1 : q == 3 ? 2 : 0;
    static const AdjFn f[3][4] = {
        {adjoint_forward_kernel<0, 0>, adjoint_forward_kernel<0, 1>, adjoint_forward_kernel<0, 2>,
         adjoint_forward_kernel<0, 3>},
        {adjoint_forward_kernel<2, 0>, adjoint_forward_kernel<2, 1>, adjoint_forward_kernel<2, 2>,
         adjoint_forward_kernel<2, 3>},
        {adjoint_forward_kernel<3, 0>, adjoint_forward_kernel<3, 1>, adjoint_forward_kernel<3, 2>,
         adjoint_forward_kernel<3, 3>}};
    return f[qc][mode];
}

AdjFn recompute_fn(int q, int mode) {
    const int qc = q == 2 ? 1 : q == 3 ? 2 : 0;
    static const AdjFn f[3][4] = {
        {adjoint_recompute_kernel<0, 0>, adjoint_recompute_kernel<0, 1>,
         adjoint_recompute_kernel<0, 2>, adjoint_recompute_kernel<0, 3>},
        {adjoint_recompute_kernel<2, 0>, adjoint_recompute_kernel<2, 1>,
         adjoint_recompute_kernel<2, 2>, adjoint_recompute_kernel<2, 3>},
        {adjoint_recompute_kernel<3, 0>, adjoint_recompute_kernel<3, 1>,
         adjoint_recompute_kernel<3, 2>, adjoint_recompute_kernel<3, 3>}};
    return f[qc][mode];
}

AdjFn segment_fn(int q, int mode) {
    const int qc = q == 2 ? 1 : q == 3 ? 2 : 0;
    static const AdjFn f[3][3] = {
        {adjoint_segment_kernel<0, 0>, adjoint_segment_kernel<0, 1>, adjoint_segment_kernel<0, 2>},
        {adjoint_segment_kernel<2, 0>, adjoint_segment_kernel<2, 1>, adjoint_segment_kernel<2, 2>},
        {adjoint_segment_kernel<3, 0>, adjoint_segment_kernel<3, 1>, adjoint_segment_kernel<3, 2>}};
    return f[qc][mode];
}

int launch_adj(AdjFn fn, size_t lds, int grid, hipStream_t stream, const AdjArgs& a,
               const char* what) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_error(e, what);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kAdjTB), lds, stream, a);
    e = hipGetLastError();
    return e == hipSuccess ? OIM_OK : hip_error(e, what);
}

int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? OIM_OK : hip_error(e, what);
}

AdjArgs base_args(const Problem* p, const oim_adjoint_cfg* cfg, const float* K, const float* Ks,
                  const float* sigma, const uint64_t* seeds, int64_t step0) {
    AdjArgs a{};
    a.row_ptr = p->d_row_ptr;
    a.col = p->d_col;
    a.J = p->d_J;
    a.inst = p->d_inst;
    a.I = p->n_inst;
    a.n_total = p->n;
    a.P = p->sell_slices * 4 * kSliceQuads;
    a.R = cfg->R;
    a.q = cfg->q;
    a.steps = cfg->steps;
    a.C = cfg->checkpoint_every;
    a.nseg = (cfg->steps + cfg->checkpoint_every - 1) / cfg->checkpoint_every;
    a.step0 = step0;
    a.dt = cfg->dt;
    a.tabN = (p->max_inst_n + 3) & ~3;
    a.max_nnz = p->max_inst_nnz;
    a.max_ell = p->max_inst_ell;
    a.K = K;
    a.Ks = Ks;
    a.sigma = sigma;
    a.seeds = seeds;
    return a;
}

}  // namespace

int64_t adjoint_checkpoint_words(const Problem* p, const oim_adjoint_cfg* cfg) {
    const int64_t nseg = (cfg->steps + cfg->checkpoint_every - 1) / cfg->checkpoint_every;
    return nseg * cfg->R * (int64_t)p->sell_slices * 4 * kSliceQuads;
}

int launch_adjoint_forward(Problem* p, const oim_adjoint_cfg* cfg, const float* K, const float* Ks,
                           const float* sigma, const uint64_t* seeds, int64_t step0,
                           const float* theta0, uint32_t* ckpt, float* thetaT, double* loss,
                           hipStream_t stream) {
    AdjArgs a = base_args(p, cfg, K, Ks, sigma, seeds, step0);
    a.theta0 = theta0;
    a.ckpt = ckpt;
    a.thetaT = thetaT;
    a.loss = loss;
    size_t lds = 0;
    const int mode = csr_mode(p, a.tabN, &lds, true);
    return launch_adj(forward_fn(cfg->q, mode), lds, cfg->R * p->n_inst, stream, a,
                      "adjoint_forward_kernel");
}

namespace {

// The second stream and the events of the overlapped backward pass, made on
// a problem's first backward call (default priority, non-blocking).
int adjoint_streams(Problem* p) {
    if (p->adj_stream) return OIM_OK;
    hipError_t e = hipStreamCreateWithFlags(&p->adj_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        p->adj_stream = nullptr;
        return hip_error(e, "adjoint stream");
    }
    for (int k = 0; k < kAdjEvents; ++k) {
        e = hipEventCreateWithFlags(&p->adj_ev[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            p->adj_ev[k] = nullptr;
            return hip_error(e, "adjoint events");
        }
    }
    return OIM_OK;
}

}  // namespace

void adjoint_release(Problem* p) {
    if (p->adj_stream) {
        (void)hipStreamSynchronize(p->adj_stream);
        (void)hipStreamDestroy(p->adj_stream);
        p->adj_stream = nullptr;
    }
    for (int k = 0; k < kAdjEvents; ++k) {
        if (p->adj_ev[k]) (void)hipEventDestroy(p->adj_ev[k]);
        p->adj_ev[k] = nullptr;
    }
}

// Segments last first; segment sg's states live in buffer sg % 2.  The
// recomputation runs on the problem's second stream, the adjoint on the
// caller's: adjoint(sg) waits for recompute(sg), recompute(sg - 2) waits for
// adjoint(sg) (the buffer it overwrites), so recompute(sg - 1) overlaps
// adjoint(sg).  The caller's stream ends after every kernel of the pass.
int launch_adjoint_backward(Problem* p, const oim_adjoint_cfg* cfg, const float* K, const float* Ks,
                            const float* sigma, const uint64_t* seeds, int64_t step0,
                            const uint32_t* ckpt, double* gK, double* gKs, double* gS,
                            hipStream_t stream) {
    AdjArgs a = base_args(p, cfg, K, Ks, sigma, seeds, step0);
    if (cfg->steps == 0) return OIM_OK;
    const int nwg = cfg->R * p->n_inst;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t seg_bytes = up((size_t)(cfg->checkpoint_every + 1) * cfg->R * a.P * sizeof(uint32_t));
    const size_t lam_bytes = up((size_t)cfg->R * a.P * sizeof(float));
    const size_t part_bytes = (size_t)cfg->steps * nwg * kAdjWaves * sizeof(float4);
    const size_t need = 2 * seg_bytes + lam_bytes + part_bytes + 256;
    if (p->adj_bytes < need) {
        (void)hipFree(p->d_adj);
        p->d_adj = nullptr;
        p->adj_bytes = 0;
        const hipError_t e = hipMalloc(&p->d_adj, need);
        if (e != hipSuccess) {
            p->d_adj = nullptr;
            return e == hipErrorOutOfMemory
                       ? set_error(OIM_E_NOMEM, "adjoint workspace: out of device memory")
                       : hip_error(e, "adjoint workspace");
        }
        p->adj_bytes = need;
    }
    int st = adjoint_streams(p);
    if (st) return st;
    unsigned char* w = static_cast<unsigned char*>(p->d_adj);
    uint32_t* segbuf[2] = {reinterpret_cast<uint32_t*>(w), reinterpret_cast<uint32_t*>(w + seg_bytes)};
    a.ckpt = const_cast<uint32_t*>(ckpt);
    a.lam = reinterpret_cast<float*>(w + 2 * seg_bytes);
    a.gpart = reinterpret_cast<float4*>(w + 2 * seg_bytes + lam_bytes);
    size_t lds_rec = 0, lds_adj = 0;
    const AdjFn frec = recompute_fn(cfg->q, csr_mode(p, a.tabN, &lds_rec, true));
    const AdjFn fadj = segment_fn(cfg->q, csr_mode(p, a.tabN, &lds_adj, false));
    hipStream_t side = p->adj_stream;
    hipEvent_t* start = &p->adj_ev[0];
    hipEvent_t* rec = &p->adj_ev[1];   // [2]
    hipEvent_t* adj = &p->adj_ev[3];   // [2]
    hipError_t e = hipEventRecord(*start, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, *start, 0);
    if (e != hipSuccess) return hip_error(e, "adjoint stream fork");
    for (int sg = a.nseg - 1; sg >= 0 && !st; --sg) {
        const int buf = sg & 1;
        a.cur_seg = sg;
        a.seg = segbuf[buf];
        if (sg + 2 <= a.nseg - 1 && (e = hipStreamWaitEvent(side, adj[buf], 0)) != hipSuccess)
            return hip_error(e, "adjoint buffer wait");
        if ((st = launch_adj(frec, lds_rec, nwg, side, a, "adjoint_recompute_kernel"))) break;
        if ((e = hipEventRecord(rec[buf], side)) != hipSuccess ||
            (e = hipStreamWaitEvent(stream, rec[buf], 0)) != hipSuccess)
            return hip_error(e, "adjoint segment order");
        if ((st = launch_adj(fadj, lds_adj, nwg, stream, a, "adjoint_segment_kernel"))) break;
        if ((e = hipEventRecord(adj[buf], stream)) != hipSuccess)
            return hip_error(e, "adjoint segment order");
    }
    if (st) return st;
    hipLaunchKernelGGL(adjoint_reduce_kernel, dim3((cfg->steps + 255) / 256), dim3(256), 0, stream,
                       a.gpart, cfg->steps, nwg * kAdjWaves, gK, gKs, gS);
    return check_launch("adjoint_reduce_kernel");
}

}  // namespace oim
