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
constexpr int kCsrGlobal = 0, kCsrLdsUnit = 1, kCsrLds = 2;

struct AdjArgs {
    const int64_t* row_ptr;
    const int32_t* col;
    const float* J;
    int tabN;              // table length in LDS (largest instance, rounded up to 4)
    int64_t max_nnz;       // most stored entries of one instance
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
    uint32_t* seg;         // [C][R][P] scratch (backward)
    float4* gpart;         // [steps][R * I][kAdjWaves] (backward)
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
template <int MODE>
struct Rows {
    const AdjArgs* a;
    int off;
    const int32_t* rp;    // LDS row offsets [nb + 1]
    const uint16_t* col;  // LDS column indices
    const float* w;       // LDS weights (MODE == kCsrLds)
    __device__ __forceinline__ int64_t begin(int i) const {
        return MODE == kCsrGlobal ? a->row_ptr[off + i] : (int64_t)rp[i];
    }
    __device__ __forceinline__ int64_t end(int i) const {
        return MODE == kCsrGlobal ? a->row_ptr[off + i + 1] : (int64_t)rp[i + 1];
    }
    __device__ __forceinline__ void edge(int64_t e, int& j, float& wt) const {
        if constexpr (MODE == kCsrGlobal) {
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
__device__ __forceinline__ void gather(const Rows<MODE>& g, const float4* tab, int i,
                                       float& A, float& B, float& Cl, float& Dl) {
    const int64_t e0 = g.begin(i), e1 = g.end(i);
    float A0 = 0.f, B0 = 0.f, C0 = 0.f, D0 = 0.f, A1 = 0.f, B1 = 0.f, C1 = 0.f, D1 = 0.f;
    int64_t e = e0;
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
            for (int k = 0; k < 8; ++k) pv[k] = *reinterpret_cast<const float2*>(tab + jj[k]);
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
            const float2 p0 = *reinterpret_cast<const float2*>(tab + j0);
            const float2 p1 = *reinterpret_cast<const float2*>(tab + j1);
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
            const float2 p0 = *reinterpret_cast<const float2*>(tab + j0);
            A0 = __builtin_fmaf(w0, p0.y, A0);
            B0 = __builtin_fmaf(w0, p0.x, B0);
        }
    }
    A = A0 + A1;
    B = B0 + B1;
    Cl = C0 + C1;
    Dl = D0 + D1;
}

// Writes (s, c) of the thread's oscillators into a table.
__device__ __forceinline__ void put_sc(const Ctx& x, float4* tab, const uint32_t (&u)[kAdjQPT][4]) {
#pragma unroll
    for (int k = 0; k < kAdjQPT; ++k) {
        const int m = threadIdx.x + k * kAdjTB;
        if (m >= x.nq) break;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<float2*>(tab + 4 * m + j) = make_float2(sin_turn(u[k][j]), cos_turn(u[k][j]));
    }
}

// One synchronous Euler-Maruyama step of the thread's oscillators reading
// neighbour (s, c) from tin and writing the new (s, c) into tout.
template <int QM, int MODE>
__device__ __forceinline__ void fwd_step(const AdjArgs& a, const Ctx& x, const Rows<MODE>& g, int s,
                                         const float4* tin, float4* tout,
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
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * m + j;
            if (i >= x.nb) break;
            float A, B, Cl, Dl;
            gather<false>(g, tin, i, A, B, Cl, Dl);
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

// Dynamic LDS: two tables of tabN float4, then (CSR in LDS) the instance's
// row offsets, 16-bit column indices and FP32 weights.  Fills the CSR copy.
template <int MODE>
__device__ __forceinline__ Rows<MODE> setup_rows(const AdjArgs& a, const Ctx& x, unsigned char* smem) {
    Rows<MODE> g;
    g.a = &a;
    g.off = x.off;
    unsigned char* p = smem + (size_t)32 * a.tabN;
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
    float4* const tabs = reinterpret_cast<float4*>(smem);
    auto tab = [&](int k) { return tabs + (size_t)k * a.tabN; };
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
    const float4* fin = tab(a.steps & 1);
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

template <int QM, int MODE>
__global__ __launch_bounds__(kAdjTB) void adjoint_backward_kernel(AdjArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Ctx x = make_ctx(a);
    const Rows<MODE> g = setup_rows<MODE>(a, x, smem);
    float4* const tabs = reinterpret_cast<float4*>(smem);
    auto tab = [&](int k) { return tabs + (size_t)k * a.tabN; };
    const int q = QM ? QM : a.q;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwg = a.R * a.I;
    const float sqrt_dt = __builtin_sqrtf(a.dt);
    uint32_t u[kAdjQPT][4];
    float lam[kAdjQPT][4];
    int p = 0;  // table written next
    for (int sg = a.nseg - 1; sg >= 0; --sg) {
        const int t0 = sg * a.C;
        const int t1 = t0 + a.C < a.steps ? t0 + a.C : a.steps;
        const bool last = sg == a.nseg - 1;
        // recompute the segment's states from its checkpoint
        load_words(a, x, a.ckpt, sg, u);
        put_sc(x, tab(p), u);
        __syncthreads();
        for (int s = t0; s < t1; ++s) {
            store_words(a, x, a.seg, s - t0, u);
            if (s + 1 < t1 || last) {
                fwd_step<QM>(a, x, g, s, tab(p), tab(p ^ 1), u);
                p ^= 1;
                __syncthreads();
            }
        }
        if (last) {
            // lam_T from the final phases, whose (s, c) table is tab[p]
#pragma unroll
            for (int k = 0; k < kAdjQPT; ++k) {
                const int m = threadIdx.x + k * kAdjTB;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = 4 * m + j;
                    lam[k][j] = 0.f;
                    if (m >= x.nq || i >= x.nb) continue;
                    float A, B, Cl, Dl;
                    gather<false>(g, tab(p), i, A, B, Cl, Dl);
                    const float si = sin_turn(u[k][j]), ci = cos_turn(u[k][j]);
                    lam[k][j] = -0.5f * (si * A - ci * B);
                }
            }
            p ^= 1;
        }
        // adjoint recurrence back through the segment
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
size_t tab_bytes(int tabN) { return (size_t)32 * tabN; }
size_t csr_bytes(int tabN, int64_t nnz, bool weights) {
    size_t b = ((size_t)4 * (tabN + 1) + 15) & ~(size_t)15;
    b += ((size_t)2 * nnz + 15) & ~(size_t)15;
    if (weights) b += (size_t)4 * nnz;
    return b;
}
constexpr size_t kAdjLdsLimit = 160 * 1024 - 256;  // dynamic LDS next to the static reduction slots

// CSR placement for a problem: in LDS when it fits (unit weights need no
// weight array), else read from global memory.
int csr_mode(const Problem* p, int tabN, size_t* lds) {
    const size_t t = tab_bytes(tabN);
    const bool small_idx = p->max_inst_n <= 0x7fff;
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
    static const AdjFn f[3][3] = {
        {adjoint_forward_kernel<0, 0>, adjoint_forward_kernel<0, 1>, adjoint_forward_kernel<0, 2>},
        {adjoint_forward_kernel<2, 0>, adjoint_forward_kernel<2, 1>, adjoint_forward_kernel<2, 2>},
        {adjoint_forward_kernel<3, 0>, adjoint_forward_kernel<3, 1>, adjoint_forward_kernel<3, 2>}};
    return f[qc][mode];
}

AdjFn backward_fn(int q, int mode) {
    const int qc = q == 2 ? 1 : q == 3 ? 2 : 0;
    static const AdjFn f[3][3] = {
        {adjoint_backward_kernel<0, 0>, adjoint_backward_kernel<0, 1>, adjoint_backward_kernel<0, 2>},
        {adjoint_backward_kernel<2, 0>, adjoint_backward_kernel<2, 1>, adjoint_backward_kernel<2, 2>},
        {adjoint_backward_kernel<3, 0>, adjoint_backward_kernel<3, 1>, adjoint_backward_kernel<3, 2>}};
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
    const int mode = csr_mode(p, a.tabN, &lds);
    return launch_adj(forward_fn(cfg->q, mode), lds, cfg->R * p->n_inst, stream, a,
                      "adjoint_forward_kernel");
}

int launch_adjoint_backward(Problem* p, const oim_adjoint_cfg* cfg, const float* K, const float* Ks,
                            const float* sigma, const uint64_t* seeds, int64_t step0,
                            const uint32_t* ckpt, double* gK, double* gKs, double* gS,
                            hipStream_t stream) {
    AdjArgs a = base_args(p, cfg, K, Ks, sigma, seeds, step0);
    if (cfg->steps == 0) return OIM_OK;
    const int nwg = cfg->R * p->n_inst;
    const size_t seg_bytes = (size_t)cfg->checkpoint_every * cfg->R * a.P * sizeof(uint32_t);
    const size_t part_bytes = (size_t)cfg->steps * nwg * kAdjWaves * sizeof(float4);
    const size_t need = seg_bytes + part_bytes + 256;
    if (p->adj_bytes < need) {
        hipFree(p->d_adj);
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
    unsigned char* w = static_cast<unsigned char*>(p->d_adj);
    a.ckpt = const_cast<uint32_t*>(ckpt);
    a.seg = reinterpret_cast<uint32_t*>(w);
    a.gpart = reinterpret_cast<float4*>(w + (seg_bytes + 255) / 256 * 256);
    size_t lds = 0;
    const int mode = csr_mode(p, a.tabN, &lds);
    int st = launch_adj(backward_fn(cfg->q, mode), lds, nwg, stream, a, "adjoint_backward_kernel");
    if (st) return st;
    hipLaunchKernelGGL(adjoint_reduce_kernel, dim3((cfg->steps + 255) / 256), dim3(256), 0, stream,
                       a.gpart, cfg->steps, nwg * kAdjWaves, gK, gKs, gS);
    return check_launch("adjoint_reduce_kernel");
}

}  // namespace oim
