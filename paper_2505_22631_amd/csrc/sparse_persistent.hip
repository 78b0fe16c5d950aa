// sparse_persistent.hip -- the whole Euler-Maruyama loop of Algorithm 1 for a
// sparse coupling in ONE launch, one workgroup per replica, the replica's
// state resident in LDS.
//
// Per step t (Sec. II-E Eq. 5 with the descent sign, Algorithm 1):
//   phase A  every oscillator's coupling sum from the phases of step t,
//            c_i = sum_j J_ij sin(th_i - th_j) = s_i sum_j J_ij c_j - c_i sum_j J_ij s_j,
//            gathered over the sliced-ELL rows from the (sin, cos) table in LDS,
//            folded with the SHIL term into drift_i (registers)
//   barrier
//   phase B  Philox noise, Euler-Maruyama update, wrap, and the (sin, cos)
//            table refreshed for step t+1
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
#include <float.h>

#include "internal.hpp"
#include "noise.hpp"
#include "phase.hpp"

namespace oim {

namespace {

struct PersistArgs {
    const int2* sell;
    const int32_t* desc;
    int32_t S;        // slices
    int32_t plane;    // S * 64: length of one LDS plane
    int32_t n;
    int32_t q;
    int32_t steps;
    int32_t M;        // readout period (0 = none)
    int64_t step0;
    float dt;
    const float* K;
    const float* Ks;
    const float* sigma;
    const uint64_t* seeds;
    float* theta;     // [R][n]
    uint32_t* phase;  // [R][n] or null
    double* trace;    // [ceil(steps/M)][R]
    double* best_h;   // [R]
    int32_t* best_step;
    int8_t* best_colour;  // [R][n]
    int32_t R;
};

template <int TB, int MS, int QM>
__global__ __launch_bounds__(TB) void persistent_sparse_kernel(PersistArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    float2* sc = reinterpret_cast<float2*>(smem);                   // [4 * plane]
    unsigned char* col8 = smem + (size_t)8 * 4 * a.plane;          // [4 * plane]
    double* red = reinterpret_cast<double*>(col8 + ((4 * a.plane + 15) & ~15));  // [W]
    int* flag = reinterpret_cast<int*>(red + TB / 64);

    constexpr int W = TB / 64;
    const int r = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = a.n, plane = a.plane, S = a.S;
    const int q = QM ? QM : a.q;
    const uint64_t seed = a.seeds[r];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    float* th = a.theta + (int64_t)r * n;
    uint32_t* pw = a.phase ? a.phase + (int64_t)r * n : nullptr;

    uint32_t ph[MS][4];
    float sn[MS][4], cs[MS][4], drift[MS][4];

#pragma unroll
    for (int k = 0; k < MS; ++k) {
        const int slice = wave + k * W;
        const int m = slice * 64 + lane;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * m + j;
            const bool valid = slice < S && i < n;
            const uint32_t u = valid ? (pw ? pw[i] : phase_from_theta(th[i])) : 0u;
            ph[k][j] = u;
            sn[k][j] = sin_turn(u);
            cs[k][j] = cos_turn(u);
            drift[k][j] = 0.0f;
            if (valid) sc[j * plane + m] = make_float2(sn[k][j], cs[k][j]);
        }
    }
    __syncthreads();

    const float sqrt_dt = __builtin_sqrtf(a.dt);
    double best = DBL_MAX;
    int32_t best_at = -1;

    for (int s = 0; s < a.steps; ++s) {
        const uint32_t t = (uint32_t)(a.step0 + s);
        const float kc = -a.dt * a.K[s] * kTurnScale;
        const float ks = -a.dt * a.Ks[s] * kTurnScale;
        const float ns = a.sigma[s] * sqrt_dt * kTurnScale;

        // ---- phase A: coupling sums over the sliced-ELL rows ----
#pragma unroll
        for (int k = 0; k < MS; ++k) {
            const int slice = wave + k * W;
            if (slice < S) {
                const int32_t* d = a.desc + slice * 8;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int32_t off = d[j], deg = d[4 + j];
                    const int2* ep = a.sell + (int64_t)off * 64 + lane;
                    float A0 = 0.f, B0 = 0.f, A1 = 0.f, B1 = 0.f;
                    int e = 0;
                    for (; e + 4 <= deg; e += 4) {
                        const int2 v0 = ep[(e + 0) * 64];
                        const int2 v1 = ep[(e + 1) * 64];
                        const int2 v2 = ep[(e + 2) * 64];
                        const int2 v3 = ep[(e + 3) * 64];
                        const float2 p0 = *reinterpret_cast<const float2*>(smem + v0.x);
                        const float2 p1 = *reinterpret_cast<const float2*>(smem + v1.x);
                        const float2 p2 = *reinterpret_cast<const float2*>(smem + v2.x);
                        const float2 p3 = *reinterpret_cast<const float2*>(smem + v3.x);
                        A0 = __builtin_fmaf(__int_as_float(v0.y), p0.y, A0);
                        B0 = __builtin_fmaf(__int_as_float(v0.y), p0.x, B0);
                        A1 = __builtin_fmaf(__int_as_float(v1.y), p1.y, A1);
                        B1 = __builtin_fmaf(__int_as_float(v1.y), p1.x, B1);
                        A0 = __builtin_fmaf(__int_as_float(v2.y), p2.y, A0);
                        B0 = __builtin_fmaf(__int_as_float(v2.y), p2.x, B0);
                        A1 = __builtin_fmaf(__int_as_float(v3.y), p3.y, A1);
                        B1 = __builtin_fmaf(__int_as_float(v3.y), p3.x, B1);
                    }
                    for (; e < deg; ++e) {
                        const int2 v = ep[e * 64];
                        const float2 p = *reinterpret_cast<const float2*>(smem + v.x);
                        A0 = __builtin_fmaf(__int_as_float(v.y), p.y, A0);
                        B0 = __builtin_fmaf(__int_as_float(v.y), p.x, B0);
                    }
                    const float A = A0 + A1, B = B0 + B1;
                    const float coup = sn[k][j] * A - cs[k][j] * B;
                    drift[k][j] = kc * coup + ks * sin_q<QM>(sn[k][j], cs[k][j], ph[k][j], q);
                }
            }
        }
        __syncthreads();

        // ---- phase B: noise, Euler-Maruyama update, wrap, table refresh ----
#pragma unroll
        for (int k = 0; k < MS; ++k) {
            const int slice = wave + k * W;
            const int m = slice * 64 + lane;
            if (slice < S && 4 * m < n) {
                float z[4];
                normals4((uint32_t)m, t, k0, k1, z);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t u = advance(ph[k][j], __builtin_fmaf(ns, z[j], drift[k][j]));
                    ph[k][j] = u;
                    sn[k][j] = sin_turn(u);
                    cs[k][j] = cos_turn(u);
                    if (4 * m + j < n) sc[j * plane + m] = make_float2(sn[k][j], cs[k][j]);
                }
            }
        }
        __syncthreads();

        // ---- optional readout: threshold, Eq. 1 / Eq. 2, best-so-far ----
        if (a.M > 0 && ((s + 1) % a.M == 0 || s + 1 == a.steps)) {
#pragma unroll
            for (int k = 0; k < MS; ++k) {
                const int slice = wave + k * W;
                const int m = slice * 64 + lane;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (slice < S && 4 * m + j < n) {
                        col8[j * plane + m] = (unsigned char)nearest_state(ph[k][j], q);
                    }
                }
            }
            __syncthreads();
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < MS; ++k) {
                const int slice = wave + k * W;
                if (slice < S) {
                    const int m = slice * 64 + lane;
                    const int32_t* d = a.desc + slice * 8;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (4 * m + j >= n) continue;
                        const int ci = col8[j * plane + m];
                        const int32_t off = d[j], deg = d[4 + j];
                        const int2* ep = a.sell + (int64_t)off * 64 + lane;
                        double row = 0.0;
                        for (int e = 0; e < deg; ++e) {
                            const int2 v = ep[e * 64];
                            const int cj = col8[v.x >> 3];
                            const float w = __int_as_float(v.y);
                            const float term = (q == 2) ? (ci == cj ? w : -w) : (ci == cj ? w : 0.f);
                            row += (double)term;
                        }
                        acc += row;
                    }
                }
            }
            // workgroup reduction (fixed order: lanes by xor butterfly, then waves)
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (lane == 0) red[wave] = acc;
            __syncthreads();
            if (threadIdx.x == 0) {
                double tot = 0.0;
                for (int w = 0; w < W; ++w) tot += red[w];
                const double H = -0.5 * tot;
                const int kread = (s + a.M) / a.M - 1;
                if (a.trace) a.trace[(int64_t)kread * a.R + r] = H;
                int improved = 0;
                if (H < best) {
                    best = H;
                    best_at = (int32_t)(a.step0 + s + 1);
                    improved = 1;
                }
                *flag = improved;
            }
            __syncthreads();
            if (*flag && a.best_colour) {
                int8_t* bc = a.best_colour + (int64_t)r * n;
#pragma unroll
                for (int k = 0; k < MS; ++k) {
                    const int slice = wave + k * W;
                    const int m = slice * 64 + lane;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (slice < S && 4 * m + j < n) bc[4 * m + j] = (int8_t)col8[j * plane + m];
                }
            }
            __syncthreads();
        }
    }

    // ---- final phases ----
#pragma unroll
    for (int k = 0; k < MS; ++k) {
        const int slice = wave + k * W;
        const int m = slice * 64 + lane;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * m + j;
            if (slice < S && i < n) {
                th[i] = theta_from_phase(ph[k][j]);
                if (pw) pw[i] = ph[k][j];
            }
        }
    }
    if (threadIdx.x == 0) {
        if (a.best_h) a.best_h[r] = best_at >= 0 ? best : __builtin_inf();
        if (a.best_step) a.best_step[r] = best_at;
    }
}

using KernelFn = void (*)(PersistArgs);

struct Variant {
    int tb, ms;
    KernelFn fn[3];  // QM = 0 (generic), 2, 3
};

#define OIM_VARIANT(TB, MS)                                                              \
    Variant {                                                                            \
        TB, MS, {                                                                        \
            persistent_sparse_kernel<TB, MS, 0>, persistent_sparse_kernel<TB, MS, 2>,    \
                persistent_sparse_kernel<TB, MS, 3>                                      \
        }                                                                                \
    }

const Variant kVariants[] = {
    OIM_VARIANT(256, 1),  OIM_VARIANT(256, 2),  OIM_VARIANT(256, 3),  OIM_VARIANT(256, 4),
    OIM_VARIANT(256, 6),  OIM_VARIANT(256, 8),  OIM_VARIANT(256, 10), OIM_VARIANT(256, 12),
    OIM_VARIANT(512, 1),  OIM_VARIANT(512, 2),  OIM_VARIANT(512, 3),  OIM_VARIANT(512, 4),
    OIM_VARIANT(512, 5),  OIM_VARIANT(512, 6),  OIM_VARIANT(512, 8),  OIM_VARIANT(512, 10),
    OIM_VARIANT(1024, 1), OIM_VARIANT(1024, 2), OIM_VARIANT(1024, 3), OIM_VARIANT(1024, 4),
    OIM_VARIANT(1024, 5),
};

constexpr size_t kLdsLimit = 160 * 1024;

size_t lds_bytes(int plane, int tb) {
    size_t b = (size_t)8 * 4 * plane;                 // (sin, cos) table
    b += ((size_t)4 * plane + 15) & ~(size_t)15;      // colours for readout
    b += sizeof(double) * (tb / 64) + 16;             // reduction scratch + flag
    return b;
}

// Pick the variant: fewest waves that still cover every slice with the
// registers of one variant, preferring 8 waves per workgroup.
const Variant* pick_variant(int S, int tb_hint) {
    const Variant* best = nullptr;
    for (const Variant& v : kVariants) {
        const int W = v.tb / 64;
        if (tb_hint && v.tb != tb_hint) continue;
        if (W * v.ms < S) continue;
        if (!best) { best = &v; continue; }
        // smallest ms*W (least idle), then the preferred block size
        const int cv = W * v.ms, cb = (best->tb / 64) * best->ms;
        const int pv = v.tb == 512 ? 0 : 1, pb = best->tb == 512 ? 0 : 1;
        if (cv < cb || (cv == cb && pv < pb)) best = &v;
    }
    return best;
}

int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    return v ? atoi(v) : dflt;
}

}  // namespace

bool persistent_sparse_fits(const Problem* p) {
    if (p->dense || p->sell_slices == 0) return false;
    if (lds_bytes(p->sell_slices * 64, 1024) > kLdsLimit) return false;
    return pick_variant(p->sell_slices, 0) != nullptr;
}

int launch_persistent_sparse(const Problem* p, const oim_run_cfg* cfg, const float* K,
                             const float* Ks, const float* sigma, const uint64_t* seeds,
                             int64_t step0, float* theta, uint32_t* phase,
                             const oim_readout* ro, hipStream_t stream) {
    const int S = p->sell_slices;
    const Variant* v = pick_variant(S, env_int("OIM_PERSIST_TB", 0));
    if (!v) v = pick_variant(S, 0);
    if (!v || !persistent_sparse_fits(p))
        return set_error(OIM_E_UNSUPPORTED, "replica does not fit the LDS-resident kernel");
    PersistArgs a{};
    a.sell = p->d_sell;
    a.desc = p->d_sell_desc;
    a.S = S;
    a.plane = S * 64;
    a.n = p->n;
    a.q = cfg->q;
    a.steps = cfg->steps;
    a.M = cfg->readout_every;
    a.step0 = step0;
    a.dt = cfg->dt;
    a.K = K;
    a.Ks = Ks;
    a.sigma = sigma;
    a.seeds = seeds;
    a.theta = theta;
    a.phase = phase;
    a.trace = ro ? ro->trace : nullptr;
    a.best_h = ro ? ro->best_h : nullptr;
    a.best_step = ro ? ro->best_step : nullptr;
    a.best_colour = ro ? ro->best_colour : nullptr;
    a.R = cfg->R;
    const int qi = cfg->q == 2 ? 1 : cfg->q == 3 ? 2 : 0;
    KernelFn fn = v->fn[qi];
    const size_t lds = lds_bytes(a.plane, v->tb);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");
    hipLaunchKernelGGL(fn, dim3(cfg->R), dim3(v->tb), lds, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "persistent_sparse_kernel launch");
    return OIM_OK;
}

}  // namespace oim
