// sparse_persistent.hip -- launch variants of the LDS-resident kernel
// (persistent_kernel.hpp), the default choice, the launch and the autotuner.
#include <float.h>

#include "persistent_kernel.hpp"

namespace oim {

namespace {

using namespace persist;


struct Variant {
    int tb, ms, rpl;
    KernelFn fn[3];  // QM = 0 (generic), 2, 3
    // slices covered: (waves / waves per slice) x slices per wave group
    int covers() const { return (tb / 64) / (4 / rpl) * ms; }
};

#define OIM_VARIANT_ENTRY(TB, MS, RPL)                                                   \
    Variant{TB, MS, RPL,                                                                 \
            {persistent_sparse_kernel<TB, MS, 0, RPL, false>,                            \
             persistent_sparse_kernel<TB, MS, 2, RPL, false>,                            \
             persistent_sparse_kernel<TB, MS, 3, RPL, false>}},

const Variant kVariants[kVariantCount] = {OIM_PERSIST_VARIANTS(OIM_VARIANT_ENTRY)};

constexpr size_t kLdsLimit = 160 * 1024;

// LDS of a launch; with slice_sums, room for the readout's per-slice sums
// (slices covered by the variant) too.
size_t lds_bytes(int plane, int tb, int rpl, int covered = 0) {
    size_t b = (size_t)8 * 4 * plane;                 // (sin, cos) table
    b += (size_t)4 * plane + 16;                      // colours for readout, zero entry
    b += sizeof(double) * (tb / 64 + kSliceTreeLevels) + 32;  // reduction, tree levels, readout state
    if (rpl < 4) b += sizeof(double) * (size_t)tb;    // quads' partial row sums (readout)
    b += sizeof(double) * (size_t)covered;            // per-slice sums (readout), if used
    return b;
}

constexpr uint64_t kMaxSellBytes = 0x7fffffffull;

// Default choice without tuning: fewest waves that still cover every slice
// with the registers of one variant, preferring 8 waves per workgroup, among
// blocks of at least 256 threads.
const Variant* pick_variant(int S, int tb_hint) {
    const Variant* best = nullptr;
    for (const Variant& v : kVariants) {
        const int W = v.tb / 64;
        if (v.rpl != 4) continue;
        if (tb_hint ? v.tb != tb_hint : v.tb < 256) continue;
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

const Variant* find_variant(int tb, int ms, int rpl) {
    for (const Variant& v : kVariants)
        if (v.tb == tb && v.ms == ms && v.rpl == rpl) return &v;
    return nullptr;
}

// The variant covers every slice of the largest instance and its LDS fits.
bool variant_ok(const Problem* p, const Variant& v) {
    return v.covers() >= p->max_slices &&
           lds_bytes(p->max_slices * 64, v.tb, v.rpl) <= kLdsLimit;
}

int q_class(int q) { return q == 2 ? 1 : q == 3 ? 2 : 0; }

// The variant a run uses: the tuned one for this SHIL order if set, else an
// OIM_PERSIST_TB block-size hint, else the default choice.
const Variant* run_variant(const Problem* p, int q) {
    const int qc = q_class(q);
    if (p->tuned_tb[qc]) {
        const Variant* v = find_variant(p->tuned_tb[qc], p->tuned_ms[qc], p->tuned_rpl[qc]);
        if (v && variant_ok(p, *v)) return v;
    }
    const Variant* v = pick_variant(p->max_slices, env_int("OIM_PERSIST_TB", 0));
    return v ? v : pick_variant(p->max_slices, 0);
}

}  // namespace

bool persistent_variant_fits(const Problem* p, int tb, int ms, int rpl) {
    const Variant* v = find_variant(tb, ms, rpl);
    return v && variant_ok(p, *v);
}

bool persistent_sparse_fits(const Problem* p) {
    if (p->dense || p->max_slices == 0) return false;
    if (lds_bytes(p->max_slices * 64, 1024, 4) > kLdsLimit) return false;
    if ((uint64_t)p->sell_entries * 8 > kMaxSellBytes) return false;
    return pick_variant(p->max_slices, 0) != nullptr;
}

namespace {
// sched_stride: the row length of per-replica schedules ([R][sched_stride]),
// or 0 for one schedule shared by every replica.
int launch_variant(const Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                   const float* sigma, const uint64_t* seeds, int64_t step0, float* theta,
                   uint32_t* phase, const oim_readout* ro, hipStream_t stream,
                   const Variant* forced, int32_t sched_stride) {
    const int S = p->max_slices;
    const Variant* v = forced ? forced : run_variant(p, cfg->q);
    if (!v || !persistent_sparse_fits(p) || !variant_ok(p, *v))
        return set_error(OIM_E_UNSUPPORTED, "replica does not fit the LDS-resident kernel");
    PersistArgs a{};
    a.sell = reinterpret_cast<const int4*>(p->d_sell);
    a.row_split = p->d_row_split;
    a.desc = p->d_sell_desc;
    a.sell_bytes = (uint32_t)(p->sell_entries * 8);
    a.inst = p->d_inst;
    a.order = p->d_order;
    a.I = p->n_inst;
    a.n_total = p->n;
    const int plane = S * 64;
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
    a.sched_stride = sched_stride;
    const int qi = cfg->q == 2 ? 1 : cfg->q == 3 ? 2 : 0;
    KernelFn fn = v->fn[qi];
    if (p->d_sell_uw) {
        a.sell_uw = reinterpret_cast<const int4*>(p->d_sell_uw);
        a.sell_uw_bytes = (uint32_t)(p->sell_entries * 4);
        a.w0 = p->uniform_w;
        fn = kUniformKernels[v - kVariants][qi];
    }
    // the readout keeps per-slice sums in LDS when there is room for them
    const size_t lds_fast = lds_bytes(plane, v->tb, v->rpl, v->covers());
    a.slice_sums = (a.M > 0 && lds_fast <= kLdsLimit) ? 1 : 0;
    const size_t lds = a.slice_sums ? lds_fast : lds_bytes(plane, v->tb, v->rpl);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");
    if ((int64_t)cfg->R * p->n_inst > 0x7fffffff)
        return set_error(OIM_E_ARG, "R * instances too large");
    hipLaunchKernelGGL(fn, dim3(cfg->R * p->n_inst), dim3(v->tb), lds, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "persistent_sparse_kernel launch");
    return OIM_OK;
}
}  // namespace

int launch_persistent_sparse(const Problem* p, const oim_run_cfg* cfg, const float* K,
                             const float* Ks, const float* sigma, const uint64_t* seeds,
                             int64_t step0, float* theta, uint32_t* phase,
                             const oim_readout* ro, hipStream_t stream) {
    return launch_variant(p, cfg, K, Ks, sigma, seeds, step0, theta, phase, ro, stream, nullptr,
                          (cfg->flags & OIM_SCHED_PER_REPLICA) ? cfg->steps : 0);
}

// Autotuner: every variant whose waves cover the largest instance runs the
// first trial_steps steps of the caller's schedule on a scratch copy of
// theta (no readout), twice; the faster of the two timings (HIP events on the
// caller's stream) ranks it.  The four fastest then run three times on up to
// twice as many steps, and the smallest median wins.  The winner is recorded
// in the problem for this SHIL order.  Results do not depend on the variant:
// every oscillator's arithmetic is the same in all of them.
int tune_persistent(Problem* p, const oim_run_cfg* cfg, const float* K, const float* Ks,
                    const float* sigma, const uint64_t* seeds, const float* theta,
                    int32_t trial_steps, oim_tune_report* rep, hipStream_t stream) {
    if (!persistent_sparse_fits(p))
        return set_error(OIM_E_UNSUPPORTED, "replica does not fit the LDS-resident kernel");
    const size_t bytes = (size_t)cfg->R * p->n * sizeof(float);
    float* scratch = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&scratch), bytes);
    if (e != hipSuccess) {
        return e == hipErrorOutOfMemory ? set_error(OIM_E_NOMEM, "autotune scratch: out of device memory")
                                        : hip_error(e, "autotune scratch");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = OIM_OK;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        st = hip_error(e, "autotune events");
    oim_run_cfg c = *cfg;
    c.readout_every = 0;
    // per-replica schedules keep the caller's row length while the trials
    // run a prefix of each row
    const int32_t stride = (cfg->flags & OIM_SCHED_PER_REPLICA) ? cfg->steps : 0;
    // times one variant `reps` times on `steps` steps of the schedule
    auto time_variant = [&](const Variant& v, int steps, int reps, float* out) {
        c.steps = steps;
        for (int rep_i = 0; rep_i < reps && !st; ++rep_i) {
            if ((e = hipMemcpyAsync(scratch, theta, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess ||
                (e = hipEventRecord(e0, stream)) != hipSuccess) {
                st = hip_error(e, "autotune copy");
                break;
            }
            st = launch_variant(p, &c, K, Ks, sigma, seeds, 0, scratch, nullptr, nullptr, stream, &v,
                                stride);
            if (st) break;
            float ms = 0.f;
            if ((e = hipEventRecord(e1, stream)) != hipSuccess ||
                (e = hipEventSynchronize(e1)) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
                st = hip_error(e, "autotune timing");
                break;
            }
            out[rep_i] = ms;
        }
    };
    // first pass: every covering variant, best of two short trials
    constexpr int kFinalists = 4;
    const Variant* fin[kFinalists] = {};
    float fin_ms[kFinalists] = {};
    int tried = 0;
    for (const Variant& v : kVariants) {
        if (st) break;
        if (!variant_ok(p, v)) continue;
        float t[2] = {0.f, 0.f};
        time_variant(v, trial_steps, 2, t);
        if (st) break;
        const float t_min = t[0] < t[1] ? t[0] : t[1];
        if (rep && tried < OIM_TUNE_MAX) {
            rep->block[tried] = v.tb;
            rep->slices_per_wave[tried] = v.ms;
            rep->rows_per_lane[tried] = v.rpl;
            rep->ms[tried] = t_min;
        }
        ++tried;
        // keep the kFinalists fastest, sorted
        for (int f = 0; f < kFinalists; ++f) {
            if (!fin[f] || t_min < fin_ms[f]) {
                for (int g2 = kFinalists - 1; g2 > f; --g2) {
                    fin[g2] = fin[g2 - 1];
                    fin_ms[g2] = fin_ms[g2 - 1];
                }
                fin[f] = &v;
                fin_ms[f] = t_min;
                break;
            }
        }
    }
    // second pass: the finalists on trials twice as long (within the schedule),
    // three times each; the smallest median wins (short trials alone picked
    // variants up to 15 % apart from run to run on the 1024-graph batch)
    const Variant* best = nullptr;
    float best_ms = 0.f;
    const int final_steps = 2 * trial_steps < cfg->steps ? 2 * trial_steps : cfg->steps;
    for (int f = 0; f < kFinalists && fin[f] && !st; ++f) {
        float t[3] = {0.f, 0.f, 0.f};
        time_variant(*fin[f], final_steps, 3, t);
        if (st) break;
        const float lo = t[0] < t[1] ? t[0] : t[1], hi = t[0] < t[1] ? t[1] : t[0];
        const float med = t[2] < lo ? lo : (t[2] > hi ? hi : t[2]);
        if (!best || med < best_ms) {
            best = fin[f];
            best_ms = med;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(scratch);
    if (st) return st;
    if (!best) return set_error(OIM_E_UNSUPPORTED, "no variant covers the largest instance");
    const int qc = q_class(cfg->q);
    p->tuned_tb[qc] = (int16_t)best->tb;
    p->tuned_ms[qc] = (int16_t)best->ms;
    p->tuned_rpl[qc] = (int16_t)best->rpl;
    if (rep) {
        rep->n_tried = tried < OIM_TUNE_MAX ? tried : OIM_TUNE_MAX;
        rep->chosen_block = best->tb;
        rep->chosen_slices_per_wave = best->ms;
        rep->chosen_rows_per_lane = best->rpl;
        rep->chosen_ms = best_ms;
    }
    return OIM_OK;
}

}  // namespace oim
