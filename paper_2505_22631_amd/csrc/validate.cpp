// validate.cpp -- host-only argument checks and the sliced-ELL builder.
// Nothing here touches the HIP runtime, so every rejection path can be
// exercised on a machine without a GPU.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>

#include "internal.hpp"

namespace oim {

static thread_local std::string g_last_error;

int set_error(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

void clear_error() { g_last_error.clear(); }

int hip_error(hipError_t e, const char* what) {
    return set_error(OIM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

const char* last_error_cstr() { return g_last_error.c_str(); }

static uint32_t bits(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return u;
}

int validate_csr(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                 const float* J) {
    if (n < 1 || n > (1 << 24)) return set_error(OIM_E_ARG, "n must be in [1, 2^24]");
    if (nnz < 0) return set_error(OIM_E_ARG, "nnz must be >= 0");
    if (!row_ptr) return set_error(OIM_E_ARG, "row_ptr is NULL");
    if (nnz > 0 && (!col_idx || !J)) return set_error(OIM_E_ARG, "col_idx or J is NULL");
    if (row_ptr[0] != 0) return set_error(OIM_E_CSR, "row_ptr[0] != 0");
    if (row_ptr[n] != nnz) return set_error(OIM_E_CSR, "row_ptr[n] != nnz");
    for (int32_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i])
            return set_error(OIM_E_CSR, "row_ptr decreases at row " + std::to_string(i));
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col_idx[e];
            if (j < 0 || j >= n)
                return set_error(OIM_E_CSR, "column out of range in row " + std::to_string(i));
            if (j == i)
                return set_error(OIM_E_CSR, "diagonal entry in row " + std::to_string(i));
            if (e > row_ptr[i] && col_idx[e - 1] >= j)
                return set_error(OIM_E_CSR,
                                 "columns not strictly increasing in row " + std::to_string(i));
        }
    }
    for (int64_t e = 0; e < nnz; ++e)
        if (!std::isfinite(J[e])) return set_error(OIM_E_NONFINITE, "non-finite J entry");
    // symmetry: (j, i) exists with the same bits for every stored (i, j)
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col_idx[e];
            const int32_t* b = col_idx + row_ptr[j];
            const int32_t* en = col_idx + row_ptr[j + 1];
            const int32_t* hit = std::lower_bound(b, en, i);
            if (hit == en || *hit != i)
                return set_error(OIM_E_ASYM, "entry (" + std::to_string(i) + "," +
                                                 std::to_string(j) + ") has no transpose");
            if (bits(J[hit - col_idx]) != bits(J[e]))
                return set_error(OIM_E_ASYM, "J(" + std::to_string(i) + "," + std::to_string(j) +
                                                 ") != J(" + std::to_string(j) + "," +
                                                 std::to_string(i) + ")");
        }
    }
    return OIM_OK;
}

int validate_dense(int32_t n, const float* J) {
    if (n < 1 || n > 65536) return set_error(OIM_E_ARG, "dense n must be in [1, 65536]");
    if (!J) return set_error(OIM_E_ARG, "J is NULL");
    const int64_t nn = (int64_t)n * n;
    for (int64_t k = 0; k < nn; ++k) {
        if ((k / n) == (k % n)) continue;  // diagonal ignored
        if (!std::isfinite(J[k])) return set_error(OIM_E_NONFINITE, "non-finite J entry");
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j)
            if (bits(J[(int64_t)i * n + j]) != bits(J[(int64_t)j * n + i]))
                return set_error(OIM_E_ASYM, "J(" + std::to_string(i) + "," + std::to_string(j) +
                                                 ") != J(" + std::to_string(j) + "," +
                                                 std::to_string(i) + ")");
    return OIM_OK;
}

namespace {
std::mutex g_registry_mu;
std::unordered_map<uint64_t, Problem*> g_registry;
uint64_t g_next_handle = 1;
}  // namespace

oim_problem register_problem(Problem* p) {
    std::lock_guard<std::mutex> lock(g_registry_mu);
    p->handle = g_next_handle++;
    g_registry.emplace(p->handle, p);
    return reinterpret_cast<oim_problem>(static_cast<uintptr_t>(p->handle));
}

Problem* checked(oim_problem h) {
    const uint64_t key = static_cast<uint64_t>(reinterpret_cast<uintptr_t>(h));
    if (key == 0) return nullptr;
    std::lock_guard<std::mutex> lock(g_registry_mu);
    const auto it = g_registry.find(key);
    return it == g_registry.end() ? nullptr : it->second;
}

void unregister_problem(Problem* p) {
    std::lock_guard<std::mutex> lock(g_registry_mu);
    g_registry.erase(p->handle);
}

int validate_cfg(const Problem* p, const oim_run_cfg* cfg) {
    if (!cfg) return set_error(OIM_E_ARG, "cfg is NULL");
    if (cfg->q < 2 || cfg->q > kMaxQ) return set_error(OIM_E_ARG, "q must be in [2, 16]");
    if (cfg->R < 1) return set_error(OIM_E_ARG, "R must be >= 1");
    if (cfg->steps < 0) return set_error(OIM_E_ARG, "steps must be >= 0");
    if (!(cfg->dt > 0.0f) || !std::isfinite(cfg->dt))
        return set_error(OIM_E_ARG, "dt must be finite and > 0");
    if (cfg->readout_every < 0) return set_error(OIM_E_ARG, "readout_every must be >= 0");
    const uint32_t known = OIM_LOOP_MASK | OIM_PREC_MASK | OIM_SCHED_PER_REPLICA;
    if (cfg->flags & ~known) return set_error(OIM_E_ARG, "unknown flag bits");
    const uint32_t loop = cfg->flags & OIM_LOOP_MASK;
    const uint32_t prec = cfg->flags & OIM_PREC_MASK;
    if (loop == OIM_LOOP_MASK) return set_error(OIM_E_ARG, "two loop forms requested");
    if (prec != OIM_PREC_FP32 && prec != OIM_PREC_BF16X3)
        return set_error(OIM_E_ARG, "unknown precision");
    if (prec == OIM_PREC_BF16X3 && !p->dense)
        return set_error(OIM_E_UNSUPPORTED, "BF16X3 applies to dense problems only");
    if ((int64_t)cfg->R * p->n > ((int64_t)1 << 40))
        return set_error(OIM_E_ARG, "R * n too large");
    return OIM_OK;
}

int validate_adjoint_cfg(const Problem* p, const oim_adjoint_cfg* cfg) {
    if (!cfg) return set_error(OIM_E_ARG, "cfg is NULL");
    if (cfg->q < 2 || cfg->q > kMaxQ) return set_error(OIM_E_ARG, "q must be in [2, 16]");
    if (cfg->R < 1) return set_error(OIM_E_ARG, "R must be >= 1");
    if (cfg->steps < 0) return set_error(OIM_E_ARG, "steps must be >= 0");
    if (!(cfg->dt > 0.0f) || !std::isfinite(cfg->dt))
        return set_error(OIM_E_ARG, "dt must be finite and > 0");
    if (cfg->checkpoint_every < 1) return set_error(OIM_E_ARG, "checkpoint_every must be >= 1");
    if (cfg->flags != 0) return set_error(OIM_E_ARG, "flags must be 0");
    if (p->dense) return set_error(OIM_E_UNSUPPORTED, "the adjoint runs on sparse problems");
    if (p->max_inst_n > kAdjMaxN)
        return set_error(OIM_E_UNSUPPORTED, "adjoint: an instance has more than 4096 oscillators");
    if ((int64_t)cfg->R * p->n_inst > (int64_t)INT32_MAX / 2)
        return set_error(OIM_E_ARG, "R * instances too large");
    return OIM_OK;
}

int validate_blocks(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t n_inst,
                    const int32_t* inst_off) {
    if (n_inst < 1 || n_inst > n) return set_error(OIM_E_ARG, "n_inst must be in [1, n]");
    if (n_inst == 1 && !inst_off) return OIM_OK;
    if (!inst_off) return set_error(OIM_E_ARG, "inst_off is NULL");
    if (inst_off[0] != 0 || inst_off[n_inst] != n)
        return set_error(OIM_E_ARG, "inst_off must start at 0 and end at n");
    for (int32_t b = 0; b < n_inst; ++b) {
        if (inst_off[b + 1] <= inst_off[b])
            return set_error(OIM_E_ARG, "inst_off must be strictly increasing");
        for (int32_t i = inst_off[b]; i < inst_off[b + 1]; ++i)
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                if (col_idx[e] < inst_off[b] || col_idx[e] >= inst_off[b + 1])
                    return set_error(OIM_E_CSR, "entry couples two instances in row " +
                                                    std::to_string(i));
    }
    return OIM_OK;
}

void build_sell(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const float* J,
                int32_t n_inst, const int32_t* inst_off, SellImage& out, float uniform_w) {
    out.desc.clear();
    out.entries.clear();
    out.entries_uw.clear();
    out.row_split.clear();
    const bool uw = uniform_w == 1.0f || uniform_w == -1.0f;
    out.inst.clear();
    out.max_slices = 0;
    int64_t rows4 = 0;  // running offset in int4 rows (64 int4 per row)
    int32_t slice_base = 0;
    for (int32_t b = 0; b < n_inst; ++b) {
        const int32_t o = inst_off ? inst_off[b] : 0;
        const int32_t nb = inst_off ? inst_off[b + 1] - inst_off[b] : n;
        const int32_t quads = (nb + 3) / 4;
        const int32_t S = (quads + kSliceQuads - 1) / kSliceQuads;
        out.inst.push_back(int4{slice_base, S, o, nb});
        out.max_slices = std::max(out.max_slices, S);
        // LDS position of local oscillator i: plane (i % 4) of length S*64, slot i / 4.
        const int64_t plane = (int64_t)S * kSliceQuads;
        auto lds_off = [plane](int64_t i) { return (int32_t)(8 * ((i & 3) * plane + (i >> 2))); };
        for (int32_t s = 0; s < S; ++s) {
            int32_t mx = 0;
            const int64_t lo = 4LL * s * kSliceQuads, hi = std::min<int64_t>(nb, 4LL * (s + 1) * kSliceQuads);
            for (int64_t i = lo; i < hi; ++i)
                mx = std::max<int32_t>(mx, (int32_t)(row_ptr[o + i + 1] - row_ptr[o + i]));
            const int32_t deg = (mx + 3) & ~3;
            out.desc.push_back(int2{(int32_t)rows4, deg});
            const size_t first = out.entries.size();
            out.entries.resize(first + (size_t)4 * deg / 2 * kSliceQuads * 2, int2{0, 0});
            const size_t first_uw = out.entries_uw.size();
            if (uw) out.entries_uw.resize(first_uw + (size_t)4 * deg * kSliceQuads, 0u);
            const uint32_t zero_off = (uint32_t)(36 * plane);  // after table and colours
            for (int j = 0; j < 4; ++j) {
                for (int l = 0; l < kSliceQuads; ++l) {
                    const int64_t i = 4LL * (s * kSliceQuads + l) + j;  // local index
                    const int32_t self = (int32_t)std::min<int64_t>(i, nb - 1);
                    const int64_t rb = i < nb ? row_ptr[o + i] : 0;
                    const int64_t rl = i < nb ? row_ptr[o + i + 1] - row_ptr[o + i] : 0;
                    int32_t first_up = 0;  // columns ascend along a row
                    while (first_up < rl && col_idx[rb + first_up] - o <= i) ++first_up;
                    out.row_split.push_back(int2{first_up, (int32_t)rl});
                    for (int32_t e = 0; e < deg; ++e) {
                        int2 v;
                        if (e < rl) {
                            v.x = lds_off(col_idx[rb + e] - o);
                            float w = J[rb + e];
                            std::memcpy(&v.y, &w, 4);
                        } else {
                            v.x = lds_off(self);
                            v.y = 0;
                        }
                        const int64_t q4 = ((int64_t)j * (deg / 2) + e / 2) * kSliceQuads + l;
                        out.entries[first + (size_t)(q4 * 2 + (e & 1))] = v;
                        if (uw) {
                            const int64_t u4 = ((int64_t)j * (deg / 4) + e / 4) * kSliceQuads + l;
                            out.entries_uw[first_uw + (size_t)(u4 * 4 + (e & 3))] =
                                e < rl ? (uint32_t)v.x : zero_off;
                        }
                    }
                }
            }
            rows4 += 4LL * deg / 2;
        }
        slice_base += S;
    }
    out.slices = slice_base;
    out.order.resize(n_inst);
    for (int32_t b = 0; b < n_inst; ++b) out.order[b] = b;
    std::stable_sort(out.order.begin(), out.order.end(), [&](int32_t x, int32_t y) {
        return out.inst[x].y > out.inst[y].y || (out.inst[x].y == out.inst[y].y && out.inst[x].w > out.inst[y].w);
    });
}

bool ell_wanted(int32_t n, const int64_t* row_ptr, int mode) {
    if (mode == 0 || n <= 0) return false;
    int64_t dmax = 0, csr_groups = 0;
    for (int32_t m = 0; 4 * m < n; ++m) {
        int64_t qmax = 0;
        for (int32_t i = 4 * m; i < std::min(n, 4 * m + 4); ++i)
            qmax = std::max<int64_t>(qmax, row_ptr[i + 1] - row_ptr[i]);
        dmax = std::max(dmax, qmax);
        csr_groups += std::max<int64_t>(1, (qmax + 3) / 4);
    }
    const int64_t quads = (n + 3) / 4;
    if (quads * 4 * std::max<int64_t>(4, (dmax + 3) & ~int64_t(3)) > (int64_t)1 << 26)
        return false;  // at most 64 Mi entries (512 MiB)
    if (mode == 1) return true;
    const int64_t ell_groups = quads * std::max<int64_t>(1, (dmax + 3) / 4);
    return 4 * ell_groups <= 5 * csr_groups;
}

void build_ell(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const float* J,
               EllImage& out) {
    int64_t dmax = 0;
    for (int32_t i = 0; i < n; ++i) dmax = std::max<int64_t>(dmax, row_ptr[i + 1] - row_ptr[i]);
    const int32_t D = (int32_t)std::max<int64_t>(4, (dmax + 3) & ~int64_t(3));
    const size_t np = (size_t)(n + 3) / 4 * 4;
    out.D = D;
    out.col.assign(np * D, 0);
    out.J.assign(np * D, 0.f);
    for (size_t i = 0; i < np; ++i) {
        const int32_t self = (int32_t)std::min<size_t>(i, (size_t)n - 1);
        const int64_t b = i < (size_t)n ? row_ptr[i] : 0;
        const int64_t len = i < (size_t)n ? row_ptr[i + 1] - b : 0;
        for (int32_t e = 0; e < D; ++e) {
            const size_t x = (i / 4) * 4 * (size_t)D + (size_t)(e / 4) * 16 + (i % 4) * 4 + e % 4;
            out.col[x] = e < len ? col_idx[b + e] : self;
            out.J[x] = e < len ? J[b + e] : 0.f;
        }
    }
}

}  // namespace oim
