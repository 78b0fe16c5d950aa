// readout.hip -- thresholding and objective readouts.
//
//   round      nearest stable phase k = floor(q theta / 2pi + 1/2) mod q, the
//              "phase threshold kernel" of Sec. III-B, FP32 decision
//   cut        max-cut value sum_{i<j} w_ij [k_i != k_j] with w = -J (Sec. II-C)
//   conflicts  colouring conflicts #{i<j : J_ij != 0, k_i == k_j}
//   energy     Eq. 1 (q = 2) or Eq. 2 (q >= 3) at the colours, and Eq. 6 with
//              w = -J at the continuous phases, FP64
//
// One workgroup per replica walks the upper triangle of the coupling (CSR
// rows, or the dense matrix).  Every FP64 sum follows one fixed order, the
// same in every readout of the library: each row i sums its terms over
// j > i in ascending column order, from +0, and the row sums are combined by
// the pairwise tree over rows (zero-padded to a power of two, adjacent pairs
// first, the lower rows on the left).  Here a thread owns one row of a block
// of 256; the block's tree runs over lanes (xor butterfly, partner distance
// 1, 2, ..., 32) and then over the four waves; the blocks are combined by
// the same tree, built incrementally in the order the blocks complete
// (tree_push / tree_finish).  Integer weights are accumulated in int64 and
// are exact.
#include "internal.hpp"
#include "phase.hpp"
#include "tree.hpp"

// products and sums of the readouts are rounded one by one, as written
#pragma clang fp contract(off)

namespace oim {

namespace {

constexpr int kTB = 256;

// Sum of a 256-thread block's values, one per row of the block, by the
// pairwise tree over the rows (thread t = row t); valid in thread 0.
template <typename T>
__device__ T block_tree(T v, T* scratch) {
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    T tot = 0;
    if (threadIdx.x == 0) tot = (scratch[0] + scratch[1]) + (scratch[2] + scratch[3]);
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(256) void round_kernel(int64_t count, const float* theta, int q,
                                                    float scale, int8_t* colour) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        const float th = theta[k];
        int8_t c = -1;
        if (__builtin_isfinite(th) && __builtin_fabsf(th) < 1048576.0f) {
            const int x = (int)__builtin_floorf(__builtin_fmaf(th, scale, 0.5f));
            int m = x % q;
            if (m < 0) m += q;
            c = (int8_t)m;
        }
        colour[k] = c;
    }
}

__global__ __launch_bounds__(256) void phase_convert_kernel(int64_t count, const float* theta_in,
                                                            uint32_t* phase_out,
                                                            const uint32_t* phase_in,
                                                            float* theta_out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (theta_in) {
            const float th = theta_in[k];
            phase_out[k] = phase_from_theta(th);
        } else {
            theta_out[k] = theta_from_phase(phase_in[k]);
        }
    }
}

// mode 0: cut (int64 + f64), 1: conflicts, 2: energies.  Thread t of the
// workgroup owns row 256 b + t of block b; the block sums are combined in
// thread 0 by the pairwise tree over blocks.
template <int MODE, bool DENSE>
__global__ __launch_bounds__(kTB) void pair_sum_kernel(
    int n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const float* __restrict__ J, const float* __restrict__ Jd, const int8_t* __restrict__ colour,
    const float* __restrict__ theta, int q, int64_t* out_i64, double* out_f64a, double* out_f64b) {
    __shared__ int64_t si[kTB / 64];
    __shared__ double sd[kTB / 64];
    __shared__ double stack[2][TreeAcc::kLevels];
    const int r = blockIdx.x;
    const int8_t* k = colour ? colour + (int64_t)r * n : nullptr;
    const float* th = theta ? theta + (int64_t)r * n : nullptr;
    int64_t tot_i = 0;
    TreeAcc tree_a(stack[0]), tree_b(stack[1]);
    for (int i0 = 0; i0 < n; i0 += kTB) {
        const int i = i0 + (int)threadIdx.x;
        int64_t acc_i = 0;
        double acc_a = 0.0, acc_b = 0.0;
        if (i < n) {
            const int ki = k ? k[i] : 0;
            const double ti = th ? (double)th[i] : 0.0;
            auto visit = [&](int j, float w) {
                if (MODE == 0) {
                    if (ki != k[j]) {
                        acc_i += (int64_t)(-w);
                        acc_a += -(double)w;
                    }
                } else if (MODE == 1) {
                    if (w != 0.0f && ki == k[j]) acc_i += 1;
                } else {
                    if (k) {
                        if (q == 2) acc_a += (ki == k[j]) ? -(double)w : (double)w;
                        else if (ki == k[j]) acc_a += -(double)w;
                    }
                    if (th) {
                        const double c = cos(ti - (double)th[j]);
                        const double term = -(double)w * c;
                        acc_b += term;
                    }
                }
            };
            if (DENSE) {
                const float* rowJ = Jd + (int64_t)i * n;
                for (int j = i + 1; j < n; ++j) visit(j, rowJ[j]);
            } else {
                for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                    const int j = col[e];
                    if (j > i) visit(j, J[e]);
                }
            }
        }
        if (MODE == 0 || MODE == 1) {
            const int64_t bi = block_tree<int64_t>(acc_i, si);
            if (threadIdx.x == 0) tot_i += bi;
        }
        if (MODE == 0 || MODE == 2) {
            const double ba = block_tree<double>(acc_a, sd);
            if (threadIdx.x == 0) tree_a.push(ba);
        }
        if (MODE == 2) {
            const double bb = block_tree<double>(acc_b, sd);
            if (threadIdx.x == 0) tree_b.push(bb);
        }
    }
    if (threadIdx.x == 0) {
        if ((MODE == 0 || MODE == 1) && out_i64) out_i64[r] = tot_i;
        if ((MODE == 0 || MODE == 2) && out_f64a) out_f64a[r] = tree_a.finish();
        if (MODE == 2 && out_f64b) out_f64b[r] = tree_b.finish();
    }
}

template <int MODE>
int launch_pairs(const Problem* p, int R, const int8_t* colour, const float* theta, int q,
                 int64_t* oi, double* oa, double* ob, hipStream_t s) {
    if (R < 1) return set_error(OIM_E_ARG, "R must be >= 1");
    if (p->dense)
        hipLaunchKernelGGL((pair_sum_kernel<MODE, true>), dim3(R), dim3(kTB), 0, s, p->n,
                           nullptr, nullptr, nullptr, p->d_Jdense, colour, theta, q, oi, oa, ob);
    else
        hipLaunchKernelGGL((pair_sum_kernel<MODE, false>), dim3(R), dim3(kTB), 0, s, p->n,
                           p->d_row_ptr, p->d_col, p->d_J, nullptr, colour, theta, q, oi, oa,
                           ob);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "readout launch");
    return OIM_OK;
}

}  // namespace

int launch_round(int32_t q, int64_t count, const float* theta, int8_t* colour, hipStream_t s) {
    if (count == 0) return OIM_OK;
    const float scale = (float)((double)q / 6.283185307179586476925286766559);
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(round_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count, theta, q,
                       scale, colour);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "round launch");
    return OIM_OK;
}

int launch_phase_convert(int64_t count, const float* theta_in, uint32_t* phase_out,
                         const uint32_t* phase_in, float* theta_out, hipStream_t s) {
    if (count == 0) return OIM_OK;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(phase_convert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count,
                       theta_in, phase_out, phase_in, theta_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "phase conversion launch");
    return OIM_OK;
}

int launch_cut(const Problem* p, int32_t R, const int8_t* colour, int64_t* cut_i64,
               double* cut_f64, hipStream_t s) {
    return launch_pairs<0>(p, R, colour, nullptr, 2, cut_i64, cut_f64, nullptr, s);
}

int launch_conflicts(const Problem* p, int32_t R, const int8_t* colour, int64_t* conflicts,
                     hipStream_t s) {
    return launch_pairs<1>(p, R, colour, nullptr, 2, conflicts, nullptr, nullptr, s);
}

int launch_energy(const Problem* p, int32_t q, int32_t R, const float* theta,
                  const int8_t* colour, double* h_model, double* h_eq6, hipStream_t s) {
    return launch_pairs<2>(p, R, h_model ? colour : nullptr, h_eq6 ? theta : nullptr, q, nullptr,
                           h_model, h_eq6, s);
}

}  // namespace oim
