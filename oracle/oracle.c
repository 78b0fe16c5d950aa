/*
 * oracle.c -- plain FP64 CPU reference of the simulated oscillator Ising/Potts
 * machine (arXiv 2505.22631).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source, header, table or constant with the
 * GPU library.
 *
 * What it computes, in the paper's order (Algorithm 1, Sec. II-E Eq. 5):
 *   for each step t: first every oscillator's coupling sum is formed from the
 *   phases of step t (the derivative loop), then every phase is advanced by
 *   forward Euler with the SHIL term and a Gaussian noise kick and wrapped back
 *   into one period (the update loop).
 *
 * Readings of the paper that this file follows (all phases in radians, period
 * 2*pi; the paper's normalised phase is theta / (2*pi)):
 *   - J is the Ising coupling of Eq. 1 (H = -sum_{i<j} J_ij s_i s_j); max-cut
 *     maps to J = -w (Sec. II-C).  The drift that descends this energy is
 *       f_i = -K * sum_{j != i} J_ij sin(theta_i - theta_j) - Ks sin(q theta_i)
 *     (the sign printed in Eq. 5 would synchronise max-cut edge partners; the
 *     descent sign is the one whose fixed points minimise Eq. 1 / Eq. 6).
 *   - SHIL: -Ks sin(q theta) has its stable points at 2*pi*k/q (Sec. II-D).
 *   - Noise: theta += sigma_t * sqrt(dt) * xi, xi ~ N(0,1) (the Algorithm 1
 *     form, sigma playing the role of K_n).
 *   - Schedules K, Ks, sigma are per-step arrays indexed by the local step.
 *   - The noise is a counter-based stream: Philox4x32-10 (Salmon, Moraes, Dror,
 *     Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11) keyed by the
 *     replica's 64-bit seed, counter (i/4, t, b, 0) with i the oscillator's
 *     index within its instance and b the instance of a block-diagonal batch
 *     (a single graph is instance 0), followed by Box-Muller
 *     (Box & Muller 1958) on 24-bit uniforms.  Words (x0,x1) serve oscillators
 *     i = 0,1 mod 4 and (x2,x3) serve i = 2,3 mod 4; the even member of a pair
 *     takes rho*cos(2 pi u2), the odd one rho*sin(2 pi u2).
 *   - Thresholding (readout only, never fed back): k = floor(q theta/(2 pi) + 1/2)
 *     mod q, evaluated in FP32 as floor(fmaf(theta, (float)(q/(2 pi)), 0.5f)),
 *     the precision the GPU takes the same decision in.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11, Sec. 4.2): ten rounds of two 32x32->64 products     */
/* with the Weyl-sequence key schedule.                                      */
/* ------------------------------------------------------------------------ */
static void philox_one_round(uint32_t x[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x[1] ^ k[0];
    const uint32_t y1 = lo1;
    const uint32_t y2 = hi0 ^ x[3] ^ k[1];
    const uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u; /* golden ratio */
            k[1] += 0xBB67AE85u; /* sqrt(3) - 1  */
        }
        philox_one_round(x, k);
    }
    memcpy(out, x, sizeof x);
}

/* One standard normal for oscillator i (index within instance b) at global
 * step t of the replica whose seed is `seed`. */
double orc_normal_b(uint64_t seed, uint32_t i, uint32_t t, uint32_t b) {
    const uint32_t ctr[4] = {i >> 2, t, b, 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const int pair = (int)((i >> 1) & 1u);
    const uint32_t xa = x[2 * pair], xb = x[2 * pair + 1];
    const double u1 = ((double)(xa >> 8) + 1.0) / 16777216.0; /* (0, 1] */
    const double u2 = (double)(xb >> 8) / 16777216.0;         /* [0, 1) */
    const double rho = sqrt(-2.0 * log(u1));
    return (i & 1u) ? rho * sin(ORC_TWO_PI * u2) : rho * cos(ORC_TWO_PI * u2);
}

double orc_normal(uint64_t seed, uint32_t i, uint32_t t) { return orc_normal_b(seed, i, t, 0u); }

void orc_normals(uint64_t seed, uint32_t i0, int64_t count, uint32_t t, double* out) {
    for (int64_t k = 0; k < count; ++k) out[k] = orc_normal(seed, (uint32_t)(i0 + k), t);
}

static double wrap_2pi(double th) {
    double w = th - ORC_TWO_PI * floor(th / ORC_TWO_PI);
    if (w >= ORC_TWO_PI) w -= ORC_TWO_PI;
    if (w < 0.0) w = 0.0;
    return w;
}

/* ------------------------------------------------------------------------ */
/* Integrators.  theta is [R][n], FP64, in/out.  J is the Ising coupling.    */
/* Returns 0, or -1 on a bad argument.                                       */
/* ------------------------------------------------------------------------ */
/* The derivative loop of Algorithm 1 for oscillators i0 .. i1-1: each
 * coupling sum c_i = sum_{j != i} J_ij sin(th_i - th_j) from the phases of
 * step t, in row order. */
static void coupling_rows(int32_t i0, int32_t i1, int32_t n, const int64_t* row_ptr,
                          const int32_t* col, const double* Jv, const double* Jdense,
                          const double* th, double* coup) {
    for (int32_t i = i0; i < i1; ++i) {
        double acc = 0.0;
        if (Jdense) {
            for (int32_t j = 0; j < n; ++j)
                if (j != i) acc += Jdense[(int64_t)i * n + j] * sin(th[i] - th[j]);
        } else {
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                acc += Jv[e] * sin(th[i] - th[col[e]]);
        }
        coup[i] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* BF16x3 split products for a dense coupling (the precision of the dense   */
/* all-to-all workload; the paper computes in FP32).  The coupling sum is    */
/* taken through the identity sin(a - b) = sin a cos b - cos a sin b:        */
/*   c_i = sin th_i * Y_C,i - cos th_i * Y_S,i,  Y_X,i = sum_{j != i} J_ij X_j */
/* where every GEMM operand x (J_ij, and sin th_j / cos th_j rounded to      */
/* FP32) is split as x = x_hi + x_lo + e, x_hi = bf16(x),                    */
/* x_lo = bf16(x - x_hi), and each product J_ij X_j is replaced by           */
/* J_hi X_hi + J_hi X_lo + J_lo X_hi (the J_lo X_lo term dropped).  Products */
/* and sums here are FP64 in row order, so the only departures from the      */
/* exact coupling are the splits and the dropped term:                       */
/*   |c_i(bf16x3) - c_i| <= ~3 * 2^-16 * sum_j |J_ij|.                        */
/* ------------------------------------------------------------------------ */
/* BF16 of an FP32 value: the FP32 bit pattern rounded to its top 16 bits,  */
/* to nearest, ties to even (finite inputs). */
static float bf16_round(float x) {
    uint32_t u;
    memcpy(&u, &x, sizeof u);
    const uint32_t keep_lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + keep_lsb) & 0xffff0000u;
    float r;
    memcpy(&r, &u, sizeof r);
    return r;
}

float orc_bf16_round(float x) { return bf16_round(x); }

/* hi and lo halves of the split of one FP32 value (x - hi is exact in FP32) */
static void split3(float x, double* hi, double* lo) {
    const float h = bf16_round(x);
    *hi = (double)h;
    *lo = (double)bf16_round(x - h);
}

/* The split GEMM operands of the phases of rows i0 .. i1-1: xs holds four
 * planes of n, (sin_hi, sin_lo, cos_hi, cos_lo). */
static void split_x_rows(int32_t i0, int32_t i1, int32_t n, const double* th, double* xs) {
    for (int32_t j = i0; j < i1; ++j) {
        split3((float)sin(th[j]), &xs[j], &xs[n + j]);
        split3((float)cos(th[j]), &xs[2 * n + j], &xs[3 * n + j]);
    }
}

/* Coupling sums of rows i0 .. i1-1 from the split J (Jsp: n*n hi, then n*n
 * lo, diagonal zero) and the split phases of every row. */
static void coupling_rows_bf16x3(int32_t i0, int32_t i1, int32_t n, const double* Jsp,
                                 const double* xs, const double* th, double* coup) {
    const double* Jh = Jsp;
    const double* Jl = Jsp + (size_t)n * n;
    const double *sh = xs, *sl = xs + n, *ch = xs + 2 * n, *cl = xs + 3 * n;
    for (int32_t i = i0; i < i1; ++i) {
        double ys = 0.0, yc = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double h = Jh[(int64_t)i * n + j], l = Jl[(int64_t)i * n + j];
            ys += h * sh[j] + h * sl[j] + l * sh[j];
            yc += h * ch[j] + h * cl[j] + l * ch[j];
        }
        coup[i] = sin(th[i]) * yc - cos(th[i]) * ys;
    }
}

void orc_coupling_dense_bf16x3(int32_t n, const double* J, const double* theta, double* out) {
    double* Jsp = (double*)malloc(sizeof(double) * 2 * (size_t)n * n);
    double* xs = (double*)malloc(sizeof(double) * 4 * (size_t)n);
    if (!Jsp || !xs) {
        free(Jsp);
        free(xs);
        for (int32_t i = 0; i < n; ++i) out[i] = NAN;
        return;
    }
    for (int64_t k = 0; k < (int64_t)n * n; ++k) split3((float)J[k], &Jsp[k], &Jsp[(size_t)n * n + k]);
    split_x_rows(0, n, n, theta, xs);
    coupling_rows_bf16x3(0, n, n, Jsp, xs, theta, out);
    free(Jsp);
    free(xs);
}

/* The update loop of Algorithm 1 for oscillators i0 .. i1-1: forward Euler
 * with the SHIL term and the noise kick, then the wrap into one period. */
static void update_rows(int32_t i0, int32_t i1, int32_t q, double dt, double Kt, double Kst,
                        double sigt, uint64_t seed, uint32_t t, const uint32_t* inst_of,
                        const uint32_t* local, const double* coup, double* th) {
    const double sq = sqrt(dt);
    for (int32_t i = i0; i < i1; ++i) {
        const double f = -Kt * coup[i] - Kst * sin((double)q * th[i]);
        const double xi = orc_normal_b(seed, local[i], t, inst_of[i]);
        th[i] = wrap_2pi(th[i] + dt * f + sigt * sq * xi);
    }
}

static int run_common(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* Jv,
                      const double* Jdense, const double* Jsplit, int32_t q, int32_t R, int32_t steps, int64_t step0,
                      double dt, const double* K, const double* Ks, const double* sigma,
                      const uint64_t* seeds, double* theta, int32_t nthreads, int32_t n_inst,
                      const int32_t* inst_off, uint32_t inst_base) {
    if (n < 1 || R < 1 || steps < 0 || q < 2 || !(dt > 0.0)) return -1;
    /* instance of every oscillator and its index within the instance */
    uint32_t* inst_of = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t* local = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    if (!inst_of || !local) { free(inst_of); free(local); return -1; }
    for (int32_t i = 0; i < n; ++i) { inst_of[i] = inst_base; local[i] = (uint32_t)i; }
    if (inst_off && n_inst > 1) {
        for (int32_t b = 0; b < n_inst; ++b)
            for (int32_t i = inst_off[b]; i < inst_off[b + 1]; ++i) {
                inst_of[i] = inst_base + (uint32_t)b;
                local[i] = (uint32_t)(i - inst_off[b]);
            }
    }
    int threads = 1;
#ifdef _OPENMP
    threads = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
    int bad = 0;
    if (R >= threads || threads == 1) {
        /* replicas are independent: one replica per thread at a time */
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
        for (int32_t r = 0; r < R; ++r) {
            double* th = theta + (int64_t)r * n;
            double* coup = (double*)malloc(sizeof(double) * (size_t)n);
            double* xs = Jsplit ? (double*)malloc(sizeof(double) * 4 * (size_t)n) : NULL;
            if (!coup || (Jsplit && !xs)) { free(coup); free(xs); bad = 1; continue; }
            for (int32_t s = 0; s < steps; ++s) {
                if (Jsplit) {
                    split_x_rows(0, n, n, th, xs);
                    coupling_rows_bf16x3(0, n, n, Jsplit, xs, th, coup);
                } else {
                    coupling_rows(0, n, n, row_ptr, col, Jv, Jdense, th, coup);
                }
                update_rows(0, n, q, dt, K[s], Ks[s], sigma[s], seeds[r], (uint32_t)(step0 + s),
                            inst_of, local, coup, th);
            }
            free(coup);
            free(xs);
        }
    } else {
        /* fewer replicas than threads: the oscillators of one replica are
         * split into contiguous ranges, one per thread, with a barrier
         * between the two loops of every step; every oscillator's arithmetic
         * is the same as in the serial loops */
        double* coup = (double*)malloc(sizeof(double) * (size_t)n);
        double* xs = Jsplit ? (double*)malloc(sizeof(double) * 4 * (size_t)n) : NULL;
        if (!coup || (Jsplit && !xs)) bad = 1;
        for (int32_t r = 0; r < R && !bad; ++r) {
            double* th = theta + (int64_t)r * n;
#pragma omp parallel num_threads(threads)
            {
                int me = 0, nt = 1;
#ifdef _OPENMP
                me = omp_get_thread_num();
                nt = omp_get_num_threads();
#endif
                const int32_t i0 = (int32_t)((int64_t)n * me / nt);
                const int32_t i1 = (int32_t)((int64_t)n * (me + 1) / nt);
                for (int32_t s = 0; s < steps; ++s) {
                    if (Jsplit) {
                        split_x_rows(i0, i1, n, th, xs);
#pragma omp barrier
                        coupling_rows_bf16x3(i0, i1, n, Jsplit, xs, th, coup);
                    } else {
                        coupling_rows(i0, i1, n, row_ptr, col, Jv, Jdense, th, coup);
                    }
#pragma omp barrier
                    update_rows(i0, i1, q, dt, K[s], Ks[s], sigma[s], seeds[r],
                                (uint32_t)(step0 + s), inst_of, local, coup, th);
#pragma omp barrier
                }
            }
        }
        free(coup);
        free(xs);
    }
    free(inst_of);
    free(local);
    return bad ? -1 : 0;
}

int orc_run_csr(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                int32_t q, int32_t R, int32_t steps, int64_t step0, double dt, const double* K,
                const double* Ks, const double* sigma, const uint64_t* seeds, double* theta,
                int32_t nthreads) {
    return run_common(n, row_ptr, col, J, NULL, NULL, q, R, steps, step0, dt, K, Ks, sigma, seeds,
                      theta, nthreads, 1, NULL, 0u);
}

/* A single graph integrated as instance `b` of a block-diagonal batch: the
 * same trajectory that instance b of the batch follows (its noise counter
 * carries b). */
int orc_run_csr_instance(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                         uint32_t b, int32_t q, int32_t R, int32_t steps, int64_t step0,
                         double dt, const double* K, const double* Ks, const double* sigma,
                         const uint64_t* seeds, double* theta, int32_t nthreads) {
    return run_common(n, row_ptr, col, J, NULL, NULL, q, R, steps, step0, dt, K, Ks, sigma, seeds,
                      theta, nthreads, 1, NULL, b);
}

/* Block-diagonal batch: instance b holds oscillators inst_off[b] .. inst_off[b+1]-1
 * (no coupling between instances); the noise of each oscillator is drawn with its
 * index within its instance and the instance number. */
int orc_run_csr_blocks(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                       int32_t n_inst, const int32_t* inst_off, int32_t q, int32_t R,
                       int32_t steps, int64_t step0, double dt, const double* K, const double* Ks,
                       const double* sigma, const uint64_t* seeds, double* theta,
                       int32_t nthreads) {
    return run_common(n, row_ptr, col, J, NULL, NULL, q, R, steps, step0, dt, K, Ks, sigma, seeds,
                      theta, nthreads, n_inst, inst_off, 0u);
}

int orc_run_dense(int32_t n, const double* J, int32_t q, int32_t R, int32_t steps, int64_t step0,
                  double dt, const double* K, const double* Ks, const double* sigma,
                  const uint64_t* seeds, double* theta, int32_t nthreads) {
    return run_common(n, NULL, NULL, NULL, J, NULL, q, R, steps, step0, dt, K, Ks, sigma, seeds, theta,
                      nthreads, 1, NULL, 0u);
}

/* Dense coupling with BF16x3 split products (see coupling_rows_bf16x3); the
 * rest of the step is the FP64 step of Algorithm 1. */
int orc_run_dense_bf16x3(int32_t n, const double* J, int32_t q, int32_t R, int32_t steps,
                         int64_t step0, double dt, const double* K, const double* Ks,
                         const double* sigma, const uint64_t* seeds, double* theta,
                         int32_t nthreads) {
    if (n < 1) return -1;
    double* Jsp = (double*)malloc(sizeof(double) * 2 * (size_t)n * n);
    if (!Jsp) return -1;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) {
            const int64_t k = (int64_t)i * n + j;
            if (i == j) { Jsp[k] = 0.0; Jsp[(size_t)n * n + k] = 0.0; }
            else split3((float)J[k], &Jsp[k], &Jsp[(size_t)n * n + k]);
        }
    const int rc = run_common(n, NULL, NULL, NULL, NULL, Jsp, q, R, steps, step0, dt, K, Ks,
                              sigma, seeds, theta, nthreads, 1, NULL, 0u);
    free(Jsp);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Thresholding (Sec. III-B "phase threshold"): nearest of the q stable      */
/* phases 2 pi k / q.  FP32 decision; -1 for non-finite or |theta| >= 2^20.  */
/* ------------------------------------------------------------------------ */
void orc_round_f32(int64_t count, const float* theta, int32_t q, int8_t* colour) {
    const float scale = (float)((double)q / ORC_TWO_PI);
    for (int64_t k = 0; k < count; ++k) {
        const float th = theta[k];
        if (!isfinite(th) || fabsf(th) >= 1048576.0f) { colour[k] = -1; continue; }
        const float x = floorf(fmaf(th, scale, 0.5f));
        int64_t c = (int64_t)x % q;
        if (c < 0) c += q;
        colour[k] = (int8_t)c;
    }
}

/* ------------------------------------------------------------------------ */
/* Readouts over the upper triangle i < j of a symmetric CSR coupling.       */
/* ------------------------------------------------------------------------ */
/* max-cut value with edge weights w = -J (Sec. II-C), integer weights */
int64_t orc_cut_int(int32_t n, const int64_t* row_ptr, const int32_t* col, const int64_t* Jint,
                    const int8_t* colour) {
    int64_t cut = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (i < j && colour[i] != colour[j]) cut += -Jint[e];
        }
    return cut;
}

double orc_cut_f64(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                   const int8_t* colour) {
    double cut = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (i < j && colour[i] != colour[j]) cut += -J[e];
        }
    return cut;
}

/* colouring conflicts: edges (J != 0) whose ends share a colour */
int64_t orc_conflicts(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                      const int8_t* colour) {
    int64_t c = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (i < j && J[e] != 0.0 && colour[i] == colour[j]) ++c;
        }
    return c;
}

/* Eq. 1 for q = 2 (spin s = 1 - 2k), Eq. 2 for q >= 3 (Kronecker delta). */
double orc_h_model(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                   int32_t q, const int8_t* colour) {
    double h = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (i >= j) continue;
            if (q == 2) {
                const double si = 1.0 - 2.0 * colour[i], sj = 1.0 - 2.0 * colour[j];
                h -= J[e] * si * sj;
            } else if (colour[i] == colour[j]) {
                h -= J[e];
            }
        }
    return h;
}

/* Eq. 6 with the weights w = -J, evaluated at the (continuous) phases. */
double orc_h_eq6(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                 const double* theta) {
    double h = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (i < j) h += -J[e] * cos(theta[i] - theta[j]);
        }
    return h;
}

/* ------------------------------------------------------------------------ */
/* Readouts in one fixed FP64 order, so that real-weighted cut and energy    */
/* values from identical spins are reproducible bit for bit (integer weights */
/* give the same value in any order).  Each row i sums its terms over the    */
/* upper triangle j > i in ascending column order, starting from +0.  The    */
/* row sums are then combined by the pairwise tree over rows: the rows are   */
/* padded with zeros to a power of two and adjacent pairs are added level    */
/* by level, the lower-indexed partial sum on the left.                      */
/* ------------------------------------------------------------------------ */
double orc_pairwise_tree(const double* v, int64_t count) {
    if (count <= 0) return 0.0;
    int64_t P = 1;
    while (P < count) P <<= 1;
    double* w = (double*)malloc(sizeof(double) * (size_t)P);
    if (!w) return NAN;
    for (int64_t k = 0; k < P; ++k) w[k] = k < count ? v[k] : 0.0;
    for (int64_t len = P; len > 1; len >>= 1)
        for (int64_t k = 0; k < len / 2; ++k) w[k] = w[2 * k] + w[2 * k + 1];
    const double s = w[0];
    free(w);
    return s;
}

/* Row sums of one readout's terms over j > i (CSR order is ascending j).
 * kind 0, cut (Sec. II-C, w = -J):  -J_ij when the colours differ, else 0
 * kind 1, Eq. 1 (q = 2):            -J_ij s_i s_j with s = 1 - 2k
 *         Eq. 2 (q >= 3):           -J_ij when the colours are equal, else 0
 * kind 2, Eq. 6 (w = -J):           -J_ij cos(theta_i - theta_j)          */
void orc_upper_row_sums(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                        int32_t kind, int32_t q, const int8_t* colour, const double* theta,
                        double* out) {
    for (int32_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (j <= i) continue;
            double term;
            if (kind == 0) {
                term = colour[i] != colour[j] ? -J[e] : 0.0;
            } else if (kind == 1) {
                if (q == 2) term = colour[i] == colour[j] ? -J[e] : J[e];
                else term = colour[i] == colour[j] ? -J[e] : 0.0;
            } else {
                const double c = cos(theta[i] - theta[j]);
                term = -J[e] * c;
            }
            acc += term;
        }
        out[i] = acc;
    }
}

int orc_abi_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* Adjoint of the fixed-noise Euler-Maruyama trajectory (schedule tuning).   */
/*   loss      L = sum_r sum_{i<j} w_ij (1 - cos(th_T,i - th_T,j)) / 2,      */
/*             w = -J  (the relaxed cut at the final phases)                 */
/*   lam_T,i   = dL/dth_T,i = 1/2 sum_j w_ij sin(th_i - th_j)                */
/*   step      th_{t+1} = th_t + dt f(th_t) + sigma_t sqrt(dt) xi_t,         */
/*             f_i = -K_t sum_j J_ij sin(th_i - th_j) - Ks_t sin(q th_i)     */
/*   lam_t,k   = lam_{t+1,k} + dt sum_i lam_{t+1,i} df_i/dth_k                */
/*             = lam_{t+1,k} + dt [ K_t sum_j J_kj cos(th_k - th_j)          */
/*                 (lam_{t+1,j} - lam_{t+1,k}) - q Ks_t cos(q th_k) lam_{t+1,k} ] */
/*   dL/dK_t   = -dt sum lam_{t+1,i} sum_j J_ij sin(th_t,i - th_t,j)          */
/*   dL/dKs_t  = -dt sum lam_{t+1,i} sin(q th_t,i)                           */
/*   dL/dsig_t = sqrt(dt) sum lam_{t+1,i} xi_t,i                             */
/* The wrap into one period has derivative 1 almost everywhere.  All sums    */
/* run over replicas too (one schedule drives every replica).                */
/* ------------------------------------------------------------------------ */
/* A block-diagonal batch (instances [inst_off[b], inst_off[b+1])) draws its */
/* noise per instance, as the forward integrator does; the loss and the      */
/* gradients are sums over instances and replicas.                           */
int orc_adjoint_csr_blocks(int32_t n, const int64_t* row_ptr, const int32_t* col,
                           const double* J, int32_t n_inst, const int32_t* inst_off, int32_t q,
                           int32_t R, int32_t steps, int64_t step0, double dt, const double* K,
                           const double* Ks, const double* sigma, const uint64_t* seeds,
                           const double* theta0, double* loss, double* gK, double* gKs,
                           double* gS) {
    if (n < 1 || R < 1 || steps < 0 || q < 2 || !(dt > 0.0) || n_inst < 1) return -1;
    const size_t N = (size_t)n;
    uint32_t* inst_of = (uint32_t*)malloc(sizeof(uint32_t) * N);
    uint32_t* local = (uint32_t*)malloc(sizeof(uint32_t) * N);
    if (!inst_of || !local) { free(inst_of); free(local); return -1; }
    for (int32_t i = 0; i < n; ++i) { inst_of[i] = 0; local[i] = (uint32_t)i; }
    if (inst_off && n_inst > 1)
        for (int32_t b = 0; b < n_inst; ++b)
            for (int32_t i = inst_off[b]; i < inst_off[b + 1]; ++i) {
                inst_of[i] = (uint32_t)b;
                local[i] = (uint32_t)(i - inst_off[b]);
            }
    double* traj = (double*)malloc(sizeof(double) * N * (size_t)(steps + 1));
    double* lam = (double*)malloc(sizeof(double) * N);
    double* nxt = (double*)malloc(sizeof(double) * N);
    if (!traj || !lam || !nxt) {
        free(traj); free(lam); free(nxt); free(inst_of); free(local);
        return -1;
    }
    for (int32_t s = 0; s < steps; ++s) gK[s] = gKs[s] = gS[s] = 0.0;
    double total = 0.0;
    const double sq = sqrt(dt);
    for (int32_t r = 0; r < R; ++r) {
        /* forward, keeping every state */
        memcpy(traj, theta0 + (size_t)r * N, sizeof(double) * N);
        if (run_common(n, row_ptr, col, J, NULL, NULL, q, 1, 0, step0, dt, K, Ks, sigma, seeds + r,
                       traj, 1, n_inst, inst_off, 0u) != 0) { total = NAN; break; }
        for (int32_t s = 0; s < steps; ++s) {
            memcpy(traj + N * (s + 1), traj + N * s, sizeof(double) * N);
            if (run_common(n, row_ptr, col, J, NULL, NULL, q, 1, 1, step0 + s, dt, K + s, Ks + s,
                           sigma + s, seeds + r, traj + N * (s + 1), 1, n_inst, inst_off, 0u) != 0) {
                total = NAN;
                break;
            }
        }
        const double* thT = traj + N * (size_t)steps;
        for (int32_t i = 0; i < n; ++i) {
            double g = 0.0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                const int32_t j = col[e];
                const double w = -J[e];
                g += 0.5 * w * sin(thT[i] - thT[j]);
                if (i < j) total += 0.5 * w * (1.0 - cos(thT[i] - thT[j]));
            }
            lam[i] = g;
        }
        for (int32_t s = steps - 1; s >= 0; --s) {
            const double* th = traj + N * (size_t)s;
            const uint32_t t = (uint32_t)(step0 + s);
            for (int32_t k = 0; k < n; ++k) {
                double cc = 0.0, csin = 0.0;
                for (int64_t e = row_ptr[k]; e < row_ptr[k + 1]; ++e) {
                    const int32_t j = col[e];
                    cc += J[e] * cos(th[k] - th[j]) * (lam[j] - lam[k]);
                    csin += J[e] * sin(th[k] - th[j]);
                }
                nxt[k] = lam[k] + dt * (K[s] * cc - (double)q * Ks[s] * cos((double)q * th[k]) * lam[k]);
                gK[s] += -dt * lam[k] * csin;
                gKs[s] += -dt * lam[k] * sin((double)q * th[k]);
                gS[s] += sq * lam[k] * orc_normal_b(seeds[r], local[k], t, inst_of[k]);
            }
            memcpy(lam, nxt, sizeof(double) * N);
        }
    }
    *loss = total;
    free(traj);
    free(lam);
    free(nxt);
    free(inst_of);
    free(local);
    return 0;
}

int orc_adjoint_csr(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                    int32_t q, int32_t R, int32_t steps, int64_t step0, double dt,
                    const double* K, const double* Ks, const double* sigma,
                    const uint64_t* seeds, const double* theta0, double* loss, double* gK,
                    double* gKs, double* gS) {
    return orc_adjoint_csr_blocks(n, row_ptr, col, J, 1, NULL, q, R, steps, step0, dt, K, Ks,
                                  sigma, seeds, theta0, loss, gK, gKs, gS);
}
