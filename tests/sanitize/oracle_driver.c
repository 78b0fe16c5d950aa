/* Exercises every entry point of the CPU oracle on small inputs, for a build
 * with the address and undefined-behaviour sanitizers: the driver checks
 * return codes and finiteness only (the values are pinned elsewhere); the
 * sanitizers report any out-of-bounds access, use of freed memory or
 * undefined operation.  Prints "ok" and exits 0 when everything ran. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_normals(uint64_t seed, uint32_t i0, int64_t count, uint32_t t, double* out);
float orc_bf16_round(float x);
void orc_coupling_dense_bf16x3(int32_t n, const double* J, const double* theta, double* out);
int orc_run_csr(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                int32_t q, int32_t R, int32_t steps, int64_t step0, double dt, const double* K,
                const double* Ks, const double* sigma, const uint64_t* seeds, double* theta,
                int32_t nthreads);
int orc_run_csr_blocks(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                       int32_t n_inst, const int32_t* inst_off, int32_t q, int32_t R,
                       int32_t steps, int64_t step0, double dt, const double* K, const double* Ks,
                       const double* sigma, const uint64_t* seeds, double* theta,
                       int32_t nthreads);
int orc_run_dense(int32_t n, const double* J, int32_t q, int32_t R, int32_t steps, int64_t step0,
                  double dt, const double* K, const double* Ks, const double* sigma,
                  const uint64_t* seeds, double* theta, int32_t nthreads);
int orc_run_dense_bf16x3(int32_t n, const double* J, int32_t q, int32_t R, int32_t steps,
                         int64_t step0, double dt, const double* K, const double* Ks,
                         const double* sigma, const uint64_t* seeds, double* theta,
                         int32_t nthreads);
void orc_round_f32(int64_t count, const float* theta, int32_t q, int8_t* colour);
int64_t orc_cut_int(int32_t n, const int64_t* row_ptr, const int32_t* col, const int64_t* Jint,
                    const int8_t* colour);
double orc_cut_f64(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                   const int8_t* colour);
int64_t orc_conflicts(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                      const int8_t* colour);
double orc_h_model(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                   int32_t q, const int8_t* colour);
double orc_h_eq6(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                 const double* theta);
double orc_pairwise_tree(const double* v, int64_t count);
void orc_upper_row_sums(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                        int32_t kind, int32_t q, const int8_t* colour, const double* theta,
                        double* out);
int orc_adjoint_csr(int32_t n, const int64_t* row_ptr, const int32_t* col, const double* J,
                    int32_t q, int32_t R, int32_t steps, int64_t step0, double dt,
                    const double* K, const double* Ks, const double* sigma,
                    const uint64_t* seeds, const double* theta0, double* loss, double* gK,
                    double* gKs, double* gS);

#define N 37
#define R 3
#define STEPS 25

static int fails = 0;
static void check(int ok, const char* what) {
    if (!ok) {
        printf("FAIL %s\n", what);
        ++fails;
    }
}
static int all_finite(const double* v, int64_t count) {
    for (int64_t k = 0; k < count; ++k)
        if (!isfinite(v[k])) return 0;
    return 1;
}

int main(void) {
    /* a symmetric random graph with an isolated vertex (N - 1) */
    static int adj[N][N];
    uint32_t s = 12345u;
    for (int i = 0; i < N - 1; ++i)
        for (int j = i + 1; j < N - 1; ++j) {
            s = s * 1664525u + 1013904223u;
            if ((s >> 24) < 52) adj[i][j] = adj[j][i] = 1 + (int)((s >> 8) % 3);
        }
    int64_t row_ptr[N + 1];
    int32_t col[N * N];
    double J[N * N];
    int64_t Jint[N * N];
    int64_t e = 0;
    for (int i = 0; i < N; ++i) {
        row_ptr[i] = e;
        for (int j = 0; j < N; ++j)
            if (adj[i][j]) {
                col[e] = j;
                Jint[e] = (adj[i][j] % 2) ? -adj[i][j] : adj[i][j];
                J[e] = 0.75 * (double)Jint[e];
                ++e;
            }
    }
    row_ptr[N] = e;
    double Jd[N * N];
    for (int i = 0; i < N * N; ++i) Jd[i] = 0.0;
    for (int i = 0; i < N; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) Jd[i * N + col[k]] = J[k];

    double K[STEPS], Ks[STEPS], sg[STEPS];
    for (int t = 0; t < STEPS; ++t) {
        K[t] = 0.2 * t;
        Ks[t] = 0.1 * t;
        sg[t] = 0.05;
    }
    uint64_t seeds[R] = {1u, 77u, 0xfedcba9876543210ull};
    double th0[R * N], th[R * N];
    for (int k = 0; k < R * N; ++k) th0[k] = fmod(0.37 * k, 6.2);

    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out4[4];
    orc_philox4x32_10(ctr, key, out4);
    double nz[9];
    orc_normals(seeds[2], 0xfffffff8u, 9, 0x7fffffffu, nz);
    check(all_finite(nz, 9), "normals");
    check(orc_bf16_round(1.0f + 1.0f / 256.0f) == 1.0f, "bf16 tie");

    for (int q = 2; q <= 5; ++q)
        for (int threads = 1; threads <= 2; ++threads) {
            for (int k = 0; k < R * N; ++k) th[k] = th0[k];
            check(orc_run_csr(N, row_ptr, col, J, q, R, STEPS, 1000, 0.01, K, Ks, sg, seeds, th,
                              threads) == 0, "run_csr");
            check(all_finite(th, R * N), "run_csr finite");
        }
    const int32_t inst_off[3] = {0, 20, N};
    for (int k = 0; k < R * N; ++k) th[k] = th0[k];
    check(orc_run_csr_blocks(N, row_ptr, col, J, 2, inst_off, 3, R, STEPS, 0, 0.01, K, Ks, sg,
                             seeds, th, 2) == 0, "run_csr_blocks");
    for (int k = 0; k < R * N; ++k) th[k] = th0[k];
    check(orc_run_dense(N, Jd, 2, R, STEPS, 5, 0.01, K, Ks, sg, seeds, th, 2) == 0, "run_dense");
    for (int k = 0; k < R * N; ++k) th[k] = th0[k];
    check(orc_run_dense_bf16x3(N, Jd, 2, R, STEPS, 5, 0.01, K, Ks, sg, seeds, th, 1) == 0,
          "run_dense_bf16x3");
    check(all_finite(th, R * N), "dense finite");
    double coup[N];
    orc_coupling_dense_bf16x3(N, Jd, th0, coup);
    check(all_finite(coup, N), "coupling bf16x3");

    float thf[N + 3];
    for (int i = 0; i < N; ++i) thf[i] = (float)th[i];
    thf[N] = NAN;
    thf[N + 1] = INFINITY;
    thf[N + 2] = -3.0e9f;
    int8_t colour[N + 3];
    orc_round_f32(N + 3, thf, 3, colour);
    check(colour[N] == -1 && colour[N + 1] == -1 && colour[N + 2] == -1, "round specials");
    orc_round_f32(N, thf, 2, colour);
    (void)orc_cut_int(N, row_ptr, col, Jint, colour);
    check(isfinite(orc_cut_f64(N, row_ptr, col, J, colour)), "cut_f64");
    (void)orc_conflicts(N, row_ptr, col, J, colour);
    check(isfinite(orc_h_model(N, row_ptr, col, J, 2, colour)), "h_model");
    check(isfinite(orc_h_eq6(N, row_ptr, col, J, th)), "h_eq6");
    double rows[N];
    for (int kind = 0; kind < 4; ++kind) {
        orc_upper_row_sums(N, row_ptr, col, J, kind, 2, colour, th, rows);
        check(all_finite(rows, N), "upper_row_sums");
    }
    check(orc_pairwise_tree(rows, 0) == 0.0, "tree empty");
    check(orc_pairwise_tree(rows, 1) == rows[0], "tree one");
    check(isfinite(orc_pairwise_tree(rows, N)), "tree");

    double loss[1], gK[STEPS], gKs[STEPS], gS[STEPS];
    check(orc_adjoint_csr(N, row_ptr, col, J, 2, R, STEPS, 3, 0.01, K, Ks, sg, seeds, th0, loss,
                          gK, gKs, gS) == 0, "adjoint");
    check(all_finite(gK, STEPS) && all_finite(gKs, STEPS) && all_finite(gS, STEPS), "adjoint finite");
    /* error paths */
    check(orc_run_csr(0, row_ptr, col, J, 2, R, STEPS, 0, 0.01, K, Ks, sg, seeds, th, 1) != 0,
          "n = 0 rejected");
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
