/* The oracle (test infrastructure) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every topology and model through RK4 with R and
 * the mean phase velocity recorded, the right-hand side alone, Dormand-Prince
 * with and without dense output, and the argument checks.  Small sizes; exits
 * non-zero on a failed check, the sanitizers abort on the first error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_rhs(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
            const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
            const double* per_elem, int reverse, const double* z, double* f);
int orc_run(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
            const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
            const double* per_elem, int reverse, double* y, double dt, int64_t steps, double* R,
            int64_t record_every, double* mean_vel, int64_t mv_start);
int orc_run_dopri(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
                  const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
                  const double* per_elem, double* y, double t_end, double rtol, double atol, double dt0,
                  int64_t max_steps, double* stats);
int orc_run_dopri_dense(int model, int topo, int64_t n, int64_t radius, int64_t n1, int64_t n2, int64_t n3,
                        const int64_t* row_ptr, const int32_t* col, const double* w, const double* prm,
                        const double* per_elem, double* y, double t_end, double rtol, double atol, double dt0,
                        int64_t max_steps, double* stats, double t_out, double* Rout, double* Yout);

#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

enum { KUR = 0, FHN = 1, HH = 2, INERTIA = 3 };
enum { RING = 0, CUBE = 1, CSR = 2, BALL = 3, DISK = 4, LINKS = 5 };

static double* state(int nv, int64_t n, unsigned seed) {
    double* y = malloc(sizeof(double) * nv * n);
    srand(seed);
    for (int64_t i = 0; i < nv * n; ++i) y[i] = 6.0 * rand() / (double)RAND_MAX - 3.0;
    return y;
}

static int finite_all(const double* y, int64_t m) {
    for (int64_t i = 0; i < m; ++i)
        if (!isfinite(y[i])) return 0;
    return 1;
}

int main(void) {
    const double kprm[3] = {0.1, 1.0, 1.46}, iprm[5] = {0.0, 0.5, 0.45, 1.0, 0.05};
    const double fprm[4] = {0.05, 0.5, 0.1, 1.4707963267948966};
    const double hprm[10] = {1.0, 120.0, 36.0, 0.3, 50.0, -77.0, -54.387, 0.0, 0.0, 2.0};
    double R[64], mv[4096], f[4096], stats[8], Rout[64], Yout[64 * 200];
    /* rings: Kuramoto, inertia, FHN; P up to (n-1)/2 */
    for (int model = 0; model < 4; ++model) {
        if (model == HH) continue;
        const int nv = model == KUR ? 1 : 2;
        const double* prm = model == KUR ? kprm : (model == FHN ? fprm : iprm);
        for (int64_t n = 3; n <= 40; n += 37 / 3) {
            for (int64_t P = 1; 2 * P + 1 <= n; P += 3) {
                double* y = state(nv, n, (unsigned)(n * 31 + P));
                CHECK(orc_rhs(model, RING, n, P, 0, 0, 0, NULL, NULL, NULL, prm, NULL, 0, y, f) == 0);
                CHECK(orc_rhs(model, RING, n, P, 0, 0, 0, NULL, NULL, NULL, prm, NULL, 1, y, f) == 0);
                CHECK(orc_run(model, RING, n, P, 0, 0, 0, NULL, NULL, NULL, prm, NULL, 0, y, 0.01, 12, R, 3,
                              model == INERTIA ? NULL : mv, 4) == 0);
                CHECK(finite_all(y, nv * n));
                free(y);
            }
        }
        double* y = state(nv, 9, 5);
        CHECK(orc_run(model, RING, 9, 5, 0, 0, 0, NULL, NULL, NULL, prm, NULL, 0, y, 0.01, 3, NULL, 0, NULL, -1) != 0);
        free(y);
    }
    /* lattices: cube, ball, disk with non-cubic extents */
    for (int model = 0; model < 4; model += 3) {
        const int nv = model == KUR ? 1 : 2;
        const double* prm = model == KUR ? kprm : iprm;
        double* y = state(nv, 7 * 8 * 9, 11);
        CHECK(orc_run(model, CUBE, 7 * 8 * 9, 3, 7, 8, 9, NULL, NULL, NULL, prm, NULL, 0, y, 0.05, 4, R, 1,
                      model == KUR ? mv : NULL, 2) == 0);
        CHECK(orc_run(model, BALL, 7 * 8 * 9, 3, 7, 8, 9, NULL, NULL, NULL, prm, NULL, 0, y, 0.05, 4, R, 2, NULL, -1) ==
              0);
        CHECK(orc_run(model, DISK, 11 * 9, 4, 11, 9, 1, NULL, NULL, NULL, prm, NULL, 0, y, 0.05, 4, R, 4, NULL, -1) ==
              0);
        CHECK(finite_all(y, nv * 7 * 8 * 9));
        CHECK(orc_run(model, CUBE, 7 * 8 * 9, 4, 7, 8, 9, NULL, NULL, NULL, prm, NULL, 0, y, 0.05, 1, NULL, 0, NULL,
                      -1) != 0); /* 2h+1 > 7 */
        free(y);
    }
    /* row lists (compressed-matrix topology) and a CSR graph for HH, with empty rows and self links */
    {
        enum { N = 60 };
        int64_t rp[N + 1];
        int32_t col[N * 6];
        double w[N * 6], iapp[N];
        int64_t e = 0;
        rp[0] = 0;
        for (int i = 0; i < N; ++i) {
            const int deg = i % 7 == 0 ? 0 : 1 + i % 6;
            for (int k = 0; k < deg; ++k) {
                col[e] = (int32_t)((i + 5 * k) % N);
                w[e] = 0.01 * (k + 1);
                ++e;
            }
            rp[i + 1] = e;
            iapp[i] = 8.0 + (i % 5);
        }
        for (int model = 0; model < 4; ++model) {
            if (model == HH) continue;
            const int nv = model == KUR ? 1 : 2;
            const double* prm = model == KUR ? kprm : (model == FHN ? fprm : iprm);
            double* y = state(nv, N, 17);
            CHECK(orc_run(model, LINKS, N, 0, 0, 0, 0, rp, col, NULL, prm, NULL, 0, y, 0.01, 5, R, 1,
                          model == INERTIA ? NULL : mv, 1) == 0);
            CHECK(finite_all(y, nv * N));
            free(y);
        }
        double* y = malloc(sizeof(double) * 4 * N);
        for (int i = 0; i < N; ++i) {
            y[i] = -65.0 + 0.1 * i;
            y[N + i] = 0.05, y[2 * N + i] = 0.6, y[3 * N + i] = 0.32;
        }
        CHECK(orc_rhs(HH, CSR, N, 0, 0, 0, 0, rp, col, w, hprm, iapp, 0, y, f) == 0);
        CHECK(orc_run(HH, CSR, N, 0, 0, 0, 0, rp, col, w, hprm, iapp, 0, y, 0.01, 50, NULL, 0, NULL, -1) == 0);
        CHECK(finite_all(y, 4 * N));
        col[3] = N; /* source out of range */
        CHECK(orc_run(HH, CSR, N, 0, 0, 0, 0, rp, col, w, hprm, iapp, 0, y, 0.01, 1, NULL, 0, NULL, -1) != 0);
        col[3] = 0;
        rp[5] = rp[6] + 1; /* row offsets not monotone */
        CHECK(orc_run(HH, CSR, N, 0, 0, 0, 0, rp, col, w, hprm, iapp, 0, y, 0.01, 1, NULL, 0, NULL, -1) != 0);
        free(y);
    }
    /* Dormand-Prince: controlled, fixed step, dense output, a NaN state */
    {
        double* y = state(2, 50, 23);
        CHECK(orc_run_dopri(FHN, RING, 50, 10, 0, 0, 0, NULL, NULL, NULL, fprm, NULL, y, 1.0, 1e-6, 1e-9, 1e-3,
                            100000, stats) == 0);
        CHECK(orc_run_dopri(KUR, RING, 50, 10, 0, 0, 0, NULL, NULL, NULL, kprm, NULL, y, 0.5, 0.0, 0.0, 0.01,
                            100000, stats) == 0);
        CHECK(orc_run_dopri_dense(INERTIA, RING, 50, 10, 0, 0, 0, NULL, NULL, NULL, iprm, NULL, y, 2.0, 1e-8, 1e-10,
                                  1e-3, 100000, stats, 0.25, Rout, Yout) == 0);
        CHECK(finite_all(Rout, 9));
        y[7] = NAN;
        CHECK(orc_run_dopri(FHN, RING, 50, 10, 0, 0, 0, NULL, NULL, NULL, fprm, NULL, y, 1.0, 1e-6, 1e-9, 1e-3,
                            100000, stats) != 0);
        free(y);
    }
    printf("oracle clean\n");
    return 0;
}
