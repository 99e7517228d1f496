/*
 * Calls every exported function of oracle/oracle.c on small inputs, with the
 * edge cases the pins use (empty target lists, a single particle, zero and
 * non-finite tidal tensors), and checks a few identities that hold for any
 * input.  Built together with oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py; a sanitizer
 * report or a failed check ends the program with a non-zero status.
 *
 * Test infrastructure only: nothing in the library links this file.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_kernel(int64_t n, const double *r, double h, double *f, double *D, double *W);
void orc_field(int64_t n, const double *x, const double *v, const double *m, double eps, double G,
               int64_t np, const double *p, const double *pv, const int64_t *excl,
               double *acc, double *jerk, double *tidal);
void orc_direct_box(int64_t n, const double *x, const double *v, const double *m, double eps, double G,
                    double box, int64_t ntgt, const int64_t *tgt, double *acc, double *jerk, double *tidal);
void orc_direct(int64_t n, const double *x, const double *v, const double *m, double eps, double G,
                int64_t ntgt, const int64_t *tgt, double *acc, double *jerk, double *tidal);
void orc_abs_scale_box(int64_t n, const double *x, const double *m, double eps, double G, double box,
                       int64_t ntgt, const int64_t *tgt, double *scale);
void orc_abs_scale(int64_t n, const double *x, const double *m, double eps, double G,
                   int64_t ntgt, const int64_t *tgt, double *scale);
void orc_field_soft(int64_t n, const double *x, const double *v, const double *m, const double *hs,
                    double G, int64_t np, const double *p, const double *pv, const double *hp,
                    const int64_t *excl, double *acc, double *jerk, double *tidal);
void orc_ewald_unit(int64_t n, const double *d, double L, double alpha, int nr, int nk,
                    double *g, double *T, double *dg, double *dT);
void orc_direct_ewald(int64_t n, const double *x, const double *v, const double *m, double eps, double G,
                      double box, int64_t ntgt, const int64_t *tgt, double *acc, double *jerk, double *tidal);
void orc_timestep(int64_t n, const double *tidal, double eta, double dt_max, int32_t k_max,
                  double *dt_grav, int8_t *bin);
int64_t orc_select(int64_t n, int64_t *tf, const int8_t *bin, int64_t step_ticks, int32_t tick_bin,
                   double q_f, uint8_t *active);
void orc_predict(int64_t n, const double *a0, const double *jerk, const double *t0, double t, double *acc);
void orc_adjoint(int64_t n, const double *x, const double *m, const double *w, double eps, double G,
                 int64_t nk, const int64_t *kidx, double *dldx, double *dldm);
void orc_moments(int64_t cnt, const int64_t *idx, const double *x, const double *v, const double *m,
                 double *out);
int orc_num_threads(void);
void orc_set_threads(int k);

static int failures = 0;
#define CHECK(cond, what)                                           \
    do {                                                            \
        if (!(cond)) {                                              \
            fprintf(stderr, "check failed: %s (%s:%d)\n", what, __FILE__, __LINE__); \
            ++failures;                                             \
        }                                                           \
    } while (0)

/* a fixed linear congruential sequence in [0, 1) (no libc state) */
static uint64_t lcg_state = 12345u;
static double urand(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static int all_finite(const double *a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

enum { N = 11 };

int main(void)
{
    double x[3 * N], v[3 * N], m[N], w[3 * N];
    int64_t all[N];
    for (int i = 0; i < N; ++i) {
        for (int c = 0; c < 3; ++c) {
            x[3 * i + c] = urand();
            v[3 * i + c] = urand() - 0.5;
            w[3 * i + c] = urand() - 0.5;
        }
        m[i] = 0.5 + urand();
        all[i] = i;
    }
    const double eps = 0.05, G = 1.0;

    /* kernel: Newtonian (f = 1/r^3, D = -3/r^5) at and beyond the softening length */
    {
        const double h = 0.2, r[6] = {0.0, 0.03, 0.1, 0.19, 0.2, 0.4};
        double f[6], D[6], Wk[6];
        orc_kernel(6, r, h, f, D, Wk);
        CHECK(all_finite(f, 6) && all_finite(D, 6) && all_finite(Wk, 6), "kernel finite");
        for (int k = 4; k < 6; ++k) {
            CHECK(fabs(f[k] * r[k] * r[k] * r[k] - 1.0) < 1e-13, "kernel f Newtonian");
            CHECK(fabs(-D[k] * pow(r[k], 5) / 3.0 - 1.0) < 1e-13, "kernel D Newtonian");
        }
    }

    /* direct sum over every particle: finite, and sum m a = 0 (pairwise equal and opposite) */
    double acc[3 * N], jerk[3 * N], tid[6 * N], scale[N];
    {
        orc_direct(N, x, v, m, eps, G, N, all, acc, jerk, tid);
        CHECK(all_finite(acc, 3 * N) && all_finite(jerk, 3 * N) && all_finite(tid, 6 * N), "direct finite");
        for (int c = 0; c < 3; ++c) {
            double s = 0.0, sa = 0.0;
            for (int i = 0; i < N; ++i) {
                s += m[i] * acc[3 * i + c];
                sa += fabs(m[i] * acc[3 * i + c]);
            }
            CHECK(fabs(s) <= 1e-12 * sa, "momentum");
        }
        orc_abs_scale(N, x, m, eps, G, N, all, scale);
        for (int i = 0; i < N; ++i) {
            const double a = sqrt(acc[3 * i] * acc[3 * i] + acc[3 * i + 1] * acc[3 * i + 1] +
                                  acc[3 * i + 2] * acc[3 * i + 2]);
            CHECK(a <= scale[i] * (1.0 + 1e-12), "scale bounds |a|");
        }
        /* empty target list and a single particle */
        orc_direct(N, x, v, m, eps, G, 0, all, acc, jerk, tid);
        orc_direct(1, x, v, m, eps, G, 1, all, acc, jerk, tid);
        CHECK(acc[0] == 0.0 && acc[1] == 0.0 && acc[2] == 0.0, "lone particle feels nothing");
    }

    /* periodic: nearest image and Ewald */
    {
        orc_direct_box(N, x, v, m, eps, G, 1.0, N, all, acc, jerk, tid);
        CHECK(all_finite(acc, 3 * N) && all_finite(tid, 6 * N), "box finite");
        orc_abs_scale_box(N, x, m, eps, G, 1.0, N, all, scale);
        CHECK(all_finite(scale, N), "box scale finite");
        orc_direct_ewald(5, x, v, m, eps, G, 1.0, 5, all, acc, jerk, tid);
        CHECK(all_finite(acc, 15) && all_finite(jerk, 15) && all_finite(tid, 30), "ewald finite");
        const double d[9] = {0.0, 0.0, 0.0, 0.1, -0.2, 0.3, 0.5, 0.5, 0.5};
        double g[9], T[18], dg[9], dT[18];
        orc_ewald_unit(3, d, 1.0, 2.0, 3, 4, g, T, dg, dT);
        CHECK(all_finite(dg, 9) && all_finite(dT, 18), "ewald unit finite");
        /* at zero separation: no correction force (by symmetry, up to rounding), and the
         * tide of the neutralising background, 4 pi / 3 per unit volume, on the diagonal */
        CHECK(fabs(dg[0]) + fabs(dg[1]) + fabs(dg[2]) < 1e-12, "no correction force at zero separation");
        for (int c = 0; c < 3; ++c) CHECK(fabs(dT[c] - 4.0 * 3.14159265358979323846 / 3.0) < 1e-10, "background tide");
    }

    /* per-particle softening with every length equal to eps reproduces the single-length field */
    {
        double hs[N], a2[3 * N], j2[3 * N], t2[6 * N];
        for (int i = 0; i < N; ++i) hs[i] = eps;
        orc_field(N, x, v, m, eps, G, N, x, v, all, acc, jerk, tid);
        orc_field_soft(N, x, v, m, hs, G, N, x, v, hs, all, a2, j2, t2);
        for (int i = 0; i < 3 * N; ++i)
            CHECK(fabs(a2[i] - acc[i]) <= 1e-13 * (fabs(acc[i]) + 1e-300) + 1e-300, "soft == single length");
        orc_field_soft(N, x, v, m, hs, G, 0, x, v, hs, NULL, a2, j2, t2);
    }

    /* timestep bins: zero tensor -> bin 0, non-finite -> k_max, all in range */
    {
        double T[6 * 4] = {0};
        for (int k = 0; k < 6; ++k) T[6 + k] = 1e3 * (k + 1);
        for (int k = 0; k < 6; ++k) T[12 + k] = 1e-3 * (k + 1);
        T[18] = NAN;
        double dt[4];
        int8_t bin[4];
        orc_timestep(4, T, 0.01, 0.0625, 20, dt, bin);
        CHECK(bin[0] == 0, "zero tensor bin");
        CHECK(bin[3] == 20, "non-finite tensor bin");
        for (int k = 0; k < 4; ++k) CHECK(bin[k] >= 0 && bin[k] <= 20, "bin range");
    }

    /* Eq. 3-4 bookkeeping: counts agree with the flags; predictor exact for zero jerk */
    {
        int64_t tf[N];
        int8_t bin[N];
        uint8_t act[N];
        for (int i = 0; i < N; ++i) {
            tf[i] = i;
            bin[i] = (int8_t)(i % 5);
        }
        for (int s = 0; s < 6; ++s) {
            const int64_t cnt = orc_select(N, tf, bin, 1, 4, 0.25, act);
            int64_t c2 = 0;
            for (int i = 0; i < N; ++i) c2 += act[i];
            CHECK(cnt == c2, "select count");
        }
        double a0[3 * N], jz[3 * N], t0[N], out[3 * N];
        for (int i = 0; i < 3 * N; ++i) {
            a0[i] = urand();
            jz[i] = 0.0;
        }
        for (int i = 0; i < N; ++i) t0[i] = 0.1 * i;
        orc_predict(N, a0, jz, t0, 2.0, out);
        CHECK(memcmp(a0, out, sizeof(a0)) == 0, "zero-jerk prediction");
    }

    /* adjoint and moments */
    {
        double dx[3 * N], dm[N], mo[25];
        orc_adjoint(N, x, m, w, eps, G, N, all, dx, dm);
        CHECK(all_finite(dx, 3 * N) && all_finite(dm, N), "adjoint finite");
        orc_adjoint(N, x, m, w, eps, G, 0, all, dx, dm);
        orc_moments(N, all, x, v, m, mo);
        double M = 0.0;
        for (int i = 0; i < N; ++i) M += m[i];
        CHECK(fabs(mo[0] - M) <= 1e-14 * M, "moment mass");
        CHECK(fabs(mo[7] + mo[8] + mo[9]) <= 1e-12 * (fabs(mo[7]) + fabs(mo[8]) + fabs(mo[9])),
              "quadrupole traceless");
        CHECK(fabs(mo[13] + mo[14] + mo[15]) <= 1e-12 * (fabs(mo[13]) + fabs(mo[14]) + fabs(mo[15]) + 1e-300),
              "quadrupole rate traceless");
    }

    orc_set_threads(2);
    CHECK(orc_num_threads() >= 1, "threads");
    orc_set_threads(0);

    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitize run: all checks passed\n");
    return 0;
}
