/*
 * oracle.c -- plain, slow FP64 reference for the adaptive-force-update gravity
 * path of Grudic (2020), "Accelerating self-gravitating hydrodynamics
 * simulations with adaptive force updates".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the HIP path.
 *
 * Every routine is the textbook definition written out in double precision,
 * looping over all pairs in index order with no blocking, reordering or
 * approximation:
 *
 *   - field():      softened direct sum for acceleration g, jerk j = dg/dt
 *                   (the discretised form of the paper's jerk integral,
 *                   Sec. 2.2, Eq. 5) and tidal tensor T = grad g (Sec. 3,
 *                   Eq. 7 uses its Frobenius norm).
 *   - timestep():   tidal timestep Eq. 7 and its power-of-two block bin
 *                   (the hierarchical block steps of Sec. 3).
 *   - select():     force-age counter Eq. 3 and update test Eq. 4 (Sec. 2.1).
 *   - predict():    first-order jerk predictor Eq. 6 in closed form
 *                   a0 + j (t - t0) (Sec. 2.2).
 *   - adjoint():    exact gradient of L = sum_i w_i . a_i with respect to
 *                   positions and masses (not in the paper; the analytic
 *                   derivative of the direct sum above).
 *   - moments():    mass, centre of mass, mean velocity, traceless quadrupole
 *                   and its time derivative for a particle set (the node
 *                   multipoles of an oct-tree, Sec. 3).
 *
 * Softening kernel (a reading; the paper only says softening follows the
 * hydro kernel): cubic-spline M4 density kernel with compact support h = eps,
 * W(r) = 8/(pi h^3) w(u), u = r/h,
 *     w = 1 - 6u^2 + 6u^3 (u < 1/2), 2(1-u)^3 (1/2 <= u < 1), 0 (u >= 1).
 * The pair force factor is f(r) = mu(u)/r^3, mu(u) the kernel mass inside r,
 * so g_i = G sum_j m_j f(r) d_ij with d_ij = x_j - x_i; D(r) = f'(r)/r.
 * Written in the u^3-cancelled form, exactly equal algebraically:
 *     u < 1/2:   f = h^-3 (32/3 - 192/5 u^2 + 32 u^3),  D = h^-5 (96u - 384/5)
 *     1/2<=u<1:  f = h^-3 (64/3 - 48u + 192/5 u^2 - 32/3 u^3 - 1/(15u^3)),
 *                D = h^-5 (-48/u + 384/5 - 32u + 1/(5u^5))
 *     u >= 1:    f = r^-3, D = -3 r^-5 (Newtonian).
 * The self pair (j == i) is excluded from every sum.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ---- softening kernel --------------------------------------------------- */

static void kernel_fd(double r, double h, double *f, double *D)
{
    if (r >= h) {
        double r2 = r * r;
        *f = 1.0 / (r2 * r);
        *D = -3.0 / (r2 * r2 * r);
        return;
    }
    double hi = 1.0 / h;
    double h3 = hi * hi * hi;
    double h5 = h3 * hi * hi;
    double u = r * hi;
    if (u < 0.5) {
        *f = h3 * (32.0 / 3.0 - 192.0 / 5.0 * u * u + 32.0 * u * u * u);
        *D = h5 * (96.0 * u - 384.0 / 5.0);
    } else {
        double u3 = u * u * u;
        *f = h3 * (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u * u
                   - 32.0 / 3.0 * u3 - 1.0 / (15.0 * u3));
        *D = h5 * (-48.0 / u + 384.0 / 5.0 - 32.0 * u + 1.0 / (5.0 * u3 * u * u));
    }
}

static double kernel_w(double r, double h)
{
    double u = r / h;
    double c = 8.0 / (ORC_PI * h * h * h);
    if (u < 0.5) return c * (1.0 - 6.0 * u * u + 6.0 * u * u * u);
    if (u < 1.0) { double t = 1.0 - u; return c * 2.0 * t * t * t; }
    return 0.0;
}

/* Exported for the kernel pins: f, D and W at separation r. */
void orc_kernel(int64_t n, const double *r, double h, double *f, double *D, double *W)
{
    for (int64_t k = 0; k < n; ++k) {
        kernel_fd(r[k], h, &f[k], &D[k]);
        W[k] = kernel_w(r[k], h);
    }
}

/* ---- direct-sum field ---------------------------------------------------- */
/*
 * Field at np probe points p (np x 3, row-major) moving with velocity pv, due
 * to n sources (x, v: n x 3 row-major; m: n).  excl[k] names a source index
 * skipped for probe k (the probe's own particle), or -1; excl may be NULL.
 * Outputs (np rows): acc (3), jerk (3), tidal (6: xx yy zz xy xz yz).
 *
 *   g  =  G sum_j m_j f d
 *   j  =  G sum_j m_j [ f nu + D (d.nu) d ]          nu = v_j - pv
 *   T  = -G sum_j m_j [ f I  + D d d^T ]             (T = grad g)
 */
/* Nearest periodic image of a separation in a cubic box of side L:
 * d - L * round(d / L), ties to even (L <= 0: no box, d unchanged). */
static double nearest_image(double d, double L)
{
    if (L <= 0) return d;
    return d - L * nearbyint(d / L);
}

void orc_field_box(int64_t n, const double *x, const double *v, const double *m,
                   double eps, double G, double box,
                   int64_t np, const double *p, const double *pv, const int64_t *excl,
                   double *acc, double *jerk, double *tidal)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < np; ++k) {
        double px = p[3 * k], py = p[3 * k + 1], pz = p[3 * k + 2];
        double qx = pv[3 * k], qy = pv[3 * k + 1], qz = pv[3 * k + 2];
        int64_t skip = excl ? excl[k] : -1;
        double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0;
        double txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == skip) continue;
            double dx = nearest_image(x[3 * j] - px, box);
            double dy = nearest_image(x[3 * j + 1] - py, box);
            double dz = nearest_image(x[3 * j + 2] - pz, box);
            double nx = v[3 * j] - qx, ny = v[3 * j + 1] - qy, nz = v[3 * j + 2] - qz;
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double f, D;
            kernel_fd(r, eps, &f, &D);
            double mj = m[j];
            double dn = dx * nx + dy * ny + dz * nz;
            ax += mj * f * dx; ay += mj * f * dy; az += mj * f * dz;
            jx += mj * (f * nx + D * dn * dx);
            jy += mj * (f * ny + D * dn * dy);
            jz += mj * (f * nz + D * dn * dz);
            txx -= mj * (f + D * dx * dx);
            tyy -= mj * (f + D * dy * dy);
            tzz -= mj * (f + D * dz * dz);
            txy -= mj * (D * dx * dy);
            txz -= mj * (D * dx * dz);
            tyz -= mj * (D * dy * dz);
        }
        acc[3 * k] = G * ax; acc[3 * k + 1] = G * ay; acc[3 * k + 2] = G * az;
        jerk[3 * k] = G * jx; jerk[3 * k + 1] = G * jy; jerk[3 * k + 2] = G * jz;
        tidal[6 * k] = G * txx; tidal[6 * k + 1] = G * tyy; tidal[6 * k + 2] = G * tzz;
        tidal[6 * k + 3] = G * txy; tidal[6 * k + 4] = G * txz; tidal[6 * k + 5] = G * tyz;
    }
}

void orc_field(int64_t n, const double *x, const double *v, const double *m,
               double eps, double G,
               int64_t np, const double *p, const double *pv, const int64_t *excl,
               double *acc, double *jerk, double *tidal)
{
    orc_field_box(n, x, v, m, eps, G, 0.0, np, p, pv, excl, acc, jerk, tidal);
}

/* Direct sum at the particles listed in tgt (self excluded); outputs have
 * ntgt rows in the order of tgt.  box > 0: every pair at its nearest
 * periodic image in a cube of that side. */
void orc_direct_box(int64_t n, const double *x, const double *v, const double *m,
                    double eps, double G, double box, int64_t ntgt, const int64_t *tgt,
                    double *acc, double *jerk, double *tidal)
{
    double *p = (double *)malloc(sizeof(double) * 3 * (size_t)(ntgt > 0 ? ntgt : 1));
    double *q = (double *)malloc(sizeof(double) * 3 * (size_t)(ntgt > 0 ? ntgt : 1));
    for (int64_t k = 0; k < ntgt; ++k)
        for (int c = 0; c < 3; ++c) {
            p[3 * k + c] = x[3 * tgt[k] + c];
            q[3 * k + c] = v[3 * tgt[k] + c];
        }
    orc_field_box(n, x, v, m, eps, G, box, ntgt, p, q, tgt, acc, jerk, tidal);
    free(p);
    free(q);
}

void orc_direct(int64_t n, const double *x, const double *v, const double *m,
                double eps, double G, int64_t ntgt, const int64_t *tgt,
                double *acc, double *jerk, double *tidal)
{
    orc_direct_box(n, x, v, m, eps, G, 0.0, ntgt, tgt, acc, jerk, tidal);
}

/* Sum of |pair acceleration terms| G sum_j m_j |f d|, the scale against which
 * the FP64 direct sum's cancellation error is normalised. */
void orc_abs_scale_box(int64_t n, const double *x, const double *m, double eps, double G, double box,
                       int64_t ntgt, const int64_t *tgt, double *scale)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ntgt; ++k) {
        int64_t i = tgt[k];
        double s = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = nearest_image(x[3 * j] - x[3 * i], box);
            double dy = nearest_image(x[3 * j + 1] - x[3 * i + 1], box);
            double dz = nearest_image(x[3 * j + 2] - x[3 * i + 2], box);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double f, D;
            kernel_fd(r, eps, &f, &D);
            s += m[j] * f * r;
        }
        scale[k] = G * s;
    }
}

void orc_abs_scale(int64_t n, const double *x, const double *m, double eps, double G,
                   int64_t ntgt, const int64_t *tgt, double *scale)
{
    orc_abs_scale_box(n, x, m, eps, G, 0.0, ntgt, tgt, scale);
}

/* ---- per-particle softening ---------------------------------------------- */
/*
 * Softening lengths that differ between particles (the paper's fully
 * adaptive softening, Sec. 3, with the lengths given): the pair kernel is
 * the mean of the two particles' kernels, so the pair force stays equal and
 * opposite,
 *   f_ij = (f(r, h_i) + f(r, h_j)) / 2,   D_ij = (D(r, h_i) + D(r, h_j)) / 2,
 * and g, j, T follow from f_ij and D_ij exactly as with one softening.
 * hs (n) holds the sources' lengths, hp (np) the probes'.
 */
void orc_field_soft(int64_t n, const double *x, const double *v, const double *m, const double *hs,
                    double G, int64_t np, const double *p, const double *pv, const double *hp,
                    const int64_t *excl, double *acc, double *jerk, double *tidal)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < np; ++k) {
        double px = p[3 * k], py = p[3 * k + 1], pz = p[3 * k + 2];
        double qx = pv[3 * k], qy = pv[3 * k + 1], qz = pv[3 * k + 2];
        int64_t skip = excl ? excl[k] : -1;
        double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0;
        double txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == skip) continue;
            double dx = x[3 * j] - px, dy = x[3 * j + 1] - py, dz = x[3 * j + 2] - pz;
            double nx = v[3 * j] - qx, ny = v[3 * j + 1] - qy, nz = v[3 * j + 2] - qz;
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double f1, D1, f2, D2;
            kernel_fd(r, hp[k], &f1, &D1);
            kernel_fd(r, hs[j], &f2, &D2);
            double f = 0.5 * (f1 + f2), D = 0.5 * (D1 + D2);
            double mj = m[j];
            double dn = dx * nx + dy * ny + dz * nz;
            ax += mj * f * dx; ay += mj * f * dy; az += mj * f * dz;
            jx += mj * (f * nx + D * dn * dx);
            jy += mj * (f * ny + D * dn * dy);
            jz += mj * (f * nz + D * dn * dz);
            txx -= mj * (f + D * dx * dx);
            tyy -= mj * (f + D * dy * dy);
            tzz -= mj * (f + D * dz * dz);
            txy -= mj * (D * dx * dy);
            txz -= mj * (D * dx * dz);
            tyz -= mj * (D * dy * dz);
        }
        acc[3 * k] = G * ax; acc[3 * k + 1] = G * ay; acc[3 * k + 2] = G * az;
        jerk[3 * k] = G * jx; jerk[3 * k + 1] = G * jy; jerk[3 * k + 2] = G * jz;
        tidal[6 * k] = G * txx; tidal[6 * k + 1] = G * tyy; tidal[6 * k + 2] = G * tzz;
        tidal[6 * k + 3] = G * txy; tidal[6 * k + 4] = G * txz; tidal[6 * k + 5] = G * tyz;
    }
}

/* ---- Ewald summation in a periodic cube ----------------------------------- */
#define ORC_PI 3.14159265358979323846
/*
 * Field of a unit mass (G = 1) and all its periodic images in a cube of side
 * L, with a uniform neutralising background (the k = 0 mode removed), at
 * separation d = x_source - x_target, split with parameter alpha:
 *   g(d) = sum_n B(|d_n|) d_n
 *          + (4 pi / L^3) sum_{k != 0} k / k^2 exp(-k^2 / (4 alpha^2)) sin(k.d),
 *   d_n = d + n L,  B(r) = erfc(alpha r) / r^3 + (2 alpha / sqrt(pi)) exp(-alpha^2 r^2) / r^2,
 *   T(d) = dg / dx_target = -grad_d g
 *        = -sum_n [B I + (B'(r) / r) d_n d_n^T]
 *          - (4 pi / L^3) sum_{k != 0} k k^T / k^2 exp(-k^2 / (4 alpha^2)) cos(k.d),
 *   B'(r) = -3 erfc(alpha r) / r^4 - (2 alpha / sqrt(pi)) exp(-alpha^2 r^2) (3 / r^3 + 2 alpha^2 / r),
 * over images |n_a| <= nr and wave vectors k = 2 pi h / L, |h_a| <= nk.
 * The correction is what the periodic field adds to the Newtonian field of
 * the single image d:  dg = g - d / r^3,  dT = T + (I / r^3 - 3 d d^T / r^5).
 * In the n = 0 term the Newtonian part is subtracted analytically: with
 * z = alpha r, h(r) = B(r) - 1/r^3 has the series
 *   h = (2 / sqrt(pi)) sum_{k >= 1} (-1)^k 2k / ((2k + 1) k!) alpha^(2k+1) r^(2k-2),
 * used for z < 0.5 (the closed form loses digits to cancellation there), so
 * the correction is exact to rounding down to d = 0, where dg = 0 and dT is
 * the background's tide.
 */
static void ewald_h(double r, double alpha, double *h, double *hp_r)
{
    const double sp = 2.0 / sqrt(ORC_PI);
    const double z = alpha * r;
    if (z < 0.5) {
        /* h = sp sum_{k>=1} c_k r^(2k-2) and h'(r)/r = sp sum_{k>=2} c_k (2k-2) r^(2k-4),
         * c_k = (-1)^k 2k / ((2k+1) k!) alpha^(2k+1); terms fall like z^(2k) / k! */
        double sh = 0.0, shp = 0.0;
        double ak = alpha * alpha * alpha;   /* alpha^(2k+1) */
        double fact = 1.0;                   /* k! */
        double rp = 1.0;                     /* r^(2k-2) */
        double rq = 1.0;                     /* r^(2k-4), from k = 2 */
        for (int k = 1; k <= 30; ++k) {
            if (k > 1) {
                ak *= alpha * alpha;
                fact *= k;
                rp *= r * r;
            }
            if (k > 2) rq *= r * r;
            const double c = ((k & 1) ? -1.0 : 1.0) * (2.0 * k) / ((2.0 * k + 1.0) * fact) * ak;
            sh += c * rp;
            if (k >= 2) shp += c * (2.0 * k - 2.0) * rq;
        }
        *h = sp * sh;
        *hp_r = sp * shp;
        return;
    }
    const double e = exp(-z * z);
    const double ec = erfc(z);
    const double r2 = r * r, r3 = r2 * r;
    const double B = ec / r3 + sp * alpha * e / r2;
    const double Bp = -3.0 * ec / (r2 * r2) - sp * alpha * e * (3.0 / r3 + 2.0 * alpha * alpha / r);
    *h = B - 1.0 / r3;
    *hp_r = (Bp + 3.0 / (r2 * r2)) / r;
}

/* Periodic field g, T of a unit mass at separation d and its correction dg,
 * dT to the single image (see above).  T and dT in xx yy zz xy xz yz order. */
static void ewald_unit(const double d[3], double L, double alpha, int nr, int nk,
                       double g[3], double T[6], double dg[3], double dT[6])
{
    const double sp = 2.0 / sqrt(ORC_PI);
    double gs[3] = {0, 0, 0}, ts[6] = {0, 0, 0, 0, 0, 0};
    for (int a = -nr; a <= nr; ++a)
        for (int b = -nr; b <= nr; ++b)
            for (int c = -nr; c <= nr; ++c) {
                const double y[3] = {d[0] + a * L, d[1] + b * L, d[2] + c * L};
                const double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
                double Bv, Bp_r;
                if (a == 0 && b == 0 && c == 0) {
                    /* the single image itself, Newtonian part removed */
                    ewald_h(r, alpha, &Bv, &Bp_r);
                } else {
                    const double z = alpha * r, e = exp(-z * z), ec = erfc(z);
                    const double r2 = r * r, r3 = r2 * r;
                    Bv = ec / r3 + sp * alpha * e / r2;
                    Bp_r = (-3.0 * ec / (r2 * r2) - sp * alpha * e * (3.0 / r3 + 2.0 * alpha * alpha / r)) / r;
                }
                for (int q = 0; q < 3; ++q) gs[q] += Bv * y[q];
                ts[0] -= Bv + Bp_r * y[0] * y[0];
                ts[1] -= Bv + Bp_r * y[1] * y[1];
                ts[2] -= Bv + Bp_r * y[2] * y[2];
                ts[3] -= Bp_r * y[0] * y[1];
                ts[4] -= Bp_r * y[0] * y[2];
                ts[5] -= Bp_r * y[1] * y[2];
            }
    const double pre = 4.0 * ORC_PI / (L * L * L);
    const double kf = 2.0 * ORC_PI / L;
    for (int a = -nk; a <= nk; ++a)
        for (int b = -nk; b <= nk; ++b)
            for (int c = -nk; c <= nk; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                const double k[3] = {kf * a, kf * b, kf * c};
                const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                const double w = pre * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                const double ph = k[0] * d[0] + k[1] * d[1] + k[2] * d[2];
                const double sn = sin(ph), cs = cos(ph);
                for (int q = 0; q < 3; ++q) gs[q] += w * k[q] * sn;
                ts[0] -= w * k[0] * k[0] * cs;
                ts[1] -= w * k[1] * k[1] * cs;
                ts[2] -= w * k[2] * k[2] * cs;
                ts[3] -= w * k[0] * k[1] * cs;
                ts[4] -= w * k[0] * k[2] * cs;
                ts[5] -= w * k[1] * k[2] * cs;
            }
    /* gs, ts hold the correction (n = 0 entered without its Newtonian part) */
    for (int q = 0; q < 3; ++q) dg[q] = gs[q];
    for (int q = 0; q < 6; ++q) dT[q] = ts[q];
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r > 0) {
        const double r3 = r * r * r, r5 = r3 * r * r;
        for (int q = 0; q < 3; ++q) g[q] = dg[q] + d[q] / r3;
        T[0] = dT[0] - (1.0 / r3 - 3.0 * d[0] * d[0] / r5);
        T[1] = dT[1] - (1.0 / r3 - 3.0 * d[1] * d[1] / r5);
        T[2] = dT[2] - (1.0 / r3 - 3.0 * d[2] * d[2] / r5);
        T[3] = dT[3] + 3.0 * d[0] * d[1] / r5;
        T[4] = dT[4] + 3.0 * d[0] * d[2] / r5;
        T[5] = dT[5] + 3.0 * d[1] * d[2] / r5;
    } else {
        for (int q = 0; q < 3; ++q) g[q] = NAN;
        for (int q = 0; q < 6; ++q) T[q] = NAN;
    }
}

void orc_ewald_unit(int64_t n, const double *d, double L, double alpha, int nr, int nk,
                    double *g, double *T, double *dg, double *dT)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        ewald_unit(d + 3 * i, L, alpha, nr, nk, g + 3 * i, T + 6 * i, dg + 3 * i, dT + 6 * i);
}

/* Periodic direct sum with Ewald's method for g and T (the jerk keeps the
 * nearest image only, as Sec. 3.4 states for its periodic problem):
 *   g_i = G sum_{j != i} m_j f(r) d_ij  +  G sum_j m_j dg(d_ij),
 *   T_i = (nearest-image T)             +  G sum_j m_j dT(d_ij),
 * d_ij the nearest image; the softened single-image terms as in
 * orc_direct_box; the correction sums include j = i (dg(0) = 0, dT(0) the
 * tide of the background that neutralises particle i's own images).
 * alpha = 2 / L, images |n_a| <= 3, wave vectors |h_a| <= 4 (omitted terms
 * below 1e-20 of the kept ones). */
void orc_direct_ewald(int64_t n, const double *x, const double *v, const double *m,
                      double eps, double G, double box, int64_t ntgt, const int64_t *tgt,
                      double *acc, double *jerk, double *tidal)
{
    orc_direct_box(n, x, v, m, eps, G, box, ntgt, tgt, acc, jerk, tidal);
    const double alpha = 2.0 / box;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < ntgt; ++k) {
        const int64_t i = tgt[k];
        double sg[3] = {0, 0, 0}, st[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double d[3];
            for (int q = 0; q < 3; ++q) d[q] = nearest_image(x[3 * j + q] - x[3 * i + q], box);
            double g[3], T[6], dg[3], dT[6];
            ewald_unit(d, box, alpha, 3, 4, g, T, dg, dT);
            for (int q = 0; q < 3; ++q) sg[q] += m[j] * dg[q];
            for (int q = 0; q < 6; ++q) st[q] += m[j] * dT[q];
        }
        for (int q = 0; q < 3; ++q) acc[3 * k + q] += G * sg[q];
        for (int q = 0; q < 6; ++q) tidal[6 * k + q] += G * st[q];
    }
}

/* ---- tidal timestep (Eq. 7) and block bin --------------------------------- */
/*
 * dt_grav = sqrt(eta) * (|T|_F^2 / 6)^(-1/4),
 * |T|_F^2 = Txx^2 + Tyy^2 + Tzz^2 + 2 (Txy^2 + Txz^2 + Tyz^2).
 * Bin: the smallest k >= 0 with dt_max 2^-k <= dt_grav, clamped to k_max;
 * |T| = 0 gives k = 0 (dt_max).  The bin is decided on the exactly defined
 * ratio Q = (dt_max/dt_grav)^4 = |T|^2 dt_max^4 / (6 eta^2), evaluated as
 *     a = dt_max*dt_max; b = a*a; e2 = eta*eta; Q = (n2*b)/(6*e2)
 * with each operation rounded once (no fused multiply-add), and
 * dt_max 2^-k <= dt_grav  <=>  Q <= 2^(4k).
 * Non-finite Q (a non-finite tensor) is put in bin k_max.
 */
static int bin_of(double n2, double eta, double dt_max, int k_max)
{
    double a = dt_max * dt_max;
    double b = a * a;
    double e2 = eta * eta;
    double den = 6.0 * e2;
    double num = n2 * b;
    double Q = num / den;
    if (!(Q == Q) || Q > 1.7976931348623157e308) return k_max;
    if (Q <= 0.0) return 0;
    int e;
    double fr = frexp(Q, &e);            /* Q = fr 2^e, fr in [1/2, 1) */
    int mexp = (fr == 0.5) ? e - 1 : e;  /* smallest integer m with Q <= 2^m */
    int k = mexp <= 0 ? 0 : (mexp + 3) / 4;
    if (k > k_max) k = k_max;
    return k;
}

void orc_timestep(int64_t n, const double *tidal, double eta, double dt_max, int32_t k_max,
                  double *dt_grav, int8_t *bin)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *t = tidal + 6 * i;
        double d2 = t[0] * t[0] + t[1] * t[1];
        d2 = d2 + t[2] * t[2];
        double o2 = t[3] * t[3] + t[4] * t[4];
        o2 = o2 + t[5] * t[5];
        double n2 = d2 + 2.0 * o2;
        dt_grav[i] = (n2 > 0.0) ? sqrt(eta) * pow(n2 / 6.0, -0.25) : INFINITY;
        bin[i] = (int8_t)bin_of(n2, eta, dt_max, k_max);
    }
}

/* ---- force-age bookkeeping (Eq. 3, Eq. 4) -------------------------------- */
/*
 * Integer time: one tick is the step of bin `tick_bin`, so bin k spans
 * 2^(tick_bin - min(k, tick_bin)) ticks.  At the start of a step, for every
 * particle: T_f += step_ticks (Eq. 3); it is due iff T_f >= q_f dt_bin
 * (Eq. 4, inclusive); a due particle gets T_f = 0.  active[i] is set to 1 for
 * due particles and 0 otherwise; returns the number due.
 */
int64_t orc_select(int64_t n, int64_t *tf, const int8_t *bin, int64_t step_ticks,
                   int32_t tick_bin, double q_f, uint8_t *active)
{
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i) {
        int k = bin[i];
        if (k > tick_bin) k = tick_bin;
        if (k < 0) k = 0;
        int64_t span = (int64_t)1 << (tick_bin - k);
        tf[i] += step_ticks;
        double thresh = q_f * (double)span;
        if ((double)tf[i] >= thresh) {
            active[i] = 1;
            tf[i] = 0;
            ++count;
        } else {
            active[i] = 0;
        }
    }
    return count;
}

/* ---- jerk predictor (Eq. 6), closed form ----------------------------------- */
/* acc = a0 + j (t - t0), row by row; each operation rounded once. */
void orc_predict(int64_t n, const double *a0, const double *jerk, const double *t0, double t,
                 double *acc)
{
    for (int64_t i = 0; i < n; ++i) {
        double dt = t - t0[i];
        for (int c = 0; c < 3; ++c) {
            double jd = jerk[3 * i + c] * dt;
            acc[3 * i + c] = a0[3 * i + c] + jd;
        }
    }
}

/* ---- adjoint of L = sum_i w_i . a_i ----------------------------------------- */
/*
 * For each listed particle k:
 *   dL/dx_k = G m_k sum_{j != k} J(d_kj) w_j  +  T_k w_k,
 *   dL/dm_k = -G sum_{j != k} f(r_kj) d_kj . w_j,
 * with d_kj = x_j - x_k, J = f I + D d d^T, and T_k the tidal tensor at k.
 * Derivation: a_i depends on x_k through the pair (i, k) twice -- as the
 * target (i = k, giving T_k w_k) and as a source (j = k, giving
 * G m_k J(x_k - x_i) w_i, and J is even in d).
 */
void orc_adjoint(int64_t n, const double *x, const double *m, const double *w,
                 double eps, double G, int64_t nk, const int64_t *kidx,
                 double *dldx, double *dldm)
{
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nk; ++t) {
        int64_t k = kidx[t];
        double vx = 0, vy = 0, vz = 0, s = 0;
        double txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            double dx = x[3 * j] - x[3 * k], dy = x[3 * j + 1] - x[3 * k + 1],
                   dz = x[3 * j + 2] - x[3 * k + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double f, D;
            kernel_fd(r, eps, &f, &D);
            double wx = w[3 * j], wy = w[3 * j + 1], wz = w[3 * j + 2];
            double dw = dx * wx + dy * wy + dz * wz;
            vx += f * wx + D * dw * dx;
            vy += f * wy + D * dw * dy;
            vz += f * wz + D * dw * dz;
            s += f * dw;
            double mj = m[j];
            txx -= mj * (f + D * dx * dx);
            tyy -= mj * (f + D * dy * dy);
            tzz -= mj * (f + D * dz * dz);
            txy -= mj * (D * dx * dy);
            txz -= mj * (D * dx * dz);
            tyz -= mj * (D * dy * dz);
        }
        double wkx = w[3 * k], wky = w[3 * k + 1], wkz = w[3 * k + 2];
        double twx = G * (txx * wkx + txy * wky + txz * wkz);
        double twy = G * (txy * wkx + tyy * wky + tyz * wkz);
        double twz = G * (txz * wkx + tyz * wky + tzz * wkz);
        dldx[3 * t] = G * m[k] * vx + twx;
        dldx[3 * t + 1] = G * m[k] * vy + twy;
        dldx[3 * t + 2] = G * m[k] * vz + twz;
        dldm[t] = -G * s;
    }
}

/* ---- node multipoles ------------------------------------------------------- */
/*
 * For the particles idx[0..cnt):  out[0] = M,  out[1..3] = centre of mass c,
 * out[4..6] = mass-weighted mean velocity u,
 * out[7..12]  = Q    = sum m (3 y y^T - |y|^2 I),              y = x - c,
 * out[13..18] = Qdot = sum m (3 (y w^T + w y^T) - 2 (y.w) I),  w = v - u,
 * (tensors in xx yy zz xy xz yz order), out[19..24] = AABB min xyz, max xyz.
 */
void orc_moments(int64_t cnt, const int64_t *idx, const double *x, const double *v,
                 const double *m, double *out)
{
    double M = 0, cx = 0, cy = 0, cz = 0, ux = 0, uy = 0, uz = 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t i = idx[t];
        M += m[i];
        cx += m[i] * x[3 * i]; cy += m[i] * x[3 * i + 1]; cz += m[i] * x[3 * i + 2];
        ux += m[i] * v[3 * i]; uy += m[i] * v[3 * i + 1]; uz += m[i] * v[3 * i + 2];
        for (int c = 0; c < 3; ++c) {
            if (x[3 * i + c] < lo[c]) lo[c] = x[3 * i + c];
            if (x[3 * i + c] > hi[c]) hi[c] = x[3 * i + c];
        }
    }
    cx /= M; cy /= M; cz /= M; ux /= M; uy /= M; uz /= M;
    double q[6] = {0}, qd[6] = {0};
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t i = idx[t];
        double y[3] = {x[3 * i] - cx, x[3 * i + 1] - cy, x[3 * i + 2] - cz};
        double w[3] = {v[3 * i] - ux, v[3 * i + 1] - uy, v[3 * i + 2] - uz};
        double y2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
        double yw = y[0] * w[0] + y[1] * w[1] + y[2] * w[2];
        const int a[6] = {0, 1, 2, 0, 0, 1}, b[6] = {0, 1, 2, 1, 2, 2};
        for (int c = 0; c < 6; ++c) {
            double del = (a[c] == b[c]) ? 1.0 : 0.0;
            q[c] += m[i] * (3.0 * y[a[c]] * y[b[c]] - y2 * del);
            qd[c] += m[i] * (3.0 * (y[a[c]] * w[b[c]] + w[a[c]] * y[b[c]]) - 2.0 * yw * del);
        }
    }
    out[0] = M;
    out[1] = cx; out[2] = cy; out[3] = cz;
    out[4] = ux; out[5] = uy; out[6] = uz;
    for (int c = 0; c < 6; ++c) { out[7 + c] = q[c]; out[13 + c] = qd[c]; }
    for (int c = 0; c < 3; ++c) { out[19 + c] = lo[c]; out[22 + c] = hi[c]; }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later calls (k <= 0: the OpenMP default). */
void orc_set_threads(int k)
{
#ifdef _OPENMP
    static int dflt = 0;
    if (dflt == 0) dflt = omp_get_max_threads();
    omp_set_num_threads(k > 0 ? k : dflt);
#else
    (void)k;
#endif
}
