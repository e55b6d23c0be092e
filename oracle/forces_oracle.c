/*
 * FP64 CPU oracle for the cylindrical (S1 x R2) direct-sum gravity.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU library.
 *
 * Everything is written as the plain definition: for every target i,
 *
 *   a_i   = sum_{j != i} sum_{n} -G m_j F(|s|, h_i + h_j) s / |s|
 *   phi_i = sum_{j != i} sum_{n}  G m_j P(|s|, h_i + h_j)
 *
 * with s = (x_i - x_j, y_i - y_j, w(z_i - z_j) - n L) and the image index n
 * running over -n_img..n_img in ascending order, j ascending, all in FP64.
 *
 *  - pair equation of motion with pair softening h_i + h_j: Sect. 2.1,
 *    eq. (ComovingEquationsOfMotion);
 *  - F(r, h), the cubic-spline softened force law: Sect. 2.1,
 *    eq. (Force_spline_kernel), middle branch read with a single minus sign
 *    (the only reading that is continuous at r = h/2 and r = h);
 *  - direction and sign, attractive along -(x_i - x_j): Sect. 2.1,
 *    eq. (NewtonianForce);
 *  - the image sum along z: Sect. 2.1, eq. (ForceCylindrical);
 *  - P(r, h) is the potential belonging to F, P(r) = -int_r^inf F(s) ds,
 *    which the paper does not print; integrated by hand from F.
 *
 * Positions are first wrapped into [0, L) along z:
 *     z <- z - L floor(z / L), and z == L is mapped to 0.
 * The pair's minimum-image separation is w(t) = t - L floor(t / L + 1/2).
 *
 * Image windows (the paper fixes the set only through its cut-off):
 *   window 0: n = -n_img..n_img about the minimum image, i.e. a cylinder of
 *             half-height (n_img + 1/2) L centred on the target;
 *   window 1: the printed condition taken literally on the unwrapped
 *             separation r_z = z_i - z_j (both in [0, L)):
 *             n = -N_cut..N_cut with |r_z - n L| < N_cut L, N_cut = n_img.
 *
 * Self pairs (j == i) are excluded, images included.  Coincident distinct
 * particles (|s| == 0) feel no force and contribute P(0) = -2.8 / h.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

/* number of threads the parallel loops below use */
int oracle_num_threads(void) { return omp_get_max_threads(); }

/* F(r, h): magnitude of the softened force per unit G m_j (Force_spline_kernel). */
double oracle_spline_force(double r, double h)
{
    double u = r / h;
    if (u < 0.5) {
        return 32.0 * pow(r, 4) / pow(h, 6) - 38.4 * pow(r, 3) / pow(h, 5)
               + 32.0 * r / (3.0 * pow(h, 3));
    }
    if (u < 1.0) {
        return -32.0 * pow(r, 4) / (3.0 * pow(h, 6)) + 38.4 * pow(r, 3) / pow(h, 5)
               - 48.0 * r * r / pow(h, 4) + 64.0 * r / (3.0 * pow(h, 3))
               - 1.0 / (15.0 * r * r);
    }
    return 1.0 / (r * r);
}

/* P(r, h): potential per unit G m_j, with dP/dr = F and P -> 0 at infinity.
 * Integrating F from r to infinity piece by piece gives, with u = r / h,
 *   u <  1/2:  h P = -2.8 + 16/3 u^2 - 9.6 u^4 + 6.4 u^5
 *   u <  1  :  h P = -3.2 + 1/(15 u) + 32/3 u^2 - 16 u^3 + 9.6 u^4 - 32/15 u^5
 *   u >= 1  :    P = -1 / r                                                  */
double oracle_spline_potential(double r, double h)
{
    double u = r / h;
    if (u < 0.5) {
        return (-2.8 + 16.0 / 3.0 * u * u - 9.6 * pow(u, 4) + 6.4 * pow(u, 5)) / h;
    }
    if (u < 1.0) {
        return (-3.2 + 1.0 / (15.0 * u) + 32.0 / 3.0 * u * u - 16.0 * pow(u, 3)
                + 9.6 * pow(u, 4) - 32.0 / 15.0 * pow(u, 5)) / h;
    }
    return -1.0 / r;
}

double oracle_wrap_position(double z, double L)
{
    double w = z - L * floor(z / L);
    if (w >= L) w = 0.0;
    return w;
}

double oracle_min_image(double t, double L)
{
    return t - L * floor(t / L + 0.5);
}

/* add the contribution of one image (offset s, softening h, mass m) */
static void add_image(double sx, double sy, double sz, double h, double m,
                      double acc[3], double *pot)
{
    double r = sqrt(sx * sx + sy * sy + sz * sz);
    if (r > 0.0) {
        double f = oracle_spline_force(r, h);
        acc[0] += -m * f * sx / r;
        acc[1] += -m * f * sy / r;
        acc[2] += -m * f * sz / r;
    }
    *pot += m * oracle_spline_potential(r, h);
}

/*
 * Accelerations and potentials (G = 1, scale factor 1) of the targets listed
 * in tgt[0..n_tgt) (or of every particle when tgt == NULL, n_tgt = N).
 * Inputs are SoA: x, y, z, m, h each of length N.  Outputs:
 * acc[3 * n_tgt] as (x block | y block | z block), pot[n_tgt] (may be NULL).
 * Returns 0 on success, -1 on invalid arguments.
 */
int oracle_forces(const double *x, const double *y, const double *z,
                  const double *m, const double *h, int64_t N, double L,
                  int n_img, int window, const int64_t *tgt, int64_t n_tgt,
                  double *acc, double *pot)
{
    if (N <= 0 || !(L > 0.0) || n_img < 0 || (window != 0 && window != 1))
        return -1;
    if (tgt == NULL) n_tgt = N;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n_tgt; ++k) {
        int64_t i = tgt ? tgt[k] : k;
        double a[3] = {0.0, 0.0, 0.0};
        double p = 0.0;
        double zi = oracle_wrap_position(z[i], L);
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double sx = x[i] - x[j];
            double sy = y[i] - y[j];
            double zj = oracle_wrap_position(z[j], L);
            double hij = h[i] + h[j];
            if (window == 0) {
                double d = oracle_min_image(zi - zj, L);
                for (int n = -n_img; n <= n_img; ++n)
                    add_image(sx, sy, d - n * L, hij, m[j], a, &p);
            } else {
                double rz = zi - zj;
                for (int n = -n_img; n <= n_img; ++n) {
                    if (fabs(rz - n * L) < n_img * L)
                        add_image(sx, sy, rz - n * L, hij, m[j], a, &p);
                }
            }
        }
        acc[k] = a[0];
        acc[n_tgt + k] = a[1];
        acc[2 * n_tgt + k] = a[2];
        if (pot) pot[k] = p;
    }
    return 0;
}

/*
 * Image sum of one unit point mass (G = 1, unsoftened), as seen at axial
 * offset d and radial distance rho from it, over the images n with
 * n_lo <= |n| <= n_hi (ascending n):
 *   Fz   = sum -(d - n L) / r_n^3,
 *   Frho = sum -rho / r_n^3,          r_n^2 = rho^2 + (d - n L)^2,
 *   Pot  = sum -1 / r_n.
 * This is the per-pair quantity of eq. (ForceCylindrical) restricted to a
 * band of images; with n_lo = 2 it is the far-image remainder.
 */
/* The pair sum of eq. ForceCylindrical for arbitrary lists: targets t
 * (positions, softening, id) against sources s (positions, mass, softening,
 * id), images |n| <= n_img about the minimum image, pairs with equal ids
 * skipped.  acc is [3][n_t] (accumulated into, not cleared). */
int oracle_pairs(const double *tx, const double *ty, const double *tz, const double *th,
                 const int64_t *tid, int64_t n_t,
                 const double *sx, const double *sy, const double *sz, const double *sm,
                 const double *sh, const int64_t *sid, int64_t n_s, double L, int n_img,
                 double *acc)
{
    if (n_t < 0 || n_s < 0 || !(L > 0.0) || n_img < 0) return -1;
    for (int64_t k = 0; k < n_t; ++k) {
        double a[3] = {0.0, 0.0, 0.0};
        double p = 0.0;
        double zi = oracle_wrap_position(tz[k], L);
        for (int64_t j = 0; j < n_s; ++j) {
            if (tid[k] == sid[j]) continue;
            double d = oracle_min_image(zi - oracle_wrap_position(sz[j], L), L);
            for (int n = -n_img; n <= n_img; ++n)
                add_image(tx[k] - sx[j], ty[k] - sy[j], d - n * L, th[k] + sh[j], sm[j], a, &p);
        }
        acc[k] += a[0];
        acc[n_t + k] += a[1];
        acc[2 * n_t + k] += a[2];
    }
    return 0;
}

int oracle_image_band(const double *d, const double *rho, int64_t n, double L,
                      int n_lo, int n_hi, double *Fz, double *Frho, double *Pot)
{
    if (n < 0 || !(L > 0.0) || n_lo < 0 || n_hi < n_lo) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double fz = 0.0, fr = 0.0, pp = 0.0;
        for (int64_t q = -n_hi; q <= n_hi; ++q) {
            int64_t aq = q < 0 ? -q : q;
            if (aq < n_lo) continue;
            double sz = d[k] - (double)q * L;
            double r = sqrt(rho[k] * rho[k] + sz * sz);
            fz += -sz / (r * r * r);
            fr += -rho[k] / (r * r * r);
            pp += -1.0 / r;
        }
        Fz[k] = fz;
        Frho[k] = fr;
        if (Pot) Pot[k] = pp;
    }
    return 0;
}
