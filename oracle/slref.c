/*
 * slref.c -- plain, slow, double-precision reference for the regularized Stokes
 * single layer.  TEST INFRASTRUCTURE ONLY: used by the test-suite, by the
 * smoke check and by the benchmark's CPU-baseline leg.  Nothing on the product
 * path links or calls this file.  It shares no code with the GPU library.
 *
 * What it computes (Agarwal & Biros, Sec. 3.4, eq. (regstokes), discretized by
 * the trapezoid-POU rule of Sec. 3.3, eq. (smoothint)):
 *
 *   u(x_i) = 1/(8 pi mu) * sum_j w_j [ f_j s1(r/d)/r + (f_j . (x_i - x_j)) (x_i - x_j) s2(r/d)/r^3 ]
 *
 * with r = |x_i - x_j|, d = delta (or delta_tgt[i] when a per-target value is
 * given), and the smoothing factors of Sec. 3.4
 *
 *   s1(p) = erf(p) - (2/3) p (2 p^2 - 5) exp(-p^2) / sqrt(pi)
 *   s2(p) = erf(p) - (2/3) p (4 p^4 - 14 p^2 + 3) exp(-p^2) / sqrt(pi).
 *
 * At r = 0 the factors are replaced by their limits stated in Sec. 3.4:
 * s1(r/d)/r -> 16 / (3 d sqrt(pi)); the s2 term carries (x_i - x_j) twice and
 * therefore vanishes.  Every source is summed for every target, including the
 * target's own node (the trapezoid rule samples the smooth regularized
 * integrand at every node).  No cut-off, no tiling: the full formula for every
 * pair, glibc erf/exp, Neumaier-compensated sums per component, ascending j.
 * Build with -O2, without -ffast-math.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SLREF_PI 3.14159265358979323846264338327950288

/* s1(p), s2(p) exactly as printed in Sec. 3.4. */
void slref_smoothing(double p, double *s1, double *s2)
{
    const double e = exp(-p * p) / sqrt(SLREF_PI);
    const double erfp = erf(p);
    *s1 = erfp - (2.0 / 3.0) * p * (2.0 * p * p - 5.0) * e;
    *s2 = erfp - (2.0 / 3.0) * p * (4.0 * p * p * p * p - 14.0 * p * p + 3.0) * e;
}

/* K1 = s1(r/d)/r and K2 = s2(r/d)/r^3, with the r = 0 limits of Sec. 3.4. */
void slref_kernel(double r, double d, double *K1, double *K2)
{
    if (r == 0.0) {
        *K1 = 16.0 / (3.0 * d * sqrt(SLREF_PI));
        *K2 = 32.0 / (3.0 * d * d * d * sqrt(SLREF_PI));
        return;
    }
    double s1, s2;
    slref_smoothing(r / d, &s1, &s2);
    *K1 = s1 / r;
    *K2 = s2 / (r * r * r);
}

typedef struct { double s, c; } neumaier;

static void nm_add(neumaier *a, double t)
{
    const double s = a->s + t;
    if (fabs(a->s) >= fabs(t))
        a->c += (a->s - s) + t;
    else
        a->c += (t - s) + a->s;
    a->s = s;
}

/*
 * Host pointers, structure-of-arrays, all double.
 * tx/ty/tz == NULL means targets = sources (n_tgt must then equal n_src).
 * delta_tgt == NULL means the scalar delta for every target.
 * nthreads <= 0 leaves the OpenMP default.
 * Returns 0 on success, -1 on invalid arguments (nothing written).
 */
int slref_eval(int64_t n_src, const double *sx, const double *sy, const double *sz,
               const double *w, const double *fx, const double *fy, const double *fz,
               int64_t n_tgt, const double *tx, const double *ty, const double *tz,
               double delta, const double *delta_tgt, double mu,
               double *ux, double *uy, double *uz, int nthreads)
{
    if (n_src < 0 || n_tgt < 0 || !(mu > 0.0) || !isfinite(mu))
        return -1;
    if (delta_tgt == NULL && (!(delta > 0.0) || !isfinite(delta)))
        return -1;
    if (tx == NULL) {
        if (n_tgt != n_src)
            return -1;
        tx = sx; ty = sy; tz = sz;
    }
    const double scale = 1.0 / (8.0 * SLREF_PI * mu);
#ifdef _OPENMP
    /* this call only: the process-wide default stays as it was */
    const int team = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 16) num_threads(team)
    for (int64_t i = 0; i < n_tgt; ++i) {
        const double d = delta_tgt ? delta_tgt[i] : delta;
        neumaier ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (int64_t j = 0; j < n_src; ++j) {
            const double dx = tx[i] - sx[j], dy = ty[i] - sy[j], dz = tz[i] - sz[j];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            double K1, K2;
            slref_kernel(r, d, &K1, &K2);
            const double fd = fx[j] * dx + fy[j] * dy + fz[j] * dz;
            nm_add(&ax, w[j] * (K1 * fx[j] + K2 * fd * dx));
            nm_add(&ay, w[j] * (K1 * fy[j] + K2 * fd * dy));
            nm_add(&az, w[j] * (K1 * fz[j] + K2 * fd * dz));
        }
        ux[i] = (ax.s + ax.c) * scale;
        uy[i] = (ay.s + ay.c) * scale;
        uz[i] = (az.s + az.c) * scale;
    }
    return 0;
}

int slref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Per-patch regularization parameter, Sec. 3.4, eq. (regparam):
 *
 *   delta_{j,k}^{i} = C delta*_i,
 *   delta*_i = max over the nodes X_{l,l'} of patch i of the largest Euclidean distance from
 *              X_{l,l'} to its adjacent nodes X_{l-a,l'-b}, a, b in {-1, 0, 1}.
 *
 * Nodes are given patch-major, n x n per patch, (l, l') row-major (l, l' = 1..m-1, m = n + 1).
 * Reading: the adjacent nodes are those of the patch's own grid, so a node on the edge of the
 * grid has fewer neighbours (the grid of eq. (grid) has no nodes at l = 0 or m).  Every node of
 * patch i receives C delta*_i.  Plain loops over the definition.
 */
int slref_patch_delta(int64_t n_patches, int64_t n, const double *x, const double *y,
                      const double *z, double C, double *delta)
{
    if (n_patches < 1 || n < 1 || !(C > 0.0) || !isfinite(C)) return -1;
    for (int64_t i = 0; i < n_patches; ++i) {
        const int64_t base = i * n * n;
        double dstar = 0.0;
        for (int64_t l = 0; l < n; ++l)
            for (int64_t lp = 0; lp < n; ++lp) {
                const int64_t p = base + l * n + lp;
                double de = 0.0;   /* d_e(X_{l,l'}, neighbours) */
                for (int a = -1; a <= 1; ++a)
                    for (int b = -1; b <= 1; ++b) {
                        const int64_t ll = l - a, llp = lp - b;
                        if (ll < 0 || ll >= n || llp < 0 || llp >= n) continue;
                        const int64_t q = base + ll * n + llp;
                        const double dx = x[p] - x[q], dy = y[p] - y[q], dz = z[p] - z[q];
                        const double d = sqrt(dx * dx + dy * dy + dz * dz);
                        if (d > de) de = d;
                    }
                if (de > dstar) dstar = de;
            }
        for (int64_t p = base; p < base + n * n; ++p) delta[p] = C * dstar;
    }
    return 0;
}

/*
 * Plain (unregularized) Stokeslet sum, the kernel of the single-level FMM's far field
 * (Sec. 5): the limit of the sum above where s1 = s2 = 1,
 *
 *   v(t_i) = sum_j [ g_j / r + (g_j . (t_i - y_j)) (t_i - y_j) / r^3 ],  r = |t_i - y_j| > 0,
 *
 * with the densities g_j given directly (no weights, no 1/(8 pi mu)).  A pair with r = 0 is
 * skipped (the FMM never evaluates one).  Host pointers, structure-of-arrays; Neumaier sums,
 * ascending j.  Returns 0, or -1 on invalid sizes.
 */
int slref_stokeslet(int64_t n_src, const double *sx, const double *sy, const double *sz,
                    const double *gx, const double *gy, const double *gz, int64_t n_tgt,
                    const double *tx, const double *ty, const double *tz, double *vx, double *vy,
                    double *vz, int nthreads)
{
    if (n_src < 0 || n_tgt < 0) return -1;
#ifdef _OPENMP
    const int team = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16) num_threads(team)
    for (int64_t i = 0; i < n_tgt; ++i) {
        neumaier ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        for (int64_t j = 0; j < n_src; ++j) {
            const double dx = tx[i] - sx[j], dy = ty[i] - sy[j], dz = tz[i] - sz[j];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            const double r = sqrt(r2);
            const double gd = gx[j] * dx + gy[j] * dy + gz[j] * dz;
            nm_add(&ax, gx[j] / r + gd * dx / (r2 * r));
            nm_add(&ay, gy[j] / r + gd * dy / (r2 * r));
            nm_add(&az, gz[j] / r + gd * dz / (r2 * r));
        }
        vx[i] = ax.s + ax.c;
        vy[i] = ay.s + ay.c;
        vz[i] = az.s + az.c;
    }
    return 0;
}
