/*
 * bf_oracle.c -- plain, slow, obviously-correct FP64 CPU reference for the
 * direct-summation pass of the hierarchical fourth-order forward symplectic
 * integrator (HHS-FSI) of Rantala et al. 2022 (BIFROST, arXiv 2210.02472).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the GPU kernels.
 *
 * Conventions shared by every routine below:
 *   - particle arrays are particle-indexed (length n, structure of arrays);
 *   - `tgt` (length nt) and `src` (length ns) are particle indices;
 *   - outputs are indexed by target slot k = 0..nt-1 (not by particle);
 *   - r_ji = x_j - x_i and s^2 = |r_ji|^2 + eps2 (Plummer softening, eps2 = 0
 *     gives the paper's unsoftened form);
 *   - a source equal to the target (j == i) is skipped; a distinct source at
 *     zero separation (only possible with eps2 == 0) contributes nothing and
 *     increments *n_coincident (reading of an undefined case).
 *
 *   - `sub` (particle-indexed subsystem labels, or NULL): a pair whose two
 *     particles carry the same label is skipped.  Accelerations, gradient
 *     sums and time-steps ignore intra-subsystem pairs (Sec. 3.3, Alg. 1 and
 *     the time-step assignment of subsystem particles).
 *
 * Each target is independent, so the outer loop carries an OpenMP pragma; the
 * inner loop is the definition summed in source order.
 */
#include <math.h>
#include <stdint.h>

/* Newtonian acceleration, Sec. 2.1 (Eq. new-newton-acc); softened form as in
 * the comparison runs of Sec. 5.2 (Plummer softening).  Also returns, per target,
 * the sum of the magnitudes of the individual terms (a conditioning scale used
 * to state FP64 tolerances). */
void oracle_forces(const double *x, const double *y, const double *z, const double *m,
                   int64_t nt, const int64_t *tgt, int64_t ns, const int64_t *src,
                   const int64_t *sub, double G, double eps2,
                   double *ax, double *ay, double *az, double *mag, int64_t *n_coincident)
{
    int64_t coinc = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : coinc)
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t i = tgt[k];
        double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
        for (int64_t q = 0; q < ns; ++q) {
            const int64_t j = src[q];
            if (j == i) continue;
            if (sub && sub[j] == sub[i]) continue;  /* same subsystem */
            const double rx = x[j] - x[i], ry = y[j] - y[i], rz = z[j] - z[i];
            const double s2 = rx * rx + ry * ry + rz * rz + eps2;
            if (s2 == 0.0) { ++coinc; continue; }
            const double s = sqrt(s2);
            const double w = G * m[j] / (s2 * s);      /* G m_j / s^3 */
            sx += w * rx; sy += w * ry; sz += w * rz;
            sm += fabs(w) * sqrt(rx * rx + ry * ry + rz * rz);
        }
        ax[k] = sx; ay[k] = sy; az[k] = sz;
        if (mag) mag[k] = sm;
    }
    if (n_coincident) *n_coincident = coinc;
}

/* Force-gradient sum, Sec. 2.1 (Eq. new-grad-acc) and the inter-level form of
 * Sec. 2.2:  Gsum_i = sum_j G m_j / s^5 * ( s^2 a_ji - 3 (a_ji . r_ji) r_ji ),
 * a_ji = a_j - a_i, with a given particle-indexed.  The gradient acceleration is
 * then a_i + eps^2/24 Gsum_i (eps = time-step).  With softening the exact
 * Jacobian of the softened acceleration is used (s replaces |r|).  `mag`
 * receives sum_j of the magnitudes of the individual terms. */
void oracle_gradient(const double *x, const double *y, const double *z, const double *m,
                     const double *ax, const double *ay, const double *az,
                     int64_t nt, const int64_t *tgt, int64_t ns, const int64_t *src,
                     const int64_t *sub, double G, double eps2,
                     double *gx, double *gy, double *gz, double *mag, int64_t *n_coincident)
{
    int64_t coinc = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : coinc)
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t i = tgt[k];
        double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
        for (int64_t q = 0; q < ns; ++q) {
            const int64_t j = src[q];
            if (j == i) continue;
            if (sub && sub[j] == sub[i]) continue;  /* same subsystem */
            const double rx = x[j] - x[i], ry = y[j] - y[i], rz = z[j] - z[i];
            const double s2 = rx * rx + ry * ry + rz * rz + eps2;
            if (s2 == 0.0) { ++coinc; continue; }
            const double dax = ax[j] - ax[i], day = ay[j] - ay[i], daz = az[j] - az[i];
            const double s = sqrt(s2);
            const double s5 = s2 * s2 * s;
            const double adotr = dax * rx + day * ry + daz * rz;
            const double w = G * m[j] / s5;
            const double tx = w * (s2 * dax - 3.0 * adotr * rx);
            const double ty = w * (s2 * day - 3.0 * adotr * ry);
            const double tz = w * (s2 * daz - 3.0 * adotr * rz);
            sx += tx; sy += ty; sz += tz;
            sm += sqrt(tx * tx + ty * ty + tz * tz);
        }
        gx[k] = sx; gy[k] = sy; gz[k] = sz;
        if (mag) mag[k] = sm;
    }
    if (n_coincident) *n_coincident = coinc;
}

/* Pairwise time-steps, Sec. 3.5.3 (Eqs. dt-freefall and dt-flyby):
 *   dt_ff,i = eta_ff * min_j ( |r_ij|^3 / (G (m_i + m_j)) )^(1/2)
 *   dt_fb,i = eta_fb * min_j |r_ij| / |v_ij|
 * Unsoftened separations.  A pair with |v_ij| = 0 gives no fly-by bound; a
 * target with no valid source gets +inf. */
void oracle_dt_min(const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz, const double *m,
                   int64_t nt, const int64_t *tgt, int64_t ns, const int64_t *src,
                   const int64_t *sub, double G, double eta_ff, double eta_fb,
                   double *dt_ff, double *dt_fb, int64_t *n_coincident)
{
    int64_t coinc = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : coinc)
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t i = tgt[k];
        double tff = INFINITY, tfb = INFINITY;
        for (int64_t q = 0; q < ns; ++q) {
            const int64_t j = src[q];
            if (j == i) continue;
            if (sub && sub[j] == sub[i]) continue;  /* same subsystem */
            const double rx = x[j] - x[i], ry = y[j] - y[i], rz = z[j] - z[i];
            const double r = sqrt(rx * rx + ry * ry + rz * rz);
            if (r == 0.0) { ++coinc; continue; }
            const double ff = sqrt(r * r * r / (G * (m[i] + m[j])));
            if (ff < tff) tff = ff;
            const double ux = vx[j] - vx[i], uy = vy[j] - vy[i], uz = vz[j] - vz[i];
            const double u = sqrt(ux * ux + uy * uy + uz * uz);
            if (u > 0.0) {
                const double fb = r / u;
                if (fb < tfb) tfb = fb;
            }
        }
        dt_ff[k] = eta_ff * tff;
        dt_fb[k] = eta_fb * tfb;
    }
    if (n_coincident) *n_coincident = coinc;
}

/* Global PN1.0 term, Sec. 3.8 (Eqs. subsyspn and subsyspn-mass): the pairwise
 * first post-Newtonian acceleration summed over pairs in which either particle
 * is flagged massive (is_bh[p] != 0).  The paper does not print the two-body
 * PN1.0 acceleration; this is the standard harmonic-gauge (EIH) two-body form
 * with n = (x_i - x_j)/r, v_ij = v_i - v_j:
 *   a_i += G m_j / (c^2 r^2) * { [ G (5 m_i + 4 m_j) / r + 3/2 (n.v_j)^2
 *                                  - v_i^2 + 4 v_i.v_j - 2 v_j^2 ] n
 *                                + [ 4 n.v_i - 3 n.v_j ] v_ij }             */
void oracle_pn1(const double *x, const double *y, const double *z,
                const double *vx, const double *vy, const double *vz, const double *m,
                const unsigned char *is_bh,
                int64_t nt, const int64_t *tgt, int64_t ns, const int64_t *src,
                double G, double c,
                double *px, double *py, double *pz, int64_t *n_coincident)
{
    int64_t coinc = 0;
    const double c2 = c * c;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : coinc)
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t i = tgt[k];
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t q = 0; q < ns; ++q) {
            const int64_t j = src[q];
            if (j == i) continue;
            if (!is_bh[i] && !is_bh[j]) continue;
            const double rx = x[i] - x[j], ry = y[i] - y[j], rz = z[i] - z[j];
            const double r = sqrt(rx * rx + ry * ry + rz * rz);
            if (r == 0.0) { ++coinc; continue; }
            const double nx = rx / r, ny = ry / r, nz = rz / r;
            const double vi2 = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
            const double vj2 = vx[j] * vx[j] + vy[j] * vy[j] + vz[j] * vz[j];
            const double vivj = vx[i] * vx[j] + vy[i] * vy[j] + vz[i] * vz[j];
            const double nvi = nx * vx[i] + ny * vy[i] + nz * vz[i];
            const double nvj = nx * vx[j] + ny * vy[j] + nz * vz[j];
            const double A = G * (5.0 * m[i] + 4.0 * m[j]) / r + 1.5 * nvj * nvj - vi2 + 4.0 * vivj - 2.0 * vj2;
            const double B = 4.0 * nvi - 3.0 * nvj;
            const double pre = G * m[j] / (c2 * r * r);
            sx += pre * (A * nx + B * (vx[i] - vx[j]));
            sy += pre * (A * ny + B * (vy[i] - vy[j]));
            sz += pre * (A * nz + B * (vz[i] - vz[j]));
        }
        px[k] = sx; py[k] = sy; pz[k] = sz;
    }
    if (n_coincident) *n_coincident = coinc;
}

/* Newtonian energy of a particle set, Sec. 2.1 (the N-body Hamiltonian):
 *   T = sum_i 1/2 m_i |v_i|^2,  U = - sum_{i<j} G m_i m_j / s_ij.
 * Sums are Neumaier-compensated in source order so the result does not depend
 * on the thread count. */
static void neumaier_add(double *sum, double *comp, double v)
{
    const double t = *sum + v;
    if (fabs(*sum) >= fabs(v)) *comp += (*sum - t) + v;
    else *comp += (v - t) + *sum;
    *sum = t;
}

void oracle_energy(const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz, const double *m,
                   int64_t ns, const int64_t *set, double G, double eps2,
                   double *kinetic, double *potential, double *rowbuf)
{
    /* rowbuf (length ns) holds the per-row pair sums so that the final reduction
     * is in a fixed order. */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < ns; ++a) {
        const int64_t i = set[a];
        double s = 0.0, cmp = 0.0;
        for (int64_t b = a + 1; b < ns; ++b) {
            const int64_t j = set[b];
            const double rx = x[j] - x[i], ry = y[j] - y[i], rz = z[j] - z[i];
            const double s2 = rx * rx + ry * ry + rz * rz + eps2;
            if (s2 == 0.0) continue;
            neumaier_add(&s, &cmp, G * m[i] * m[j] / sqrt(s2));
        }
        rowbuf[a] = s + cmp;
    }
    double ts = 0.0, tc = 0.0, us = 0.0, uc = 0.0;
    for (int64_t a = 0; a < ns; ++a) {
        const int64_t i = set[a];
        neumaier_add(&ts, &tc, 0.5 * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]));
        neumaier_add(&us, &uc, -rowbuf[a]);
    }
    *kinetic = ts + tc;
    *potential = us + uc;
}

/* Number of OpenMP threads a parallel region uses (for reporting). */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int oracle_num_threads(void) { return 1; }
void oracle_set_num_threads(int n) { (void)n; }
#endif

/* Subsystem neighbour criterion (Sec. 3.3, Eqs. ngb-bound and ngb-unbound) for
 * every target/source pair: out[k * ns + q] = 1 if source src[q] is a neighbour
 * of target tgt[k], else 0.  Only pairs closer than r_max are examined.  With
 * mu = G (m_i + m_j), relative separation r and velocity v, specific energy
 * E = v^2/2 - mu/r and specific angular momentum h = |r x v|:
 *   bound (E < 0), semi-major axis a = -mu / (2E):  a < r_ngb  or  r < r_ngb;
 *   unbound (E >= 0): periapsis r_p = h^2 / (mu (1 + e)), e = sqrt(1 + 2 E h^2 / mu^2);
 *     r < r_ngb,  or  r_p < r_ngb and C r / |v| < tau.                            */
void oracle_neighbours(const double *x, const double *y, const double *z,
                       const double *vx, const double *vy, const double *vz, const double *m,
                       int64_t nt, const int64_t *tgt, int64_t ns, const int64_t *src,
                       double G, double r_ngb, double r_max, double C, double tau,
                       unsigned char *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t i = tgt[k];
        for (int64_t q = 0; q < ns; ++q) {
            const int64_t j = src[q];
            unsigned char nb = 0;
            if (j != i) {
                const double rx = x[j] - x[i], ry = y[j] - y[i], rz = z[j] - z[i];
                const double ux = vx[j] - vx[i], uy = vy[j] - vy[i], uz = vz[j] - vz[i];
                const double r = sqrt(rx * rx + ry * ry + rz * rz);
                if (r < r_max) {
                    const double mu = G * (m[i] + m[j]);
                    const double v2 = ux * ux + uy * uy + uz * uz;
                    const double E = 0.5 * v2 - mu / r;
                    if (E < 0.0) {
                        const double a = -mu / (2.0 * E);
                        nb = (a < r_ngb) || (r < r_ngb);
                    } else {
                        const double hx = ry * uz - rz * uy, hy = rz * ux - rx * uz, hz = rx * uy - ry * ux;
                        const double h2 = hx * hx + hy * hy + hz * hz;
                        const double e = sqrt(1.0 + 2.0 * E * h2 / (mu * mu));
                        const double rp = h2 / (mu * (1.0 + e));
                        nb = (r < r_ngb) || (rp < r_ngb && C * r / sqrt(v2) < tau);
                    }
                }
            }
            out[k * ns + q] = nb;
        }
    }
}
