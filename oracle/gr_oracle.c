/*
 * FP64 brute-force oracle for the ray / 3D-Gaussian line-integral projector.
 *
 * TEST INFRASTRUCTURE ONLY. It exists to check the HIP library; only the test
 * suite, the smoke entry point and the benchmark's CPU-baseline leg may load
 * it. It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Radioactive 3D Gaussian Ray Tracing, Sec. 3):
 *   - a Gaussian is exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)) scaled by a peak density
 *     rho (Eq. 2), with Sigma = R S S^T R^T (Sec. 3.1), R from a unit
 *     quaternion (w, x, y, z) and S = diag(s);
 *   - a ray is o + t d for t over the whole real line (Eq. 3);
 *   - per pair: delta = o - mu, A = d^T P d, B = d^T P delta,
 *     C = delta^T P delta with P = Sigma^-1 (Eq. 7), and the closed form
 *     rho sqrt(2 pi / A) exp(-(C - B^2/A)/2) (Eq. 11);
 *   - per ray: the order-free sum over Gaussians (Eq. 4 and the boxed Eq. 12).
 * The paper skips contributions it calls negligible without giving a rule
 * (Sec. 4.1, implementation details). Here a pair counts iff
 * D = C - B^2/A <= kappa^2, i.e. the line meets the kappa-sigma ellipsoid.
 * kappa = +inf gives the untruncated Eq. 12.
 *
 * Every pair of every ray is evaluated: no acceleration structure, no culling.
 * Sums use Neumaier's compensated summation. All arithmetic is double.
 *
 * The gradient (not derived in the paper) follows from differentiating Eq. 11:
 * with t* = -B/A and p = delta + t* d (the point of the line closest to mu in
 * the metric P, taken relative to mu), D = p^T P p, and
 *   dT/drho   = T / rho
 *   dT/dmu    = T P p
 *   dT/dP     = -(T/2) (p p^T + d d^T / A)        (D is a minimum over t)
 * then chained through P = R diag(s^-2) R^T and through the normalisation of q.
 * The indicator D <= kappa^2 is held fixed (its derivative is taken as zero).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TWO_PI 6.283185307179586476925286766559

typedef struct {
    double mu[3];
    double s[3];
    double qn[4];   /* normalised quaternion (w, x, y, z) */
    double qnorm;   /* |q| before normalisation */
    double R[3][3]; /* columns are the local axes in world coordinates */
    double P[3][3]; /* Sigma^-1 = R diag(s^-2) R^T */
    double rho;
    int valid;
} orc_gauss;

/* Rotation matrix of a unit quaternion (w, x, y, z), Hamilton convention,
 * acting on column vectors. */
static void quat_to_rot(const double q[4], double R[3][3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

/* Partial derivatives of R(q) with respect to each component of the unit
 * quaternion, dR[c][a][b] = d R_ab / d q_c. */
static void quat_rot_jacobian(const double q[4], double dR[4][3][3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    /* d/dw */
    double Dw[3][3] = {{0, -2 * z, 2 * y}, {2 * z, 0, -2 * x}, {-2 * y, 2 * x, 0}};
    /* d/dx */
    double Dx[3][3] = {{0, 2 * y, 2 * z}, {2 * y, -4 * x, -2 * w}, {2 * z, 2 * w, -4 * x}};
    /* d/dy */
    double Dy[3][3] = {{-4 * y, 2 * x, 2 * w}, {2 * x, 0, 2 * z}, {-2 * w, 2 * z, -4 * y}};
    /* d/dz */
    double Dz[3][3] = {{-4 * z, -2 * w, 2 * x}, {2 * w, -4 * z, 2 * y}, {2 * x, 2 * y, 0}};
    memcpy(dR[0], Dw, sizeof(Dw));
    memcpy(dR[1], Dx, sizeof(Dx));
    memcpy(dR[2], Dy, sizeof(Dy));
    memcpy(dR[3], Dz, sizeof(Dz));
}

static void load_gauss(int64_t n, int64_t i, const double *mean, const double *scale,
                       const double *quat, const double *dens, orc_gauss *g) {
    int k, a, b;
    double qq = 0.0;
    g->valid = 1;
    for (k = 0; k < 3; ++k) {
        g->mu[k] = mean[k * n + i];
        g->s[k] = scale[k * n + i];
        if (!(g->s[k] > 0.0) || !isfinite(g->s[k]) || !isfinite(g->mu[k])) g->valid = 0;
    }
    for (k = 0; k < 4; ++k) {
        g->qn[k] = quat[k * n + i];
        if (!isfinite(g->qn[k])) g->valid = 0;
        qq += g->qn[k] * g->qn[k];
    }
    g->rho = dens[i];
    if (!isfinite(g->rho)) g->valid = 0;
    g->qnorm = sqrt(qq);
    if (!(g->qnorm > 0.0)) g->valid = 0;
    if (!g->valid) return;
    for (k = 0; k < 4; ++k) g->qn[k] /= g->qnorm;
    quat_to_rot(g->qn, g->R);
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (k = 0; k < 3; ++k) acc += g->R[a][k] * g->R[b][k] / (g->s[k] * g->s[k]);
            g->P[a][b] = acc;
        }
}

/* A, B, C of Eq. 7 for one ray and one Gaussian (literal formulas). */
static void pair_abc(const orc_gauss *g, const double o[3], const double d[3],
                     double *A, double *B, double *C, double delta[3]) {
    double Pd[3], Pdel[3];
    int a;
    for (a = 0; a < 3; ++a) delta[a] = o[a] - g->mu[a];
    for (a = 0; a < 3; ++a) {
        Pd[a] = g->P[a][0] * d[0] + g->P[a][1] * d[1] + g->P[a][2] * d[2];
        Pdel[a] = g->P[a][0] * delta[0] + g->P[a][1] * delta[1] + g->P[a][2] * delta[2];
    }
    *A = d[0] * Pd[0] + d[1] * Pd[1] + d[2] * Pd[2];
    *B = delta[0] * Pd[0] + delta[1] * Pd[1] + delta[2] * Pd[2];
    *C = delta[0] * Pdel[0] + delta[1] * Pdel[1] + delta[2] * Pdel[2];
}

typedef struct {
    double s, c;
} nsum;

static inline void nsum_add(nsum *acc, double x) {
    double t = acc->s + x;
    if (fabs(acc->s) >= fabs(x))
        acc->c += (acc->s - t) + x;
    else
        acc->c += (x - t) + acc->s;
    acc->s = t;
}
static inline double nsum_get(const nsum *acc) { return acc->s + acc->c; }

static orc_gauss *load_all(int64_t n, const double *mean, const double *scale,
                           const double *quat, const double *dens) {
    orc_gauss *G = (orc_gauss *)malloc(sizeof(orc_gauss) * (size_t)(n > 0 ? n : 1));
    int64_t i;
    if (!G) return NULL;
    for (i = 0; i < n; ++i) load_gauss(n, i, mean, scale, quat, dens, &G[i]);
    return G;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Per-ray projection (Eq. 12). Outputs (each may be NULL):
 *   I_kappa: sum over pairs with D <= kappa^2
 *   I_inf:   sum over all pairs (untruncated Eq. 12)
 *   I_in:    sum over pairs with D <= kappa^2 (1 - tau)
 *   I_hi:    sum over pairs with D <= kappa^2 (1 + tau)
 *   hits:    number of pairs with D <= kappa^2
 * Invalid Gaussians (s <= 0, q = 0, non-finite values) contribute nothing.
 * Returns 0, or -1 on allocation failure.
 */
int orc_project(int64_t n, const double *mean, const double *scale, const double *quat,
                const double *dens, double kappa, double tau, int64_t nr, const double *ro,
                const double *rd, double *I_kappa, double *I_inf, double *I_in, double *I_hi,
                int64_t *hits, int nthreads) {
    orc_gauss *G = load_all(n, mean, scale, quat, dens);
    const double k2 = kappa * kappa;
    const double k2_in = k2 * (1.0 - tau), k2_hi = k2 * (1.0 + tau);
    int64_t r;
    if (!G) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (r = 0; r < nr; ++r) {
        double o[3] = {ro[r], ro[nr + r], ro[2 * nr + r]};
        double d[3] = {rd[r], rd[nr + r], rd[2 * nr + r]};
        nsum sk = {0, 0}, sinf = {0, 0}, sin_ = {0, 0}, shi = {0, 0};
        int64_t h = 0, i;
        for (i = 0; i < n; ++i) {
            const orc_gauss *g = &G[i];
            double A, B, C, delta[3], D, T;
            if (!g->valid) continue;
            pair_abc(g, o, d, &A, &B, &C, delta);
            D = C - B * B / A;
            T = g->rho * sqrt(ORC_TWO_PI / A) * exp(-0.5 * D);
            nsum_add(&sinf, T);
            if (D <= k2) {
                nsum_add(&sk, T);
                ++h;
            }
            if (D <= k2_in) nsum_add(&sin_, T);
            if (D <= k2_hi) nsum_add(&shi, T);
        }
        if (I_kappa) I_kappa[r] = nsum_get(&sk);
        if (I_inf) I_inf[r] = nsum_get(&sinf);
        if (I_in) I_in[r] = nsum_get(&sin_);
        if (I_hi) I_hi[r] = nsum_get(&shi);
        if (hits) hits[r] = h;
    }
    free(G);
    return 0;
}

/*
 * Contribution of ONE Gaussian (parameters given as 11 doubles:
 * mu(3), s(3), q(4) raw, rho) to each ray, with no cutoff applied:
 * T[r] = rho sqrt(2 pi/A) exp(-D/2) and D[r]. Used for finite differences
 * with a frozen inclusion set. Either output may be NULL.
 */
int orc_pair_values(const double *theta, int64_t nr, const double *ro, const double *rd,
                    double *T_out, double *D_out) {
    double mean[3] = {theta[0], theta[1], theta[2]};
    double scale[3] = {theta[3], theta[4], theta[5]};
    double quat[4] = {theta[6], theta[7], theta[8], theta[9]};
    double dens[1] = {theta[10]};
    orc_gauss g;
    int64_t r;
    load_gauss(1, 0, mean, scale, quat, dens, &g);
    if (!g.valid) return -1;
    for (r = 0; r < nr; ++r) {
        double o[3] = {ro[r], ro[nr + r], ro[2 * nr + r]};
        double d[3] = {rd[r], rd[nr + r], rd[2 * nr + r]};
        double A, B, C, delta[3], D;
        pair_abc(&g, o, d, &A, &B, &C, delta);
        D = C - B * B / A;
        if (T_out) T_out[r] = g.rho * sqrt(ORC_TWO_PI / A) * exp(-0.5 * D);
        if (D_out) D_out[r] = D;
    }
    return 0;
}

/* Chain rule from dL/dP (GP, the 9 entries of P taken as independent) to the
 * scale and quaternion entries out[3..9], through P = R diag(s^-2) R^T and the
 * normalisation of q. */
static void chain_from_P(const orc_gauss *g, double GP[3][3], double out[11]) {
    double GR[3][3], dR[4][3][3], gqn[4], qdot;
    int a, b, c, k;
    /* P = sum_k lam_k r_k r_k^T with lam_k = s_k^-2 and r_k the k-th column of R. */
    for (k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (a = 0; a < 3; ++a)
            for (b = 0; b < 3; ++b) acc += GP[a][b] * g->R[a][k] * g->R[b][k];
        out[3 + k] = acc * (-2.0) / (g->s[k] * g->s[k] * g->s[k]);
    }
    /* dL/dR_ab = sum_c (GP_ac + GP_ca) R_cb lam_b */
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) {
            double acc = 0.0, lam = 1.0 / (g->s[b] * g->s[b]);
            for (c = 0; c < 3; ++c) acc += (GP[a][c] + GP[c][a]) * g->R[c][b];
            GR[a][b] = acc * lam;
        }
    quat_rot_jacobian(g->qn, dR);
    for (c = 0; c < 4; ++c) {
        double acc = 0.0;
        for (a = 0; a < 3; ++a)
            for (b = 0; b < 3; ++b) acc += GR[a][b] * dR[c][a][b];
        gqn[c] = acc;
    }
    /* q_hat = q / |q|: dL/dq = (I - q_hat q_hat^T) dL/dq_hat / |q| */
    qdot = gqn[0] * g->qn[0] + gqn[1] * g->qn[1] + gqn[2] * g->qn[2] + gqn[3] * g->qn[3];
    for (c = 0; c < 4; ++c) out[6 + c] = (gqn[c] - g->qn[c] * qdot) / g->qnorm;
}

/* Gradient of T for one included pair with respect to the 11 raw parameters
 * mu(3), s(3), q(4), rho, scaled by w; also returns T and D. */
static void pair_grad(const orc_gauss *g, const double o[3], const double d[3], double w,
                      double out[11], double *T_out, double *D_out) {
    double A, B, C, delta[3], D, E, T, p[3], Pp[3], GP[3][3];
    int a, b;
    pair_abc(g, o, d, &A, &B, &C, delta);
    D = C - B * B / A;
    E = sqrt(ORC_TWO_PI / A) * exp(-0.5 * D);
    T = g->rho * E;
    for (a = 0; a < 3; ++a) p[a] = delta[a] - (B / A) * d[a];
    for (a = 0; a < 3; ++a) Pp[a] = g->P[a][0] * p[0] + g->P[a][1] * p[1] + g->P[a][2] * p[2];
    /* dL/dmu = w T P p */
    for (a = 0; a < 3; ++a) out[a] = w * T * Pp[a];
    /* dL/dP = -(w T / 2)(p p^T + d d^T / A) */
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) GP[a][b] = -0.5 * w * T * (p[a] * p[b] + d[a] * d[b] / A);
    chain_from_P(g, GP, out);
    out[10] = w * E;
    if (T_out) *T_out = T;
    if (D_out) *D_out = D;
}

/*
 * Analytic gradient of L = sum_r w[r] I_kappa[r] with respect to the raw
 * parameters of the Gaussians listed in sel[0..nsel) (sel = NULL: all, in
 * order). Output g[11 * nsel] per selected Gaussian: mu(3), s(3), q(4), rho.
 * gabs[11 * nsel] (may be NULL): sum over pairs of |per-pair contribution|.
 * gband[11 * nsel] (may be NULL): the same sum restricted to pairs whose D
 * lies within kappa^2 (1 +- tau), whose inclusion is decided by rounding.
 */
int orc_grad(int64_t n, const double *mean, const double *scale, const double *quat,
             const double *dens, double kappa, double tau, int64_t nr, const double *ro,
             const double *rd, const double *w, const int64_t *sel, int64_t nsel, double *g,
             double *gabs, double *gband, int nthreads) {
    orc_gauss *G = load_all(n, mean, scale, quat, dens);
    const double k2 = kappa * kappa;
    const double k2_lo = k2 * (1.0 - tau), k2_hi = k2 * (1.0 + tau);
    int64_t m;
    if (!G) return -1;
    if (!sel) nsel = n;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (m = 0; m < nsel; ++m) {
        const int64_t i = sel ? sel[m] : m;
        const orc_gauss *gg = &G[i];
        nsum acc[11], aabs[11], aband[11];
        int k;
        int64_t r;
        memset(acc, 0, sizeof(acc));
        memset(aabs, 0, sizeof(aabs));
        memset(aband, 0, sizeof(aband));
        if (gg->valid) {
            for (r = 0; r < nr; ++r) {
                double o[3] = {ro[r], ro[nr + r], ro[2 * nr + r]};
                double d[3] = {rd[r], rd[nr + r], rd[2 * nr + r]};
                double A, B, C, delta[3], D, pg[11], T;
                pair_abc(gg, o, d, &A, &B, &C, delta);
                D = C - B * B / A;
                if (!(D <= k2_hi)) continue;
                pair_grad(gg, o, d, w[r], pg, &T, &D);
                if (D <= k2) {
                    for (k = 0; k < 11; ++k) {
                        nsum_add(&acc[k], pg[k]);
                        nsum_add(&aabs[k], fabs(pg[k]));
                    }
                }
                if (D > k2_lo)
                    for (k = 0; k < 11; ++k) nsum_add(&aband[k], fabs(pg[k]));
            }
        }
        for (k = 0; k < 11; ++k) {
            g[11 * m + k] = nsum_get(&acc[k]);
            if (gabs) gabs[11 * m + k] = nsum_get(&aabs[k]);
            if (gband) gband[11 * m + k] = nsum_get(&aband[k]);
        }
    }
    free(G);
    return 0;
}

/*
 * Voxelisation of the Gaussian mixture (Fig. 1: the reconstruction is the
 * optimised Gaussians voxelised). The field is Eq. 2's sum of Gaussians,
 *   V(x) = sum_i rho_i exp(-D_i(x) / 2),  D_i(x) = (x - mu_i)^T P_i (x - mu_i),
 * with the same kappa cutoff as the projection (a Gaussian counts where
 * D_i(x) <= kappa^2). Voxel (ix, iy, iz) has centre origin + (ix, iy, iz) .*
 * spacing and output index (iz * ny + iy) * nx + ix. Outputs (each may be
 * NULL): V with the cutoff, V_inf without it, V_in / V_hi at kappa^2 (1 -+ tau),
 * counts[0] / counts[1] the (voxel, Gaussian) pairs inside kappa^2 (1 -+ tau).
 * Returns 0, or -1 on allocation failure.
 */
int orc_voxelize(int64_t n, const double *mean, const double *scale, const double *quat,
                 const double *dens, double kappa, double tau, const double *origin,
                 const double *spacing, const int64_t *dims, double *V, double *V_inf,
                 double *V_in, double *V_hi, int64_t *counts, int nthreads) {
    orc_gauss *G = load_all(n, mean, scale, quat, dens);
    int64_t c_in = 0, c_hi = 0;
    const double k2 = kappa * kappa;
    const double k2_in = k2 * (1.0 - tau), k2_hi = k2 * (1.0 + tau);
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t nv = nx * ny * nz;
    int64_t v;
    if (!G) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : c_in, c_hi)
    for (v = 0; v < nv; ++v) {
        const int64_t ix = v % nx, iy = (v / nx) % ny, iz = v / (nx * ny);
        const double x[3] = {origin[0] + (double)ix * spacing[0], origin[1] + (double)iy * spacing[1],
                             origin[2] + (double)iz * spacing[2]};
        nsum sk = {0, 0}, sinf = {0, 0}, sin_ = {0, 0}, shi = {0, 0};
        int64_t i;
        for (i = 0; i < n; ++i) {
            const orc_gauss *g = &G[i];
            double del[3], D = 0.0, T;
            int a, b;
            if (!g->valid) continue;
            for (a = 0; a < 3; ++a) del[a] = x[a] - g->mu[a];
            for (a = 0; a < 3; ++a)
                for (b = 0; b < 3; ++b) D += del[a] * g->P[a][b] * del[b];
            T = g->rho * exp(-0.5 * D);
            nsum_add(&sinf, T);
            if (D <= k2) nsum_add(&sk, T);
            if (D <= k2_in) {
                nsum_add(&sin_, T);
                ++c_in;
            }
            if (D <= k2_hi) {
                nsum_add(&shi, T);
                ++c_hi;
            }
        }
        if (V) V[v] = nsum_get(&sk);
        if (V_inf) V_inf[v] = nsum_get(&sinf);
        if (V_in) V_in[v] = nsum_get(&sin_);
        if (V_hi) V_hi[v] = nsum_get(&shi);
    }
    if (counts) {
        counts[0] = c_in;
        counts[1] = c_hi;
    }
    free(G);
    return 0;
}

/*
 * One Adam step (Kingma and Ba; the paper optimises with Adam, Sec. 4.1) on
 * count parameters: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
 * p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = step >= 1.
 */
void orc_adam(int64_t count, double *p, const double *g, double *m, double *v, double lr, double b1,
              double b2, double eps, int64_t step) {
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    int64_t i;
    for (i = 0; i < count; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* Precision matrix P = Sigma^-1 and rotation R of each Gaussian, row-major
 * 3x3 each (for cross-checks against an independent inverse). */
int orc_precision(int64_t n, const double *mean, const double *scale, const double *quat,
                  const double *dens, double *P_out, double *R_out) {
    orc_gauss *G = load_all(n, mean, scale, quat, dens);
    int64_t i;
    int a, b;
    if (!G) return -1;
    for (i = 0; i < n; ++i)
        for (a = 0; a < 3; ++a)
            for (b = 0; b < 3; ++b) {
                if (P_out) P_out[9 * i + 3 * a + b] = G[i].valid ? G[i].P[a][b] : NAN;
                if (R_out) R_out[9 * i + 3 * a + b] = G[i].valid ? G[i].R[a][b] : NAN;
            }
    free(G);
    return 0;
}

/*
 * Time-of-flight PET projection with attenuation. The paper names both as the
 * projector's next extensions (Sec. 5, future works); the model here is the
 * standard one. Bin b of ray r weighs the line by the TOF kernel
 *   h_b(t) = (bin_width / (sqrt(2 pi) sigma)) exp(-(t - tau_b)^2 / (2 sigma^2)),
 *   tau_b  = center[r] + (b - (n_bins - 1) / 2) bin_width,
 * t the ray parameter (mm along unit directions), and the attenuation factor
 * atten[r] multiplies every bin of the ray:
 *   I_b(r) = atten[r] sum_i rho_i Int G_i(o + t d) h_b(t) dt.
 * The exponents of the Gaussian and of the kernel are both quadratics in t,
 * so the integral stays in closed form (Eq. 9-11 with the sum quadratic):
 *   A' = A + 1/sigma^2, B' = B - tau_b/sigma^2, C' = C + tau_b^2/sigma^2,
 *   I_b = atten sum_i rho_i (bin_width / (sqrt(2 pi) sigma)) sqrt(2 pi / A')
 *         exp(-(C' - B'^2/A') / 2).
 * A pair counts as in the projection: D = C - B^2/A <= kappa^2 (the line meets
 * the kappa ellipsoid), whatever the bin. n_bins = 0 means no TOF kernel: one
 * output per ray, atten[r] times the projection. center and atten may be
 * NULL (0 and 1). Outputs are [nb][nr] with nb = max(1, n_bins), each may be
 * NULL: I_kappa, I_in / I_hi (pairs inside kappa^2 (1 -+ tau)), I_inf (no
 * cutoff). Returns 0, -1 on allocation failure, -2 on bad TOF parameters.
 */
static double tof_pair(double A, double B, double C, double rho, int n_bins, double sigma,
                       double bin_width, double tau_b) {
    double lam, A2, B2, C2;
    if (n_bins == 0) return rho * sqrt(ORC_TWO_PI / A) * exp(-0.5 * (C - B * B / A));
    lam = 1.0 / (sigma * sigma);
    A2 = A + lam;
    B2 = B - tau_b * lam;
    C2 = C + tau_b * tau_b * lam;
    return rho * (bin_width / (sqrt(ORC_TWO_PI) * sigma)) * sqrt(ORC_TWO_PI / A2) *
           exp(-0.5 * (C2 - B2 * B2 / A2));
}

static double tof_center(int n_bins, double bin_width, const double *center, int64_t r, int b) {
    const double c = center ? center[r] : 0.0;
    return c + ((double)b - 0.5 * (double)(n_bins - 1)) * bin_width;
}

int orc_project_tof(int64_t n, const double *mean, const double *scale, const double *quat,
                    const double *dens, double kappa, double tau, int64_t nr, const double *ro,
                    const double *rd, int n_bins, double sigma, double bin_width, const double *center,
                    const double *atten, double *I_kappa, double *I_in, double *I_hi, double *I_inf,
                    int nthreads) {
    orc_gauss *G;
    const double k2 = kappa * kappa;
    const double k2_in = k2 * (1.0 - tau), k2_hi = k2 * (1.0 + tau);
    const int nb = n_bins > 0 ? n_bins : 1;
    int64_t r;
    if (n_bins < 0 || (n_bins > 0 && !(sigma > 0.0 && bin_width > 0.0))) return -2;
    G = load_all(n, mean, scale, quat, dens);
    if (!G) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (r = 0; r < nr; ++r) {
        double o[3] = {ro[r], ro[nr + r], ro[2 * nr + r]};
        double d[3] = {rd[r], rd[nr + r], rd[2 * nr + r]};
        const double a_r = atten ? atten[r] : 1.0;
        int b;
        for (b = 0; b < nb; ++b) {
            const double tb = tof_center(n_bins, bin_width, center, r, b);
            nsum sk = {0, 0}, sinf = {0, 0}, sin_ = {0, 0}, shi = {0, 0};
            int64_t i;
            for (i = 0; i < n; ++i) {
                const orc_gauss *g = &G[i];
                double A, B, C, delta[3], D, T;
                if (!g->valid) continue;
                pair_abc(g, o, d, &A, &B, &C, delta);
                D = C - B * B / A;
                T = tof_pair(A, B, C, g->rho, n_bins, sigma, bin_width, tb);
                nsum_add(&sinf, T);
                if (D <= k2) nsum_add(&sk, T);
                if (D <= k2_in) nsum_add(&sin_, T);
                if (D <= k2_hi) nsum_add(&shi, T);
            }
            if (I_kappa) I_kappa[(int64_t)b * nr + r] = a_r * nsum_get(&sk);
            if (I_inf) I_inf[(int64_t)b * nr + r] = a_r * nsum_get(&sinf);
            if (I_in) I_in[(int64_t)b * nr + r] = a_r * nsum_get(&sin_);
            if (I_hi) I_hi[(int64_t)b * nr + r] = a_r * nsum_get(&shi);
        }
    }
    free(G);
    return 0;
}

/* Gradient of one pair's weighted value with respect to the 11 raw
 * parameters, from its partial derivatives in A, B, C and rho (LA, LB, LC,
 * Lrho): with delta = o - mu, A = d^T P d, B = d^T P delta, C = delta^T P delta,
 *   dL/dP_ab = LA d_a d_b + LB d_a delta_b + LC delta_a delta_b,
 *   dL/dmu   = -LB P d - 2 LC P delta,
 * then through P = R diag(s^-2) R^T and the normalisation of q. */
static void pair_grad_abc(const orc_gauss *g, const double d[3], const double delta[3], double LA,
                          double LB, double LC, double Lrho, double out[11]) {
    double GP[3][3], Pd[3], Pdl[3];
    int a, b;
    for (a = 0; a < 3; ++a) {
        Pd[a] = g->P[a][0] * d[0] + g->P[a][1] * d[1] + g->P[a][2] * d[2];
        Pdl[a] = g->P[a][0] * delta[0] + g->P[a][1] * delta[1] + g->P[a][2] * delta[2];
    }
    for (a = 0; a < 3; ++a) out[a] = -LB * Pd[a] - 2.0 * LC * Pdl[a];
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) GP[a][b] = LA * d[a] * d[b] + LB * d[a] * delta[b] + LC * delta[a] * delta[b];
    chain_from_P(g, GP, out);
    out[10] = Lrho;
}

/*
 * Analytic gradient of L = sum_{b,r} w[b nr + r] I_b(r) (orc_project_tof, same
 * model and cutoff) with respect to the raw parameters of the Gaussians in
 * sel[0..nsel) (NULL: all). For one bin, with F = I_b / atten of one pair,
 *   dF/drho = F/rho, dF/dC = -F/2, dF/dB = F B'/A',
 *   dF/dA   = F (-1/(2 A') - B'^2/(2 A'^2))
 * (A', B', C' as in orc_project_tof; without a TOF kernel the unprimed
 * values), summed over the bins with weights atten w, then chained by
 * pair_grad_abc. Outputs as orc_grad: g, gabs, gband [11 nsel].
 */
int orc_grad_tof(int64_t n, const double *mean, const double *scale, const double *quat,
                 const double *dens, double kappa, double tau, int64_t nr, const double *ro,
                 const double *rd, int n_bins, double sigma, double bin_width, const double *center,
                 const double *atten, const double *w, const int64_t *sel, int64_t nsel, double *g,
                 double *gabs, double *gband, int nthreads) {
    orc_gauss *G;
    const double k2 = kappa * kappa;
    const double k2_lo = k2 * (1.0 - tau), k2_hi = k2 * (1.0 + tau);
    const int nb = n_bins > 0 ? n_bins : 1;
    const double lam = n_bins > 0 ? 1.0 / (sigma * sigma) : 0.0;
    int64_t m;
    if (n_bins < 0 || (n_bins > 0 && !(sigma > 0.0 && bin_width > 0.0))) return -2;
    G = load_all(n, mean, scale, quat, dens);
    if (!G) return -1;
    if (!sel) nsel = n;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (m = 0; m < nsel; ++m) {
        const int64_t i = sel ? sel[m] : m;
        const orc_gauss *gg = &G[i];
        nsum acc[11], aabs[11], aband[11];
        int k;
        int64_t r;
        memset(acc, 0, sizeof(acc));
        memset(aabs, 0, sizeof(aabs));
        memset(aband, 0, sizeof(aband));
        if (gg->valid) {
            for (r = 0; r < nr; ++r) {
                double o[3] = {ro[r], ro[nr + r], ro[2 * nr + r]};
                double d[3] = {rd[r], rd[nr + r], rd[2 * nr + r]};
                const double a_r = atten ? atten[r] : 1.0;
                double A, B, C, delta[3], D, LA = 0.0, LB = 0.0, LC = 0.0, Lrho = 0.0, pg[11];
                int b;
                pair_abc(gg, o, d, &A, &B, &C, delta);
                D = C - B * B / A;
                if (!(D <= k2_hi)) continue;
                for (b = 0; b < nb; ++b) {
                    const double tb = tof_center(n_bins, bin_width, center, r, b);
                    const double A2 = A + lam, B2 = B - tb * lam;
                    const double E = tof_pair(A, B, C, 1.0, n_bins, sigma, bin_width, tb);  /* F / rho */
                    const double F = gg->rho * E;
                    const double wb = a_r * w[(int64_t)b * nr + r];
                    LA += wb * F * (-0.5 / A2 - 0.5 * B2 * B2 / (A2 * A2));
                    LB += wb * F * B2 / A2;
                    LC += wb * F * (-0.5);
                    Lrho += wb * E;
                }
                pair_grad_abc(gg, d, delta, LA, LB, LC, Lrho, pg);
                if (D <= k2) {
                    for (k = 0; k < 11; ++k) {
                        nsum_add(&acc[k], pg[k]);
                        nsum_add(&aabs[k], fabs(pg[k]));
                    }
                }
                if (D > k2_lo)
                    for (k = 0; k < 11; ++k) nsum_add(&aband[k], fabs(pg[k]));
            }
        }
        for (k = 0; k < 11; ++k) {
            g[11 * m + k] = nsum_get(&acc[k]);
            if (gabs) gabs[11 * m + k] = nsum_get(&aabs[k]);
            if (gband) gband[11 * m + k] = nsum_get(&aband[k]);
        }
    }
    free(G);
    return 0;
}
