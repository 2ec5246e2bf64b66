/*
 * FP64 CPU oracle for entropy-regularised OT device association.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library with a plain,
 * slow, obviously correct reference. It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Every function follows the paper's definitions directly, in double
 * precision, with index-ordered compensated (Neumaier) sums and the C
 * library's exp/log. Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp.
 *
 * Contents
 *   - per-link shadowing draw: SplitMix64 (Steele, Lea & Flood, 2014) of a
 *     (key, device, RRH) counter, turned into a standard normal by the
 *     Box-Muller transform (1958);
 *   - downlink rate R_ij = W log2(1 + SINR_ji), SINR with interference from
 *     every other RRH at full power (Sec. II-A, "Downlink Model");
 *   - cost C_ij = (1/R_ij) / median(1/R): the load-per-unit-traffic cost of
 *     Sec. IV choice (ii), normalised by its lower median;
 *   - log-domain Sinkhorn: the iteration of the Sinkhorn algorithm of
 *     Sec. III-B written on f = eps log(row scaling), g = eps log(column
 *     scaling), starting from the all-ones column scaling, stopping on the
 *     total absolute marginal residual (the stop rule of the Sinkhorn-vs-LP
 *     experiment of Sec. III);
 *   - plan statistics: marginals, transport cost <C,pi>, the regularised
 *     objective of eq. (5) with the "-1" of the entropy definition, and the
 *     dual value implied by the KKT form of the Lagrangian.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_WARN_MAXITER 1
#define ORA_EINVAL -1
#define ORA_ENOMEM -2
#define ORA_ENUMERIC -4

/* ---------------------------------------------------------------- sums -- */

/* Neumaier's improved Kahan summation, in index order. */
typedef struct { double s, c; } nsum;
static inline void nsum_add(nsum *acc, double x) {
    double t = acc->s + x;
    if (fabs(acc->s) >= fabs(x)) acc->c += (acc->s - t) + x;
    else acc->c += (x - t) + acc->s;
    acc->s = t;
}
static inline double nsum_get(const nsum *acc) { return acc->s + acc->c; }

double ora_sum(const double *x, int64_t n) {
    nsum acc = {0.0, 0.0};
    for (int64_t k = 0; k < n; ++k) nsum_add(&acc, x[k]);
    return nsum_get(&acc);
}

/* ------------------------------------------------------ shadowing draw -- */

/* SplitMix64 output for state x: add the golden-ratio increment, then the
 * 64-bit mixer with shifts 30/27/31 and the two published multipliers. */
uint64_t ora_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Standard normal for link (i, j): hash key ^ (i * 2^32 + j); the high and
 * low 32-bit halves give u1, u2 = (h + 1/2) 2^-32 in (0, 1); Box-Muller
 * X = sqrt(-2 ln u1) cos(2 pi u2). */
double ora_shadow_normal(uint64_t key, int64_t i, int64_t j) {
    uint64_t ctr = ((uint64_t)i << 32) + (uint64_t)j;
    uint64_t h = ora_splitmix64(key ^ ctr);
    double u1 = ((double)(h >> 32) + 0.5) * 0x1p-32;
    double u2 = ((double)(h & 0xFFFFFFFFULL) + 0.5) * 0x1p-32;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* ------------------------------------------------------------- radio ----- */

typedef struct {
    double tx_power_w, ref_gain, pathloss_exp, min_dist_m, shadow_sigma_db, noise_w, bandwidth_hz;
    uint64_t shadow_key;
} ora_radio;

/* Path gain G_ji = K0 * max(d, d_min)^(-alpha) * 10^(sigma X_ij / 10). */
static double gain(const ora_radio *r, const float *dev_xy, const float *rrh_xy, int64_t i, int64_t j) {
    double dx = (double)dev_xy[2 * i] - (double)rrh_xy[2 * j];
    double dy = (double)dev_xy[2 * i + 1] - (double)rrh_xy[2 * j + 1];
    double d = sqrt(dx * dx + dy * dy);
    if (d < r->min_dist_m) d = r->min_dist_m;
    double X = ora_shadow_normal(r->shadow_key, i, j);
    return r->ref_gain * pow(d, -r->pathloss_exp) * pow(10.0, r->shadow_sigma_db * X / 10.0);
}

/* Rates of device i to every RRH: R[j] = W log2(1 + SINR_ji),
 * SINR_ji = P G_ji / (sum_{l != j} P G_li + N0). The interference sum over
 * every other RRH is taken directly, as two index-ordered compensated sums:
 * the RRHs before j (ascending) and the RRHs after j (descending), so a row
 * costs O(J) and no term is ever subtracted. log2(1 + x) is evaluated as
 * log1p(x)/ln 2 so that weak links keep their digits. pg, pre (J each) are
 * scratch. */
static void rate_row(const float *dev_xy, const float *rrh_xy, int64_t J, const ora_radio *r, int64_t i,
                     double *pg, double *pre, double *R) {
    for (int64_t j = 0; j < J; ++j) pg[j] = r->tx_power_w * gain(r, dev_xy, rrh_xy, i, j);
    nsum lo = {0.0, 0.0};
    for (int64_t j = 0; j < J; ++j) {
        pre[j] = nsum_get(&lo);
        nsum_add(&lo, pg[j]);
    }
    nsum hi = {0.0, 0.0};
    for (int64_t j = J - 1; j >= 0; --j) {
        double sinr = pg[j] / ((pre[j] + nsum_get(&hi)) + r->noise_w);
        R[j] = r->bandwidth_hz * log1p(sinr) / M_LN2;
        nsum_add(&hi, pg[j]);
    }
}

/* Rates of the listed rows: R[k*J + j] = rate of device rows[k] to RRH j. */
int ora_rates_rows(const float *dev_xy, const float *rrh_xy, int64_t J, const ora_radio *r,
                   const int64_t *rows, int64_t nrows, double *R) {
    if (!dev_xy || !rrh_xy || !r || !rows || !R || J < 1 || nrows < 0) return ORA_EINVAL;
    int err = 0;
#pragma omp parallel
    {
        double *pg = (double *)malloc(sizeof(double) * (size_t)J * 2);
        if (!pg) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t k = 0; k < nrows; ++k) rate_row(dev_xy, rrh_xy, J, r, rows[k], pg, pg + J, R + k * J);
            free(pg);
        }
    }
    return err ? ORA_ENOMEM : ORA_OK;
}

int ora_rates(const float *dev_xy, const float *rrh_xy, int64_t I, int64_t J, const ora_radio *r, double *R) {
    if (I < 1) return ORA_EINVAL;
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)I);
    if (!rows) return ORA_ENOMEM;
    for (int64_t i = 0; i < I; ++i) rows[i] = i;
    int st = ora_rates_rows(dev_xy, rrh_xy, J, r, rows, I, R);
    free(rows);
    return st;
}

static int cmp_double(const void *x, const void *y) {
    double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

/* Lower median: element floor((n-1)/2) of the sorted values. */
double ora_lower_median(const double *x, int64_t n) {
    if (n < 1) return NAN;
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    if (!t) return NAN;
    memcpy(t, x, sizeof(double) * (size_t)n);
    qsort(t, (size_t)n, sizeof(double), cmp_double);
    double m = t[(n - 1) / 2];
    free(t);
    return m;
}

/* Cost from rates: C_ij = (1 / R_ij) / scale. If scale <= 0 the scale is
 * the lower median of all 1/R_ij and is written back to *scale. */
int ora_cost_from_rates(const double *R, int64_t n, double *scale, double *C) {
    if (!R || !C || !scale || n < 1) return ORA_EINVAL;
    for (int64_t k = 0; k < n; ++k) {
        if (!(R[k] > 0.0) || !isfinite(R[k])) return ORA_EINVAL;
        C[k] = 1.0 / R[k];
    }
    if (!(*scale > 0.0)) *scale = ora_lower_median(C, n);
    for (int64_t k = 0; k < n; ++k) C[k] = C[k] / *scale;
    return ORA_OK;
}

/* ---------------------------------------------------- Sinkhorn (FP64) ---- */

static int validate(const double *C, int64_t I, int64_t J, const double *a, const double *b,
                    double eps, double tol, int32_t max_iter) {
    if (!C || !a || !b || I < 1 || J < 1) return ORA_EINVAL;
    if (!(eps > 0.0) || !isfinite(eps) || !(tol >= 0.0) || max_iter < 1) return ORA_EINVAL;
    for (int64_t i = 0; i < I; ++i) if (!(a[i] > 0.0) || !isfinite(a[i])) return ORA_EINVAL;
    for (int64_t j = 0; j < J; ++j) if (!(b[j] > 0.0) || !isfinite(b[j])) return ORA_EINVAL;
    for (int64_t k = 0; k < I * J; ++k) if (!isfinite(C[k])) return ORA_EINVAL;
    double sa = ora_sum(a, I), sb = ora_sum(b, J);
    if (fabs(sa - sb) > 1e-12 * sa) return ORA_EINVAL;
    return ORA_OK;
}

/* eps * log(sum_k exp((v_k - C_k) / eps)) over a strided line of C, with the
 * maximum exponent taken out first. */
static double eps_lse(const double *v, const double *Cline, int64_t n, double eps) {
    double m = -INFINITY;
    for (int64_t k = 0; k < n; ++k) {
        double x = (v[k] - Cline[k]) / eps;
        if (x > m) m = x;
    }
    nsum s = {0.0, 0.0};
    for (int64_t k = 0; k < n; ++k) nsum_add(&s, exp((v[k] - Cline[k]) / eps - m));
    return eps * (m + log(nsum_get(&s)));
}

/* Row sums r_i and column sums c_j of pi_ij = exp((f_i + g_j - C_ij) / eps). */
static void plan_marginals(const double *C, const double *Ct, int64_t I, int64_t J, const double *f,
                           const double *g, double eps, double *r, double *c) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < I; ++i) {
        nsum s = {0.0, 0.0};
        for (int64_t j = 0; j < J; ++j) nsum_add(&s, exp((f[i] + g[j] - C[i * J + j]) / eps));
        r[i] = nsum_get(&s);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < J; ++j) {
        nsum s = {0.0, 0.0};
        for (int64_t i = 0; i < I; ++i) nsum_add(&s, exp((f[i] + g[j] - Ct[j * I + i]) / eps));
        c[j] = nsum_get(&s);
    }
}

static double total_residual(const double *r, const double *a, int64_t I, const double *c,
                             const double *b, int64_t J, double mass) {
    nsum s = {0.0, 0.0};
    for (int64_t i = 0; i < I; ++i) nsum_add(&s, fabs(r[i] - a[i]));
    for (int64_t j = 0; j < J; ++j) nsum_add(&s, fabs(c[j] - b[j]));
    return nsum_get(&s) / mass;
}

/*
 * Log-domain Sinkhorn, FP64.
 *   f_i <- eps log a_i - eps LSE_j((g_j - C_ij) / eps)      (row scaling update)
 *   g_j <- eps log b_j - eps LSE_i((f_i - C_ij) / eps)      (column scaling update)
 * g starts at g0 (NULL: zero, i.e. the all-ones column scaling). After every
 * full iteration k the residual r_k = (sum_i |rowsum_i - a_i| +
 * sum_j |colsum_j - b_j|) / sum(a) of the iterate pi^(k) is formed; the loop
 * stops when r_k < tol (ORA_OK) or k == max_iter (ORA_WARN_MAXITER).
 * hist (optional, max_iter entries) receives r_1, r_2, ...
 */
int ora_sinkhorn(const double *C, int64_t I, int64_t J, const double *a, const double *b, double eps,
                 double tol, int32_t max_iter, const double *g0, double *f, double *g, double *r_out,
                 int32_t *iters_out, double *hist) {
    int st = validate(C, I, J, a, b, eps, tol, max_iter);
    if (st) return st;
    if (!f || !g) return ORA_EINVAL;
    double *Ct = (double *)malloc(sizeof(double) * (size_t)(I * J));
    double *rs = (double *)malloc(sizeof(double) * (size_t)I);
    double *cs = (double *)malloc(sizeof(double) * (size_t)J);
    if (!Ct || !rs || !cs) { free(Ct); free(rs); free(cs); return ORA_ENOMEM; }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < J; ++j)
        for (int64_t i = 0; i < I; ++i) Ct[j * I + i] = C[i * J + j];
    for (int64_t j = 0; j < J; ++j) g[j] = g0 ? g0[j] : 0.0;
    double mass = ora_sum(a, I);
    double r = INFINITY;
    int32_t k = 0;
    st = ORA_WARN_MAXITER;
    while (k < max_iter) {
        ++k;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < I; ++i) f[i] = eps * log(a[i]) - eps_lse(g, C + i * J, J, eps);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < J; ++j) g[j] = eps * log(b[j]) - eps_lse(f, Ct + j * I, I, eps);
        plan_marginals(C, Ct, I, J, f, g, eps, rs, cs);
        r = total_residual(rs, a, I, cs, b, J, mass);
        if (hist) hist[k - 1] = r;
        if (!isfinite(r)) { st = ORA_ENUMERIC; break; }
        if (r < tol) { st = ORA_OK; break; }
    }
    if (r_out) *r_out = r;
    if (iters_out) *iters_out = k;
    free(Ct); free(rs); free(cs);
    return st;
}

/* pi_ij = exp((f_i + g_j - C_ij) / eps), row-major I x J. */
int ora_plan(const double *C, int64_t I, int64_t J, const double *f, const double *g, double eps, double *pi) {
    if (!C || !f || !g || !pi || I < 1 || J < 1 || !(eps > 0.0)) return ORA_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < I; ++i)
        for (int64_t j = 0; j < J; ++j) pi[i * J + j] = exp((f[i] + g[j] - C[i * J + j]) / eps);
    return ORA_OK;
}

/*
 * Statistics of the plan pi(f, g) = exp((f + g - C) / eps):
 *   out[0] = marginal residual (sum|rowsum - a| + sum|colsum - b|) / sum(a)
 *   out[1] = transport cost <C, pi>
 *   out[2] = regularised objective of eq. (5): <C,pi> + eps sum pi (log pi - 1)
 *   out[3] = dual value <f,a> + <g,b> - eps sum pi
 *   out[4] = total mass sum pi
 * row_sums (I) and col_sums (J) are optional outputs. Every sum is
 * index-ordered and compensated.
 */
int ora_plan_stats(const double *C, int64_t I, int64_t J, const double *a, const double *b,
                   const double *f, const double *g, double eps, double *out, double *row_sums,
                   double *col_sums) {
    if (!C || !a || !b || !f || !g || !out || I < 1 || J < 1 || !(eps > 0.0)) return ORA_EINVAL;
    double *rs = row_sums ? row_sums : (double *)malloc(sizeof(double) * (size_t)I);
    double *cs = col_sums ? col_sums : (double *)malloc(sizeof(double) * (size_t)J);
    double *cost_r = (double *)malloc(sizeof(double) * (size_t)I);
    double *ent_r = (double *)malloc(sizeof(double) * (size_t)I);
    if (!rs || !cs || !cost_r || !ent_r) {
        if (!row_sums) free(rs);
        if (!col_sums) free(cs);
        free(cost_r); free(ent_r);
        return ORA_ENOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < I; ++i) {
        nsum s = {0.0, 0.0}, sc = {0.0, 0.0}, se = {0.0, 0.0};
        for (int64_t j = 0; j < J; ++j) {
            double lp = (f[i] + g[j] - C[i * J + j]) / eps; /* log pi_ij */
            double p = exp(lp);
            nsum_add(&s, p);
            nsum_add(&sc, C[i * J + j] * p);
            nsum_add(&se, p * (lp - 1.0));
        }
        rs[i] = nsum_get(&s);
        cost_r[i] = nsum_get(&sc);
        ent_r[i] = nsum_get(&se);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < J; ++j) {
        nsum s = {0.0, 0.0};
        for (int64_t i = 0; i < I; ++i) nsum_add(&s, exp((f[i] + g[j] - C[i * J + j]) / eps));
        cs[j] = nsum_get(&s);
    }
    double mass_a = ora_sum(a, I);
    nsum res = {0.0, 0.0};
    for (int64_t i = 0; i < I; ++i) nsum_add(&res, fabs(rs[i] - a[i]));
    for (int64_t j = 0; j < J; ++j) nsum_add(&res, fabs(cs[j] - b[j]));
    double cost = ora_sum(cost_r, I), ent = ora_sum(ent_r, I), mass_pi = ora_sum(rs, I);
    nsum dual = {0.0, 0.0};
    for (int64_t i = 0; i < I; ++i) nsum_add(&dual, f[i] * a[i]);
    for (int64_t j = 0; j < J; ++j) nsum_add(&dual, g[j] * b[j]);
    nsum_add(&dual, -eps * mass_pi);
    out[0] = nsum_get(&res) / mass_a;
    out[1] = cost;
    out[2] = cost + eps * ent;
    out[3] = nsum_get(&dual);
    out[4] = mass_pi;
    if (!row_sums) free(rs);
    if (!col_sums) free(cs);
    free(cost_r); free(ent_r);
    return ORA_OK;
}

/*
 * Statistics of the plan pi(f, g) = exp((f_i + g_j - C_ij) / eps) for the
 * rate cost C_ij = (1 / R_ij) / scale of a geometry (Sec. II-A, Sec. IV cost
 * choice (ii)), with each row of C regenerated when it is needed and never
 * held whole, so that instances whose cost does not fit in memory can be
 * checked (the same quantities as ora_plan_stats):
 *   out[0] = marginal residual (sum|rowsum - a| + sum|colsum - b|) / sum(a)
 *   out[1] = transport cost <C, pi>
 *   out[2] = total mass sum pi
 * row_sums (I) and col_sums (J) are optional outputs. Row quantities are
 * compensated sums in column order; a column sum is compensated within each
 * thread's contiguous block of rows and the blocks are added in row order.
 */
int ora_geometry_plan_stats(const float *dev_xy, const float *rrh_xy, int64_t I, int64_t J, const ora_radio *r,
                            double scale, const double *a, const double *b, const double *f, const double *g,
                            double eps, double *out, double *row_sums, double *col_sums) {
    if (!dev_xy || !rrh_xy || !r || !a || !b || !f || !g || !out || I < 1 || J < 1 || !(eps > 0.0) ||
        !(scale > 0.0))
        return ORA_EINVAL;
    double *rs = row_sums ? row_sums : (double *)malloc(sizeof(double) * (size_t)I);
    double *cost_r = (double *)malloc(sizeof(double) * (size_t)I);
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    nsum *cacc = (nsum *)calloc((size_t)nt * (size_t)J, sizeof(nsum));
    int used = 1, err = (!rs || !cost_r || !cacc) ? 1 : 0;
    if (!err) {
#pragma omp parallel num_threads(nt)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#pragma omp single
            used = omp_get_num_threads();
#endif
            double *w = (double *)malloc(sizeof(double) * (size_t)J * 3);
            nsum *ca = cacc + (size_t)t * (size_t)J;
            if (!w) {
#pragma omp atomic write
                err = 1;
            }
#pragma omp barrier
            if (!err) {
#pragma omp for schedule(static)
                for (int64_t i = 0; i < I; ++i) {
                    double *Rr = w + 2 * J;
                    rate_row(dev_xy, rrh_xy, J, r, i, w, w + J, Rr);
                    nsum s = {0.0, 0.0}, sc = {0.0, 0.0};
                    for (int64_t j = 0; j < J; ++j) {
                        double c = (1.0 / Rr[j]) / scale;
                        double p = exp((f[i] + g[j] - c) / eps);
                        nsum_add(&s, p);
                        nsum_add(&sc, c * p);
                        nsum_add(&ca[j], p);
                    }
                    rs[i] = nsum_get(&s);
                    cost_r[i] = nsum_get(&sc);
                }
            }
            free(w);
        }
    }
    if (!err) {
        /* static scheduling gives thread t the t-th contiguous block of rows */
        double *cs = col_sums ? col_sums : (double *)malloc(sizeof(double) * (size_t)J);
        if (!cs) {
            err = 1;
        } else {
            for (int64_t j = 0; j < J; ++j) {
                nsum s = {0.0, 0.0};
                for (int t = 0; t < used; ++t) {
                    nsum_add(&s, cacc[(size_t)t * (size_t)J + j].s);
                    nsum_add(&s, cacc[(size_t)t * (size_t)J + j].c);
                }
                cs[j] = nsum_get(&s);
            }
            nsum res = {0.0, 0.0};
            for (int64_t i = 0; i < I; ++i) nsum_add(&res, fabs(rs[i] - a[i]));
            for (int64_t j = 0; j < J; ++j) nsum_add(&res, fabs(cs[j] - b[j]));
            out[0] = nsum_get(&res) / ora_sum(a, I);
            out[1] = ora_sum(cost_r, I);
            out[2] = ora_sum(rs, I);
            if (!col_sums) free(cs);
        }
    }
    if (!row_sums) free(rs);
    free(cost_r);
    free(cacc);
    return err ? ORA_ENOMEM : ORA_OK;
}
