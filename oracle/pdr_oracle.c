/*
 * Plain FP64 CPU oracle of the Potential Difference Reduction (PDR) method
 * (Liu, "A Localized Method for Multicommodity Flow Problem", arXiv 2108.07549).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the reference that the GPU library is
 * checked against. Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the GPU product path never calls into it. It shares no
 * code, header or constant with the GPU library.
 *
 * Every routine follows the paper's definitions in the paper's order, in FP64,
 * with plain loops. OpenMP is used only over outputs that are independent by
 * definition (vertex/commodity entries, edges), so results do not depend on
 * the thread count.
 *
 * Layouts (no padding): f[e*K + k] edge-major in the caller's CSR arc order,
 * Delta/h[i*K + k] vertex-major. Arc e has tail i (row_ptr[i] <= e <
 * row_ptr[i+1]) and head col[e].
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *  - the degree of a vertex in a directed graph is in-degree + out-degree,
 *    counting arcs (Section 3.4: the edge-sum rewrite and the convergence
 *    proof count each incident arc once);
 *  - a vertex of degree 0 has height 0;
 *  - Algorithm 2 treats s <= u as the uncongested case (at s == u both
 *    cases give psi = 0; the congested branch would find no interval);
 *  - if rounding makes every interval test of Algorithm 2 fail, the largest
 *    p with 2 c_(p) > psi_p is taken (that predicate is monotone in p);
 *  - the AGD objective change is the exact change of the edge subproblem
 *    objective (Expression 13) with the optimal slack r >= 0, evaluated in a
 *    form free of cancellation (a difference of squares is factored);
 *  - the AGD periodic increase multiplies beta_ij by alpha_inc and caps it at
 *    beta_max, after the accept/reject step, including at t = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ESO 0
#define ORC_AGD 1
#define ORC_GDM 2
#define ORC_CAP 3
/* parallel regions are used only when a loop has this much work */
#define ORC_PAR_MIN 65536

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel regions (timing only: no result depends on it). */
void orc_set_num_threads(int nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

/* Tail of every arc. */
void orc_tails(int32_t n, int32_t m, const int64_t *row_ptr, int32_t *tails)
{
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) tails[e] = i;
    (void)m;
}

/* Degree delta_i = number of out-arcs + number of in-arcs (notation table,
 * Expression 4). */
void orc_degrees(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col, int32_t *deg)
{
    for (int32_t i = 0; i < n; ++i) deg[i] = (int32_t)(row_ptr[i + 1] - row_ptr[i]);
    for (int32_t e = 0; e < m; ++e) deg[col[e]] += 1;
}

/* Excess (Expression 2 with the injection of Expression 3) and height
 * (Expression 4): Delta_ik = sum_{in} f - sum_{out} f + hatDelta_ik,
 * h_ik = Delta_ik / delta_i. */
void orc_excess(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col, int32_t K,
                const int32_t *s, const int32_t *t, const double *d, const double *f,
                double *Delta, double *h)
{
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *tails = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    orc_degrees(n, m, row_ptr, col, deg);
    orc_tails(n, m, row_ptr, tails);

    /* hatDelta: +d_k at s_k, -d_k at t_k, 0 elsewhere */
    memset(Delta, 0, sizeof(double) * (size_t)n * (size_t)K);
    for (int32_t k = 0; k < K; ++k) {
        Delta[(size_t)s[k] * K + k] += d[k];
        Delta[(size_t)t[k] * K + k] -= d[k];
    }
    /* each arc e = (i, j) carries f_e,k out of i and into j; commodities are
     * independent, so threads split the commodity range */
#pragma omp parallel if ((int64_t)m * K >= ORC_PAR_MIN)
    {
        int32_t nt = 1, id = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        id = omp_get_thread_num();
#endif
        int32_t k0 = (int32_t)((int64_t)K * id / nt), k1 = (int32_t)((int64_t)K * (id + 1) / nt);
        for (int32_t e = 0; e < m; ++e) {
            const double *fe = f + (size_t)e * K;
            double *Di = Delta + (size_t)tails[e] * K;
            double *Dj = Delta + (size_t)col[e] * K;
            for (int32_t k = k0; k < k1; ++k) {
                Dj[k] += fe[k];
                Di[k] -= fe[k];
            }
        }
    }
#pragma omp parallel for schedule(static) if ((int64_t)n * K >= ORC_PAR_MIN)
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < K; ++k)
            h[(size_t)i * K + k] = deg[i] > 0 ? Delta[(size_t)i * K + k] / (double)deg[i] : 0.0;
    free(deg);
    free(tails);
}

/* Congestion (Expression 5): F_e = sum_k f_e,k, psi_e = max(0, F_e - u_e). */
void orc_congestion(int32_t m, int32_t K, const double *f, const double *u, double *F, double *psi)
{
#pragma omp parallel for schedule(static) if ((int64_t)m * K >= ORC_PAR_MIN)
    for (int32_t e = 0; e < m; ++e) {
        double acc = 0.0;
        for (int32_t k = 0; k < K; ++k) acc += f[(size_t)e * K + k];
        F[e] = acc;
        psi[e] = acc > u[e] ? acc - u[e] : 0.0;
    }
}

/* Objective as Algorithm 1 computes it: z = 1/2 sum_e psi_e^2 + 1/2 sum_{i,k} delta_i h_ik^2.
 * out[0] = z, out[1] = z_psi, out[2] = z_h. */
void orc_objective(int32_t n, int32_t m, const int32_t *deg, int32_t K, const double *h,
                   const double *psi, double *out)
{
    double zp = 0.0, zh = 0.0;
    for (int32_t e = 0; e < m; ++e) zp += psi[e] * psi[e];
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < K; ++k) {
            double v = h[(size_t)i * K + k];
            zh += (double)deg[i] * v * v;
        }
    out[0] = 0.5 * zp + 0.5 * zh;
    out[1] = 0.5 * zp;
    out[2] = 0.5 * zh;
}

/* The edge-sum form of the same objective (Expression 8):
 * z = 1/2 sum_{(i,j)} [psi_ij^2 + sum_k h_ik^2 + sum_k h_jk^2]. */
double orc_objective_edge_form(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col,
                               int32_t K, const double *h, const double *psi)
{
    double z = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            double acc = psi[e] * psi[e];
            for (int32_t k = 0; k < K; ++k) {
                double a = h[(size_t)i * K + k], b = h[(size_t)j * K + k];
                acc += a * a + b * b;
            }
            z += 0.5 * acc;
        }
    (void)m;
    return z;
}

static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* Algorithm 2 (solver for the edge subproblem, Expression 14) for one arc.
 * hi, hj, fe: the K heights at the tail and head and the K current flows.
 * Writes the K new flows, and psi (new congestion) and r (slack).
 * work: scratch of K doubles. Returns 1 for the congested case, 0 otherwise. */
int orc_eso_edge(int32_t K, const double *hi, const double *hj, const double *fe, double u,
                 double *fout, double *work, double *psi_out, double *r_out)
{
    /* 1. potentials c_k = ((h_ik + f_ij,k) - (h_jk - f_ij,k)) / 2 */
    double s = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double c = 0.5 * ((hi[k] + fe[k]) - (hj[k] - fe[k]));
        fout[k] = c; /* hold c in the output until step 3 */
        if (c > 0.0) s += c;
    }
    double psi = 0.0, r = 0.0;
    int congested = 0;
    /* 2. uncongested if the potential flow fits (s <= u, see header) */
    if (s <= u) {
        r = u - s;
        psi = 0.0;
    } else {
        congested = 1;
        r = 0.0;
        int32_t M = 0;
        for (int32_t k = 0; k < K; ++k)
            if (fout[k] > 0.0) work[M++] = fout[k];
        qsort(work, (size_t)M, sizeof(double), cmp_desc);
        double sum_c = 0.0;
        int found = 0;
        double best = 0.0; /* fallback: largest p with 2 c_(p) > psi_p */
        for (int32_t p = 1; p <= M; ++p) {
            sum_c += work[p - 1];
            double cand = (sum_c - u) / (1.0 + (double)p / 2.0);
            double upper = work[p - 1];
            double lower = (p < M) ? work[p] : 0.0;
            if (2.0 * lower < cand && cand <= 2.0 * upper) {
                psi = cand;
                found = 1;
                break;
            }
            if (2.0 * upper > cand) best = cand;
        }
        if (!found) psi = best;
    }
    /* 3. f'_k = max(0, c_k - psi/2) */
    for (int32_t k = 0; k < K; ++k) {
        double v = fout[k] - 0.5 * psi;
        fout[k] = v > 0.0 ? v : 0.0;
    }
    *psi_out = psi;
    *r_out = r;
    return congested;
}

/* Capacity-enforcing edge step (the formulation of Section 6: conservation
 * relaxed, capacity kept). The arc's part of the edge-form objective of
 * Expression 8 without the congestion term, 1/2 sum_k [(h_ik - x_k)^2 +
 * (h_jk + x_k)^2] over the step x = f' - f, is minimised subject to
 * sum_k f'_k <= u and f' >= 0: up to a constant this is the Euclidean
 * projection of c_k = ((h_ik + f_k) - (h_jk - f_k)) / 2 onto the capped
 * simplex. Its KKT conditions give f'_k = max(0, c_k - lambda) with lambda >= 0
 * and lambda (sum f' - u) = 0: lambda = 0 when sum max(0, c) <= u; otherwise,
 * with the positive c sorted descending and prefix sums S_p, lambda =
 * (S_p - u) / p for the first p with c_(p+1) <= lambda <= c_(p)
 * (c_(M+1) := 0; lambda = c_(p) happens at u = 0).
 * Writes the new flows and *lambda_out; returns 1 when the capacity binds. */
int orc_cap_edge(int32_t K, const double *hi, const double *hj, const double *fe, double u,
                 double *fout, double *work, double *lambda_out)
{
    double s = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double c = 0.5 * ((hi[k] + fe[k]) - (hj[k] - fe[k]));
        fout[k] = c;
        if (c > 0.0) s += c;
    }
    double lambda = 0.0;
    int binds = 0;
    if (s > u) {
        binds = 1;
        int32_t M = 0;
        for (int32_t k = 0; k < K; ++k)
            if (fout[k] > 0.0) work[M++] = fout[k];
        qsort(work, (size_t)M, sizeof(double), cmp_desc);
        double sum_c = 0.0, best = 0.0;
        int found = 0;
        for (int32_t p = 1; p <= M; ++p) {
            sum_c += work[p - 1];
            const double cand = (sum_c - u) / (double)p;
            const double lower = (p < M) ? work[p] : 0.0;
            if (lower <= cand && cand <= work[p - 1]) {
                lambda = cand;
                found = 1;
                break;
            }
            if (work[p - 1] >= cand) best = cand;  /* rounding fallback: largest p with c_(p) >= lambda_p */
        }
        if (!found) lambda = best;
    }
    for (int32_t k = 0; k < K; ++k) {
        double v = fout[k] - lambda;
        fout[k] = v > 0.0 ? v : 0.0;
    }
    *lambda_out = lambda;
    return binds;
}

/* One AGD edge step (Algorithm 3, inner loop) for one arc with pre-update
 * congestion psi = max(0, F - u). Updates fout (= new flows) and *beta.
 * Returns 1 if the step was accepted. */
int orc_agd_edge(int32_t K, const double *hi, const double *hj, const double *fe, double F,
                 double u, double psi, int64_t t, double *beta, double beta_min, double beta_max,
                 double alpha_inc, double alpha_dec, int32_t inc_period, double *fout,
                 double *dz_out)
{
    double b = *beta;
    double sum_df = 0.0, quad = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double g = hi[k] - hj[k];
        double phi = g - psi;
        double step = b * phi;
        double df = step > -fe[k] ? step : -fe[k];
        fout[k] = df; /* hold the step until the decision */
        sum_df += df;
        /* change of the two height terms of Expression 13 for this commodity:
         * 1/2[(h_i - df)^2 - h_i^2 + (h_j + df)^2 - h_j^2] = df (df - (h_i - h_j)) */
        quad += df * (df - g);
    }
    /* change of the congestion term, 1/2[(F + S - u)_+^2 - (F - u)_+^2] with
     * S = sum df. When the arc is over capacity before and after, it equals
     * S (F - u + S/2) (difference of squares), which avoids cancelling two
     * large squares when the step is small. */
    double before = F - u, after = F + sum_df - u;
    double dcong;
    if (before > 0.0 && after > 0.0)
        dcong = sum_df * (before + 0.5 * sum_df);
    else
        dcong = 0.5 * ((after > 0.0 ? after * after : 0.0) - (before > 0.0 ? before * before : 0.0));
    double dz = dcong + quad;
    (void)psi;
    int accept = dz <= 0.0;
    for (int32_t k = 0; k < K; ++k) fout[k] = accept ? fe[k] + fout[k] : fe[k];
    if (!accept) {
        b = b * alpha_dec;
        if (b < beta_min) b = beta_min;
    }
    if (inc_period > 0 && t % inc_period == 0) {
        b = b * alpha_inc;
        if (b > beta_max) b = beta_max;
    }
    *beta = b;
    if (dz_out) *dz_out = dz;
    return accept;
}

/* One GDM arc step (Algorithm 4, inner loop): the step df_k = max(-f_k,
 * beta phi_k) and its objective change are those of Algorithm 3; if the change
 * is <= 0 the velocity becomes v' = gamma v + df and the flow max(0, f + v'),
 * else flow and velocity are kept and beta decreases. The periodic increase of
 * beta follows Algorithm 3's reading (after the decision, capped at beta_max).
 * Writes the new flows to fout and velocities to vout; returns 1 if accepted. */
int orc_gdm_edge(int32_t K, const double *hi, const double *hj, const double *fe, const double *ve,
                 double F, double u, double psi, int64_t t, double *beta, double beta_min,
                 double beta_max, double alpha_inc, double alpha_dec, int32_t inc_period,
                 double gamma, double *fout, double *vout, double *dz_out)
{
    double b = *beta;
    double sum_df = 0.0, quad = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double g = hi[k] - hj[k];
        double step = b * (g - psi);
        double df = step > -fe[k] ? step : -fe[k];
        fout[k] = df; /* hold the step until the decision */
        sum_df += df;
        quad += df * (df - g);
    }
    double before = F - u, after = F + sum_df - u;
    double dcong;
    if (before > 0.0 && after > 0.0)
        dcong = sum_df * (before + 0.5 * sum_df);
    else
        dcong = 0.5 * ((after > 0.0 ? after * after : 0.0) - (before > 0.0 ? before * before : 0.0));
    double dz = dcong + quad;
    int accept = dz <= 0.0;
    for (int32_t k = 0; k < K; ++k) {
        if (accept) {
            double vn = gamma * ve[k] + fout[k];
            double fn = fe[k] + vn;
            vout[k] = vn;
            fout[k] = fn > 0.0 ? fn : 0.0;
        } else {
            vout[k] = ve[k];
            fout[k] = fe[k];
        }
    }
    if (!accept) {
        b = b * alpha_dec;
        if (b < beta_min) b = beta_min;
    }
    if (inc_period > 0 && t % inc_period == 0) {
        b = b * alpha_inc;
        if (b > beta_max) b = beta_max;
    }
    *beta = b;
    if (dz_out) *dz_out = dz;
    return accept;
}

typedef struct {
    double beta_init, beta_min, beta_max, alpha_inc, alpha_dec;
    int32_t inc_period;
    double gamma; /* momentum coefficient (Algorithm 4 only) */
} orc_agd_params;

/*
 * Algorithm 1 (method ORC_ESO), Algorithm 3 (ORC_AGD) or Algorithm 4 (ORC_GDM),
 * or the same loop with the capacity-enforcing edge step of Section 6's
 * formulation (ORC_CAP, orc_cap_edge), resumable.
 *
 * State in/out: f (m*K), beta (m, AGD/GDM), v (m*K, GDM velocities; else may
 * be NULL), *t (iteration counter), *z_prev (previous objective, +inf at the
 * start; Algorithm 4 does not initialise it, read as +inf like Algorithms 1, 3).
 * Runs at most max_iter loop passes. Each pass computes heights, congestion and
 * z, records z into z_hist[pass] (if z_hist), applies the stop test
 * |z - z_prev| < eps_obj (eps_obj > 0) or z <= z_target (z_target > 0), and
 * otherwise updates every arc from the pass's heights (Jacobi) and increments t.
 * Returns the number of updates done; *stopped = 1 if the stop test fired.
 */
int64_t orc_run(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col, const double *u,
                int32_t K, const int32_t *s, const int32_t *t_sink, const double *d, int32_t method,
                const orc_agd_params *prm, int64_t max_iter, double eps_obj, double z_target,
                double *f, double *beta, double *v, int64_t *t, double *z_prev, double *z_hist,
                int32_t *stopped)
{
    size_t nK = (size_t)n * K, mK = (size_t)m * K;
    double *Delta = (double *)malloc(sizeof(double) * (nK ? nK : 1));
    double *h = (double *)malloc(sizeof(double) * (nK ? nK : 1));
    double *F = (double *)malloc(sizeof(double) * (size_t)(m ? m : 1));
    double *psi = (double *)malloc(sizeof(double) * (size_t)(m ? m : 1));
    double *fnew = (double *)malloc(sizeof(double) * (mK ? mK : 1));
    double *vnew = method == ORC_GDM ? (double *)malloc(sizeof(double) * (mK ? mK : 1)) : NULL;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *tails = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    orc_degrees(n, m, row_ptr, col, deg);
    orc_tails(n, m, row_ptr, tails);
    double beta_min = prm ? prm->beta_min : 0.0;
    if (prm && beta_min <= 0.0) beta_min = 1.0 / (double)K;

    int64_t done = 0;
    *stopped = 0;
    for (int64_t pass = 0; pass < max_iter; ++pass) {
        orc_excess(n, m, row_ptr, col, K, s, t_sink, d, f, Delta, h);
        orc_congestion(m, K, f, u, F, psi);
        double zz[3];
        orc_objective(n, m, deg, K, h, psi, zz);
        double z = zz[0];
        if (z_hist) z_hist[pass] = z;
        if ((eps_obj > 0.0 && fabs(z - *z_prev) < eps_obj) || (z_target > 0.0 && z <= z_target)) {
            *stopped = 1;
            break;
        }
        *z_prev = z;
        int64_t tt = *t;
#pragma omp parallel if ((int64_t)m * K >= ORC_PAR_MIN)
        {
            double *work = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
#pragma omp for schedule(static)
            for (int32_t e = 0; e < m; ++e) {
                const double *hi = h + (size_t)tails[e] * K;
                const double *hj = h + (size_t)col[e] * K;
                const double *fe = f + (size_t)e * K;
                double *fo = fnew + (size_t)e * K;
                if (method == ORC_ESO) {
                    double ps, r;
                    orc_eso_edge(K, hi, hj, fe, u[e], fo, work, &ps, &r);
                } else if (method == ORC_CAP) {
                    double lam;
                    orc_cap_edge(K, hi, hj, fe, u[e], fo, work, &lam);
                } else if (method == ORC_GDM) {
                    orc_gdm_edge(K, hi, hj, fe, v + (size_t)e * K, F[e], u[e], psi[e], tt, &beta[e],
                                 beta_min, prm->beta_max, prm->alpha_inc, prm->alpha_dec,
                                 prm->inc_period, prm->gamma, fo, vnew + (size_t)e * K, NULL);
                } else {
                    orc_agd_edge(K, hi, hj, fe, F[e], u[e], psi[e], tt, &beta[e], beta_min,
                                 prm->beta_max, prm->alpha_inc, prm->alpha_dec, prm->inc_period,
                                 fo, NULL);
                }
            }
            free(work);
        }
        memcpy(f, fnew, sizeof(double) * mK);
        if (vnew) memcpy(v, vnew, sizeof(double) * mK);
        *t = tt + 1;
        ++done;
    }
    free(Delta); free(h); free(F); free(psi); free(fnew); free(vnew); free(deg); free(tails);
    return done;
}

/* Forward-mode derivative of T PDR-ESO sweeps (Algorithm 1 with Algorithm 2)
 * along a direction (du, dd) of the capacities and demands, the starting flows
 * f held fixed.
 *
 * The pass map is piecewise linear. The excess and heights are linear in (f, d),
 * so their tangents are orc_excess applied to (fdot, dd). Per arc, Algorithm 2's
 * result is f'_k = max(0, c_k - psi/2): when the arc is uncongested (psi = 0)
 * the tangent is cdot_k where c_k > 0 and 0 elsewhere; when it is congested,
 * psi = (sum_A c - u) / (1 + |A|/2) over the active set A = {k : f'_k > 0}, so
 * psidot = (sum_A cdot - udot) / (1 + |A|/2) and f'dot_k = cdot_k - psidot/2 on A,
 * 0 off it. On the measure-zero boundaries the branch Algorithm 2 takes is
 * differentiated (a one-sided derivative).
 *
 * f: in the starting flows (m x K), out f^(T). fdot: out the tangent of f^(T).
 * z_out / zdot_out: z(f^(T)) of Algorithm 1 and its directional derivative
 * zdot = sum_e psi_e psidot_e + sum_{i,k} Delta_ik hdot_ik, with
 * psidot_e = sum_k fdot_e,k - du_e when F_e > u_e, else 0. */
void orc_eso_tangent(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col,
                     const double *u, int32_t K, const int32_t *s, const int32_t *t_sink,
                     const double *d, const double *du, const double *dd, int64_t T, double *f,
                     double *fdot, double *z_out, double *zdot_out)
{
    const size_t mK = (size_t)m * K, nK = (size_t)n * K;
    int32_t *tails = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *Delta = (double *)malloc(sizeof(double) * (nK ? nK : 1));
    double *h = (double *)malloc(sizeof(double) * (nK ? nK : 1));
    double *Ddot = (double *)malloc(sizeof(double) * (nK ? nK : 1));
    double *hdot = (double *)malloc(sizeof(double) * (nK ? nK : 1));
    double *fn = (double *)malloc(sizeof(double) * (mK ? mK : 1));
    double *fdn = (double *)malloc(sizeof(double) * (mK ? mK : 1));
    orc_tails(n, m, row_ptr, tails);
    orc_degrees(n, m, row_ptr, col, deg);
    memset(fdot, 0, sizeof(double) * mK);
    for (int64_t pass = 0; pass < T; ++pass) {
        orc_excess(n, m, row_ptr, col, K, s, t_sink, d, f, Delta, h);
        orc_excess(n, m, row_ptr, col, K, s, t_sink, dd, fdot, Ddot, hdot);
        /* arcs are independent: threads split them, each with its own scratch */
#pragma omp parallel if ((int64_t)m * K >= ORC_PAR_MIN)
        {
        double *work = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
        double *cdot = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
#pragma omp for schedule(static)
        for (int32_t e = 0; e < m; ++e) {
            const double *hi = h + (size_t)tails[e] * K, *hj = h + (size_t)col[e] * K;
            const double *hdi = hdot + (size_t)tails[e] * K, *hdj = hdot + (size_t)col[e] * K;
            const double *fe = f + (size_t)e * K, *fde = fdot + (size_t)e * K;
            double *fo = fn + (size_t)e * K, *fdo = fdn + (size_t)e * K;
            double psi, r;
            const int congested = orc_eso_edge(K, hi, hj, fe, u[e], fo, work, &psi, &r);
            for (int32_t k = 0; k < K; ++k)
                cdot[k] = 0.5 * ((hdi[k] + fde[k]) - (hdj[k] - fde[k]));
            if (!congested) {
                for (int32_t k = 0; k < K; ++k) fdo[k] = fo[k] > 0.0 ? cdot[k] : 0.0;
            } else {
                double sum_cdot = 0.0;
                int32_t na = 0;
                for (int32_t k = 0; k < K; ++k)
                    if (fo[k] > 0.0) {
                        sum_cdot += cdot[k];
                        ++na;
                    }
                const double psidot = (sum_cdot - du[e]) / (1.0 + 0.5 * (double)na);
                for (int32_t k = 0; k < K; ++k) fdo[k] = fo[k] > 0.0 ? cdot[k] - 0.5 * psidot : 0.0;
            }
        }
        free(work);
        free(cdot);
        }
        memcpy(f, fn, sizeof(double) * mK);
        memcpy(fdot, fdn, sizeof(double) * mK);
    }
    /* the objective at f^(T) and its tangent */
    orc_excess(n, m, row_ptr, col, K, s, t_sink, d, f, Delta, h);
    orc_excess(n, m, row_ptr, col, K, s, t_sink, dd, fdot, Ddot, hdot);
    double z_psi = 0.0, z_h = 0.0, zdot = 0.0;
    for (int32_t e = 0; e < m; ++e) {
        double F = 0.0, Fd = 0.0;
        for (int32_t k = 0; k < K; ++k) {
            F += f[(size_t)e * K + k];
            Fd += fdot[(size_t)e * K + k];
        }
        if (F > u[e]) {
            const double psi = F - u[e];
            z_psi += 0.5 * psi * psi;
            zdot += psi * (Fd - du[e]);
        }
    }
    for (size_t q = 0; q < nK; ++q) {
        z_h += 0.5 * Delta[q] * h[q];
        zdot += Delta[q] * hdot[q];
    }
    *z_out = z_psi + z_h;
    *zdot_out = zdot;
    free(tails);
    free(deg);
    free(Delta);
    free(h);
    free(Ddot);
    free(hdot);
    free(fn);
    free(fdn);
}

/*
 * Residual report for a pseudo-flow f (FP64):
 * out[0] z, out[1] z_psi, out[2] z_h, out[3] kkt_sq = sum rho^2 with
 * rho = phi if f > 0 else max(0, phi) (residual of the stable-flow optimality
 * conditions, Section 3.3), out[4] max |Delta|, out[5] max psi,
 * out[6] Farkas gap G = sum_k d_k (h_sk - h_tk) - sum_e u_e max(0, max_k (h_ik - h_jk)),
 * out[7] the rounding margin tau_G of G.
 * Returns the verdict: 2 infeasible if G > tau_G, else 1 feasible if
 * z <= z_feasible_tol, else 0 undecided.
 *
 * G <= 0 for every h on a feasible instance (weak duality with y = -h and
 * l_e = max(0, max_k (h_ik - h_jk))), so G > 0 certifies infeasibility.
 */
int32_t orc_report(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col,
                   const double *u, int32_t K, const int32_t *s, const int32_t *t_sink,
                   const double *d, const double *f, double z_feasible_tol, double *out)
{
    size_t nK = (size_t)n * K;
    double *Delta = (double *)malloc(sizeof(double) * (nK ? nK : 1));
    double *h = (double *)malloc(sizeof(double) * (nK ? nK : 1));
    double *F = (double *)malloc(sizeof(double) * (size_t)(m ? m : 1));
    double *psi = (double *)malloc(sizeof(double) * (size_t)(m ? m : 1));
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    orc_degrees(n, m, row_ptr, col, deg);
    orc_excess(n, m, row_ptr, col, K, s, t_sink, d, f, Delta, h);
    orc_congestion(m, K, f, u, F, psi);
    double zz[3];
    orc_objective(n, m, deg, K, h, psi, zz);

    double kkt = 0.0, maxpsi = 0.0, maxD = 0.0, ul = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            double lmax = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                double g = h[(size_t)i * K + k] - h[(size_t)j * K + k];
                double phi = g - psi[e];
                double rho = f[(size_t)e * K + k] > 0.0 ? phi : (phi > 0.0 ? phi : 0.0);
                kkt += rho * rho;
                if (g > lmax) lmax = g;
            }
            ul += u[e] * lmax;
            if (psi[e] > maxpsi) maxpsi = psi[e];
        }
    for (size_t q = 0; q < nK; ++q)
        if (fabs(Delta[q]) > maxD) maxD = fabs(Delta[q]);
    double dh = 0.0, dh_abs = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double g = h[(size_t)s[k] * K + k] - h[(size_t)t_sink[k] * K + k];
        dh += d[k] * g;
        dh_abs += d[k] * fabs(g);
    }
    double G = dh - ul;
    double tau = 64.0 * 2.220446049250313e-16 * (dh_abs + ul);
    out[0] = zz[0]; out[1] = zz[1]; out[2] = zz[2];
    out[3] = kkt; out[4] = maxD; out[5] = maxpsi; out[6] = G; out[7] = tau;
    free(Delta); free(h); free(F); free(psi); free(deg);
    if (G > tau) return 2;
    if (zz[0] <= z_feasible_tol) return 1;
    return 0;
}
