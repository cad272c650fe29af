/*
 * The paper's own evaluation method on the CPU (Sec. 2.2-2.4): the distinct
 * spin determinants are visited in the sorted (omega) order of Sec. 2.1;
 * the first one is factorised (LU with partial pivoting, then the inverse),
 * every following one is reached from the previous one by in-place
 * Sherman-Morrison column substitutions (Eq. sherman), one column at a
 * time.  A substitution whose ratio has |r| < threshold (1e-3 in the paper)
 * is postponed to a list of failed updates; the list is retried until it is
 * empty, and when a pass leaves as many failed updates as the previous one
 * (the first "previous" length being the full substitution count) the
 * updates are abandoned and the determinant is recomputed from scratch.
 * The derivatives use the current inverse: grad~_e D / D = sum_c
 * S^-1[c][e] grad~ phi_{col_c}(r_e) (Sec. 2.3, row-replacement form).
 *
 * TEST INFRASTRUCTURE ONLY: a CPU baseline of the paper's method, checked
 * against the direct-LU oracle (oracle.c); the library uses neither.
 *
 * Column scaling by powers of two (exact) keeps the synthetic workloads'
 * determinants inside the FP64 range; it does not change any ratio.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void orc_orbitals(int n_mo, int n_prim, const int32_t *pw, const double *alpha,
                  const double *coef, const double *r, double *out);

static int occ_list(int n_int, const uint64_t *d, int *occ)
{
    int n = 0;
    for (int w = 0; w < n_int; ++w)
        for (int b = 0; b < 64; ++b)
            if ((d[w] >> b) & 1ULL) occ[n++] = 64 * w + b;
    return n;
}

/* LU with partial pivoting of the n x n matrix S (row-major, destroyed),
 * inverse into X (row-major); det = sign * 2^ex * mant.  Returns 1 if singular. */
static int lu_inverse(int n, double *S, double *X, double *sign, double *logabs)
{
    int piv[64];
    double sg = 1.0, la = 0.0;
    for (int j = 0; j < n; ++j) {
        int p = j;
        double best = fabs(S[j * n + j]);
        for (int i = j + 1; i < n; ++i)
            if (fabs(S[i * n + j]) > best) { best = fabs(S[i * n + j]); p = i; }
        piv[j] = p;
        if (best == 0.0) return 1;
        if (p != j) {
            for (int c = 0; c < n; ++c) {
                double t = S[j * n + c]; S[j * n + c] = S[p * n + c]; S[p * n + c] = t;
            }
            sg = -sg;
        }
        const double d = S[j * n + j];
        if (d < 0) sg = -sg;
        la += log(fabs(d));
        for (int i = j + 1; i < n; ++i) {
            const double l = S[i * n + j] / d;
            S[i * n + j] = l;
            for (int c = j + 1; c < n; ++c) S[i * n + c] -= l * S[j * n + c];
        }
    }
    double y[64];
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < n; ++i) y[i] = (i == k) ? 1.0 : 0.0;
        for (int j = 0; j < n; ++j) {
            const int p = piv[j];
            if (p != j) { double t = y[j]; y[j] = y[p]; y[p] = t; }
        }
        for (int i = 0; i < n; ++i) {
            double s = y[i];
            for (int j = 0; j < i; ++j) s -= S[i * n + j] * y[j];
            y[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int j = i + 1; j < n; ++j) s -= S[i * n + j] * y[j];
            y[i] = s / S[i * n + i];
        }
        for (int c = 0; c < n; ++c) X[c * n + k] = y[c];
    }
    *sign = sg;
    *logabs = la;
    return 0;
}

/* sign of the permutation that sorts col[0..n) ascending */
static double perm_sign(int n, const int *col)
{
    int inv = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (col[i] > col[j]) ++inv;
    return (inv & 1) ? -1.0 : 1.0;
}

typedef struct { int k, p; } subst;

/*
 * One spin channel of one walker.  P: [5][n][M] scaled orbitals (q = 0 the
 * values, 1..4 the derivatives) of the channel's n electrons; occ: [U][n]
 * occupied orbitals of the distinct determinants in chain order, ascending
 * within a determinant; kx[m]: column m of P is the orbital times 2^-kx[m].
 * Outputs per determinant d: sgn[d], lg[d] = ln |D| (unscaled),
 * rat[d][e][q] = grad~_{e,q} D / D.
 * stats: [0] successful substitutions, [1] factorisations from scratch,
 * [2] postponed (failed) substitution attempts.
 */
static void chain(int n, int M, const double *P, const int *kx, int64_t U, const int *occ,
                  double threshold, double *sgn, double *lg, double *rat, int64_t *stats)
{
    double *S = malloc(sizeof(double) * n * n), *X = malloc(sizeof(double) * n * n);
    double w[64], rowk[64];
    int col[64], in_new[1024];
    subst todo[64], failed[64];
    double cur_sign = 0.0, cur_log = -INFINITY;  /* det of the matrix with columns col */
    int have = 0;
    for (int64_t d = 0; d < U; ++d) {
        const int *o = occ + d * n;
        int recompute = !have;
        if (have) {
            /* substitutions: holes (columns whose orbital left) paired in
             * ascending column-orbital order with the new orbitals ascending */
            memset(in_new, 0, sizeof(int) * (M < 1024 ? M : 1024));
            for (int c = 0; c < n; ++c) in_new[o[c]] = 1;
            int holes[64], nh = 0, parts[64], np = 0;
            int in_cur[1024];
            memset(in_cur, 0, sizeof(int) * (M < 1024 ? M : 1024));
            for (int c = 0; c < n; ++c) in_cur[col[c]] = 1;
            for (int m = 0; m < M; ++m) {
                if (in_cur[m] && !in_new[m]) {
                    for (int c = 0; c < n; ++c)
                        if (col[c] == m) holes[nh++] = c;
                }
                if (in_new[m] && !in_cur[m]) parts[np++] = m;
            }
            int nt = nh;
            for (int t = 0; t < nt; ++t) { todo[t].k = holes[t]; todo[t].p = parts[t]; }
            int prev = nt;
            while (nt > 0) {
                int nf = 0;
                for (int t = 0; t < nt; ++t) {
                    const int k = todo[t].k, p = todo[t].p;
                    /* w = S^-1 phi_p; ratio r = w[k] */
                    for (int i = 0; i < n; ++i) {
                        double s = 0.0;
                        for (int e = 0; e < n; ++e) s += X[i * n + e] * P[e * M + p];
                        w[i] = s;
                    }
                    const double r = w[k];
                    if (!(fabs(r) >= threshold)) {
                        failed[nf++] = todo[t];
                        stats[2]++;
                        continue;
                    }
                    /* (S + u e_k^T)^-1 = S^-1 - (S^-1 u)(e_k^T S^-1) / r, S^-1 u = w - e_k */
                    for (int e = 0; e < n; ++e) rowk[e] = X[k * n + e];
                    for (int i = 0; i < n; ++i) {
                        const double f = (i == k) ? (w[i] - 1.0) / r : w[i] / r;
                        for (int e = 0; e < n; ++e) X[i * n + e] -= f * rowk[e];
                    }
                    cur_log += log(fabs(r));
                    if (r < 0) cur_sign = -cur_sign;
                    col[k] = p;
                    stats[0]++;
                }
                if (nf == 0) break;
                if (nf == prev) { recompute = 1; break; }
                prev = nf;
                nt = nf;
                memcpy(todo, failed, sizeof(subst) * nf);
            }
        }
        if (recompute) {
            for (int c = 0; c < n; ++c) col[c] = o[c];
            for (int e = 0; e < n; ++e)
                for (int c = 0; c < n; ++c) S[e * n + c] = P[e * M + col[c]];
            double sg, la;
            if (lu_inverse(n, S, X, &sg, &la)) {
                cur_sign = 0.0;
                cur_log = -INFINITY;
                have = 0;  /* singular: the next determinant starts afresh */
            } else {
                cur_sign = sg;
                cur_log = la;
                have = 1;
            }
            stats[1]++;
        }
        if (cur_sign == 0.0) {
            sgn[d] = 0.0;
            lg[d] = -INFINITY;
            for (int t = 0; t < 4 * n; ++t) rat[d * 4 * n + t] = 0.0;
            continue;
        }
        int ksum = 0;
        for (int c = 0; c < n; ++c) ksum += kx[col[c]];
        sgn[d] = cur_sign * perm_sign(n, col);
        lg[d] = cur_log + ksum * M_LN2;
        for (int e = 0; e < n; ++e)
            for (int q = 0; q < 4; ++q) {
                double s = 0.0;
                for (int c = 0; c < n; ++c) s += X[c * n + e] * P[((1 + q) * n + e) * M + col[c]];
                rat[d * 4 * n + e * 4 + q] = s;
            }
    }
    free(S);
    free(X);
}

/*
 * Psi, grad~Psi / Psi of W walkers by the paper's method.  uniq_up [U][n_int]
 * and uniq_dn [V][n_int]: distinct determinants in chain (omega) order;
 * row_i, col_j, val [nnz]: the coefficients in those indices.  Outputs as
 * orc_eval: sign [W], logabs [W], gl [W][N][4]; stats [3] summed over walkers.
 */
int orc_sm_eval(int n_up, int n_dn, int n_mo, int n_prim, const int32_t *pw, const double *alpha,
                const double *coef, const int32_t *pw_dn, const double *alpha_dn,
                const double *coef_dn, int n_int, int64_t U, const uint64_t *uniq_up, int64_t V,
                const uint64_t *uniq_dn, int64_t nnz, const int32_t *row_i, const int32_t *col_j,
                const double *val, int64_t W, const double *R, double threshold, int n_threads,
                double *sign, double *logabs, double *gl, int64_t *stats)
{
    const int N = n_up + n_dn, M = n_mo;
    if (n_mo > 1024 || n_up > 64 || n_dn > 64) return 2;
    int *occu = malloc(sizeof(int) * (size_t)U * (n_up > 0 ? n_up : 1));
    int *occd = malloc(sizeof(int) * (size_t)V * (n_dn > 0 ? n_dn : 1));
    for (int64_t i = 0; i < U; ++i) occ_list(n_int, uniq_up + i * n_int, occu + i * n_up);
    for (int64_t j = 0; j < V; ++j) occ_list(n_int, uniq_dn + j * n_int, occd + j * n_dn);
    int64_t st[3] = {0, 0, 0};
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        int64_t lst[3] = {0, 0, 0};
        double *phi = malloc(sizeof(double) * (size_t)N * 5 * M);
        double *Pu = malloc(sizeof(double) * 5 * (size_t)n_up * M);
        double *Pd = malloc(sizeof(double) * 5 * (size_t)(n_dn > 0 ? n_dn : 1) * M);
        int *kxu = malloc(sizeof(int) * M), *kxd = malloc(sizeof(int) * M);
        double *sgu = malloc(sizeof(double) * U), *lgu = malloc(sizeof(double) * U);
        double *sgd = malloc(sizeof(double) * V), *lgd = malloc(sizeof(double) * V);
        double *rtu = malloc(sizeof(double) * U * 4 * n_up);
        double *rtd = malloc(sizeof(double) * V * 4 * (n_dn > 0 ? n_dn : 1));
#pragma omp for schedule(dynamic)
        for (int64_t w = 0; w < W; ++w) {
            for (int e = 0; e < N; ++e) {
                const int dn = e >= n_up && alpha_dn;  /* the down electrons' own set, if any */
                orc_orbitals(n_mo, n_prim, dn ? pw_dn : pw, dn ? alpha_dn : alpha,
                             dn ? coef_dn : coef, R + (w * N + e) * 3,
                             phi + (size_t)e * 5 * M);  /* [e][5][M] */
            }
            /* per spin: power-of-two column scaling, layout [q][e][m] */
            for (int s = 0; s < 2; ++s) {
                const int n = s ? n_dn : n_up, e0 = s ? n_up : 0;
                double *P = s ? Pd : Pu;
                int *kx = s ? kxd : kxu;
                for (int m = 0; m < M; ++m) {
                    double mx = 0.0;
                    for (int e = 0; e < n; ++e) mx = fmax(mx, fabs(phi[((size_t)(e0 + e) * 5) * M + m]));
                    int k = 0;
                    if (mx > 0.0) frexp(mx, &k);
                    kx[m] = k;
                    const double sc = ldexp(1.0, -k);
                    for (int q = 0; q < 5; ++q)
                        for (int e = 0; e < n; ++e)
                            P[((size_t)q * n + e) * M + m] = phi[((size_t)(e0 + e) * 5 + q) * M + m] * sc;
                }
            }
            chain(n_up, M, Pu, kxu, U, occu, threshold, sgu, lgu, rtu, lst);
            if (n_dn > 0) chain(n_dn, M, Pd, kxd, V, occd, threshold, sgd, lgd, rtd, lst);
            /* Psi = sum_k c_k D_up D_dn, relative to the largest product */
            double L = -INFINITY;
            for (int64_t k = 0; k < nnz; ++k) {
                const double t = lgu[row_i[k]] + (n_dn > 0 ? lgd[col_j[k]] : 0.0);
                if (val[k] != 0.0 && t > L) L = t;
            }
            double ps = 0.0, pc = 0.0;  /* Neumaier sum */
            double *g = gl + (size_t)w * N * 4;
            for (int t = 0; t < 4 * N; ++t) g[t] = 0.0;
            for (int64_t k = 0; k < nnz; ++k) {
                const int i = row_i[k], j = col_j[k];
                const double sd = n_dn > 0 ? sgd[j] : 1.0, ld = n_dn > 0 ? lgd[j] : 0.0;
                if (sgu[i] == 0.0 || sd == 0.0 || val[k] == 0.0) continue;
                const double x = val[k] * sgu[i] * sd * exp(lgu[i] + ld - L);
                const double tt = ps + x;
                pc += (fabs(ps) >= fabs(x)) ? (ps - tt) + x : (x - tt) + ps;
                ps = tt;
                for (int e = 0; e < n_up; ++e)
                    for (int q = 0; q < 4; ++q) g[e * 4 + q] += x * rtu[(i * n_up + e) * 4 + q];
                for (int e = 0; e < n_dn; ++e)
                    for (int q = 0; q < 4; ++q)
                        g[(n_up + e) * 4 + q] += x * rtd[(j * n_dn + e) * 4 + q];
            }
            const double psi = ps + pc;
            if (!(psi != 0.0) || !isfinite(psi)) {
                sign[w] = 0.0;
                logabs[w] = -INFINITY;
                for (int t = 0; t < 4 * N; ++t) g[t] = 0.0;
                continue;
            }
            sign[w] = psi > 0 ? 1.0 : -1.0;
            logabs[w] = log(fabs(psi)) + L;
            for (int t = 0; t < 4 * N; ++t) g[t] /= psi;
        }
#pragma omp critical
        {
            st[0] += lst[0];
            st[1] += lst[1];
            st[2] += lst[2];
        }
        free(phi); free(Pu); free(Pd); free(sgu); free(lgu); free(sgd); free(lgd);
        free(rtu); free(rtd); free(kxu); free(kxd);
    }
    free(occu);
    free(occd);
    if (stats) { stats[0] = st[0]; stats[1] = st[1]; stats[2] = st[2]; }
    return 0;
}
