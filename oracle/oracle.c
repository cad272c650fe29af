/*
 * Plain FP64 CPU oracle for the multideterminant wavefunction evaluator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library.
 *
 * What it computes, for one walker R = (r_1..r_N), N = n_up + n_dn, electrons
 * 0..n_up-1 spin up and n_up..N-1 spin down:
 *
 *   * the molecular orbitals and their derivatives at every electron (the
 *     arrays Phi, grad Phi, lap Phi of Sec. 2), evaluated analytically from
 *     Gaussian primitives x^a y^b z^c exp(-alpha r^2) centred at the origin;
 *   * every distinct spin determinant D = det S with [S]_{e,c} = phi_{o_c}(r_e)
 *     (o_1 < ... < o_n the occupied orbitals, Eq. (1)), by LU with partial
 *     pivoting after exact power-of-two column scaling (so that nothing
 *     underflows);
 *   * the derivative ratios grad~_e D / D = sum_c [S^-1]_{c,e} grad~ phi_{o_c}(r_e)
 *     (the row-replacement reading of the derivative formula of Sec. 2.3:
 *     D is linear in row e, so replacing row e by its gradient or Laplacian
 *     gives grad~_e D; the printed formula is garbled, this is its exact form);
 *   * Psi = sum_k c_k D_up[k] D_dn[k] (Eq. (1)) and, per electron, the four
 *     components [d/dx, d/dy, d/dz, Laplacian] of Psi (the grad~ vector of
 *     Sec. 2.3, cross-spin terms vanish), summed over k with Neumaier
 *     compensation in a log-shifted frame; or, in mode 1, the same quantities
 *     through the bilinear form D_up^T C D_dn of Eq. (main) with the two
 *     matrix-vector products of Secs. 2.3-2.4 (a cross-check of mode 0).
 *
 * Outputs per walker: sign(Psi), ln|Psi|, grad~Psi/Psi [N][4], and the
 * absolute-sum scales S_Psi/|Psi| and S_{e,q}/|Psi| (S = sum of |terms|) used
 * by the scaled error metric.  A node (Psi == 0 exactly) gives sign 0,
 * ln|Psi| = -inf, zero derivatives and infinite scales.  An exactly singular
 * spin determinant contributes zero to every sum.
 *
 * Duplicated spin determinants are evaluated once: the distinct lists come
 * from a plain lexicographic sort of the bit strings (unrelated to the
 * paper's xor-key ordering, which is checked separately).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Orbitals                                                            */
/* ------------------------------------------------------------------ */

static double ipow(double x, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

/* Factors of d^j/dx^j [x^a exp(-alpha x^2)] / exp(-alpha x^2), j = 0,1,2. */
static void axis_factors(double x, int a, double alpha, double f[3])
{
    f[0] = ipow(x, a);
    double d1 = -2.0 * alpha * ipow(x, a + 1);
    if (a >= 1) d1 += (double)a * ipow(x, a - 1);
    f[1] = d1;
    double d2 = -2.0 * alpha * (double)(2 * a + 1) * ipow(x, a)
              + 4.0 * alpha * alpha * ipow(x, a + 2);
    if (a >= 2) d2 += (double)(a * (a - 1)) * ipow(x, a - 2);
    f[2] = d2;
}

/* out[q*n_mo + m], q = 0 value, 1..3 gradient x,y,z, 4 Laplacian. */
void orc_orbitals(int n_mo, int n_prim, const int32_t *pw, const double *alpha,
                  const double *coef, const double *r, double *out)
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    for (int m = 0; m < n_mo; ++m) {
        double v = 0, gx = 0, gy = 0, gz = 0, lap = 0;
        for (int p = 0; p < n_prim; ++p) {
            const int32_t *abc = pw + 3 * (m * n_prim + p);
            double al = alpha[m * n_prim + p];
            double e = coef[m * n_prim + p] * exp(-al * r2);
            double fx[3], fy[3], fz[3];
            axis_factors(r[0], abc[0], al, fx);
            axis_factors(r[1], abc[1], al, fy);
            axis_factors(r[2], abc[2], al, fz);
            v += e * fx[0] * fy[0] * fz[0];
            gx += e * fx[1] * fy[0] * fz[0];
            gy += e * fx[0] * fy[1] * fz[0];
            gz += e * fx[0] * fy[0] * fz[1];
            lap += e * (fx[2] * fy[0] * fz[0] + fx[0] * fy[2] * fz[0] + fx[0] * fy[0] * fz[2]);
        }
        out[0 * n_mo + m] = v;
        out[1 * n_mo + m] = gx;
        out[2 * n_mo + m] = gy;
        out[3 * n_mo + m] = gz;
        out[4 * n_mo + m] = lap;
    }
}

/* ------------------------------------------------------------------ */
/* One Slater determinant by LU with partial pivoting                  */
/* ------------------------------------------------------------------ */

/*
 * S: n x n row-major (rows = electrons, columns = occupied orbitals), G: the
 * four derivative matrices with the same layout ([q][e][c]).  Columns of both
 * are scaled by the same power of two (exact).  On return: *sign, *logabs of
 * det S (unscaled) and ratio[e*4+q] = grad~_{e,q} D / D.  Returns 0, or 1 if
 * S is exactly singular (then sign = 0 and ratios are zero).
 * work: at least 2*n*n + n doubles.
 */
int orc_slater(int n, const double *S_in, const double *G, double *sign,
               double *logabs, double *ratio, double *work)
{
    double *S = work;             /* n*n  LU factors */
    double *X = work + n * n;     /* n*n  inverse, X[c*n+e] */
    double *y = work + 2 * n * n; /* n    solve scratch */
    int piv[64];
    double colexp_sum = 0.0;
    memcpy(S, S_in, sizeof(double) * n * n);
    /* column scaling by 2^-k, k = exponent of the largest |entry| */
    double cscale[64];
    for (int c = 0; c < n; ++c) {
        double mx = 0.0;
        for (int e = 0; e < n; ++e) mx = fmax(mx, fabs(S[e * n + c]));
        int k = 0;
        if (mx > 0.0) frexp(mx, &k);
        cscale[c] = ldexp(1.0, -k);
        colexp_sum += (double)k;
        for (int e = 0; e < n; ++e) S[e * n + c] *= cscale[c];
    }
    /* LU, row pivoting */
    double sg = 1.0, la = 0.0;
    for (int j = 0; j < n; ++j) {
        int p = j;
        double best = fabs(S[j * n + j]);
        for (int i = j + 1; i < n; ++i)
            if (fabs(S[i * n + j]) > best) { best = fabs(S[i * n + j]); p = i; }
        piv[j] = p;
        if (best == 0.0) {
            *sign = 0.0;
            *logabs = -INFINITY;
            for (int i = 0; i < 4 * n; ++i) ratio[i] = 0.0;
            return 1;
        }
        if (p != j) {
            for (int c = 0; c < n; ++c) {
                double t = S[j * n + c]; S[j * n + c] = S[p * n + c]; S[p * n + c] = t;
            }
            sg = -sg;
        }
        double d = S[j * n + j];
        if (d < 0) sg = -sg;
        la += log(fabs(d));
        for (int i = j + 1; i < n; ++i) {
            double l = S[i * n + j] / d;
            S[i * n + j] = l;
            for (int c = j + 1; c < n; ++c) S[i * n + c] -= l * S[j * n + c];
        }
    }
    *sign = sg;
    *logabs = la + colexp_sum * log(2.0);
    /* inverse of the scaled matrix: solve (P A) X = P e_k column by column */
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < n; ++i) y[i] = (i == k) ? 1.0 : 0.0;
        for (int j = 0; j < n; ++j) {
            int p = piv[j];
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
    /* ratio: sum_c Xs[c,e] * Gs[e,c]; scaled X = diag(1/cs) S^-1, scaled G = G diag(cs) */
    for (int e = 0; e < n; ++e)
        for (int q = 0; q < 4; ++q) {
            double s = 0.0;
            for (int c = 0; c < n; ++c) s += X[c * n + e] * G[(q * n + e) * n + c] * cscale[c];
            ratio[e * 4 + q] = s;
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Distinct spin determinants (plain lexicographic order)              */
/* ------------------------------------------------------------------ */

static int g_nint; /* comparator context; set under a lock-free single thread */

static int cmp_words(const void *a, const void *b)
{
    const uint64_t *x = (const uint64_t *)a, *y = (const uint64_t *)b;
    for (int w = g_nint - 1; w >= 0; --w) {
        if (x[w] < y[w]) return -1;
        if (x[w] > y[w]) return 1;
    }
    return 0;
}

/* returns number of distinct strings; uniq must hold n_det*n_int words */
static int64_t distinct(int n_int, int64_t n_det, const uint64_t *d, uint64_t *uniq)
{
    memcpy(uniq, d, sizeof(uint64_t) * n_int * n_det);
    g_nint = n_int;
    qsort(uniq, (size_t)n_det, sizeof(uint64_t) * n_int, cmp_words);
    int64_t u = 0;
    for (int64_t k = 0; k < n_det; ++k) {
        if (u > 0 && cmp_words(uniq + (u - 1) * n_int, uniq + k * n_int) == 0) continue;
        if (u != k) memmove(uniq + u * n_int, uniq + k * n_int, sizeof(uint64_t) * n_int);
        ++u;
    }
    return u;
}

static int64_t find(int n_int, int64_t u, const uint64_t *uniq, const uint64_t *key)
{
    int64_t lo = 0, hi = u - 1;
    g_nint = n_int;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int c = cmp_words(uniq + mid * n_int, key);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int popcount64(uint64_t x)
{
    int c = 0;
    while (x) { x &= x - 1; ++c; }
    return c;
}

/* occupied orbitals in ascending order; returns count */
static int occupied(int n_int, const uint64_t *d, int *occ)
{
    int n = 0;
    for (int w = 0; w < n_int; ++w)
        for (int b = 0; b < 64; ++b)
            if ((d[w] >> b) & 1u) occ[n++] = 64 * w + b;
    return n;
}

/* ------------------------------------------------------------------ */
/* Neumaier compensated accumulator                                    */
/* ------------------------------------------------------------------ */

typedef struct { double s, c; } nsum;

static inline void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static inline double nval(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Whole-wavefunction evaluation                                       */
/* ------------------------------------------------------------------ */

/*
 * mode 0: Eq. (1), a compensated sum over the n_det products.
 * mode 1: Eq. (main), D_up^T (C D_dn) and the two derivative mat-vecs.
 * max_degree (nullable, [n_walk]): walker w keeps only products whose two
 * spin determinants both differ from the reference product (the one with the
 * largest |c_k|, earliest on ties) by at most max_degree[w] excitations.
 * Returns 0 on success, <0 on bad input.
 */
int orc_eval(int n_up, int n_dn, int n_mo, int n_prim, const int32_t *pw,
             const double *alpha, const double *coef, const int32_t *pw_dn,
             const double *alpha_dn, const double *coef_dn, int n_int, int64_t n_det,
             const uint64_t *det_up, const uint64_t *det_dn, const double *c,
             int64_t n_walk, const double *R, const int8_t *max_degree, int mode,
             double *sign_out, double *logabs_out, double *gl_out,
             double *rs_psi_out, double *rs_gl_out, int n_threads)
{
    const int N = n_up + n_dn;
    if (n_up < 1 || n_dn < 0 || n_up > 64 || n_dn > 64 || n_det < 1 || n_walk < 0) return -1;
    uint64_t *uu = (uint64_t *)malloc(sizeof(uint64_t) * n_int * n_det);
    uint64_t *ud = (uint64_t *)malloc(sizeof(uint64_t) * n_int * n_det);
    int64_t *ik = (int64_t *)malloc(sizeof(int64_t) * n_det);
    int64_t *jk = (int64_t *)malloc(sizeof(int64_t) * n_det);
    int64_t U = distinct(n_int, n_det, det_up, uu);
    int64_t V = distinct(n_int, n_det, det_dn, ud);
    for (int64_t k = 0; k < n_det; ++k) {
        ik[k] = find(n_int, U, uu, det_up + k * n_int);
        jk[k] = find(n_int, V, ud, det_dn + k * n_int);
    }
    /* reference product: largest |c|, earliest on ties */
    int64_t kref = 0;
    for (int64_t k = 1; k < n_det; ++k)
        if (fabs(c[k]) > fabs(c[kref])) kref = k;
    int *deg_u = (int *)malloc(sizeof(int) * U);
    int *deg_d = (int *)malloc(sizeof(int) * (V > 0 ? V : 1));
    for (int64_t i = 0; i < U; ++i) {
        int pc = 0;
        for (int w = 0; w < n_int; ++w) pc += popcount64(uu[i * n_int + w] ^ uu[ik[kref] * n_int + w]);
        deg_u[i] = pc / 2;
    }
    for (int64_t j = 0; j < V; ++j) {
        int pc = 0;
        for (int w = 0; w < n_int; ++w) pc += popcount64(ud[j * n_int + w] ^ ud[jk[kref] * n_int + w]);
        deg_d[j] = pc / 2;
    }
    int *occ_u = (int *)malloc(sizeof(int) * U * (n_up > 0 ? n_up : 1));
    int *occ_d = (int *)malloc(sizeof(int) * V * (n_dn > 0 ? n_dn : 1));
    int bad = 0;
    for (int64_t i = 0; i < U; ++i)
        if (occupied(n_int, uu + i * n_int, occ_u + i * n_up) != n_up) bad = 1;
    for (int64_t j = 0; j < V; ++j)
        if (occupied(n_int, ud + j * n_int, occ_d + j * n_dn) != n_dn) bad = 1;
    for (int64_t i = 0; i < U * n_up && !bad; ++i) if (occ_u[i] >= n_mo) bad = 1;
    for (int64_t j = 0; j < V * n_dn && !bad; ++j) if (occ_d[j] >= n_mo) bad = 1;
    if (bad) {
        free(uu); free(ud); free(ik); free(jk); free(deg_u); free(deg_d); free(occ_u); free(occ_d);
        return -2;
    }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif

#pragma omp parallel
    {
        double *orb = (double *)malloc(sizeof(double) * 5 * n_mo * N);
        int nmax = n_up > n_dn ? n_up : n_dn;
        double *S = (double *)malloc(sizeof(double) * nmax * nmax);
        double *G = (double *)malloc(sizeof(double) * 4 * nmax * nmax);
        double *work = (double *)malloc(sizeof(double) * (2 * nmax * nmax + nmax));
        double *sg_u = (double *)malloc(sizeof(double) * U), *la_u = (double *)malloc(sizeof(double) * U);
        double *sg_d = (double *)malloc(sizeof(double) * V), *la_d = (double *)malloc(sizeof(double) * V);
        double *rt_u = (double *)malloc(sizeof(double) * U * 4 * n_up);
        double *rt_d = (double *)malloc(sizeof(double) * V * 4 * (n_dn > 0 ? n_dn : 1));
        double *cd = (double *)malloc(sizeof(double) * U);  /* mode 1: C D_dn  */
        double *dc = (double *)malloc(sizeof(double) * V);  /* mode 1: D_up^T C */
        double *du = (double *)malloc(sizeof(double) * U);
        double *dd = (double *)malloc(sizeof(double) * V);
        nsum *acc = (nsum *)malloc(sizeof(nsum) * (1 + 4 * N));
        double *aabs = (double *)malloc(sizeof(double) * (1 + 4 * N));

#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < n_walk; ++w) {
            const double *Rw = R + w * N * 3;
            for (int e = 0; e < N; ++e) {
                /* Eq. (1): S^sigma_k[i][j] = phi^sigma_j(r_i); one common set unless the
                 * down electrons have their own */
                const int dn = e >= n_up && alpha_dn;
                orc_orbitals(n_mo, n_prim, dn ? pw_dn : pw, dn ? alpha_dn : alpha,
                             dn ? coef_dn : coef, Rw + 3 * e, orb + e * 5 * n_mo);
            }
            /* spin determinants */
            for (int spin = 0; spin < 2; ++spin) {
                int n = spin == 0 ? n_up : n_dn;
                int e0 = spin == 0 ? 0 : n_up;
                int64_t cnt = spin == 0 ? U : V;
                const int *occ = spin == 0 ? occ_u : occ_d;
                double *sg = spin == 0 ? sg_u : sg_d, *la = spin == 0 ? la_u : la_d;
                double *rt = spin == 0 ? rt_u : rt_d;
                if (n == 0) { for (int64_t i = 0; i < cnt; ++i) { sg[i] = 1.0; la[i] = 0.0; } continue; }
                for (int64_t i = 0; i < cnt; ++i) {
                    const int *o = occ + i * n;
                    for (int e = 0; e < n; ++e)
                        for (int cc = 0; cc < n; ++cc) {
                            const double *ob = orb + (e0 + e) * 5 * n_mo;
                            S[e * n + cc] = ob[o[cc]];
                            for (int q = 0; q < 4; ++q) G[(q * n + e) * n + cc] = ob[(q + 1) * n_mo + o[cc]];
                        }
                    orc_slater(n, S, G, sg + i, la + i, rt + i * 4 * n, work);
                }
            }
            int dw = max_degree ? (int)max_degree[w] : 1 << 30;
            /* log shift: largest included product magnitude */
            double L = -INFINITY;
            for (int64_t k = 0; k < n_det; ++k) {
                int64_t i = ik[k], j = jk[k];
                if (deg_u[i] > dw || deg_d[j] > dw) continue;
                if (sg_u[i] == 0.0 || sg_d[j] == 0.0 || c[k] == 0.0) continue;
                double l = la_u[i] + la_d[j];
                if (l > L) L = l;
            }
            for (int t = 0; t < 1 + 4 * N; ++t) { acc[t].s = acc[t].c = 0.0; aabs[t] = 0.0; }
            if (L > -INFINITY) {
                if (mode == 0) {
                    for (int64_t k = 0; k < n_det; ++k) {
                        int64_t i = ik[k], j = jk[k];
                        if (deg_u[i] > dw || deg_d[j] > dw) continue;
                        if (sg_u[i] == 0.0 || sg_d[j] == 0.0) continue;
                        double term = c[k] * sg_u[i] * sg_d[j] * exp(la_u[i] + la_d[j] - L);
                        nadd(&acc[0], term);
                        aabs[0] += fabs(term);
                        const double *ru = rt_u + i * 4 * n_up;
                        for (int e = 0; e < n_up; ++e)
                            for (int q = 0; q < 4; ++q) {
                                double x = term * ru[e * 4 + q];
                                nadd(&acc[1 + e * 4 + q], x);
                                aabs[1 + e * 4 + q] += fabs(x);
                            }
                        const double *rd = rt_d + j * 4 * n_dn;
                        for (int e = 0; e < n_dn; ++e)
                            for (int q = 0; q < 4; ++q) {
                                double x = term * rd[e * 4 + q];
                                nadd(&acc[1 + (n_up + e) * 4 + q], x);
                                aabs[1 + (n_up + e) * 4 + q] += fabs(x);
                            }
                    }
                } else {
                    /* separate shifts per spin; the frame becomes L = Lu + Ld */
                    double Lu = -INFINITY, Ld = -INFINITY;
                    for (int64_t i = 0; i < U; ++i) if (sg_u[i] != 0.0 && deg_u[i] <= dw && la_u[i] > Lu) Lu = la_u[i];
                    for (int64_t j = 0; j < V; ++j) if (sg_d[j] != 0.0 && deg_d[j] <= dw && la_d[j] > Ld) Ld = la_d[j];
                    L = Lu + Ld;
                    for (int64_t i = 0; i < U; ++i) {
                        du[i] = (sg_u[i] == 0.0 || deg_u[i] > dw) ? 0.0 : sg_u[i] * exp(la_u[i] - Lu);
                        cd[i] = 0.0;
                    }
                    for (int64_t j = 0; j < V; ++j) {
                        dd[j] = (sg_d[j] == 0.0 || deg_d[j] > dw) ? 0.0 : sg_d[j] * exp(la_d[j] - Ld);
                        dc[j] = 0.0;
                    }
                    for (int64_t k = 0; k < n_det; ++k) {  /* the fused double mat-vec of Sec. 2.4 */
                        cd[ik[k]] += c[k] * dd[jk[k]];
                        dc[jk[k]] += c[k] * du[ik[k]];
                    }
                    for (int64_t j = 0; j < V; ++j) nadd(&acc[0], dc[j] * dd[j]);
                    for (int64_t i = 0; i < U; ++i) {
                        const double *ru = rt_u + i * 4 * n_up;
                        for (int e = 0; e < n_up; ++e)
                            for (int q = 0; q < 4; ++q) nadd(&acc[1 + e * 4 + q], du[i] * ru[e * 4 + q] * cd[i]);
                    }
                    for (int64_t j = 0; j < V; ++j) {
                        const double *rd = rt_d + j * 4 * n_dn;
                        for (int e = 0; e < n_dn; ++e)
                            for (int q = 0; q < 4; ++q)
                                nadd(&acc[1 + (n_up + e) * 4 + q], dc[j] * dd[j] * rd[e * 4 + q]);
                    }
                    for (int t = 0; t < 1 + 4 * N; ++t) aabs[t] = NAN; /* not defined in mode 1 */
                }
            }
            double psi = nval(&acc[0]);
            if (psi == 0.0) {
                sign_out[w] = 0.0;
                logabs_out[w] = -INFINITY;
                for (int t = 0; t < 4 * N; ++t) gl_out[w * 4 * N + t] = 0.0;
                if (rs_psi_out) rs_psi_out[w] = INFINITY;
                if (rs_gl_out) for (int t = 0; t < 4 * N; ++t) rs_gl_out[w * 4 * N + t] = INFINITY;
            } else {
                sign_out[w] = psi > 0 ? 1.0 : -1.0;
                logabs_out[w] = L + log(fabs(psi));
                for (int t = 0; t < 4 * N; ++t) gl_out[w * 4 * N + t] = nval(&acc[1 + t]) / psi;
                if (rs_psi_out) rs_psi_out[w] = aabs[0] / fabs(psi);
                if (rs_gl_out) for (int t = 0; t < 4 * N; ++t) rs_gl_out[w * 4 * N + t] = aabs[1 + t] / fabs(psi);
            }
        }
        free(orb); free(S); free(G); free(work); free(sg_u); free(la_u); free(sg_d); free(la_d);
        free(rt_u); free(rt_d); free(cd); free(dc); free(du); free(dd); free(acc); free(aabs);
    }
    free(uu); free(ud); free(ik); free(jk); free(deg_u); free(deg_d); free(occ_u); free(occ_d);
    return 0;
}
