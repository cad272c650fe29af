// Slater-Jastrow trial function and fixed-node diffusion Monte Carlo step
// for gfx950.
//
//  * Jastrow prefactor (the paper's Sec. 1 leaves it to standard techniques
//    at O(N^2) cost): J = sum_{i<j} a_ij r_ij / (1 + b_ee r_ij)
//    + sum_i a_en r_i / (1 + b_en r_i), with a_ij = 1/2 for opposite spins
//    and 1/4 for equal spins (the electron-electron cusp conditions); a_en =
//    -Z gives the electron-nucleus cusp.  Applied to the determinant
//    outputs: ln|Psi_T| = ln|Psi| + J, grad ln Psi_T = grad J + grad Psi/Psi,
//    lap Psi_T/Psi_T = lap J + |grad J|^2 + 2 grad J . grad Psi/Psi
//    + lap Psi/Psi.
//  * DMC step: drift-diffusion move with the Metropolis-Hastings test of the
//    VMC step, a move that changes the sign of Psi is rejected (fixed node),
//    branching weight w <- w exp(-tau ((E_L + E_L')/2 - E_T)), then the
//    population is redrawn with the comb (systematic resampling at fixed
//    population: walker i is copied as often as the comb teeth
//    (j + u) sum w / W fall into its share of the cumulative weight), every
//    copy with weight 1.  Sums are taken in a fixed order (one block), so the
//    step is deterministic for given random numbers.

#include "mdet_internal.h"

#include <math.h>

namespace mdet {

namespace {

constexpr int kJBlock = 256;
constexpr int kDmcBlock = 1024;

// u(r) = a r / (1 + b r) and its first two derivatives
__device__ __forceinline__ void pade(double a, double b, double r, double &u, double &du,
                                     double &d2u) {
    const double s = 1.0 / (1.0 + b * r);
    u = a * r * s;
    du = a * s * s;
    d2u = -2.0 * a * b * s * s * s;
}

}  // namespace

// one thread per walker: J, grad J, lap J and their combination with the
// determinant outputs, in place (nodes are left as they are)
__global__ void __launch_bounds__(kJBlock) k_jastrow(int64_t W, int N, int n_up, double b_ee,
                                                     double a_en, double b_en, const double *R,
                                                     double *logabs, double *gl) {
    const int64_t w = (int64_t)blockIdx.x * kJBlock + threadIdx.x;
    if (w >= W || !(logabs[w] > -INFINITY)) return;
    const double *Rw = R + w * 3 * N;
    double *g = gl + w * 4 * N;
    double J = 0.0;
    for (int i = 0; i < N; ++i) {
        const double xi = Rw[3 * i], yi = Rw[3 * i + 1], zi = Rw[3 * i + 2];
        double gx = 0.0, gy = 0.0, gz = 0.0, lap = 0.0;
        // electron-nucleus term
        const double ri = sqrt(xi * xi + yi * yi + zi * zi);
        if (a_en != 0.0) {
            double u, du, d2u;
            pade(a_en, b_en, ri, u, du, d2u);
            J += u;
            if (ri > 0.0) {
                gx += du * xi / ri;
                gy += du * yi / ri;
                gz += du * zi / ri;
                lap += d2u + 2.0 * du / ri;
            } else {
                lap += INFINITY * a_en;
            }
        }
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            const double dx = xi - Rw[3 * j], dy = yi - Rw[3 * j + 1], dz = zi - Rw[3 * j + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double a = ((i < n_up) == (j < n_up)) ? 0.25 : 0.5;
            double u, du, d2u;
            pade(a, b_ee, r, u, du, d2u);
            if (j > i) J += u;
            if (r > 0.0) {
                gx += du * dx / r;
                gy += du * dy / r;
                gz += du * dz / r;
                lap += d2u + 2.0 * du / r;
            } else {
                lap += INFINITY;
            }
        }
        const double dgx = g[4 * i], dgy = g[4 * i + 1], dgz = g[4 * i + 2];
        g[4 * i + 3] += lap + gx * gx + gy * gy + gz * gz + 2.0 * (gx * dgx + gy * dgy + gz * dgz);
        g[4 * i] = dgx + gx;
        g[4 * i + 1] = dgy + gy;
        g[4 * i + 2] = dgz + gz;
    }
    logabs[w] += J;
}

// keep E_L(R) of every walker before the move
__global__ void __launch_bounds__(kJBlock) k_dmc_save(int64_t W, const double *elocal, double *e_old) {
    const int64_t w = (int64_t)blockIdx.x * kJBlock + threadIdx.x;
    if (w < W) e_old[w] = elocal[w];
}

// one block: branching weights, the step's sums and the cumulative weights.
// Thread t owns the contiguous walkers [t per, (t + 1) per).
// sums[0] = sum w, sums[1] = sum w E_L, sums[2] = sum w^2, sums[3] = accepted moves.
__global__ void __launch_bounds__(kDmcBlock) k_dmc_weights(int64_t W, double tau, double e_trial,
                                                           const double *e_old, const double *e_new,
                                                           const int32_t *accepted, double *weight,
                                                           double *cum, double *sums) {
    __shared__ double s0[kDmcBlock], s1[kDmcBlock], s2[kDmcBlock], s3[kDmcBlock];
    const int t = threadIdx.x;
    const int64_t per = (W + kDmcBlock - 1) / kDmcBlock;
    const int64_t w0 = (int64_t)t * per, w1 = min(W, w0 + per);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int64_t w = w0; w < w1; ++w) {
        const double eo = e_old[w], en = e_new[w];
        double x = 0.0;
        if (isfinite(eo) && isfinite(en)) x = weight[w] * exp(-tau * (0.5 * (eo + en) - e_trial));
        weight[w] = x;
        a0 += x;
        a1 += x * (isfinite(en) ? en : 0.0);
        a2 += x * x;
        a3 += (double)accepted[w];
        cum[w] = a0;  // inclusive, within the thread's walkers
    }
    s0[t] = a0;
    s1[t] = a1;
    s2[t] = a2;
    s3[t] = a3;
    __syncthreads();
    // exclusive prefix of the per-thread totals (fixed order), then the totals
    if (t == 0) {
        double run = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
        for (int k = 0; k < kDmcBlock; ++k) {
            const double v = s0[k];
            s0[k] = run;
            run += v;
            t1 += s1[k];
            t2 += s2[k];
            t3 += s3[k];
        }
        sums[0] = run;
        sums[1] = t1;
        sums[2] = t2;
        sums[3] = t3;
    }
    __syncthreads();
    const double base = s0[t];
    for (int64_t w = w0; w < w1; ++w) cum[w] += base;
}

// comb: new walker j takes the first walker i whose inclusive cumulative
// weight exceeds (j + u) sum w / W (walker j itself if the total is zero)
__global__ void __launch_bounds__(kJBlock) k_dmc_select(int64_t W, double comb_u, const double *cum,
                                                        const double *sums, int32_t *src) {
    const int64_t j = (int64_t)blockIdx.x * kJBlock + threadIdx.x;
    if (j >= W) return;
    const double tot = sums[0];
    if (!(tot > 0.0)) {
        src[j] = (int32_t)j;
        return;
    }
    const double x = ((double)j + comb_u) * (tot / (double)W);
    int64_t lo = 0, hi = W - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cum[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    src[j] = (int32_t)lo;
}

// gather the selected walkers' state into the temporaries (weights reset to 1)
__global__ void __launch_bounds__(kJBlock) k_dmc_gather(int64_t W, int N, const int32_t *src,
                                                        const double *R, const double *sign,
                                                        const double *logabs, const double *gl,
                                                        const double *elocal, double *Rt,
                                                        double *st, double *lt, double *gt,
                                                        double *et) {
    const int64_t t = (int64_t)blockIdx.x * kJBlock + threadIdx.x;
    const int per = 3 * N + 4 * N + 3;
    if (t >= W * per) return;
    const int64_t j = t / per;
    const int k = (int)(t - j * per);
    const int64_t i = src[j];
    if (k < 3 * N) Rt[j * 3 * N + k] = R[i * 3 * N + k];
    else if (k < 7 * N) gt[j * 4 * N + (k - 3 * N)] = gl[i * 4 * N + (k - 3 * N)];
    else if (k == 7 * N) st[j] = sign[i];
    else if (k == 7 * N + 1) lt[j] = logabs[i];
    else et[j] = elocal[i];
}

__global__ void __launch_bounds__(kJBlock) k_dmc_scatter(int64_t W, int N, const double *Rt,
                                                         const double *st, const double *lt,
                                                         const double *gt, const double *et,
                                                         double *R, double *sign, double *logabs,
                                                         double *gl, double *elocal,
                                                         double *weight) {
    const int64_t t = (int64_t)blockIdx.x * kJBlock + threadIdx.x;
    const int per = 3 * N + 4 * N + 3;
    if (t >= W * per) return;
    const int64_t j = t / per;
    const int k = (int)(t - j * per);
    if (k < 3 * N) R[j * 3 * N + k] = Rt[j * 3 * N + k];
    else if (k < 7 * N) gl[j * 4 * N + (k - 3 * N)] = gt[j * 4 * N + (k - 3 * N)];
    else if (k == 7 * N) sign[j] = st[j];
    else if (k == 7 * N + 1) logabs[j] = lt[j];
    else {
        elocal[j] = et[j];
        weight[j] = 1.0;
    }
}

namespace {
inline dim3 gj(int64_t n) { return dim3((unsigned)((n + kJBlock - 1) / kJBlock)); }
}  // namespace

void launch_jastrow(int64_t W, int N, int n_up, const JastrowParams &p, const double *R,
                    double *logabs, double *gl, hipStream_t st) {
    k_jastrow<<<gj(W), dim3(kJBlock), 0, st>>>(W, N, n_up, p.b_ee, p.a_en, p.b_en, R, logabs, gl);
}

void launch_dmc_save(int64_t W, const double *elocal, double *e_old, hipStream_t st) {
    k_dmc_save<<<gj(W), dim3(kJBlock), 0, st>>>(W, elocal, e_old);
}

void launch_dmc_branch(int64_t W, int N, double tau, double e_trial, double comb_u,
                       const double *e_old, const int32_t *accepted, DmcWork &d, double *R,
                       double *sign, double *logabs, double *gl, double *elocal, double *weight,
                       double *sums, hipStream_t st) {
    k_dmc_weights<<<dim3(1), dim3(kDmcBlock), 0, st>>>(W, tau, e_trial, e_old, elocal, accepted,
                                                       weight, d.cum, sums);
    k_dmc_select<<<gj(W), dim3(kJBlock), 0, st>>>(W, comb_u, d.cum, sums, d.src);
    const int64_t n = W * (7 * (int64_t)N + 3);
    k_dmc_gather<<<gj(n), dim3(kJBlock), 0, st>>>(W, N, d.src, R, sign, logabs, gl, elocal, d.R,
                                                  d.sign, d.logabs, d.gl, d.elocal);
    k_dmc_scatter<<<gj(n), dim3(kJBlock), 0, st>>>(W, N, d.R, d.sign, d.logabs, d.gl, d.elocal, R,
                                                   sign, logabs, gl, elocal, weight);
}

}  // namespace mdet
