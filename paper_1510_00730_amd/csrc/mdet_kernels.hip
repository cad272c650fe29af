// HIP kernels of the multideterminant evaluator for gfx950.
//
// Per walker w and spin sigma (electrons e of that spin, n of them):
//   Phi[e][m], grad~Phi[e][q][m]          orbitals at the electrons (Sec. 2)
//   E[m]                                  power-of-two column scale of orbital m
//   A = Phi'[:, occ0]                     scaled reference Slater matrix
//   X = A^-1 (LU with partial pivoting + one residual-correction step, Sec. 2.2)
//   T = X Phi'                            the table of the table method (Sec. 5)
//   R_d = eps_d det T[h_d, p_d] 2^dX_d    ratio D_d / D_0 of every distinct det
//   u = C R_dn, v = C^T R_up, psi = R_up.u      (the two mat-vecs of Sec. 2.4)
//   grad~_e Psi / Psi = grad~_e D0/D0 + sum_{m,c} B_q[e,m] Gamma[m,c] X[c,e] / psi
// where B_q = grad~_q Phi' - grad~_q Phi'[:,occ0] T and Gamma aggregates the
// adjugates of the small excitation matrices weighted by u (up) or v (down).
// The derivative part is the exact rewriting of Eqs. (grad_psi)-(nabla) in
// terms of the table.  A (walker, spin) whose reference is ill-conditioned is
// evaluated by direct LU of every determinant instead (the analogue of the
// paper's O(n^3) recomputation rule for failed updates, Sec. 2.2).
//
// Reductions are done in a fixed order, so FP64 results are bitwise
// reproducible run to run.

#include "mdet_internal.h"

#include <math.h>

#include <algorithm>
#include <climits>

namespace mdet {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxN = MDET_MAX_SPIN_ELEC;

__device__ __forceinline__ double pow2(int k) { return ldexp(1.0, k); }

// Axis factors of d^j/dx^j [x^a e^{-alpha x^2}] e^{+alpha x^2}, j = 0, 1, 2.
__device__ __forceinline__ void axis3(double x, int a, double al, double &f0, double &f1,
                                      double &f2) {
    double p = 1.0, pm1 = 0.0, pm2 = 0.0;  // x^a, x^(a-1), x^(a-2) (0 when negative)
    for (int i = 0; i < a; ++i) {
        pm2 = pm1;
        pm1 = p;
        p *= x;
    }
    const double da = (double)a;
    f0 = p;
    f1 = da * pm1 - 2.0 * al * p * x;
    f2 = da * (da - 1.0) * pm2 - 2.0 * al * (2.0 * da + 1.0) * p + 4.0 * al * al * p * x * x;
}

__device__ void orbital5(const Prim *prim, int P, int m, double x, double y, double z,
                         double out[5]) {
    const double r2 = x * x + y * y + z * z;
    double v = 0, gx = 0, gy = 0, gz = 0, lap = 0;
    for (int p = 0; p < P; ++p) {
        const Prim q = prim[m * P + p];
        if (q.coef == 0.0) continue;
        const double g = q.coef * exp(-q.alpha * r2);
        double x0, x1, x2, y0, y1, y2, z0, z1, z2;
        axis3(x, q.a, q.alpha, x0, x1, x2);
        axis3(y, q.b, q.alpha, y0, y1, y2);
        axis3(z, q.c, q.alpha, z0, z1, z2);
        const double yz = y0 * z0;
        v += g * x0 * yz;
        gx += g * x1 * yz;
        gy += g * x0 * y1 * z0;
        gz += g * x0 * y0 * z1;
        lap += g * (x2 * yz + x0 * (y2 * z0 + y0 * z2));
    }
    out[0] = v;
    out[1] = gx;
    out[2] = gy;
    out[3] = gz;
    out[4] = lap;
}

// exponent k with |x| = f 2^k, f in [0.5, 1); 0 for x == 0
__device__ __forceinline__ int expo(double x) {
    int k = 0;
    if (x != 0.0) (void)frexp(x, &k);
    return k;
}

// deterministic block max / sum (blockDim.x == kBlock)
__device__ int block_max_int(int v, int *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    int r = red[0];
    __syncthreads();
    return r;
}

template <typename F>
__device__ F block_sum(F v, F *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    F r = red[0];
    __syncthreads();
    return r;
}

// small determinants and cofactors (s <= 4), row-major s x s
__device__ __forceinline__ double det2(double a, double b, double c, double d) {
    return a * d - b * c;
}

__device__ double det3(const double *m, int ld) {
    return m[0] * det2(m[ld + 1], m[ld + 2], m[2 * ld + 1], m[2 * ld + 2]) -
           m[1] * det2(m[ld + 0], m[ld + 2], m[2 * ld + 0], m[2 * ld + 2]) +
           m[2] * det2(m[ld + 0], m[ld + 1], m[2 * ld + 0], m[2 * ld + 1]);
}

__device__ double small_det(const double *m, int s) {
    switch (s) {
    case 0: return 1.0;
    case 1: return m[0];
    case 2: return det2(m[0], m[1], m[2], m[3]);
    case 3: return det3(m, 3);
    default: {
        // Laplace expansion along the first two rows (products of 2x2 minors)
        const double *r0 = m, *r1 = m + 4, *r2 = m + 8, *r3 = m + 12;
        double acc = 0.0;
        const int pr[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        const double sg[6] = {1, -1, 1, 1, -1, 1};
        for (int t = 0; t < 6; ++t) {
            const int i = pr[t][0], j = pr[t][1];
            const int k = pr[5 - t][0], l = pr[5 - t][1];
            acc += sg[t] * det2(r0[i], r0[j], r1[i], r1[j]) * det2(r2[k], r2[l], r3[k], r3[l]);
        }
        return acc;
    }
    }
}

// cofactor C_{ab} = (-1)^{a+b} det(m without row a, column b)
__device__ double cofactor(const double *m, int s, int a, int b) {
    double sub[9];
    int t = 0;
    for (int i = 0; i < s; ++i) {
        if (i == a) continue;
        for (int j = 0; j < s; ++j) {
            if (j == b) continue;
            sub[t++] = m[i * s + j];
        }
    }
    const double d = small_det(sub, s - 1);
    return ((a + b) & 1) ? -d : d;
}

__device__ __forceinline__ int delta_exponent(const DetDesc &D, const int *Ex, const int *occ0) {
    int dx = 0;
    for (int a = 0; a < D.s; ++a) dx += Ex[D.p[a]] - Ex[occ0[D.h[a]]];
    return dx;
}

// Gauss-Jordan inversion with partial pivoting of an S x S matrix (row-major),
// fully unrolled so the matrix lives in registers.  Returns false on an exactly
// zero pivot.  det receives the determinant (product of pivots and row-swap signs).
template <int S>
__device__ __forceinline__ bool gj_inverse(const double *m, double *inv, double &det) {
    double a[S][S], b[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int k = 0; k < S; ++k) {
            a[i][k] = m[i * S + k];
            b[i][k] = (i == k) ? 1.0 : 0.0;
        }
    det = 1.0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        int p = j;
        double best = fabs(a[j][j]);
#pragma unroll
        for (int i = j + 1; i < S; ++i)
            if (fabs(a[i][j]) > best) {
                best = fabs(a[i][j]);
                p = i;
            }
        if (!(best > 0.0)) return false;
#pragma unroll
        for (int i = j + 1; i < S; ++i)
            if (i == p) {
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    double t = a[i][k];
                    a[i][k] = a[j][k];
                    a[j][k] = t;
                    t = b[i][k];
                    b[i][k] = b[j][k];
                    b[j][k] = t;
                }
                det = -det;
            }
        const double piv = a[j][j];
        det *= piv;
        const double r = 1.0 / piv;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            a[j][k] *= r;
            b[j][k] *= r;
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (i == j) continue;
            const double f = a[i][j];
#pragma unroll
            for (int k = 0; k < S; ++k) {
                a[i][k] -= f * a[j][k];
                b[i][k] -= f * b[j][k];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int k = 0; k < S; ++k) inv[i * S + k] = b[i][k];
    return true;
}

// LU (partial pivoting) determinant of an S x S matrix, unrolled.
template <int S>
__device__ __forceinline__ double det_lu(const double *m) {
    double a[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int k = 0; k < S; ++k) a[i][k] = m[i * S + k];
    double det = 1.0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        int p = j;
        double best = fabs(a[j][j]);
#pragma unroll
        for (int i = j + 1; i < S; ++i)
            if (fabs(a[i][j]) > best) {
                best = fabs(a[i][j]);
                p = i;
            }
        if (!(best > 0.0)) return 0.0;
#pragma unroll
        for (int i = j + 1; i < S; ++i)
            if (i == p) {
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    const double t = a[i][k];
                    a[i][k] = a[j][k];
                    a[j][k] = t;
                }
                det = -det;
            }
        det *= a[j][j];
#pragma unroll
        for (int i = j + 1; i < S; ++i) {
            const double l = a[i][j] / a[j][j];
#pragma unroll
            for (int k = j + 1; k < S; ++k) a[i][k] -= l * a[j][k];
        }
    }
    return det;
}

// Offsets of the walker-major vectors R, u, v: entry d of spin sp for walker
// w sits at w * (Upad + Vpad) + (sp ? Upad : 0) + d.
__device__ __forceinline__ size_t rv_index(const KernelArgs &a, int sp, int d, int w) {
    return (size_t)w * (size_t)(a.wk.Upad + a.wk.Vpad) + (sp ? (size_t)a.wk.Upad : 0) + d;
}

// psi of walker w: the row-split partial sums of the sparse combination
// (accumulated in FP64 in both precisions), added in a fixed order
__device__ __forceinline__ double psi_value(const KernelArgs &a, int w) {
    double s = 0.0;
    for (int k = 0; k < a.psi_nparts; ++k) s += a.wk.psi64[(size_t)w * kPsiParts + k];
    return s;
}

// s x s excitation matrix M[a][b] = T[h_a][p_b], compile-time s
template <int S>
__device__ __forceinline__ void load_exc(const DetDesc &D, const double *T, int M, double *m) {
#pragma unroll
    for (int a2 = 0; a2 < S; ++a2)
#pragma unroll
        for (int b2 = 0; b2 < S; ++b2) m[a2 * S + b2] = T[D.h[a2] * M + D.p[b2]];
}

// eps_d det M_d (the ratio D_d / D_0 before the exponent shift)
template <int S>
__device__ __forceinline__ double exc_ratio(const DetDesc &D, const double *T, int M) {
    double m[S * S];
    load_exc<S>(D, T, M, m);
    double d;
    if constexpr (S == 1) d = m[0];
    else if constexpr (S == 2) d = det2(m[0], m[1], m[2], m[3]);
    else d = det_lu<S>(m);
    return (double)D.eps * d;
}

__device__ __forceinline__ double ratio_any(const DetDesc &D, const double *T, int M) {
    switch (D.s) {
    case 0: return (double)D.eps;
    case 1: return exc_ratio<1>(D, T, M);
    case 2: return exc_ratio<2>(D, T, M);
    case 3: return exc_ratio<3>(D, T, M);
    default: return exc_ratio<4>(D, T, M);
    }
}

// coef * C_ab of M_d into dst[a*S + b] (C_ab = adj[b][a]), compile-time s
template <int S>
__device__ __forceinline__ void stage_adj(const DetDesc &D, const double *T, int M, double coef,
                                          double *dst) {
    double m[S * S], adj[S * S];
    load_exc<S>(D, T, M, m);
    if constexpr (S == 1) {
        adj[0] = 1.0;
    } else if constexpr (S == 2) {
        adj[0] = m[3];
        adj[1] = -m[1];
        adj[2] = -m[2];
        adj[3] = m[0];
    } else {
        double det = 0.0;
        if (gj_inverse<S>(m, adj, det)) {
#pragma unroll
            for (int t = 0; t < S * S; ++t) adj[t] *= det;
        } else {
            for (int a2 = 0; a2 < S; ++a2)  // exactly singular: explicit cofactors
                for (int b2 = 0; b2 < S; ++b2) adj[b2 * S + a2] = cofactor(m, S, a2, b2);
        }
    }
#pragma unroll
    for (int a2 = 0; a2 < S; ++a2)
#pragma unroll
        for (int b2 = 0; b2 < S; ++b2) dst[a2 * S + b2] = coef * adj[b2 * S + a2];
}

}  // namespace

// ---------------------------------------------------------------------------
// K1+K2+K3: orbitals, scaled reference inverse, refinement, table T, g0.
// One block per (walker, spin).
// ---------------------------------------------------------------------------
namespace {

// Gauss-Jordan elimination with partial pivoting of the n x n matrix held one
// row per lane (lanes 0..n-1 of one wave, n <= kMaxN): on return lane i
// holds row i of the inverse in x[] and every lane the log|det| and sign.
// Returns false on an exactly zero pivot.
__device__ bool wave_gauss_jordan(int n, int lane, double (&r)[kMaxN], double (&x)[kMaxN],
                                  double &logabs, double &sign) {
#pragma unroll
    for (int k = 0; k < kMaxN; ++k) x[k] = (lane == k) ? 1.0 : 0.0;
    logabs = 0.0;
    sign = 1.0;
#pragma unroll
    for (int j = 0; j < kMaxN; ++j) {
        if (j >= n) break;
        double v = (lane >= j && lane < n) ? fabs(r[j]) : -1.0;
        int id = lane;
        for (int off = 32; off > 0; off >>= 1) {
            const double v2 = __shfl_xor(v, off, 64);
            const int i2 = __shfl_xor(id, off, 64);
            if (v2 > v || (v2 == v && i2 < id)) {
                v = v2;
                id = i2;
            }
        }
        if (!(v > 0.0)) return false;
        const int src = (lane == j) ? id : ((lane == id) ? j : lane);
        double pr[kMaxN], px[kMaxN];
#pragma unroll
        for (int k = 0; k < kMaxN; ++k) {
            r[k] = __shfl(r[k], src, 64);
            x[k] = __shfl(x[k], src, 64);
        }
#pragma unroll
        for (int k = 0; k < kMaxN; ++k) {
            pr[k] = __shfl(r[k], j, 64);
            px[k] = __shfl(x[k], j, 64);
        }
        const double piv = pr[j];
        if (id != j) sign = -sign;
        if (piv < 0.0) sign = -sign;
        logabs += log(fabs(piv));
        const double rinv = 1.0 / piv;
        if (lane == j) {
#pragma unroll
            for (int k = 0; k < kMaxN; ++k) {
                r[k] = pr[k] * rinv;
                x[k] = px[k] * rinv;
            }
        } else {
            const double f = r[j] * rinv;
#pragma unroll
            for (int k = 0; k < kMaxN; ++k) {
                r[k] -= f * pr[k];
                x[k] -= f * px[k];
            }
        }
    }
    return true;
}

}  // namespace

__global__ void __launch_bounds__(kBlock) k_reference(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, N = a.N, e0 = S.e0, tid = threadIdx.x;
    extern __shared__ double lds[];
    double *phi0 = lds;             // [n][M] scaled orbital values
    double *scl = phi0 + n * M;     // [M]    2^-E[m]
    double *Aor = scl + M;          // [n][n] scaled reference
    double *Xs = Aor + n * n;       // [n][n]
    double *Rm = Xs + n * n;        // [n][n]
    int *Ex = (int *)(Rm + n * n);  // [M]
    __shared__ int s_state;         // 0 ok, 2 singular
    __shared__ double s_logabs, s_sign;
    __shared__ double colA[kMaxN], colX[kMaxN];
    const size_t ws = (size_t)w * 2 + sp;

    double *phig = a.wk.phi + (size_t)w * N * 5 * M;
    const double *Rw = a.R + (size_t)w * N * 3;
    // orbitals and derivatives, written once (unscaled)
    for (int idx = tid; idx < n * M; idx += kBlock) {
        const int e = idx / M, m = idx - e * M;
        const double *r = Rw + 3 * (e0 + e);
        double o[5];
        orbital5(a.prim, a.P, m, r[0], r[1], r[2], o);
        double *dst = phig + (size_t)(e0 + e) * 5 * M + m;
        for (int q = 0; q < 5; ++q) dst[q * M] = o[q];
        phi0[e * M + m] = o[0];
    }
    __syncthreads();
    // power-of-two column scale of every orbital over this spin's electrons
    for (int m = tid; m < M; m += kBlock) {
        double mx = 0.0;
        for (int e = 0; e < n; ++e) mx = fmax(mx, fabs(phi0[e * M + m]));
        Ex[m] = expo(mx);
        scl[m] = pow2(-Ex[m]);
        a.wk.E[ws * M + m] = Ex[m];
    }
    __syncthreads();
    for (int idx = tid; idx < n * M; idx += kBlock) phi0[idx] *= scl[idx % M];
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int e = idx / n, c = idx - e * n;
        Aor[idx] = phi0[e * M + S.occ0[c]];
    }
    __syncthreads();
    // inverse of the scaled reference by one wave (row per lane)
    if (tid < 64) {
        double r[kMaxN], x[kMaxN];
#pragma unroll
        for (int k = 0; k < kMaxN; ++k) r[k] = (tid < n && k < n) ? Aor[tid * n + k] : 0.0;
        double la, sg;
        const bool ok = wave_gauss_jordan(n, tid, r, x, la, sg);
        if (ok && tid < n)
            for (int k = 0; k < n; ++k) Xs[tid * n + k] = x[k];
        if (tid == 0) {
            s_state = ok ? 0 : 2;
            s_logabs = la;
            s_sign = sg;
        }
    }
    if (tid == 0) a.wk.Kmax[ws] = INT_MIN;
    __syncthreads();
    if (s_state) {
        if (tid == 0) {
            a.wk.flag[ws] = 2;
            a.wk.logdet0[ws] = 0.0;
            a.wk.sign0[ws] = 1.0;
        }
        return;
    }
    if (tid == 0) {
        int sx = 0;
        for (int c = 0; c < n; ++c) sx += Ex[S.occ0[c]];
        a.wk.logdet0[ws] = s_logabs + (double)sx * 0.69314718055994530942;
        a.wk.sign0[ws] = s_sign;
    }
    // one residual-correction step: X <- X + X (I - A X)
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int i = idx / n, j = idx - i * n;
        double t = (i == j) ? 1.0 : 0.0;
        for (int k = 0; k < n; ++k) t -= Aor[i * n + k] * Xs[k * n + j];
        Rm[idx] = t;
    }
    __syncthreads();
    double xr[4];
    int nx = 0;
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int i = idx / n, j = idx - i * n;
        double t = Xs[idx];
        for (int k = 0; k < n; ++k) t += Xs[i * n + k] * Rm[k * n + j];
        xr[nx++] = t;
    }
    __syncthreads();
    nx = 0;
    for (int idx = tid; idx < n * n; idx += kBlock) Xs[idx] = xr[nx++];
    __syncthreads();
    const double *X = Xs;
    if (tid < n) {
        double ca = 0.0, cx = 0.0;
        for (int i = 0; i < n; ++i) {
            ca += fabs(Aor[i * n + tid]);
            cx += fabs(X[i * n + tid]);
        }
        colA[tid] = ca;
        colX[tid] = cx;
    }
    __syncthreads();
    if (tid == 0) {
        double na = 0.0, nxm = 0.0;
        for (int c = 0; c < n; ++c) {
            na = fmax(na, colA[c]);
            nxm = fmax(nxm, colX[c]);
        }
        const double kappa = na * nxm;
        a.wk.flag[ws] = (kappa <= a.kappa_max) ? 0 : 1;  // NaN -> fallback
    }
    double *Xg = a.wk.X + ws * a.nmax * a.nmax;
    for (int idx = tid; idx < n * n; idx += kBlock) Xg[idx] = X[idx];
    double *Tg = a.wk.T + ws * a.nmax * M;
    for (int idx = tid; idx < n * M; idx += kBlock) {
        const int c = idx / M, m = idx - c * M;
        double t = 0.0;
        for (int e = 0; e < n; ++e) t += X[c * n + e] * phi0[e * M + m];
        Tg[idx] = t;
    }
    for (int idx = tid; idx < 4 * n; idx += kBlock) {
        const int e = idx >> 2, q = idx & 3;
        const double *g = phig + (size_t)(e0 + e) * 5 * M + (size_t)(1 + q) * M;
        double t = 0.0;
        for (int c = 0; c < n; ++c) t += X[c * n + e] * (g[S.occ0[c]] * scl[S.occ0[c]]);
        a.wk.g0[((size_t)w * N + e0 + e) * 4 + q] = t;
    }
}

// ---------------------------------------------------------------------------
// K4: ratios R_d / 2^K of every distinct determinant (table method).
// One block per (walker, spin); one thread per determinant.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_ratios(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] != 0) return;
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, tid = threadIdx.x;
    extern __shared__ double lds[];
    double *T = lds;                 // [n][M]
    int *Ex = (int *)(T + n * M);    // [M]
    int *occ0 = Ex + M;              // [n]
    __shared__ int red[kBlock];
    const double *Tg = a.wk.T + ws * a.nmax * M;
    for (int idx = tid; idx < n * M; idx += kBlock) T[idx] = Tg[idx];
    for (int m = tid; m < M; m += kBlock) Ex[m] = a.wk.E[ws * M + m];
    for (int c = tid; c < n; c += kBlock) occ0[c] = S.occ0[c];
    __syncthreads();
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    int kmax = INT_MIN;
    for (int d = tid; d < S.U; d += kBlock) {
        const DetDesc D = S.desc[d];
        double r = 0.0;
        if (D.s <= dmax) {
            r = ratio_any(D, T, M);
            if (r != 0.0) kmax = max(kmax, expo(r) + delta_exponent(D, Ex, occ0));
        }
        a.wk.R64[rv_index(a, sp, d, w)] = r;
    }
    int K = block_max_int(kmax, red);
    if (K == INT_MIN) K = 0;
    if (tid == 0) a.wk.K[ws] = K;
    for (int d = tid; d < S.U; d += kBlock) {
        const DetDesc D = S.desc[d];
        const size_t o = rv_index(a, sp, d, w);
        const double r = ldexp(a.wk.R64[o], delta_exponent(D, Ex, occ0) - K);
        if (a.precision == MDET_MIXED) a.wk.R32[o] = (float)r;
        else a.wk.R64[o] = r;
    }
}

// ---------------------------------------------------------------------------
// K5: the two sparse products of Sec. 2.4 for a tile of 64 walkers (one per
// lane), 16 waves per block:
//   pass 0:  u = C R_dn  (CSR rows, gathering R_dn)  and the psi partials R_up . u
//   pass 1:  v = C^T R_up (CSC columns, gathering R_up)
// A wave owns whole rows, so the entries of C are wave-uniform (scalar loads)
// and each one feeds 64 fused multiply-adds; the gathered vector of the 64
// walkers sits in LDS, CC entries at a time.  The kernel is bound by LDS
// bandwidth, which leaves ALU slack: the FP32 variant spends it on a
// compensated (TwoSum) accumulation.  grid.x = walker tiles x row splits,
// grid.y = pass.
// ---------------------------------------------------------------------------
constexpr int kSpmmWaves = 16;
constexpr int kSpmmLd = kSpmmTile + 1;  // LDS row pitch of the staged vector

// s + x with the rounding error of the addition carried in comp (TwoSum)
template <typename F>
__device__ __forceinline__ void two_sum_acc(F &s, F &comp, F x) {
#pragma clang fp contract(off)
    const F t = s + x;
    const F z = t - s;
    comp += (s - (t - z)) + (x - z);
    s = t;
}

template <typename F, int CC, bool COMP>
__global__ void __launch_bounds__(64 * kSpmmWaves)
    k_spmm(KernelArgs a, const F *__restrict__ R, F *__restrict__ uv,
           const F *__restrict__ rval, const F *__restrict__ cval,
           const int32_t *__restrict__ rcol, const int32_t *__restrict__ crow,
           const int32_t *__restrict__ rseg, const int32_t *__restrict__ cseg, int nch_r, int nch_c,
           int rsplit) {
    __shared__ F G[CC * kSpmmLd];
    __shared__ double red[kSpmmWaves][kSpmmTile];
    const int pass = blockIdx.y;
    const int tile = blockIdx.x / rsplit, rs = blockIdx.x - tile * rsplit;
    const int W = (int)a.W;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w0 = tile * kSpmmTile, w = w0 + lane;
    const bool active = w < W;
    const int nrows = pass ? a.C.V : a.C.U;
    const int ncols = pass ? a.C.U : a.C.V;
    const int nch = pass ? nch_c : nch_r;
    const int32_t *__restrict__ idx = pass ? crow : rcol;
    const int32_t *__restrict__ seg = pass ? cseg : rseg;
    const F *__restrict__ val = pass ? cval : rval;
    const size_t RV = (size_t)a.wk.Upad + a.wk.Vpad;
    const size_t goff = pass ? 0 : (size_t)a.wk.Upad;   // gathered: R_up (pass 1) / R_dn (pass 0)
    const size_t ooff = pass ? (size_t)a.wk.Upad : 0;   // written: v / u
    // uneven batches: the tile reaches only determinants (rows and columns in
    // ascending-degree execution order) up to its walkers' largest degree
    int dmax = MDET_MAX_DEGREE;
    if (a.max_degree) {
        int dm = active ? (int)a.max_degree[w] : 0;
        for (int off = 32; off > 0; off >>= 1) dm = max(dm, __shfl_xor(dm, off, 64));
        dmax = min(max(dm, 0), MDET_MAX_DEGREE);
    }
    const int32_t *__restrict__ degend = pass ? a.C.cdeg : a.C.rdeg;
    const int nrows_eff = (pass ? a.sp[1] : a.sp[0]).deg_end[dmax];
    const int ncols_eff = (pass ? a.sp[0] : a.sp[1]).deg_end[dmax];
    const int r0 = (int)((int64_t)nrows * rs / rsplit);
    const int r1 = min((int)((int64_t)nrows * (rs + 1) / rsplit), nrows_eff);
    double part = 0.0;
    for (int c = 0; c < nch; ++c) {
        const int cb = c * CC;
        if (cb >= ncols_eff) break;
        const int nc = min(CC, ncols_eff - cb);
        __syncthreads();
        // walker-major source: consecutive threads read consecutive entries of
        // one walker; the LDS row pitch kSpmmLd = 65 keeps both the stores here
        // and the lane-contiguous reads below free of bank conflicts
        for (int t = threadIdx.x; t < nc * kSpmmTile; t += 64 * kSpmmWaves) {
            const int ww = t / nc, jj = t - ww * nc;
            G[jj * kSpmmLd + ww] = (w0 + ww < W) ? R[(size_t)(w0 + ww) * RV + goff + cb + jj] : (F)0;
        }
        __syncthreads();
        for (int i = r0 + wave; i < r1; i += kSpmmWaves) {
            const int kb = seg[(size_t)c * nrows + i];
            const int ke = min(seg[(size_t)(c + 1) * nrows + i],
                               degend[(size_t)i * (MDET_MAX_DEGREE + 1) + dmax]);
            const size_t o = (size_t)w * RV + ooff + i;
            F s = (c == 0 || !active) ? (F)0 : uv[o];
            // 8 nonzeros per step: their scalar loads and LDS reads are all in
            // flight before the first multiply-add; two independent sums
            F s2 = 0, comp = 0, comp2 = 0;
            int k = kb;
            for (; k + 8 <= ke; k += 8) {
                int jx[8];
                F vx[8], gx[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    jx[t] = idx[k + t];
                    vx[t] = val[k + t];
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) gx[t] = G[(jx[t] - cb) * kSpmmLd + lane];
#pragma unroll
                for (int t = 0; t < 8; t += 2) {
                    if constexpr (COMP) {
                        two_sum_acc(s, comp, vx[t] * gx[t]);
                        two_sum_acc(s2, comp2, vx[t + 1] * gx[t + 1]);
                    } else {
                        s += vx[t] * gx[t];
                        s2 += vx[t + 1] * gx[t + 1];
                    }
                }
            }
            // tail: the same even/odd split by offset in the row, so that a
            // shorter segment (entries skipped for an uneven batch, all zero)
            // sums the remaining entries in exactly the same grouping
            for (; k < ke; ++k) {
                const F x = val[k] * G[(idx[k] - cb) * kSpmmLd + lane];
                const bool odd = ((k - kb) & 1) != 0;
                if constexpr (COMP) {
                    if (odd) two_sum_acc(s2, comp2, x);
                    else two_sum_acc(s, comp, x);
                } else {
                    if (odd) s2 += x;
                    else s += x;
                }
            }
            if constexpr (COMP) {
                two_sum_acc(s, comp, s2);
                s += comp + comp2;
            } else {
                s += s2;
            }
            if (active) uv[o] = s;
            if (pass == 0 && (c == nch - 1 || cb + CC >= ncols_eff) && active)
                part += (double)R[(size_t)w * RV + i] * (double)s;
        }
    }
    if (pass == 0) {
        red[wave][lane] = part;
        __syncthreads();
        if (wave == 0 && active) {
            double t = 0.0;
            for (int g = 0; g < kSpmmWaves; ++g) t += red[g][lane];
            a.wk.psi64[(size_t)w * kPsiParts + rs] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// K6: derivative aggregation (table method).  Per chunk of determinants the
// scaled adjugates w_d f_d adj(M_d) are staged in LDS, then every target
// (slot c, orbital m) sums its slots in a fixed order into Gamma[c][m].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_deriv(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] != 0) return;
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, N = a.N, tid = threadIdx.x;
    const int nt = n * M;
    extern __shared__ double lds[];
    double *T = lds;                  // [n][M]
    double *X = T + nt;               // [n][n]
    double *Gam = X + n * n;          // [n][M]  Gamma[c][m]
    double *Y = Gam + nt;             // [M][n]
    double *Zc = Y + nt;              // [n][n]
    double *cb = Zc + n * n;          // [kAdjChunk]
    int *Ex = (int *)(cb + kAdjChunk); // [M]
    int *occ0 = Ex + M;               // [n]
    const double *Tg = a.wk.T + ws * a.nmax * M;
    for (int i = tid; i < nt; i += kBlock) {
        T[i] = Tg[i];
        Gam[i] = 0.0;
    }
    const double *Xg = a.wk.X + ws * a.nmax * a.nmax;
    for (int i = tid; i < n * n; i += kBlock) X[i] = Xg[i];
    for (int m = tid; m < M; m += kBlock) Ex[m] = a.wk.E[ws * M + m];
    for (int c = tid; c < n; c += kBlock) occ0[c] = S.occ0[c];
    __syncthreads();
    const int K = a.wk.K[ws];
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const bool mixed = a.precision == MDET_MIXED;
    for (int k = 0; k < S.nchunk; ++k) {
        const int d0 = S.chunk_det[k], d1 = S.chunk_det[k + 1];
        const int base = S.adj_off[d0];
        for (int d = d0 + tid; d < d1; d += kBlock) {
            const DetDesc D = S.desc[d];
            const int s = D.s;
            if (s == 0) continue;
            double *dst = cb + (S.adj_off[d] - base);
            double coef = 0.0;
            if (s <= dmax) {
                const size_t o = rv_index(a, sp, d, w);
                const double wt = mixed ? (double)a.wk.uv32[o] : a.wk.uv64[o];
                coef = wt * (double)D.eps * pow2(delta_exponent(D, Ex, occ0) - K);
            }
            switch (s) {
            case 1: stage_adj<1>(D, T, M, coef, dst); break;
            case 2: stage_adj<2>(D, T, M, coef, dst); break;
            case 3: stage_adj<3>(D, T, M, coef, dst); break;
            default: stage_adj<4>(D, T, M, coef, dst); break;
            }
        }
        __syncthreads();
        const int32_t *gp = S.gptr + (size_t)k * (nt + 1);
        for (int t = tid; t < nt; t += kBlock) {
            double g = 0.0;
            for (int q = gp[t]; q < gp[t + 1]; ++q) g += cb[S.gpos[q]];
            Gam[t] += g;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < M * n; idx += kBlock) {
        const int m = idx / n, e = idx - m * n;
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += Gam[c * M + m] * X[c * n + e];
        Y[idx] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int c = idx / n, e = idx - c * n;
        double s = 0.0;
        for (int m = 0; m < M; ++m) s += T[c * M + m] * Y[m * n + e];
        Zc[idx] = s;
    }
    __syncthreads();
    const double psi = psi_value(a, w);
    const double *phig = a.wk.phi + (size_t)w * N * 5 * M;
    for (int idx = tid; idx < 4 * n; idx += kBlock) {
        const int e = idx >> 2, q = idx & 3;
        const double *Gq = phig + (size_t)(S.e0 + e) * 5 * M + (size_t)(1 + q) * M;
        double s1 = 0.0, s2 = 0.0;
        for (int m = 0; m < M; ++m) s1 += (Gq[m] * pow2(-Ex[m])) * Y[m * n + e];
        for (int c = 0; c < n; ++c) s2 += (Gq[occ0[c]] * pow2(-Ex[occ0[c]])) * Zc[c * n + e];
        const size_t o = ((size_t)w * N + S.e0 + e) * 4 + q;
        a.gl_out[o] = a.wk.g0[o] + (s1 - s2) / psi;
    }
}

// ---------------------------------------------------------------------------
// Direct-LU fallback for an ill-conditioned reference: every determinant of
// the (walker, spin) by its own LU, one thread per determinant with the
// NT x NT matrix in registers (NT = electrons of the spin), direct_split
// blocks per (walker, spin).
// ---------------------------------------------------------------------------
namespace {

constexpr int kDirectBlock = 128;

// LU with partial pivoting of a[NT][NT] in place; perm[i] = original row of
// row i.  The determinant is returned as mant * 2^ex (mant = 0 if singular).
template <int NT>
__device__ __forceinline__ void lu_regs(double (&a)[NT][NT], int (&perm)[NT], double &mant,
                                        int &ex) {
#pragma unroll
    for (int i = 0; i < NT; ++i) perm[i] = i;
    double m = 1.0;
    int k = 0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        int p = j;
        double best = fabs(a[j][j]);
#pragma unroll
        for (int i = j + 1; i < NT; ++i)
            if (fabs(a[i][j]) > best) {
                best = fabs(a[i][j]);
                p = i;
            }
        if (!(best > 0.0)) {
            mant = 0.0;
            ex = 0;
            return;
        }
#pragma unroll
        for (int i = j + 1; i < NT; ++i)
            if (i == p) {
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    const double t = a[i][c];
                    a[i][c] = a[j][c];
                    a[j][c] = t;
                }
                const int t = perm[i];
                perm[i] = perm[j];
                perm[j] = t;
                m = -m;
            }
        m *= a[j][j];
        int kk;
        m = frexp(m, &kk);
        k += kk;
#pragma unroll
        for (int i = j + 1; i < NT; ++i) {
            const double l = a[i][j] / a[j][j];
            a[i][j] = l;
#pragma unroll
            for (int c = j + 1; c < NT; ++c) a[i][c] -= l * a[j][c];
        }
    }
    mant = m;
    ex = k;
}

// occupied orbital of slot c for determinant D (reference with holes replaced)
__device__ __forceinline__ int slot_orbital(const DetDesc &D, const int *occ0, int c) {
    int o = occ0[c];
    for (int t = 0; t < D.s; ++t)
        if (D.h[t] == c) o = D.p[t];
    return o;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace

// pass 1: mantissa and exponent of every determinant of the block's range,
// and the integer maximum of the exponents per (walker, spin)
template <int NT>
__global__ void __launch_bounds__(kDirectBlock) k_direct_ratios_t(KernelArgs a, int sp) {
    const int w = blockIdx.x, part = blockIdx.y;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] == 0) return;
    const SpinDev S = a.sp[sp];
    const int M = a.M, tid = threadIdx.x;
    extern __shared__ double lds[];
    double *P0 = lds;                 // [NT][M] scaled orbital values of this spin
    int *Ex = (int *)(P0 + NT * M);   // [M]
    int *occ0 = Ex + M;               // [NT]
    __shared__ int red[kDirectBlock];
    const double *phig = a.wk.phi + (size_t)w * a.N * 5 * M;
    for (int m = tid; m < M; m += kDirectBlock) Ex[m] = a.wk.E[ws * M + m];
    for (int c = tid; c < NT; c += kDirectBlock) occ0[c] = S.occ0[c];
    __syncthreads();
    for (int i = tid; i < NT * M; i += kDirectBlock) {
        const int e = i / M, m = i - e * M;
        P0[i] = phig[(size_t)(S.e0 + e) * 5 * M + m] * pow2(-Ex[m]);
    }
    __syncthreads();
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const int d0 = (int)((int64_t)S.U * part / a.direct_split);
    const int d1 = (int)((int64_t)S.U * (part + 1) / a.direct_split);
    int kmax = INT_MIN;
    for (int d = d0 + tid; d < d1; d += kDirectBlock) {
        const DetDesc D = S.desc[d];
        double r = 0.0;
        int rexp = INT_MIN;
        if (D.s <= dmax) {
            double A[NT][NT];
            int perm[NT];
            int sx = 0;
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const int o = slot_orbital(D, occ0, c);
                sx += Ex[o];
#pragma unroll
                for (int e = 0; e < NT; ++e) A[e][c] = P0[e * M + o];
            }
            double mant;
            int ex;
            lu_regs<NT>(A, perm, mant, ex);
            if (mant != 0.0) {
                r = (double)D.eps * mant;
                rexp = ex + sx;
                kmax = max(kmax, rexp);
            }
        }
        const size_t o = rv_index(a, sp, d, w);
        a.wk.R64[o] = r;
        a.wk.Rexp[o] = rexp;
    }
    red[tid] = kmax;
    __syncthreads();
    if (tid == 0) {
        int m = INT_MIN;
        for (int t = 0; t < kDirectBlock; ++t) m = max(m, red[t]);
        if (m != INT_MIN) atomicMax(&a.wk.Kmax[ws], m);
    }
}

// pass 2: shift every ratio by the (walker, spin) maximum exponent
__global__ void __launch_bounds__(kBlock) k_direct_scale(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1, part = blockIdx.y;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] == 0) return;
    const SpinDev S = a.sp[sp];
    int K = a.wk.Kmax[ws];
    if (K == INT_MIN) K = 0;
    if (part == 0 && threadIdx.x == 0) {
        a.wk.K[ws] = K;
        a.wk.logdet0[ws] = 0.0;
        a.wk.sign0[ws] = 1.0;
    }
    const int d0 = (int)((int64_t)S.U * part / a.direct_split);
    const int d1 = (int)((int64_t)S.U * (part + 1) / a.direct_split);
    for (int d = d0 + threadIdx.x; d < d1; d += kBlock) {
        const size_t o = rv_index(a, sp, d, w);
        const int e = a.wk.Rexp[o];
        const double r = (e == INT_MIN) ? 0.0 : ldexp(a.wk.R64[o], e - K);
        if (a.precision == MDET_MIXED) a.wk.R32[o] = (float)r;
        else a.wk.R64[o] = r;
    }
}

// derivatives: partial sums over the block's determinants of
// w_d R_d grad~_e D_d / D_d (row-replacement form, columns of S_d^-1)
template <int NT>
__global__ void __launch_bounds__(kDirectBlock) k_direct_deriv_t(KernelArgs a, int sp) {
    const int w = blockIdx.x, part = blockIdx.y;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] == 0) return;
    const SpinDev S = a.sp[sp];
    const int M = a.M, N = a.N, tid = threadIdx.x;
    extern __shared__ double lds[];
    double *P = lds;                    // [5][NT][M] scaled orbitals and derivatives
    double *red = P + 5 * NT * M;       // [kDirectBlock / 64][NT * 4]
    int *Ex = (int *)(red + (kDirectBlock / 64) * NT * 4);  // [M]
    int *occ0 = Ex + M;                 // [NT]
    const double *phig = a.wk.phi + (size_t)w * N * 5 * M;
    for (int m = tid; m < M; m += kDirectBlock) Ex[m] = a.wk.E[ws * M + m];
    for (int c = tid; c < NT; c += kDirectBlock) occ0[c] = S.occ0[c];
    __syncthreads();
    for (int i = tid; i < 5 * NT * M; i += kDirectBlock) {
        const int q = i / (NT * M), r = i - q * NT * M, e = r / M, m = r - e * M;
        P[i] = phig[(size_t)(S.e0 + e) * 5 * M + (size_t)q * M + m] * pow2(-Ex[m]);
    }
    __syncthreads();
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const int K = a.wk.K[ws];
    const bool mixed = a.precision == MDET_MIXED;
    const int d0 = (int)((int64_t)S.U * part / a.direct_split);
    const int d1 = (int)((int64_t)S.U * (part + 1) / a.direct_split);
    double acc[NT][4];
#pragma unroll
    for (int e = 0; e < NT; ++e)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[e][q] = 0.0;
    for (int d = d0 + tid; d < d1; d += kDirectBlock) {
        const DetDesc D = S.desc[d];
        if (D.s > dmax) continue;
        const size_t o = rv_index(a, sp, d, w);
        const int rexp = a.wk.Rexp[o];
        if (rexp == INT_MIN) continue;
        double A[NT][NT];
        int perm[NT], occ[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            occ[c] = slot_orbital(D, occ0, c);
#pragma unroll
            for (int e = 0; e < NT; ++e) A[e][c] = P[e * M + occ[c]];
        }
        double mant;
        int ex;
        lu_regs<NT>(A, perm, mant, ex);
        if (mant == 0.0) continue;
        const double wt = mixed ? (double)a.wk.uv32[o] : a.wk.uv64[o];
        const double coef = wt * ldexp((double)D.eps * mant, rexp - K);
        // column e of S_d^-1: solve S x = e_e; grad~_e D_d / D_d = sum_c x_c G_q[e][occ_c]
#pragma unroll
        for (int e = 0; e < NT; ++e) {
            double x[NT];
#pragma unroll
            for (int i = 0; i < NT; ++i) x[i] = (perm[i] == e) ? 1.0 : 0.0;
#pragma unroll
            for (int i = 0; i < NT; ++i)
#pragma unroll
                for (int j = 0; j < i; ++j) x[i] -= A[i][j] * x[j];
#pragma unroll
            for (int i = NT - 1; i >= 0; --i) {
#pragma unroll
                for (int j = i + 1; j < NT; ++j) x[i] -= A[i][j] * x[j];
                x[i] /= A[i][i];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double *Gq = P + (size_t)(1 + q) * NT * M + e * M;
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < NT; ++c) s += x[c] * Gq[occ[c]];
                acc[e][q] += coef * s;
            }
        }
    }
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int e = 0; e < NT; ++e)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = wave_sum(acc[e][q]);
            if (lane == 0) red[wave * NT * 4 + e * 4 + q] = v;
        }
    __syncthreads();
    for (int i = tid; i < NT * 4; i += kDirectBlock) {
        double t = 0.0;
        for (int v = 0; v < kDirectBlock / 64; ++v) t += red[v * NT * 4 + i];
        a.wk.dpart[(((size_t)w * kDirectSplitMax + part) * N + S.e0) * 4 + i] = t;
    }
}

// ---------------------------------------------------------------------------
// Outputs: sign, ln|Psi|, status; the fallback's derivative partials are
// combined here; nodes get zero derivatives.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_finalize(KernelArgs a) {
    const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (w >= a.W) return;
    const double psi = psi_value(a, (int)w);
    const int f0 = a.wk.flag[2 * w], f1 = a.wk.flag[2 * w + 1];
    const bool node = !(psi != 0.0) || !isfinite(psi);
    if (node) {
        a.sign_out[w] = 0.0;
        a.logabs_out[w] = -INFINITY;
        for (int t = 0; t < 4 * a.N; ++t) a.gl_out[w * 4 * a.N + t] = 0.0;
        if (a.wstatus) a.wstatus[w] = MDET_W_NODE;
        return;
    }
    for (int sp = 0; sp < 2; ++sp) {
        if (a.wk.flag[2 * w + sp] == 0) continue;
        const int e0 = a.sp[sp].e0, n = a.sp[sp].n;
        for (int t = 4 * e0; t < 4 * (e0 + n); ++t) {
            double s = 0.0;
            for (int p = 0; p < a.direct_split; ++p)
                s += a.wk.dpart[((size_t)w * kDirectSplitMax + p) * a.N * 4 + t];
            a.gl_out[w * 4 * a.N + t] = s / psi;
        }
    }
    const double sg = a.wk.sign0[2 * w] * a.wk.sign0[2 * w + 1] * (psi > 0 ? 1.0 : -1.0);
    a.sign_out[w] = sg;
    a.logabs_out[w] = a.wk.logdet0[2 * w] + a.wk.logdet0[2 * w + 1] + log(fabs(psi)) +
                      (double)(a.wk.K[2 * w] + a.wk.K[2 * w + 1]) * 0.69314718055994530942;
    if (a.wstatus) a.wstatus[w] = (f0 || f1) ? MDET_W_FALLBACK : MDET_W_OK;
}

// ---------------------------------------------------------------------------
const char *kernel_name(int k) {
    static const char *names[kNumKernels] = {"k_reference", "k_ratios", "k_direct_ratios",
                                             "k_spmm",      "k_deriv",  "k_direct_deriv",
                                             "k_finalize"};
    return (k >= 0 && k < kNumKernels) ? names[k] : "";
}

// ---------------------------------------------------------------------------
// Uneven batches: stable counting sort of the walkers by maximum degree (one
// block, deterministic), gather of positions and degrees, scatter of outputs.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_degree_sort(int64_t W, const int8_t *md, int32_t *perm) {
    constexpr int D = MDET_MAX_DEGREE + 1;
    __shared__ int cnt[1024][D];
    __shared__ int base[D];
    const int t = threadIdx.x;
    const int64_t per = (W + 1023) / 1024;
    const int64_t b0 = t * per, b1 = min(W, b0 + per);
    int c[D] = {0};
    for (int64_t w = b0; w < b1; ++w) c[min(max((int)md[w], 0), D - 1)]++;
    for (int d = 0; d < D; ++d) cnt[t][d] = c[d];
    __syncthreads();
    if (t < D) {  // exclusive scan over threads, per degree
        int run = 0;
        for (int k = 0; k < 1024; ++k) {
            const int v = cnt[k][t];
            cnt[k][t] = run;
            run += v;
        }
        base[t] = run;
    }
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int d = 0; d < D; ++d) {
            const int v = base[d];
            base[d] = run;
            run += v;
        }
    }
    __syncthreads();
    int pos[D];
    for (int d = 0; d < D; ++d) pos[d] = base[d] + cnt[t][d];
    for (int64_t w = b0; w < b1; ++w) {
        const int d = min(max((int)md[w], 0), D - 1);
        perm[pos[d]++] = (int32_t)w;
    }
}

__global__ void __launch_bounds__(256) k_sort_gather(int64_t W, int N, const int32_t *perm,
                                                     const double *R, const int8_t *md, double *Rs,
                                                     int8_t *mds) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= W * N * 3) return;
    const int64_t k = t / (3 * N), r = t - k * 3 * N;
    const int64_t w = perm[k];
    Rs[t] = R[w * 3 * N + r];
    if (r == 0) mds[k] = md[w];
}

__global__ void __launch_bounds__(256) k_sort_scatter(int64_t W, int N, const int32_t *perm,
                                                      const double *sign_s, const double *logabs_s,
                                                      const double *gl_s, const int32_t *ws_s,
                                                      double *sign, double *logabs, double *gl,
                                                      int32_t *ws) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= W * N * 4) return;
    const int64_t k = t / (4 * N), r = t - k * 4 * N;
    const int64_t w = perm[k];
    gl[w * 4 * N + r] = gl_s[t];
    if (r == 0) {
        sign[w] = sign_s[k];
        logabs[w] = logabs_s[k];
        if (ws) ws[w] = ws_s[k];
    }
}

namespace {

template <int NT>
void launch_direct(const KernelArgs &a, hipStream_t st, int sp, bool deriv) {
    const int M = a.M, W = (int)a.W;
    const dim3 grid(W, a.direct_split);
    if (deriv) {
        const size_t lds = sizeof(double) * (5 * (size_t)NT * M + (kDirectBlock / 64) * NT * 4) +
                           sizeof(int) * (M + NT);
        k_direct_deriv_t<NT><<<grid, dim3(kDirectBlock), lds, st>>>(a, sp);
    } else {
        const size_t lds = sizeof(double) * (size_t)NT * M + sizeof(int) * (M + NT);
        k_direct_ratios_t<NT><<<grid, dim3(kDirectBlock), lds, st>>>(a, sp);
    }
}

void launch_direct_n(const KernelArgs &a, hipStream_t st, bool deriv) {
    for (int sp = 0; sp < 2; ++sp) {
        switch (a.sp[sp].n) {
        case 1: launch_direct<1>(a, st, sp, deriv); break;
        case 2: launch_direct<2>(a, st, sp, deriv); break;
        case 3: launch_direct<3>(a, st, sp, deriv); break;
        case 4: launch_direct<4>(a, st, sp, deriv); break;
        case 5: launch_direct<5>(a, st, sp, deriv); break;
        case 6: launch_direct<6>(a, st, sp, deriv); break;
        case 7: launch_direct<7>(a, st, sp, deriv); break;
        case 8: launch_direct<8>(a, st, sp, deriv); break;
        case 9: launch_direct<9>(a, st, sp, deriv); break;
        case 10: launch_direct<10>(a, st, sp, deriv); break;
        case 11: launch_direct<11>(a, st, sp, deriv); break;
        case 12: launch_direct<12>(a, st, sp, deriv); break;
        case 13: launch_direct<13>(a, st, sp, deriv); break;
        case 14: launch_direct<14>(a, st, sp, deriv); break;
        case 15: launch_direct<15>(a, st, sp, deriv); break;
        default: launch_direct<16>(a, st, sp, deriv); break;  // n <= MDET_MAX_SPIN_ELEC = 16
        }
    }
}

int psi_splits(int64_t W, int requested) {
    if (requested > 0) return std::max(1, std::min(requested, kPsiParts));
    const int64_t tiles = (W + kSpmmTile - 1) / kSpmmTile;
    const int rs = (int)((256 + tiles - 1) / tiles);
    return std::max(1, std::min(rs, kPsiParts));
}

hipError_t launch_core(const KernelArgs &a, hipStream_t st, hipEvent_t *ev);

}  // namespace

hipError_t launch_eval(const KernelArgs &args, hipStream_t st, hipEvent_t *ev) {
    const int64_t W = args.W;
    if (W == 0) return hipSuccess;
    KernelArgs a = args;
    a.psi_nparts = psi_splits(W, a.cfg.spmm_rsplit);
    a.direct_split = std::max(1, std::min((int)a.cfg.direct_split, kDirectSplitMax));
    if (!(a.max_degree && a.cfg.sort_walkers)) return launch_core(a, st, ev);
    // uneven batch: evaluate the walkers in ascending order of maximum degree
    const int N = a.N;
    k_degree_sort<<<dim3(1), dim3(1024), 0, st>>>(W, a.max_degree, a.wk.perm);
    k_sort_gather<<<dim3((unsigned)((W * N * 3 + 255) / 256)), dim3(256), 0, st>>>(
        W, N, a.wk.perm, a.R, a.max_degree, a.wk.Rs, a.wk.mds);
    KernelArgs b = a;
    b.R = a.wk.Rs;
    b.max_degree = a.wk.mds;
    b.sign_out = a.wk.sign_s;
    b.logabs_out = a.wk.logabs_s;
    b.gl_out = a.wk.gl_s;
    b.wstatus = a.wk.ws_s;
    const hipError_t e = launch_core(b, st, ev);
    if (e != hipSuccess) return e;
    k_sort_scatter<<<dim3((unsigned)((W * N * 4 + 255) / 256)), dim3(256), 0, st>>>(
        W, N, a.wk.perm, a.wk.sign_s, a.wk.logabs_s, a.wk.gl_s, a.wk.ws_s, a.sign_out, a.logabs_out,
        a.gl_out, a.wstatus);
    return hipGetLastError();
}

namespace {

hipError_t launch_core(const KernelArgs &a, hipStream_t st, hipEvent_t *ev) {
    const int W = (int)a.W;
    const int n = a.nmax, M = a.M;
    const dim3 g2(2 * W), blk(kBlock);
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    size_t lds_ref = sizeof(double) * ((size_t)n * M + M + 3 * n * n) + sizeof(int) * M;
    k_reference<<<g2, blk, lds_ref, st>>>(a);
    mark(1);
    size_t lds_rat = sizeof(double) * (size_t)n * M + sizeof(int) * (M + n);
    k_ratios<<<g2, blk, lds_rat, st>>>(a);
    mark(2);
    launch_direct_n(a, st, false);
    k_direct_scale<<<dim3(2 * W, a.direct_split), blk, 0, st>>>(a);
    mark(3);
    const int tiles = (W + kSpmmTile - 1) / kSpmmTile;
    const dim3 gs(tiles * a.psi_nparts, 2), bs(64 * kSpmmWaves);
    if (a.precision == MDET_MIXED)
        k_spmm<float, kSpmmCols32, true><<<gs, bs, 0, st>>>(
            a, a.wk.R32, a.wk.uv32, a.C.rval32, a.C.cval32, a.C.rcol, a.C.crow, a.C.rseg32,
            a.C.cseg32, a.C.nch_r32, a.C.nch_c32, a.psi_nparts);
    else
        k_spmm<double, kSpmmCols64, false><<<gs, bs, 0, st>>>(
            a, a.wk.R64, a.wk.uv64, a.C.rval, a.C.cval, a.C.rcol, a.C.crow, a.C.rseg64,
            a.C.cseg64, a.C.nch_r64, a.C.nch_c64, a.psi_nparts);
    mark(4);
    size_t lds_der = sizeof(double) * (3 * (size_t)n * M + 2 * n * n + kAdjChunk) +
                     sizeof(int) * (M + n);
    k_deriv<<<g2, blk, lds_der, st>>>(a);
    mark(5);
    launch_direct_n(a, st, true);
    mark(6);
    k_finalize<<<dim3((W + kBlock - 1) / kBlock), blk, 0, st>>>(a);
    mark(7);
    return hipGetLastError();
}

}  // namespace

}  // namespace mdet
