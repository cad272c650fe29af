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

#include "mdet_device.h"

#include <math.h>

#include <algorithm>
#include <climits>

namespace mdet {

namespace {

static_assert(kAdjChunkDets % kBlock == 0, "whole determinants per thread and chunk");

__device__ __forceinline__ double pow2(int k) { return ldexp(1.0, k); }

// Orbital m and its derivatives at one electron: value, grad x/y/z and
// Laplacian of sum_p coef x^a y^b z^c exp(-alpha r^2).  Per axis, with
// P_k = x^k:  d0 = P_a,  d1 = a P_(a-1) - 2 alpha P_(a+1),
// d2 = a (a-1) P_(a-2) - 2 alpha (2a+1) P_a + 4 alpha^2 P_(a+2)
// (the derivatives of x^a e^(-alpha x^2), divided by e^(-alpha x^2)).  The
// alpha-free factors come from a per-electron table, for each axis and power
// a = 0..4: pw[axis * kPowLd + 6 a + (0..5)] = P_a, a P_(a-1), P_(a+1),
// a (a-1) P_(a-2), (2a+1) P_a, P_(a+2), with P_(-1) = P_(-2) = 0 so the
// terms with a negative power vanish without a branch (no 0 * inf at a
// coordinate 0); then d1 = A1 - 2 alpha B1 and d2 = A2 - 2 alpha B2 +
// 4 alpha^2 C2 per primitive.  r2 = |r|^2.
constexpr int kPowLd = 30;
constexpr size_t kPrimLdsMax = 32 * 1024;  // LDS for the primitives in the orbital kernel
constexpr size_t kPrimLdsBytes = 2 * sizeof(double) + sizeof(int);  // per primitive

template <bool STAGED>
__device__ __forceinline__ void orbital5_tab(const Prim *prim, const double *s_al,
                                             const double *s_cf, const int *s_abc, int P, int M,
                                             int m, const double *pw, double r2, double out[5]) {
    double v = 0, gx = 0, gy = 0, gz = 0, lap = 0;
    for (int p = 0; p < P; ++p) {
        double alpha, coef;
        int pa[3];
        if constexpr (STAGED) {
            alpha = s_al[p * M + m];
            coef = s_cf[p * M + m];
            const int abc = s_abc[p * M + m];
            pa[0] = abc & 255;
            pa[1] = (abc >> 8) & 255;
            pa[2] = abc >> 16;
        } else {
            const Prim q = prim[m * P + p];
            alpha = q.alpha;
            coef = q.coef;
            pa[0] = q.a;
            pa[1] = q.b;
            pa[2] = q.c;
        }
        if (coef == 0.0) continue;
        const double g = coef * exp(-alpha * r2);
        const double t2 = 2.0 * alpha, t4 = t2 * t2;
        double f[3][3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const double *Q = pw + ax * kPowLd + 6 * pa[ax];
            f[ax][0] = Q[0];
            f[ax][1] = Q[1] - t2 * Q[2];
            f[ax][2] = Q[3] - t2 * Q[4] + t4 * Q[5];
        }
        const double yz = f[1][0] * f[2][0];
        v += g * f[0][0] * yz;
        gx += g * f[0][1] * yz;
        gy += g * f[0][0] * f[1][1] * f[2][0];
        gz += g * f[0][0] * f[1][0] * f[2][1];
        lap += g * (f[0][2] * yz + f[0][0] * (f[1][2] * f[2][0] + f[1][0] * f[2][2]));
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

// block max (blockDim.x == kBlock): wave maxima, then the kBlock / 64 of them
__device__ int block_max_int(int v, int *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = red[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) r = max(r, red[i]);
    __syncthreads();
    return r;
}

// small determinants, row-major
__device__ __forceinline__ double det2(double a, double b, double c, double d) {
    return a * d - b * c;
}

__device__ double det3(const double *m, int ld) {
    return m[0] * det2(m[ld + 1], m[ld + 2], m[2 * ld + 1], m[2 * ld + 2]) -
           m[1] * det2(m[ld + 0], m[ld + 2], m[2 * ld + 0], m[2 * ld + 2]) +
           m[2] * det2(m[ld + 0], m[ld + 1], m[2 * ld + 0], m[2 * ld + 1]);
}

__device__ __forceinline__ int delta_exponent(const DetDesc &D, const int *Ex, const int *occ0) {
    int dx = 0;
    for (int a = 0; a < D.s; ++a) dx += Ex[D.p[a]] - Ex[occ0[D.h[a]]];
    return dx;
}

// the same for a known degree S (static descriptor indices, all LDS reads
// issued together)
template <int S>
__device__ __forceinline__ int delta_exponent_t(const DetDesc &D, const int *Ex, const int *occ0) {
    int dx = 0;
#pragma unroll
    for (int a = 0; a < S; ++a) dx += Ex[D.p[a]] - Ex[occ0[D.h[a]]];
    return dx;
}

// a / b from the correctly rounded reciprocal rb = 1 / b and one FMA
// correction (Markstein): correctly rounded away from overflow and underflow,
// so equal rows still eliminate to exact zeros.
__device__ __forceinline__ double div_by(double a, double b, double rb) {
    const double q = a * rb;
    return fma(fma(-q, b, a), rb, q);
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
        const double rinv = 1.0 / a[j][j];
#pragma unroll
        for (int i = j + 1; i < S; ++i) {
            const double l = div_by(a[i][j], a[j][j], rinv);
#pragma unroll
            for (int k = j + 1; k < S; ++k) a[i][k] -= l * a[j][k];
        }
    }
    return det;
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
    else if constexpr (S == 3) d = det3(m, 3);
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

// In-place Gauss-Jordan inversion with partial pivoting (row interchanges,
// undone as column interchanges at the end) of a[S][S] in registers; det
// receives the determinant.  Returns false on an exactly zero pivot.
template <int S>
__device__ __forceinline__ bool gj_inplace(double (&a)[S][S], double &det) {
    int piv[S];
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
        piv[j] = p;
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
        const double pv = a[j][j];
        det *= pv;
        const double r = 1.0 / pv;
        a[j][j] = 1.0;
#pragma unroll
        for (int k = 0; k < S; ++k) a[j][k] *= r;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (i == j) continue;
            const double f = a[i][j];
            a[i][j] = 0.0;
#pragma unroll
            for (int k = 0; k < S; ++k) a[i][k] -= f * a[j][k];
        }
    }
    // inverse of P A is A^-1 P^T: undo the row interchanges on the columns
#pragma unroll
    for (int j = S - 1; j >= 0; --j)
#pragma unroll
        for (int c = j + 1; c < S; ++c)
            if (piv[j] == c) {
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    const double t = a[i][c];
                    a[i][c] = a[i][j];
                    a[i][j] = t;
                }
            }
    return true;
}

// coef * C_ab of an exactly singular 4 x 4 minor (Gauss-Jordan met a zero
// pivot): each cofactor from its 3 x 3 determinant.  Out of line: the case is
// rare and its registers stay out of the callers' hot path.
__device__ __noinline__ void adj4_singular(DetDesc D, const double *T, int M, double coef,
                                           double *dst) {
    double e[16];
    load_exc<4>(D, T, M, e);
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double sub[9];
            int t = 0;
            for (int i = 0; i < 4; ++i) {
                if (i == r) continue;
                for (int j = 0; j < 4; ++j)
                    if (j != c) sub[t++] = e[i * 4 + j];
            }
            const double d = det3(sub, 3);
            dst[r * 4 + c] = coef * (((r + c) & 1) ? -d : d);
        }
}

// coef * C_ab of M_d into dst[a*S + b] (C_ab = adj[b][a]), compile-time s
template <int S>
__device__ __forceinline__ void stage_adj(const DetDesc &D, const double *T, int M, double coef,
                                          double *dst) {
    if constexpr (S == 1) {
        dst[0] = coef;
    } else if constexpr (S == 2) {
        double m[4];
        load_exc<2>(D, T, M, m);
        dst[0] = coef * m[3];
        dst[1] = -coef * m[2];
        dst[2] = -coef * m[1];
        dst[3] = coef * m[0];
    } else if constexpr (S == 3) {
        // cofactors from 2 x 2 minors (no division, defined for any minor)
        double m[9];
        load_exc<3>(D, T, M, m);
        dst[0] = coef * (m[4] * m[8] - m[5] * m[7]);
        dst[1] = coef * (m[5] * m[6] - m[3] * m[8]);
        dst[2] = coef * (m[3] * m[7] - m[4] * m[6]);
        dst[3] = coef * (m[2] * m[7] - m[1] * m[8]);
        dst[4] = coef * (m[0] * m[8] - m[2] * m[6]);
        dst[5] = coef * (m[1] * m[6] - m[0] * m[7]);
        dst[6] = coef * (m[1] * m[5] - m[2] * m[4]);
        dst[7] = coef * (m[2] * m[3] - m[0] * m[5]);
        dst[8] = coef * (m[0] * m[4] - m[1] * m[3]);
    } else {
        // det M times M^-1 by pivoted Gauss-Jordan (cofactors from 2 x 2
        // minors cost less but lose accuracy on these minors, whose entries
        // cancel); the cofactor form serves only an exactly singular minor
        double a[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) a[i][k] = T[D.h[i] * M + D.p[k]];
        double det = 0.0;
        if (gj_inplace<4>(a, det)) {
            const double cd = coef * det;  // adj = det * inverse; C_ab = adj[b][a]
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int k = 0; k < 4; ++k) dst[i * 4 + k] = cd * a[k][i];
        } else {
            adj4_singular(D, T, M, coef, dst);
        }
    }
}

// coef * C_ab of a determinant of degree s > kFastDegree from the cofactors
// that k_ratios_hi stored (row-major s x s, global memory).
__device__ __forceinline__ void stage_hi(const double *src, int s, double coef, double *dst) {
    for (int q = 0; q < s * s; ++q) dst[q] = coef * src[q];
}

}  // namespace

// ---------------------------------------------------------------------------
// K1+K2+K3: orbitals, scaled reference inverse, refinement, g0.
// One block per walker.  The table T = X Phi' is not stored: the kernels
// that use it rebuild it in LDS from X and the orbitals (build_table).
// ---------------------------------------------------------------------------
namespace {

// The same for A in LDS (row-major, ld n) and Xo with ld n; logabs and sign
// receive ln|det A| and its sign.
__device__ bool lane_gauss_jordan(int n, int lane, const double *A, double *Xo, double *sc,
                                  double &logabs, double &sign) {
    double r[kMaxN];
#pragma unroll
    for (int k = 0; k < kMaxN; ++k) r[k] = (lane < n && k < n) ? A[lane * n + k] : 0.0;
    double mant;
    int ex;
    if (!lane_gj_core(n, lane, r, Xo, n, sc, mant, ex)) return false;
    sign = mant < 0.0 ? -1.0 : 1.0;
    logabs = log(fabs(mant)) + (double)ex * 0.69314718055994530942;
    return true;
}

// The reference elimination of one spin by one wave (lane = 0..63): the
// scaled reference matrix A (in Q) inverted by Gauss-Jordan into X, ln|det|
// and sign, one residual-correction step, the conditioning flag and
// grad~D0/D0.  A singular reference flags the pair for the fallback.
__device__ __forceinline__ void reference_tail(const KernelArgs &a, int w, int sp, int lane,
                                               const double *Q, double *Xl, double *Rl,
                                               double *gsc, const int *emax, const int *occl) {
    const int M = a.M, N = a.N, nm = a.nmax, nn = nm * nm;
    const SpinDev &S = a.sp[sp];
    const int n = S.n;
    const size_t ws = (size_t)w * 2 + sp;
    const double *A = Q + sp * 5 * nn;
    double *X = Xl + sp * nn, *Rm = Rl + sp * nn;
    double la = 0.0, sg = 1.0;
    const bool ok = lane_gauss_jordan(n, lane, A, X, gsc + sp * (2 * kMaxN + 2), la, sg);
    if (lane == 0) a.wk.Kmax[ws] = INT_MIN;
    if (!ok) {
        if (lane == 0) {
            a.wk.flag[ws] = 2;
            a.wk.logdet0[ws] = 0.0;
            a.wk.sign0[ws] = 1.0;
        }
        return;
    }
    if (lane == 0) {
        int sx = 0;
        for (int c = 0; c < n; ++c) {
            const int E = emax[sp * M + occl[sp * kMaxN + c]];
            sx += E == INT_MIN ? 0 : E;  // an all-zero column has scale 0
        }
        a.wk.logdet0[ws] = la + (double)sx * 0.69314718055994530942;
        a.wk.sign0[ws] = sg;
    }
    wave_lds_sync();
    // one residual-correction step: X <- X + X (I - A X); the n-term dot
    // products are unrolled so that their LDS reads are in flight together
#pragma unroll
    for (int t = 0; t < kMaxN * kMaxN / 64; ++t) {
        const int idx = lane + 64 * t;
        if (idx < n * n) {
            const int i = idx / n, j = idx - i * n;
            double u = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < kMaxN; ++k)
                if (k < n) u -= A[i * n + k] * X[k * n + j];
            Rm[idx] = u;
        }
    }
    wave_lds_sync();
    double xr[kMaxN * kMaxN / 64];
#pragma unroll
    for (int t = 0; t < kMaxN * kMaxN / 64; ++t) {
        const int idx = lane + 64 * t;
        if (idx < n * n) {
            const int i = idx / n, j = idx - i * n;
            double u = X[idx];
#pragma unroll
            for (int k = 0; k < kMaxN; ++k)
                if (k < n) u += X[i * n + k] * Rm[k * n + j];
            xr[t] = u;
        }
    }
    wave_lds_sync();
    double *Xg = a.wk.X + ws * nn;
#pragma unroll
    for (int t = 0; t < kMaxN * kMaxN / 64; ++t) {
        const int idx = lane + 64 * t;
        if (idx < n * n) {
            X[idx] = xr[t];
            Xg[idx] = xr[t];
        }
    }
    wave_lds_sync();
    // conditioning: kappa_1 = ||A||_1 ||X||_1 (largest column sums)
    double ca = 0.0, cx = 0.0;
    if (lane < n) {
#pragma unroll
        for (int i = 0; i < kMaxN; ++i)
            if (i < n) {
                ca += fabs(A[i * n + lane]);
                cx += fabs(X[i * n + lane]);
            }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ca = fmax(ca, __shfl_xor(ca, off, 64));
        cx = fmax(cx, __shfl_xor(cx, off, 64));
    }
    if (lane == 0) a.wk.flag[ws] = (ca * cx <= a.kappa_max) ? 0 : 1;  // NaN -> fallback
    // grad~_e D0 / D0 = sum_c X[c][e] grad~ Phi'[e][occ0[c]]
    if (lane < 4 * n) {
        const int e = lane >> 2, q = lane & 3;
        const double *G = Q + (sp * 5 + 1 + q) * nn;
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < kMaxN; ++c)
            if (c < n) t += X[c * n + e] * G[e * n + c];
        a.wk.g0[((size_t)w * N + S.e0 + e) * 4 + q] = t;
    }
}

}  // namespace

__global__ void __launch_bounds__(kBlock) k_reference(KernelArgs a) {
    const int w = blockIdx.x, tid = threadIdx.x;
    const int M = a.M, N = a.N, nm = a.nmax, nn = nm * nm, nup = a.sp[0].n;
    extern __shared__ double lds[];
    double *Q = lds;                  // [2][5][nm*nm] orbitals (q = 0) and derivatives at the
                                      // reference columns, Q[sp][q][e*n + c]
    double *Xl = Q + 10 * nn;         // [2][nm*nm]
    double *Rl = Xl + 2 * nn;         // [2][nm*nm]
    double *gsc = Rl + 2 * nn;        // [2][2 kMaxN + 2] Gauss-Jordan scratch per wave
    int *emax = (int *)(gsc + 2 * (2 * kMaxN + 2));  // [2][M] largest exponent of |phi| per column
    int *slot = emax + 2 * M;         // [2][M] reference slot of orbital m, or -1
    double *pw = (double *)(slot + 2 * M);  // [N][3][kPowLd] coordinate power factors
    double *r2s = pw + N * 3 * kPowLd;      // [N] |r|^2
    int *occl = (int *)(r2s + N);           // [2][kMaxN] reference occupations
    // the set-up's loads issued before any is used: the walker's coordinates
    // (one per thread, N * 3 <= kBlock) and the reference occupations
    const double *Rw = a.R + (size_t)w * N * 3;
    const int nocc = a.sp[0].n + a.sp[1].n;
    const double xv = tid < N * 3 ? Rw[tid] : 0.0;
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (tid < N) {
        rx = Rw[3 * tid];
        ry = Rw[3 * tid + 1];
        rz = Rw[3 * tid + 2];
    }
    const int osp = tid >= nup ? 1 : 0, oc = tid - (osp ? nup : 0);
    const int ov = tid < nocc ? a.sp[osp].occ0[oc] : 0;
    // the primitives (one set, or one per spin), staged as [set][p][m] arrays
    // when they fit (else read from HBM): consecutive orbitals in consecutive
    // LDS words
    const int MP = M * a.P;
    const int nsets = a.prim_dn != a.prim ? 2 : 1;
    const bool stage_prim = (size_t)nsets * MP * kPrimLdsBytes <= kPrimLdsMax;
    double *p_al = (double *)(occl + 2 * kMaxN), *p_cf = p_al + nsets * MP;
    int *p_abc = (int *)(p_cf + nsets * MP);
    if (stage_prim)
#pragma unroll 4
        for (int i = tid; i < nsets * MP; i += kBlock) {
            const int set = i >= MP, j = i - set * MP;
            const int m = j / a.P, p = j - m * a.P;
            const Prim q = (set ? a.prim_dn : a.prim)[j];
            const int o = set * MP + p * M + m;
            p_al[o] = q.alpha;
            p_cf[o] = q.coef;
            p_abc[o] = q.a | (q.b << 8) | (q.c << 16);
        }

    for (int i = tid; i < 2 * M; i += kBlock) {
        emax[i] = INT_MIN;
        slot[i] = -1;
    }
    __syncthreads();
    if (tid < nocc) {
        slot[osp * M + ov] = oc;
        occl[osp * kMaxN + oc] = ov;
    }
    if (tid < N * 3) {
        double P[9];  // P[2 + k] = x^k, k = -2..6
        P[0] = 0.0;
        P[1] = 0.0;
        double p = 1.0;
#pragma unroll
        for (int k = 0; k <= 6; ++k) {
            P[2 + k] = p;
            p *= xv;
        }
        double *t = pw + tid * kPowLd;
#pragma unroll
        for (int a = 0; a <= 4; ++a) {
            const double da = (double)a;
            t[6 * a + 0] = P[2 + a];
            t[6 * a + 1] = da * P[1 + a];
            t[6 * a + 2] = P[3 + a];
            t[6 * a + 3] = da * (da - 1.0) * P[a];
            t[6 * a + 4] = (2.0 * da + 1.0) * P[2 + a];
            t[6 * a + 5] = P[4 + a];
        }
    }
    if (tid < N) r2s[tid] = rx * rx + ry * ry + rz * rz;
    __syncthreads();
    double *phig = a.wk.phi + (size_t)w * N * 5 * M;
    // orbital m and its derivatives at electron e, written once (unscaled),
    // with the column's largest exponent and, for a reference column, the
    // copy in Q
    auto orbital_at = [&](int e, int m) {
        const int set = (nsets == 2 && e >= nup) ? 1 : 0;  // the down electrons' own orbitals
        double o[5];
        if (stage_prim) orbital5_tab<true>(nullptr, p_al + set * MP, p_cf + set * MP,
                                           p_abc + set * MP, a.P, M, m, pw + e * 3 * kPowLd,
                                           r2s[e], o);
        else orbital5_tab<false>(set ? a.prim_dn : a.prim, nullptr, nullptr, nullptr, a.P, M, m,
                                 pw + e * 3 * kPowLd, r2s[e], o);
        double *dst = phig + (size_t)e * 5 * M + m;
#pragma unroll
        for (int q = 0; q < 5; ++q) dst[q * M] = o[q];
        const int sp = e >= nup, el = e - (sp ? nup : 0);
        if (o[0] != 0.0) atomicMax(&emax[sp * M + m], expo(o[0]));
        const int c = slot[sp * M + m];
        if (c >= 0) {
            const int n = a.sp[sp].n;
#pragma unroll
            for (int q = 0; q < 5; ++q) Q[(sp * 5 + q) * nn + el * n + c] = o[q];
        }
    };
    // the other orbitals of every electron (those outside its spin's
    // reference), in chunks of 64 (electron, orbital) pairs that each wave
    // takes from a counter in LDS until none are left
    __shared__ int next_pair;
    auto other_orbitals = [&]() {
        const int lane = tid & 63;
        for (;;) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&next_pair, 64);
            base = __builtin_amdgcn_readfirstlane(base);
            if (base >= N * M) break;
            const int idx = base + lane;
            if (idx < N * M) {
                const int e = idx / M, m = idx - e * M;
                if (slot[(e >= nup ? M : 0) + m] < 0) orbital_at(e, m);
            }
        }
    };
    // power-of-two column scales E[sigma][m] (0 for an all-zero column)
    auto write_scales = [&]() {
        for (int i = tid; i < 2 * M; i += kBlock) {
            const int E = (emax[i] == INT_MIN) ? 0 : emax[i];
            emax[i] = E;
            a.wk.E[(size_t)w * 2 * M + i] = E;
        }
    };
    if (a.method == MDET_METHOD_SM_CHAIN) {  // the chain needs the orbitals and scales only
        for (int idx = tid; idx < N * M; idx += kBlock) orbital_at(idx / M, idx % M);
        __syncthreads();
        write_scales();
        if (tid < 2) a.wk.Kmax[(size_t)w * 2 + tid] = INT_MIN;
        if (w == 0 && tid < 4) a.wk.smstat[tid] = 0ull;
        return;
    }
    // the reference columns first (every electron at its spin's n reference
    // orbitals): their scales are then complete, and the two spins' reference
    // eliminations (waves 0 and 1) run while waves 2 and 3 evaluate the rest,
    // which waves 0 and 1 join when done
    if (tid == 0) next_pair = 0;
    {
        const int nd = nocc - nup, pu = nup * nup;
        for (int idx = tid; idx < pu + nd * nd; idx += kBlock) {
            const bool dn = idx >= pu;
            const int j = dn ? idx - pu : idx, nsp = dn ? nd : nup;
            const int e = (dn ? nup : 0) + j / nsp, c = j - (j / nsp) * nsp;
            orbital_at(e, occl[(dn ? kMaxN : 0) + c]);
        }
    }
    __syncthreads();
    for (int i = tid; i < 10 * nn; i += kBlock) {
        const int sp = i / (5 * nn), r = i % nn;
        const int n = a.sp[sp].n;
        if (r < n * n) {
            const int E = emax[sp * M + occl[sp * kMaxN + r % n]];
            Q[i] *= pow2(-(E == INT_MIN ? 0 : E));
        }
    }
    __syncthreads();
    if (tid < 128) reference_tail(a, w, tid >> 6, tid & 63, Q, Xl, Rl, gsc, emax, occl);
    other_orbitals();
    __syncthreads();
    write_scales();
}


namespace {

// Dense FP64 contractions of one (walker, spin) on the matrix cores:
// v_mfma_f64_16x16x4_f64 adds a 16 x 4 block A times a 4 x 16 block B to a
// 16 x 16 block D; lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] of a
// step and D[l / 16 + 4 i][l % 16] in accumulator i = 0..3 (the FP64 form
// interleaves the rows, unlike the FP32 one).  Every lane of the wave takes
// part (out-of-range entries are zero).
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kKSteps = kMaxN / 4;  // steps of 4 over an electron or slot index

// The orbital values of one table tile of 16 orbitals m0.. as the B operand:
// b[s] = phi[4s + l/16][m0 + l%16] (unscaled; phis has row stride 5 M).
__device__ __forceinline__ void table_tile_load(const double *phis, int n, int M, int m0, int lane,
                                                double (&b)[kKSteps]) {
    const int li = lane & 15, lk = lane >> 4, m = m0 + li;
#pragma unroll
    for (int s = 0; s < kKSteps; ++s) {
        const int e = 4 * s + lk;
        b[s] = (e < n && m < M) ? phis[(size_t)e * 5 * M + m] : 0.0;
    }
}

// T = X Phi' of one (walker, spin) into LDS: T[c][m] = sum_e X[c][e] phi[e][m]
// 2^-E[m] (X in LDS, row-major n x n), on the matrix cores: the waves of the
// block take tiles of 16 orbitals in turn, K = n in steps of 4.  The values
// of the wave's first tile come in b0 (loaded before the set-up barrier).
__device__ __forceinline__ void build_table(const double *phis, int n, int M, const int *Ex,
                                            const double *X, double *T, int tid, int nthr,
                                            double (&b0)[kKSteps]) {
    const int lane = tid & 63, wave = tid >> 6, nwave = nthr >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int ksteps = (n + 3) >> 2;
    double xa[kKSteps];
#pragma unroll
    for (int s = 0; s < kKSteps; ++s) {
        const int e = 4 * s + lk;
        xa[s] = (li < n && e < n) ? X[li * n + e] : 0.0;
    }
    for (int m0 = 16 * wave; m0 < M; m0 += 16 * nwave) {
        double b[kKSteps];
        if (m0 == 16 * wave) {
#pragma unroll
            for (int s = 0; s < kKSteps; ++s) b[s] = b0[s];
        } else {
            table_tile_load(phis, n, M, m0, lane, b);
        }
        const int m = m0 + li;
        const double sc = m < M ? pow2(-Ex[m]) : 0.0;
        v4d d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < kKSteps; ++s)
            if (s < ksteps) d = mfma_f64(xa[s], b[s] * sc, d);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = lk + 4 * i;
            if (c < n && m < M) T[c * M + m] = d[i];
        }
    }
}

// Set-up of the kernels that rebuild T for one (walker, spin): X, the column
// exponents and the reference occupation into LDS, and the orbital values of
// the wave's first table tile into b0, every load issued before the first is
// waited for (one round trip to memory, not one per array).
static_assert(kMaxN * kMaxN <= kBlock, "one X entry per thread");
__device__ __forceinline__ void pair_setup(const double *Xg, const int *Eg, const int *occg,
                                           const double *phis, int n, int M, int tid, double *X,
                                           int *Ex, int *occ0, double (&b0)[kKSteps]) {
    const double xv = tid < n * n ? Xg[tid] : 0.0;
    const int ev = tid < M ? Eg[tid] : 0;
    const int ov = tid < n ? occg[tid] : 0;
    table_tile_load(phis, n, M, 16 * (tid >> 6), tid & 63, b0);
    if (tid < n * n) X[tid] = xv;
    if (tid < M) Ex[tid] = ev;
    if (tid < n) occ0[tid] = ov;
    for (int m = tid + kBlock; m < M; m += kBlock) Ex[m] = Eg[m];
}

}  // namespace

// ---------------------------------------------------------------------------
// K4 for the determinants of degree kFastDegree < s <= MDET_MAX_DEGREE (the
// higher excitations of the paper's degree mix, Sec. 4, Table 4): one block
// per (walker, spin) rebuilds T, and each thread inverts whole s x s minors
// M_d = T[h, p] in registers by pivoted Gauss-Jordan.  It leaves the unshifted
// ratio eps det M_d and the exponent of its column scales in the ratio
// vector, the largest exponent in Kmax (k_ratios applies the shift), and the
// cofactors C_ab = det(M_d) (M_d^-1)_ba in the high-degree buffer for the
// derivative aggregation.  Runs before k_ratios, for expansions that hold
// such determinants only.
// ---------------------------------------------------------------------------
namespace {

// cofactors of an exactly singular s x s minor (Gauss-Jordan met a zero
// pivot), each from its (s-1) x (s-1) determinant by pivoted elimination.
// Out of line: rare, and its registers stay out of the caller.
__device__ __noinline__ void cofactors_singular(int S, const DetDescHi &H, const double *T, int M,
                                                double *dst) {
    for (int r = 0; r < S; ++r)
        for (int c = 0; c < S; ++c) {
            double m[(MDET_MAX_DEGREE - 1) * (MDET_MAX_DEGREE - 1)];
            const int n1 = S - 1;
            int t = 0;
            for (int i = 0; i < S; ++i) {
                if (i == r) continue;
                for (int j = 0; j < S; ++j)
                    if (j != c) m[t++] = T[H.h[i] * M + H.p[j]];
            }
            double det = 1.0;
            for (int j = 0; j < n1 && det != 0.0; ++j) {
                int p = j;
                for (int i = j + 1; i < n1; ++i)
                    if (fabs(m[i * n1 + j]) > fabs(m[p * n1 + j])) p = i;
                if (m[p * n1 + j] == 0.0) {
                    det = 0.0;
                    break;
                }
                if (p != j) {
                    for (int k = 0; k < n1; ++k) {
                        const double x = m[j * n1 + k];
                        m[j * n1 + k] = m[p * n1 + k];
                        m[p * n1 + k] = x;
                    }
                    det = -det;
                }
                det *= m[j * n1 + j];
                for (int i = j + 1; i < n1; ++i) {
                    const double l = m[i * n1 + j] / m[j * n1 + j];
                    for (int k = j + 1; k < n1; ++k) m[i * n1 + k] -= l * m[j * n1 + k];
                }
            }
            dst[r * S + c] = ((r + c) & 1) ? -det : det;
        }
}

// ratio eps det M and cofactors C_ab -> dst[a*S + b] of one determinant of
// compile-time degree S; returns the ratio
template <int S>
__device__ __forceinline__ double minor_hi(const DetDescHi &H, int eps, const double *T, int M,
                                           double *dst) {
    double m[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int k = 0; k < S; ++k) m[i][k] = T[H.h[i] * M + H.p[k]];
    double det = 0.0;
    if (gj_inplace<S>(m, det)) {
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int k = 0; k < S; ++k) dst[i * S + k] = det * m[k][i];  // C_ab = adj[b][a]
    } else {
        det = 0.0;
        cofactors_singular(S, H, T, M, dst);
    }
    return (double)eps * det;
}

}  // namespace

__global__ void __launch_bounds__(kBlock, 1) k_ratios_hi(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    const SpinDev S = a.sp[sp];
    const int Ulo = S.deg_end[kFastDegree];
    if (a.wk.flag[ws] != 0 || Ulo >= S.U) return;  // direct-LU fallback, or nothing to do
    const int n = S.n, M = a.M, tid = threadIdx.x;
    extern __shared__ double lds[];
    double *T = lds;                 // [n][M]
    double *X = T + n * M;           // [n][n]
    int *Ex = (int *)(X + n * n);    // [M]
    int *occ0 = Ex + M;              // [n]
    __shared__ int red[kBlock];
    const double *phis = a.wk.phi + ((size_t)w * a.N + S.e0) * 5 * M;
    double col0[kKSteps];
    pair_setup(a.wk.X + ws * a.nmax * a.nmax, a.wk.E + ws * M, S.occ0, phis, n, M, tid, X, Ex,
               occ0, col0);
    __syncthreads();
    build_table(phis, n, M, Ex, X, T, tid, kBlock, col0);
    __syncthreads();
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    double *adj = a.wk.adjhi + ws * a.wk.hi_stride;
    int kmax = INT_MIN;
    for (int d = Ulo + tid; d < S.U; d += kBlock) {
        const DetDesc D = S.desc[d];
        const DetDescHi H = S.desc_hi[d - Ulo];
        double *dst = adj + S.hi_off[d - Ulo];
        const size_t o = rv_index(a, sp, d, w);
        double r = 0.0;
        int dx = 0;
        if (D.s <= dmax) {
            switch (D.s) {
            case 5: r = minor_hi<5>(H, D.eps, T, M, dst); break;
            case 6: r = minor_hi<6>(H, D.eps, T, M, dst); break;
            case 7: r = minor_hi<7>(H, D.eps, T, M, dst); break;
            default: r = minor_hi<8>(H, D.eps, T, M, dst); break;
            }
            for (int t = 0; t < D.s; ++t) dx += Ex[H.p[t]] - Ex[occ0[H.h[t]]];
            if (r != 0.0) kmax = max(kmax, expo(r) + dx);
        }
        a.wk.R64[o] = r;
        a.wk.Rexp[o] = dx;  // also for a zero ratio: its cofactors need the scale
    }
    const int K = block_max_int(kmax, red);
    if (tid == 0 && K != INT_MIN) atomicMax(&a.wk.Kmax[ws], K);
}

// ---------------------------------------------------------------------------
// K4: ratios R_d / 2^K of every distinct determinant (table method).
// One block per (walker, spin); one thread per determinant.  Eight waves per
// SIMD (at most 64 VGPRs) let all pairs of a 1024-walker batch be resident
// at once.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock, 8) k_ratios(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] != 0) return;  // ill-conditioned: the direct-LU fallback takes the pair
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, tid = threadIdx.x;
    extern __shared__ double lds[];
    double *T = lds;                 // [n][M]
    double *X = T + n * M;           // [n][n]
    int *Ex = (int *)(X + n * n);    // [M]
    int *occ0 = Ex + M;              // [n]
    __shared__ int red[kBlock];
    const double *phis = a.wk.phi + ((size_t)w * a.N + S.e0) * 5 * M;
    double col0[kKSteps];
    pair_setup(a.wk.X + ws * a.nmax * a.nmax, a.wk.E + ws * M, S.occ0, phis, n, M, tid, X, Ex,
               occ0, col0);
    __syncthreads();
    build_table(phis, n, M, Ex, X, T, tid, kBlock, col0);
    __syncthreads();
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const bool mixed = a.precision == MDET_MIXED;
    // determinants of degree above kFastDegree (execution indices Ulo..U-1)
    // were evaluated by k_ratios_hi, which left their unshifted ratios and
    // exponents and the largest exponent in Kmax
    const int Ulo = S.deg_end[kFastDegree];
    // the first kKeep determinants of every thread stay in registers until the
    // shift K is known; further ones go through the ratio vector in HBM
    constexpr int kKeep = 4;
    double rk[kKeep];
    int xk[kKeep];
    int kmax = (tid == 0 && Ulo < S.U) ? a.wk.Kmax[ws] : INT_MIN;
#pragma unroll
    for (int j = 0; j < kKeep; ++j) {
        const int d = tid + j * kBlock;
        double r = 0.0;
        int dx = 0;
        if (d < Ulo) {
            const DetDesc D = S.desc[d];
            if (D.s <= dmax) {
                switch (D.s) {
                case 0: r = (double)D.eps; break;
                case 1: r = exc_ratio<1>(D, T, M); dx = delta_exponent_t<1>(D, Ex, occ0); break;
                case 2: r = exc_ratio<2>(D, T, M); dx = delta_exponent_t<2>(D, Ex, occ0); break;
                case 3: r = exc_ratio<3>(D, T, M); dx = delta_exponent_t<3>(D, Ex, occ0); break;
                default: r = exc_ratio<4>(D, T, M); dx = delta_exponent_t<4>(D, Ex, occ0); break;
                }
                if (r != 0.0) kmax = max(kmax, expo(r) + dx);
            }
        }
        rk[j] = r;
        xk[j] = dx;
    }
    for (int d = tid + kKeep * kBlock; d < Ulo; d += kBlock) {
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
    for (int d = Ulo + tid; d < S.U; d += kBlock) {  // the high-degree ones
        const size_t o = rv_index(a, sp, d, w);
        const int e = a.wk.Rexp[o];
        const double r = (e == INT_MIN) ? 0.0 : ldexp(a.wk.R64[o], e - K);
        a.wk.R64[o] = r;
        if (mixed) a.wk.R32[o] = (float)r;
    }
#pragma unroll
    for (int j = 0; j < kKeep; ++j) {
        const int d = tid + j * kBlock;
        if (d < Ulo) {
            const size_t o = rv_index(a, sp, d, w);
            const double r = ldexp(rk[j], xk[j] - K);
            a.wk.R64[o] = r;
            if (mixed) a.wk.R32[o] = (float)r;
        }
    }
    for (int d = tid + kKeep * kBlock; d < Ulo; d += kBlock) {
        const DetDesc D = S.desc[d];
        const size_t o = rv_index(a, sp, d, w);
        const double r = ldexp(a.wk.R64[o], delta_exponent(D, Ex, occ0) - K);
        a.wk.R64[o] = r;
        if (mixed) a.wk.R32[o] = (float)r;
    }
}

// ---------------------------------------------------------------------------
// K5: the two sparse products of Sec. 2.4 for a tile of 64 walkers (one per
// lane), 16 waves per block:
//   pass 0:  u = C R_dn  (CSR rows, gathering R_dn)  and the psi partials R_up . u
//   pass 1:  v = C^T R_up (CSC columns, gathering R_up) and the psi partials R_dn . v
// A wave owns whole rows, so the entries of C are wave-uniform and each one
// feeds 64 multiply-adds; the gathered vector of the 64 walkers sits in LDS,
// CC entries at a time.  F is the storage type of R, u and v and A the type
// of C and of the accumulation: FP64 in FP64 mode; in mixed precision float
// for both (half the bytes, twice the columns per LDS chunk, FP32 multiply-
// adds; the psi partials stay FP64 with the FP64 ratios, and the derivative
// aggregate uses the same stored u and v, so their rounding enters Psi and
// its derivatives alike).  grid.x = walker tiles x row splits, grid.y = pass.
// ---------------------------------------------------------------------------
constexpr int kSpmmWaves = 16;
constexpr int kSpmmLd = kSpmmTile + 1;  // LDS row pitch of the staged vector
constexpr int kSpmmGroup = 8;           // nonzeros per step of the inner loop

// LDS hand-off between the lanes of one wave (no block barrier)
__device__ __forceinline__ void spmm_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block -> (walker tile, row split): blocks are dealt to the 8 XCDs round
// robin, so the row splits of one tile are kept on one XCD (its L2 then holds
// the tile's gathered vector for all of them).  gridDim.x = ceil(tiles / 8) *
// 8 * rsplit; blocks past the last tile do nothing.
__device__ __forceinline__ void spmm_block_map(int b, int rsplit, int &tile, int &rs) {
    const int x = b & 7, y = b >> 3;
    tile = x + 8 * (y / rsplit);
    rs = y - (y / rsplit) * rsplit;
}

template <typename F, int CC, typename A>
__global__ void __launch_bounds__(64 * kSpmmWaves)
    k_spmm(KernelArgs a, const F *__restrict__ R, const double *__restrict__ R64,
           F *__restrict__ uv,
           const A *__restrict__ rval, const A *__restrict__ cval,
           const int32_t *__restrict__ rcol, const int32_t *__restrict__ crow,
           const int32_t *__restrict__ rseg, const int32_t *__restrict__ cseg, int nch_r, int nch_c,
           int rsplit) {
    __shared__ F G[CC * kSpmmLd];
    __shared__ double red[kSpmmWaves][kSpmmTile];
    __shared__ int Cj[kSpmmWaves][64];     // per wave: LDS offsets of a row's next 64 nonzeros
    __shared__ A Cv[kSpmmWaves][64];       // and their values
    const int pass = blockIdx.y;
    int tile, rs;
    spmm_block_map(blockIdx.x, rsplit, tile, rs);
    const int W = (int)a.W;
    if (tile * kSpmmTile >= W) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w0 = tile * kSpmmTile, w = w0 + lane;
    const bool active = w < W;
    const int nrows = pass ? a.C.V : a.C.U;
    const int nch = pass ? nch_c : nch_r;
    const int32_t *__restrict__ idx = pass ? crow : rcol;
    const int32_t *__restrict__ seg = pass ? cseg : rseg;
    const A *__restrict__ val = pass ? cval : rval;
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
    int *cj = Cj[wave];
    A *cv = Cv[wave];
    double part = 0.0;
    for (int c = 0; c < nch; ++c) {
        const int cb = c * CC;
        if (cb >= ncols_eff) break;
        const int nc = min(CC, ncols_eff - cb);
        __syncthreads();
        // stage G[j][walker]: each wave copies kSpmmTile / kSpmmWaves whole
        // walker rows (walker-major source, coalesced), all loads in flight
        // before the stores; the odd LDS pitch keeps the stores here and the
        // lane-contiguous reads below free of bank conflicts
        {
            constexpr int kRows = kSpmmTile / kSpmmWaves;
            constexpr int kIt = (CC + 63) / 64;
            F buf[kRows][kIt];
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const int ww = wave + kSpmmWaves * r;
                const F *src = R + (size_t)(w0 + ww) * RV + goff + cb;
                const bool ok = w0 + ww < W;
#pragma unroll
                for (int q = 0; q < kIt; ++q) {
                    const int jj = lane + 64 * q;
                    buf[r][q] = (F)0;
                    if (ok && jj < nc) buf[r][q] = src[jj];
                }
            }
#pragma unroll
            for (int r = 0; r < kRows; ++r)
#pragma unroll
                for (int q = 0; q < kIt; ++q) {
                    const int jj = lane + 64 * q;
                    if (jj < nc) G[jj * kSpmmLd + wave + kSpmmWaves * r] = buf[r][q];
                }
        }
        __syncthreads();
        // the wave's rows i = r0 + wave + kSpmmWaves * j, row bounds for up to
        // 64 rows at a time held one per lane
        for (int rb = r0 + wave; rb < r1; rb += kSpmmWaves * 64) {
            const int ir = rb + kSpmmWaves * lane;
            int kbv = 0, kev = 0;
            if (ir < r1) {
                kbv = seg[(size_t)c * nrows + ir];
                kev = min(seg[(size_t)(c + 1) * nrows + ir],
                          degend[(size_t)ir * (MDET_MAX_DEGREE + 1) + dmax]);
            }
            const int nr = min(64, (r1 - rb + kSpmmWaves - 1) / kSpmmWaves);
            for (int jr = 0; jr < nr; ++jr) {
                const int i = rb + kSpmmWaves * jr;
                const int kb = __builtin_amdgcn_readlane(kbv, jr);
                const int ke = __builtin_amdgcn_readlane(kev, jr);
                const size_t o = (size_t)w * RV + ooff + i;
                // two independent sums: even / odd offsets in the row segment
                A s = 0, s2 = 0;
                if (c != 0 && active) s = (A)uv[o];
                for (int base = kb; base < ke; base += 64) {
                    const int cnt = min(64, ke - base);
                    int jl = 0;
                    A vl = 0;
                    if (lane < cnt) {
                        jl = (idx[base + lane] - cb) * kSpmmLd;
                        vl = val[base + lane];
                    }
                    cj[lane] = jl;
                    cv[lane] = vl;
                    spmm_wave_sync();
                    int t = 0;
                    for (; t + kSpmmGroup <= cnt; t += kSpmmGroup) {
                        F gx[kSpmmGroup];
#pragma unroll
                        for (int u = 0; u < kSpmmGroup; ++u) gx[u] = G[cj[t + u] + lane];
#pragma unroll
                        for (int u = 0; u < kSpmmGroup; u += 2) {
                            s = fma(cv[t + u], (A)gx[u], s);
                            s2 = fma(cv[t + u + 1], (A)gx[u + 1], s2);
                        }
                    }
                    // tail: the same even/odd split by offset in the row, so
                    // that a shorter segment (entries skipped for an uneven
                    // batch, all zero) sums in exactly the same grouping
                    for (; t < cnt; ++t) {
                        const A x = (A)G[cj[t] + lane];
                        if ((base - kb + t) & 1) s2 = fma(cv[t], x, s2);
                        else s = fma(cv[t], x, s);
                    }
                    spmm_wave_sync();
                }
                // u and v are rounded to F here after every chunk; psi takes
                // the stored value, so it does not depend on how many chunks
                // the tile needed (walker order in an uneven batch).  Each
                // pass forms its own psi from the FP64 ratio of its row and
                // the stored weight: psi_up = R_up.u, psi_dn = R_dn.v
                const F sf = (F)(s + s2);
                if (active) uv[o] = sf;
                if ((c == nch - 1 || cb + CC >= ncols_eff) && active)
                    part += R64[(size_t)w * RV + ooff + i] * (double)sf;
            }
        }
    }
    red[wave][lane] = part;
    __syncthreads();
    if (wave == 0 && active) {
        double t = 0.0;
        for (int g = 0; g < kSpmmWaves; ++g) t += red[g][lane];
        a.wk.psi64[((size_t)w * 2 + pass) * kPsiParts + rs] = t;
    }
}

// ---------------------------------------------------------------------------
// K6: derivative aggregation (table method).  Per chunk of determinants the
// scaled adjugates w_d f_d adj(M_d) are staged in LDS, then every thread adds
// the staged slots of the targets (slot c, orbital m) it owns in this chunk,
// in a fixed order, into Gamma[c][m]: no target has two owners, so the sums
// are deterministic without atomics.
// ---------------------------------------------------------------------------
// LDS layout of k_deriv: T [n][M], X [n][n], Gam [n][M], then a region used
// first by the chunk loop (adjugates cb [kAdjChunk]) and afterwards by
// Y [M][n], Zc [n][n] and kDerivScratch partial sums; then Ex [M] and
// occ0 [n].
constexpr int kDerivScratch = 4 * 256;  // the waves' 16 x 16 partial blocks of Zc
static_assert(kDerivScratch >= (kBlock / 64) * 256, "Zc partials");
static_assert(kDerivScratch >= kBlock + 2 * kPsiParts, "s1 partials and the psi partial sums");
static_assert(kBlock == kBlockThreads, "gather lists are dealt to the block's threads");
static_assert(kGent % 4 == 0, "gather lists are loaded 16 bytes at a time");
constexpr int kS1Pre = 16;  // derivative-table values per thread loaded ahead of the s1 sums

__host__ __device__ inline size_t deriv_union_doubles(int n, int M) {
    const size_t loop = kAdjChunk;
    const size_t tail = (size_t)M * n + (size_t)n * n + kDerivScratch;
    return loop > tail ? loop : tail;
}

__global__ void __launch_bounds__(kBlock, 4) k_deriv(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] != 0 || a.sp[sp].n == 0) return;
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, N = a.N, tid = threadIdx.x;
    const int nt = n * M;
    extern __shared__ double lds[];
    double *T = lds;                  // [n][M]
    double *X = T + nt;               // [n][n]
    double *Gam = X + n * n;          // [n][M]  Gamma[c][m]
    double *un = Gam + nt;            // union region
    double *cb = un;                  // [kAdjChunk] staged adjugates
    double *Y = un;                   // [M][n]   (after the chunk loop)
    double *Zc = Y + (size_t)M * n;   // [n][n]
    double *scr = Zc + n * n;         // [kDerivScratch]
    int *Ex = (int *)(un + deriv_union_doubles(n, M));  // [M]
    int *occ0 = Ex + M;               // [n]
    const double *phis = a.wk.phi + ((size_t)w * N + S.e0) * 5 * M;
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const bool mixed = a.precision == MDET_MIXED;
    // a chunk holds at most kDetsPerThread * kBlock determinants: thread tid
    // stages the chunk's determinants tid + j * kBlock and then adds the
    // staged slots of its own targets (at most kGent).  The descriptors and
    // weights of the next chunk are fetched while this chunk's targets are
    // summed, its gather list right after (registers).
    constexpr int kDetsPerThread = kAdjChunkDets / kBlock;
    DetDesc Dc[kDetsPerThread];
    double wc[kDetsPerThread];
    int oc[kDetsPerThread];
    int hx[kDetsPerThread];  // degree above kFastDegree: exponent of the column scales
    uint32_t ge[kGent];
    const int Ulo = S.deg_end[kFastDegree];
    auto fetch = [&](int k) {
        const int dk = S.chunk_det[k], d1 = S.chunk_det[k + 1];
        const int base = S.adj_off[dk];
#pragma unroll
        for (int j = 0; j < kDetsPerThread; ++j) {
            const int d = dk + tid + j * kBlock;
            Dc[j].s = 0;
            wc[j] = 0.0;
            oc[j] = 0;
            hx[j] = 0;
            if (d < d1) {
                Dc[j] = S.desc[d];
                oc[j] = S.adj_off[d] - base;
                if (Dc[j].s <= dmax) {
                    const size_t o = rv_index(a, sp, d, w);
                    wc[j] = mixed ? (double)a.wk.uv32[o] : a.wk.uv64[o];
                    if (d >= Ulo) hx[j] = a.wk.Rexp[o];
                }
            }
        }
    };
    auto fetch_gather = [&](int k) {
        const uint4 *g = reinterpret_cast<const uint4 *>(S.gent + ((size_t)k * kBlock + tid) * kGent);
#pragma unroll
        for (int j = 0; j < kGent / 4; ++j) {
            const uint4 v = g[j];
            ge[4 * j] = v.x;
            ge[4 * j + 1] = v.y;
            ge[4 * j + 2] = v.z;
            ge[4 * j + 3] = v.w;
        }
    };
    double col0[kKSteps];
    pair_setup(a.wk.X + ws * a.nmax * a.nmax, a.wk.E + ws * M, S.occ0, phis, n, M, tid, X, Ex,
               occ0, col0);
    const int K = a.wk.K[ws];
    fetch(0);
    fetch_gather(0);
    for (int i = tid; i < nt; i += kBlock) Gam[i] = 0.0;
    __syncthreads();
    build_table(phis, n, M, Ex, X, T, tid, kBlock, col0);
    __syncthreads();
    for (int k = 0; k < S.nchunk; ++k) {
        // one determinant per pass, the thread's registers shifted down after
        // each (one inlined copy of the staging code)
#pragma unroll 1
        for (int j = 0; j < kDetsPerThread; ++j) {
            const DetDesc D = Dc[0];
            const int s = D.s;
            double *dst = cb + oc[0];
            if (s > kFastDegree) {  // cofactors left by k_ratios_hi
                const int d = S.chunk_det[k] + tid + j * kBlock;
                stage_hi(a.wk.adjhi + ws * a.wk.hi_stride + S.hi_off[d - Ulo], s,
                         (s <= dmax) ? wc[0] * (double)D.eps * pow2(hx[0] - K) : 0.0, dst);
            } else if (s > 0) {
                const double wd = (s <= dmax) ? wc[0] * (double)D.eps : 0.0;
                switch (s) {
                case 1: stage_adj<1>(D, T, M, wd * pow2(delta_exponent_t<1>(D, Ex, occ0) - K), dst); break;
                case 2: stage_adj<2>(D, T, M, wd * pow2(delta_exponent_t<2>(D, Ex, occ0) - K), dst); break;
                case 3: stage_adj<3>(D, T, M, wd * pow2(delta_exponent_t<3>(D, Ex, occ0) - K), dst); break;
                default: stage_adj<4>(D, T, M, wd * pow2(delta_exponent_t<4>(D, Ex, occ0) - K), dst); break;
                }
            }
#pragma unroll
            for (int i = 0; i + 1 < kDetsPerThread; ++i) {
                Dc[i] = Dc[i + 1];
                wc[i] = wc[i + 1];
                oc[i] = oc[i + 1];
                hx[i] = hx[i + 1];
            }
        }
        __syncthreads();
        if (k + 1 < S.nchunk) fetch(k + 1);
        // this thread's targets: all staged values read first, then summed per
        // target in list order
        {
            double v[kGent];
#pragma unroll
            for (int i = 0; i < kGent; ++i) v[i] = ge[i] != kGentNone ? cb[ge[i] & 0xFFFFu] : 0.0;
            int tc = -1;
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < kGent; ++i) {
                if (ge[i] == kGentNone) break;
                const int tt = (int)(ge[i] >> 16);
                if (tt != tc) {
                    if (tc >= 0) Gam[tc] += acc;
                    tc = tt;
                    acc = 0.0;
                }
                acc += v[i];
            }
            if (tc >= 0) Gam[tc] += acc;
        }
        if (k + 1 < S.nchunk) fetch_gather(k + 1);
        __syncthreads();
    }
    // the s1 sums' derivative-table values, loaded now and used after Y and
    // Zc: s1[e][q] = sum_m G_q[e][m] 2^-E[m] Y[m][e] in nf segments of m per
    // (e, q)
    const int nf = max(1, min(8, kBlock / (4 * n)));
    const double *phig = a.wk.phi + ((size_t)w * N + S.e0) * 5 * M;
    const bool s1t = tid < nf * 4 * n;
    const int pr = tid / nf, g1 = tid - pr * nf, e1 = pr >> 2, q1 = pr & 3;
    const double *Gq1 = phig + (size_t)e1 * 5 * M + (size_t)(1 + q1) * M;
    double gpre[kS1Pre];
#pragma unroll
    for (int u = 0; u < kS1Pre; ++u) {
        const int m = g1 + u * nf;
        gpre[u] = (s1t && m < M) ? Gq1[m] : 0.0;
    }
    // Y = Gamma^T X on the matrix cores (Y[m][e], row stride n): tiles of 16
    // orbitals m, K = the n slots c in steps of 4
    {
        const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
        const int ksteps = (n + 3) >> 2;
        double xb[kKSteps];
#pragma unroll
        for (int s = 0; s < kKSteps; ++s) {
            const int c = 4 * s + lk;
            xb[s] = (c < n && li < n) ? X[c * n + li] : 0.0;
        }
        for (int m0 = 16 * wave; m0 < M; m0 += 16 * (kBlock / 64)) {
            const int m = m0 + li;
            v4d d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < kKSteps; ++s) {
                const int c = 4 * s + lk;
                const double ga = (c < n && m < M) ? Gam[c * M + m] : 0.0;
                if (s < ksteps) d = mfma_f64(ga, xb[s], d);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = m0 + lk + 4 * i;
                if (mm < M && li < n) Y[mm * n + li] = d[i];
            }
        }
    }
    __syncthreads();
    // Zc = T Y on the matrix cores: one 16 x 16 block (c, e), K = the M
    // orbitals in steps of 4 dealt to the waves in turn; the waves' partial
    // blocks are added in wave order
    {
        const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
        v4d d = {0.0, 0.0, 0.0, 0.0};
        for (int m0 = 4 * wave; m0 < M; m0 += 4 * (kBlock / 64)) {
            const int m = m0 + lk;
            const double ta = (li < n && m < M) ? T[li * M + m] : 0.0;
            const double yb = (m < M && li < n) ? Y[m * n + li] : 0.0;
            d = mfma_f64(ta, yb, d);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) scr[wave * 256 + (lk + 4 * i) * 16 + li] = d[i];
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int c = idx / n, e = idx - c * n;
        double s = 0.0;
#pragma unroll
        for (int g = 0; g < kBlock / 64; ++g) s += scr[g * 256 + c * 16 + e];
        Zc[idx] = s;
    }
    __syncthreads();
    // the output threads' loads, issued before the s1 sums: the orbital
    // derivatives at the reference's occupied orbitals (occupied columns
    // clamped to n), the reference term and the psi partial sums (to LDS)
    const int eo = tid >> 2, qo = tid & 3;
    double go[kMaxN];
    double g0 = 0.0;
    if (tid < 4 * n) {
        const double *Gq = phig + (size_t)eo * 5 * M + (size_t)(1 + qo) * M;
#pragma unroll
        for (int c = 0; c < kMaxN; ++c) go[c] = Gq[occ0[c < n ? c : n - 1]];
        g0 = a.wk.g0[((size_t)w * N + S.e0 + eo) * 4 + qo];
    }
    double *psiP = scr + kBlock;  // [2][kPsiParts]
    if (tid < 2 * kPsiParts) psiP[tid] = a.wk.psi64[(size_t)w * 2 * kPsiParts + tid];
    if (s1t) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < kS1Pre; ++u) {
            const int m = g1 + u * nf;
            if (m < M) s += (gpre[u] * pow2(-Ex[m])) * Y[m * n + e1];
        }
        int m = g1 + kS1Pre * nf;
        for (; m + 7 * nf < M; m += 8 * nf) {
            double gv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) gv[u] = Gq1[m + u * nf];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int mm = m + u * nf;
                s += (gv[u] * pow2(-Ex[mm])) * Y[mm * n + e1];
            }
        }
        for (; m < M; m += nf) s += (Gq1[m] * pow2(-Ex[m])) * Y[m * n + e1];
        scr[tid] = s;
    }
    __syncthreads();
    if (tid < 4 * n) {
        const size_t o = ((size_t)w * N + S.e0 + eo) * 4 + qo;
        // the derivative of Psi for this spin's electrons is the numerator
        // g0 psi_sigma + (s1 - s2): psi_sigma is formed from the same ratios
        // and weights as the aggregate, so a rounding of the weights cannot
        // be amplified by a large g0; divided by psi_up, the psi that gives
        // ln|Psi|, so that the returned ratio times the returned Psi is that
        // numerator.  The partial sums are added in the order of psi_value.
        const int np = a.psi_nparts;
        double psi = 0.0, psi_s = 0.0;
        for (int k = 0; k < np; ++k) psi += psiP[k];
        if (sp)
            for (int k = 0; k < np; ++k) psi_s += psiP[kPsiParts + k];
        const double gr = sp ? g0 * (psi_s / psi) : g0;
        double s1 = 0.0, s2 = 0.0;
        for (int g = 0; g < nf; ++g) s1 += scr[tid * nf + g];
#pragma unroll
        for (int c = 0; c < kMaxN; ++c)
            if (c < n) s2 += (go[c] * pow2(-Ex[occ0[c]])) * Zc[c * n + eo];
        a.gl_out[o] = gr + (s1 - s2) / psi;
    }
}

// ---------------------------------------------------------------------------
// Direct-LU fallback for an ill-conditioned reference: every determinant of a
// flagged (walker, spin) by its own LU with partial pivoting, one thread per
// determinant with the matrix in registers (the analogue of the O(n^3)
// recomputation rule for failed updates, Sec. 2.2).  k_ratios lists the
// flagged pairs; a work item is (pair, part), part = one of direct_split
// slices of the pair's determinants, and a fixed grid walks the items.  One
// launch serves both spins: K x K matrices are compiled for K = NT and NT-1
// (NT = the larger electron count); a smaller spin is padded with an
// identity block, which changes neither its determinant nor its inverse.
// ---------------------------------------------------------------------------
namespace {

constexpr int kDirectBlock = 256;
// derivative sums of the direct-LU fallback: per wave, the 64 lanes'
// contributions of kEHalf electrons are staged in LDS (row pitch kWredLd)
// and added column by column
constexpr int kEHalf = 5;
constexpr int kWredLd = 4 * kEHalf + 1;

// LU with partial pivoting of a[K][K] in place; with PERM, perm[i] = original
// row of row i and the multipliers are kept below the diagonal (without PERM
// only what the determinant needs is updated).  The determinant is returned
// as mant * 2^ex (mant = 0 if singular).
template <int K, bool PERM>
__device__ __forceinline__ void lu_regs(double (&a)[K][K], int (&perm)[K], double &mant,
                                        int &ex) {
    if constexpr (PERM) {
#pragma unroll
        for (int i = 0; i < K; ++i) perm[i] = i;
    }
    double m = 1.0;
    int k = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        int p = j;
        double best = fabs(a[j][j]);
#pragma unroll
        for (int i = j + 1; i < K; ++i)
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
        for (int i = j + 1; i < K; ++i)
            if (i == p) {
#pragma unroll
                for (int c = PERM ? 0 : j; c < K; ++c) {
                    const double t = a[i][c];
                    a[i][c] = a[j][c];
                    a[j][c] = t;
                }
                if constexpr (PERM) {
                    const int t = perm[i];
                    perm[i] = perm[j];
                    perm[j] = t;
                }
                m = -m;
            }
        m *= a[j][j];
        int kk;
        m = frexp(m, &kk);
        k += kk;
        const double rinv = 1.0 / a[j][j];
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            const double l = div_by(a[i][j], a[j][j], rinv);
            if constexpr (PERM) a[i][j] = l;
#pragma unroll
            for (int c = j + 1; c < K; ++c) a[i][c] -= l * a[j][c];
        }
    }
    mant = m;
    ex = k;
}

// In-place Gauss-Jordan inversion of a[K][K] with column pivoting: step j
// takes as pivot the largest |entry| of row j among columns j..K-1 (the
// lowest column on ties) and exchanges that column with column j, occ[]
// along with it.  On return a = (A Q)^-1 for the column permutation Q, so
// that row c of the result belongs to orbital occ[c]; det A = mant * 2^ex
// (mant = 0 on a zero pivot, a then undefined).  Every other row is reduced
// by the multiplier a[i][j] / pivot times the unscaled pivot row, as in the
// LU, so equal rows still give an exactly zero pivot.
// one pivot step j of gj_inverse_cols (a template, so that every register
// index is static); returns false on a zero pivot
template <int K, int J>
__device__ __forceinline__ bool gj_step(double (&a)[K][K], int (&occ)[K], double &m, int &k) {
    int p = J;
    double best = fabs(a[J][J]);
#pragma unroll
    for (int c = J + 1; c < K; ++c)
        if (fabs(a[J][c]) > best) {
            best = fabs(a[J][c]);
            p = c;
        }
    if (!(best > 0.0)) return false;
    // column exchange by selects (no branches: the matrix stays in registers)
#pragma unroll
    for (int c = J + 1; c < K; ++c) {
        const bool sw = c == p;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const double x = a[r][c], y = a[r][J];
            a[r][c] = sw ? y : x;
            a[r][J] = sw ? x : y;
        }
        const int x = occ[c], y = occ[J];
        occ[c] = sw ? y : x;
        occ[J] = sw ? x : y;
    }
    if (p != J) m = -m;
    const double piv = a[J][J];
    m *= piv;
    int kk;
    m = frexp(m, &kk);
    k += kk;
    const double rinv = 1.0 / piv;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (i == J) continue;
        const double l = div_by(a[i][J], piv, rinv);
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (c != J) a[i][c] -= l * a[J][c];
        a[i][J] = -l;
    }
#pragma unroll
    for (int c = 0; c < K; ++c)
        if (c != J) a[J][c] *= rinv;
    a[J][J] = rinv;
    if constexpr (J + 1 < K) return gj_step<K, J + 1>(a, occ, m, k);
    else return true;
}

// In-place Gauss-Jordan inversion of a[K][K] with column pivoting: step j
// takes as pivot the largest |entry| of row j among columns j..K-1 (the
// lowest column on ties) and exchanges that column with column j, occ[]
// along with it.  On return a = (A Q)^-1 for the column permutation Q, so
// that row c of the result belongs to orbital occ[c]; det A = mant * 2^ex
// (mant = 0 on a zero pivot, a then undefined).  Every other row is reduced
// by the multiplier a[i][j] / pivot times the unscaled pivot row, as in the
// LU, so equal rows still give an exactly zero pivot.
template <int K>
__device__ __forceinline__ void gj_inverse_cols(double (&a)[K][K], int (&occ)[K], double &mant,
                                                int &ex) {
    double m = 1.0;
    int k = 0;
    if (gj_step<K, 0>(a, occ, m, k)) {
        mant = m;
        ex = k;
    } else {
        mant = 0.0;
        ex = 0;
    }
}

// occupied orbitals occ[c] of the slots c < n of determinant D (the
// reference's occ0 with the holes replaced by the particles), 0 beyond n;
// H: the holes and particles of a determinant of degree above kFastDegree,
// null otherwise.  Every register index is static (the holes and particles
// are unpacked from whole words), so nothing goes through scratch memory.
template <int K>
__device__ __forceinline__ void det_orbitals(const DetDesc &D, const DetDescHi *H, const int *occ0,
                                             int n, int (&occ)[K]) {
#pragma unroll
    for (int c = 0; c < K; ++c) occ[c] = (c < n) ? occ0[c] : 0;
    auto put = [&](int h, int p) {
#pragma unroll
        for (int c = 0; c < K; ++c) occ[c] = (c == h) ? p : occ[c];
    };
    if (H) {
        const uint2 hv = *reinterpret_cast<const uint2 *>(H->h);
        const uint2 p0 = *reinterpret_cast<const uint2 *>(H->p);
        const uint2 p1 = *reinterpret_cast<const uint2 *>(H->p + 4);
        const uint32_t pw[4] = {p0.x, p0.y, p1.x, p1.y};
#pragma unroll
        for (int t = 0; t < MDET_MAX_DEGREE; ++t)
            if (t < D.s)
                put((int)(((t < 4 ? hv.x : hv.y) >> (8 * (t & 3))) & 0xFFu),
                    (int)((pw[t >> 1] >> (16 * (t & 1))) & 0xFFFFu));
    } else {
#pragma unroll
        for (int t = 0; t < kFastDegree; ++t)
            if (t < D.s) put((int)D.h[t], (int)D.p[t]);
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// K x K Slater matrix of determinant D (slots in ascending order) from the
// staged scaled values P0[e*M + m] of the spin's n <= K electrons, padded
// with an identity block; occ[c] = orbital of slot c; returns sum of the
// column exponents.
template <int K>
__device__ __forceinline__ int direct_matrix(const DetDesc &D, const DetDescHi *H,
                                             const int *occ0, const double *P0, const int *Ex,
                                             int M, int n, double (&A)[K][K], int (&occ)[K]) {
    int sx = 0;
    det_orbitals<K>(D, H, occ0, n, occ);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        if (c < n) sx += Ex[occ[c]];
#pragma unroll
        for (int e = 0; e < K; ++e) {
            const double v = P0[min(e, n - 1) * M + occ[c]];
            A[e][c] = (c < n) ? ((e < n) ? v : 0.0) : ((e == c) ? 1.0 : 0.0);
        }
    }
    return sx;
}

// one work item of the ratio pass: mantissa and exponent of determinants
// [d0, d1) of (walker w, spin sp); returns the thread's largest exponent
template <int K>
__device__ __forceinline__ int direct_ratio_item(const KernelArgs &a, int sp, int w, const SpinDev &S,
                                 const int *occ0, const double *P0, const int *Ex, int d0,
                                 int d1) {
    const int M = a.M, n = S.n;
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    int kmax = INT_MIN;
    for (int d = d0 + (int)threadIdx.x; d < d1; d += kDirectBlock) {
        const DetDesc D = S.desc[d];
        const int Ulo = S.deg_end[kFastDegree];
        const DetDescHi *H = d >= Ulo ? S.desc_hi + (d - Ulo) : nullptr;
        double r = 0.0;
        int rexp = INT_MIN;
        if (D.s <= dmax) {
            double A[K][K];
            int occ[K], perm[K];
            const int sx = direct_matrix<K>(D, H, occ0, P0, Ex, M, n, A, occ);
            double mant;
            int ex;
            lu_regs<K, false>(A, perm, mant, ex);
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
    return kmax;
}

// per-thread inputs of one determinant of the derivative pass: descriptor,
// exponent of its ratio (INT_MIN if singular) and its weight u or v
struct DirectDet {
    DetDesc D;
    int rexp;
    double wt;
};

__device__ __forceinline__ DirectDet direct_det_load(const KernelArgs &a, const SpinDev &S, int sp,
                                                     int w, int d) {
    DirectDet X;
    X.D = S.desc[d];
    const size_t o = rv_index(a, sp, d, w);
    X.rexp = a.wk.Rexp[o];
    X.wt = a.precision == MDET_MIXED ? (double)a.wk.uv32[o] : a.wk.uv64[o];
    return X;
}

// one work item of the derivative pass: adds, per electron e and component
// q, the wave sums of  w_d D_d grad~_e D_d / D_d  (row-replacement form with
// column e of S_d^-1) to red[wave][e*4 + q].  P0 holds the unscaled orbital
// values, Gs (if not null) the unscaled derivatives, else Gg points at the
// orbital array; columns are scaled by 2^-Ex at the matrix and the rows of
// the inverse scaled back.  `first` is the thread's determinant d0 + tid,
// loaded before the staging.
template <int K>
__device__ __forceinline__ void direct_deriv_item(const KernelArgs &a, int sp, int w,
                                                  const SpinDev &S, const int *occ0,
                                                  const double *P0, const double *Gs,
                                                  const double *Gg, const int *Ex, int d0, int d1,
                                                  const DirectDet &first, double *red, double *wr) {
    const int M = a.M, n = S.n;
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const int Kx = a.wk.K[(size_t)w * 2 + sp];
    const int Ulo = S.deg_end[kFastDegree];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int base = d0; base < d1; base += kDirectBlock) {
        // every lane takes part in the wave sums; lanes without a valid
        // determinant contribute zeros
        const int d = base + (int)threadIdx.x;
        const bool in = d < d1;
        const int dd = in ? d : d0;
        const DirectDet X = base == d0 ? first : direct_det_load(a, S, sp, w, dd);
        const DetDescHi *H = dd >= Ulo ? S.desc_hi + (dd - Ulo) : nullptr;
        double A[K][K];
        int occ[K];
        int sx = 0;
        det_orbitals<K>(X.D, H, occ0, n, occ);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const double sc = pow2(-Ex[occ[c]]);
            if (c < n) sx += Ex[occ[c]];
#pragma unroll
            for (int e = 0; e < K; ++e) {
                const double v = P0[min(e, n - 1) * M + occ[c]] * sc;
                A[e][c] = (c < n) ? ((e < n) ? v : 0.0) : ((e == c) ? 1.0 : 0.0);
            }
        }
        double mant;
        int ex;
        gj_inverse_cols<K>(A, occ, mant, ex);
        const bool valid = in && X.D.s <= dmax && X.rexp != INT_MIN && mant != 0.0;
        const double coef =
            valid ? X.wt * ldexp((double)X.D.eps * mant, ex + sx - Kx) : 0.0;
        // row c of the inverse belongs to orbital occ[c]: scale it back
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const double sc = pow2(-Ex[occ[c]]);
#pragma unroll
            for (int e = 0; e < K; ++e) A[c][e] *= sc;
        }
#pragma unroll
        for (int g = 0; g < (K + kEHalf - 1) / kEHalf; ++g) {
#pragma unroll
            for (int i = 0; i < kEHalf; ++i) {
                const int e = g * kEHalf + i;
                if (e < K && e < n) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double *G = Gs ? Gs + (size_t)(q * n + e) * M
                                             : Gg + (size_t)e * 5 * M + (size_t)(1 + q) * M;
                        double s = 0.0;
#pragma unroll
                        for (int c = 0; c < K; ++c)
                            if (c < n) s += A[c][e < K ? e : 0] * G[occ[c]];
                        wr[lane * kWredLd + i * 4 + q] = valid ? coef * s : 0.0;
                    }
                }
            }
            // the wave's sums of this group of electrons: lane t adds column t
            // over the lanes (four interleaved partial sums)
            const int e0 = g * kEHalf, ne = min(n, e0 + kEHalf) - e0;
            wave_lds_sync();
            if (lane < ne * 4) {
                double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
                for (int l = 0; l < 64; l += 4) {
                    t0 += wr[l * kWredLd + lane];
                    t1 += wr[(l + 1) * kWredLd + lane];
                    t2 += wr[(l + 2) * kWredLd + lane];
                    t3 += wr[(l + 3) * kWredLd + lane];
                }
                red[wave * 4 * K + e0 * 4 + lane] += (t0 + t1) + (t2 + t3);
            }
            wave_lds_sync();
        }
    }
}

// stage the orbital values (and, if G is not null, the derivatives) of
// electrons e0 .. e0+n-1 of walker w: P0[e*M + m] = phi * 2^-E[m] (SCALE) or
// phi, and G[((q-1)*n + e)*M + m] = the derivative plane q = 1..4 (unscaled).
// KU loads are in flight per thread before the stores; a thread walks its
// elements with a running (electron, offset) pair instead of divisions, and
// past the end it loads element 0 again rather than skipping the load, so
// that the loads are issued together.
template <bool SCALE, int KU>
__device__ __forceinline__ void stage_orbitals(const KernelArgs &a, int w, int e0, int n,
                                               const int *Ex, double *P0, double *G) {
    const int M = a.M;
    const double *phig = a.wk.phi + ((size_t)w * a.N + e0) * 5 * M;
    // element (e, r) of the planes taken: plane q = r / M < nq, orbital r % M
    const int nq = G ? 5 : 1, nqM = nq * M;
    const int step = (int)blockDim.x;
    int e = 0, r = (int)threadIdx.x;
    while (r >= nqM) {
        r -= nqM;
        ++e;
    }
    while (e < n) {
        double v[KU];
        int ev[KU], rv[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            ev[u] = e;
            rv[u] = r;
            v[u] = phig[e < n ? (size_t)e * 5 * M + r : 0];
            r += step;
            while (r >= nqM) {
                r -= nqM;
                ++e;
            }
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            if (ev[u] < n) {
                const int rr = rv[u];
                const int q = nq == 1 ? 0
                                      : (rr >= M) + (rr >= 2 * M) + (rr >= 3 * M) + (rr >= 4 * M);
                const int m = rr - q * M;
                const double x = SCALE ? v[u] * pow2(-Ex[m]) : v[u];
                if (q == 0) P0[ev[u] * M + m] = x;
                else G[((q - 1) * n + ev[u]) * M + m] = x;
            }
        }
    }
}

}  // namespace

// the flagged (walker, spin) pairs in ascending order (one block of 1024:
// per-thread counts over contiguous ranges, a scan, then the writes)
__global__ void __launch_bounds__(1024) k_direct_list(KernelArgs a) {
    __shared__ int cnt[1024];
    const int t = threadIdx.x;
    const int64_t P = 2 * a.W, per = (P + 1023) / 1024;
    const int64_t b0 = t * per, b1 = min(P, b0 + per);
    int c = 0;
    for (int64_t i = b0; i < b1; ++i) c += a.wk.flag[i] != 0;
    cnt[t] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
        const int v = t >= off ? cnt[t - off] : 0;
        __syncthreads();
        cnt[t] += v;
        __syncthreads();
    }
    int pos = cnt[t] - c;
    for (int64_t i = b0; i < b1; ++i)
        if (a.wk.flag[i] != 0) a.wk.dlist[pos++] = (int32_t)i;
    if (t == 1023) a.wk.dcount[0] = cnt[1023];
}

// pass 1: mantissa and exponent of every determinant of the flagged pairs,
// and the integer maximum of the exponents per (walker, spin)
template <int NT>
__global__ void __launch_bounds__(kDirectBlock, 2) k_direct_ratios_t(KernelArgs a) {
    const int M = a.M, tid = threadIdx.x, split = a.direct_split;
    extern __shared__ double lds[];
    double *P0 = lds;                 // [NT][M] scaled orbital values of the pair's spin
    int *Ex = (int *)(P0 + NT * M);   // [M]
    int *occ0 = Ex + M;               // [NT]
    __shared__ int red[kDirectBlock];
    const int nitems = a.wk.dcount[0] * split;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int ws = __builtin_amdgcn_readfirstlane(a.wk.dlist[it / split]);
        const int part = it - (it / split) * split;
        const int w = ws >> 1, sp = ws & 1;
        const SpinDev &S = a.sp[sp];
        const int n = S.n;
        __syncthreads();  // the previous item is done with the LDS
        for (int m = tid; m < M; m += kDirectBlock) Ex[m] = a.wk.E[(size_t)ws * M + m];
        for (int c = tid; c < n; c += kDirectBlock) occ0[c] = S.occ0[c];
        __syncthreads();
        stage_orbitals<true, 8>(a, w, S.e0, n, Ex, P0, nullptr);
        __syncthreads();
        const int d0 = (int)((int64_t)S.U * part / split);
        const int d1 = (int)((int64_t)S.U * (part + 1) / split);
        int kmax;
        if (NT > 1 && n == NT - 1)
            kmax = direct_ratio_item<(NT > 1 ? NT - 1 : 1)>(a, sp, w, S, occ0, P0, Ex, d0, d1);
        else kmax = direct_ratio_item<NT>(a, sp, w, S, occ0, P0, Ex, d0, d1);  // n <= NT
        red[tid] = kmax;
        __syncthreads();
        if (tid == 0) {
            int mx = INT_MIN;
            for (int t = 0; t < kDirectBlock; ++t) mx = max(mx, red[t]);
            if (mx != INT_MIN) atomicMax(&a.wk.Kmax[ws], mx);
        }
    }
}

// pass 2: shift every ratio by the (walker, spin) maximum exponent
__global__ void __launch_bounds__(kBlock) k_direct_scale(KernelArgs a) {
    const int split = a.direct_split;
    const int nitems = a.wk.dcount[0] * split;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int ws = __builtin_amdgcn_readfirstlane(a.wk.dlist[it / split]);
        const int part = it - (it / split) * split;
        const int w = ws >> 1, sp = ws & 1;
        const SpinDev &S = a.sp[sp];
        int K = a.wk.Kmax[ws];
        if (K == INT_MIN) K = 0;
        if (part == 0 && threadIdx.x == 0) {
            a.wk.K[ws] = K;
            a.wk.logdet0[ws] = 0.0;
            a.wk.sign0[ws] = 1.0;
        }
        const int d0 = (int)((int64_t)S.U * part / split);
        const int d1 = (int)((int64_t)S.U * (part + 1) / split);
        for (int d = d0 + threadIdx.x; d < d1; d += kBlock) {
            const size_t o = rv_index(a, sp, d, w);
            const int e = a.wk.Rexp[o];
            const double r = (e == INT_MIN) ? 0.0 : ldexp(a.wk.R64[o], e - K);
            a.wk.R64[o] = r;
            if (a.precision == MDET_MIXED) a.wk.R32[o] = (float)r;
        }
    }
}

// pass 3 (after the sparse combination): derivative partial sums per item
template <int NT>
__global__ void __launch_bounds__(kDirectBlock, 2) k_direct_deriv_t(KernelArgs a) {
    const int M = a.M, N = a.N, tid = threadIdx.x, split = a.direct_split;
    const bool stage_g = a.direct_stage_grad != 0;
    extern __shared__ double lds[];
    double *P0 = lds;                                  // [NT][M] unscaled values
    double *G = stage_g ? P0 + NT * M : nullptr;       // [4][NT][M] unscaled derivatives
    double *red = P0 + (stage_g ? 5 : 1) * NT * M;     // [kDirectBlock / 64][NT * 4]
    double *wred = red + (kDirectBlock / 64) * NT * 4;  // [kDirectBlock / 64][64][kWredLd]
    int *Ex = (int *)(wred + (kDirectBlock / 64) * 64 * kWredLd);  // [M]
    int *occ0 = Ex + M;                                // [NT]
    const int nitems = a.wk.dcount[0] * split;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int ws = __builtin_amdgcn_readfirstlane(a.wk.dlist[it / split]);
        const int part = it - (it / split) * split;
        const int w = ws >> 1, sp = ws & 1;
        const SpinDev &S = a.sp[sp];
        const int n = S.n;
        const int d0 = (int)((int64_t)S.U * part / split);
        const int d1 = (int)((int64_t)S.U * (part + 1) / split);
        __syncthreads();  // the previous item is done with the LDS
        // the thread's first determinant and the column exponents (at most
        // MDET_MAX_MO = 2 kDirectBlock of them) are loaded while the block
        // stages the orbitals
        const DirectDet first = direct_det_load(a, S, sp, w, d0 + tid < d1 ? d0 + tid : 0);
        static_assert(MDET_MAX_MO <= 2 * kDirectBlock, "column exponents: two per thread");
        const int ex0 = a.wk.E[(size_t)ws * M + min(tid, M - 1)];
        const int ex1 = a.wk.E[(size_t)ws * M + min(tid + kDirectBlock, M - 1)];
        for (int c = tid; c < n; c += kDirectBlock) occ0[c] = S.occ0[c];
        for (int i = tid; i < (kDirectBlock / 64) * NT * 4; i += kDirectBlock) red[i] = 0.0;
        stage_orbitals<false, 24>(a, w, S.e0, n, nullptr, P0, G);
        if (tid < M) Ex[tid] = ex0;
        if (tid + kDirectBlock < M) Ex[tid + kDirectBlock] = ex1;
        __syncthreads();
        const double *Gg = a.wk.phi + ((size_t)w * N + S.e0) * 5 * M;
        int K;
        if (NT > 1 && n == NT - 1) {
            K = NT > 1 ? NT - 1 : 1;
            direct_deriv_item<(NT > 1 ? NT - 1 : 1)>(a, sp, w, S, occ0, P0, G, Gg, Ex, d0, d1,
                                                      first, red, wred + (tid >> 6) * 64 * kWredLd);
        } else {
            K = NT;  // n <= NT
            direct_deriv_item<NT>(a, sp, w, S, occ0, P0, G, Gg, Ex, d0, d1, first, red,
                                  wred + (tid >> 6) * 64 * kWredLd);
        }
        __syncthreads();
        for (int i = tid; i < n * 4; i += kDirectBlock) {
            const int e = i >> 2, q = i & 3;
            double t = 0.0;
            for (int v = 0; v < kDirectBlock / 64; ++v) t += red[v * 4 * K + e * 4 + q];
            a.wk.dpart[(((size_t)w * kDirectSplitMax + part) * N + S.e0) * 4 + i] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Outputs: sign, ln|Psi|, status; the fallback's derivative partials are
// combined here; nodes get zero derivatives.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_finalize(KernelArgs a) {
    // one thread per output entry (walker w, electron e, component q); the
    // thread with e = q = 0 also writes the walker's sign, ln|Psi| and status
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int per = 4 * a.N;
    if (i >= a.W * per) return;
    const int64_t w = i / per;
    const int t = (int)(i - w * per);
    // psi_up gives sign and ln|Psi| (and divides every derivative numerator)
    const double psi = psi_value(a, (int)w, 0);
    const double psi_dn = psi_value(a, (int)w, 1);
    const bool node = !(psi != 0.0) || !isfinite(psi) || !(psi_dn != 0.0) || !isfinite(psi_dn);
    const int sp = (t >= 4 * a.sp[1].e0) ? 1 : 0;
    const bool chain = a.method == MDET_METHOD_SM_CHAIN;
    if (node) {
        a.gl_out[i] = 0.0;
    } else if (!chain && a.wk.flag[2 * w + sp] != 0) {
        const int np = a.direct_split, last = np > 0 ? np - 1 : 0;
        double v[kDirectSplitMax];
#pragma unroll
        for (int p = 0; p < kDirectSplitMax; ++p)
            v[p] = a.wk.dpart[((size_t)w * kDirectSplitMax + (p < np ? p : last)) * per + t];
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < kDirectSplitMax; ++p)
            if (p < np) s += v[p];
        a.gl_out[i] = s / psi;  // the whole numerator: over the psi of ln|Psi|
    }
    if (t != 0) return;
    if (node) {
        a.sign_out[w] = 0.0;
        a.logabs_out[w] = -INFINITY;
        if (a.wstatus) a.wstatus[w] = MDET_W_NODE;
        return;
    }
    const double sg = a.wk.sign0[2 * w] * a.wk.sign0[2 * w + 1] * (psi > 0 ? 1.0 : -1.0);
    a.sign_out[w] = sg;
    a.logabs_out[w] = a.wk.logdet0[2 * w] + a.wk.logdet0[2 * w + 1] + log(fabs(psi)) +
                      (double)(a.wk.K[2 * w] + a.wk.K[2 * w + 1]) * 0.69314718055994530942;
    if (a.wstatus)
        a.wstatus[w] = (!chain && (a.wk.flag[2 * w] || a.wk.flag[2 * w + 1])) ? MDET_W_FALLBACK
                                                                              : MDET_W_OK;
}

// ---------------------------------------------------------------------------
uint32_t kernels_of_method(int method) {
    return method == MDET_METHOD_SM_CHAIN ? (1u << 0) | (1u << 3) | (1u << 6) | (1u << 7) | (1u << 8)
                                          : 0x7fu;
}

const char *kernel_name(int k) {
    static const char *names[kNumKernels] = {"k_reference", "k_ratios",   "k_direct_ratios",
                                             "k_spmm",      "k_deriv",    "k_direct_deriv",
                                             "k_finalize",  "k_sm_chain", "k_sm_deriv"};
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
void launch_direct(const KernelArgs &a, hipStream_t st, bool deriv, int cap) {
    const int M = a.M;
    // a fixed grid walks the (pair, part) items; at most 2 W of them per part
    const unsigned grid = (unsigned)std::min<int64_t>(2 * a.W * a.direct_split, cap);
    if (deriv) {
        const size_t lds = sizeof(double) * ((a.direct_stage_grad ? 5 : 1) * (size_t)NT * M +
                                             (kDirectBlock / 64) * (NT * 4 + 64 * kWredLd)) +
                           sizeof(int) * (M + NT);
        k_direct_deriv_t<NT><<<dim3(grid), dim3(kDirectBlock), lds, st>>>(a);
    } else {
        const size_t lds = sizeof(double) * (size_t)NT * M + sizeof(int) * (M + NT);
        k_direct_ratios_t<NT><<<dim3(grid), dim3(kDirectBlock), lds, st>>>(a);
    }
}

// cap: most blocks of the fixed grid (each block is placed on a CU before it
// finds no item left, so a grid beside another kernel is kept small)
void launch_direct_n(const KernelArgs &a, hipStream_t st, bool deriv, int cap = 1024) {
    switch (a.nmax) {  // the larger electron count (n_up)
    case 1: launch_direct<1>(a, st, deriv, cap); break;
    case 2: launch_direct<2>(a, st, deriv, cap); break;
    case 3: launch_direct<3>(a, st, deriv, cap); break;
    case 4: launch_direct<4>(a, st, deriv, cap); break;
    case 5: launch_direct<5>(a, st, deriv, cap); break;
    case 6: launch_direct<6>(a, st, deriv, cap); break;
    case 7: launch_direct<7>(a, st, deriv, cap); break;
    case 8: launch_direct<8>(a, st, deriv, cap); break;
    case 9: launch_direct<9>(a, st, deriv, cap); break;
    case 10: launch_direct<10>(a, st, deriv, cap); break;
    case 11: launch_direct<11>(a, st, deriv, cap); break;
    case 12: launch_direct<12>(a, st, deriv, cap); break;
    case 13: launch_direct<13>(a, st, deriv, cap); break;
    case 14: launch_direct<14>(a, st, deriv, cap); break;
    case 15: launch_direct<15>(a, st, deriv, cap); break;
    default: launch_direct<16>(a, st, deriv, cap); break;  // nmax <= MDET_MAX_SPIN_ELEC = 16
    }
}

// slices per flagged pair of the fallback: one determinant per thread up to
// kDirectSplitMax slices, unless requested explicitly
int direct_splits(const KernelArgs &a, int requested) {
    if (requested > 0) return std::max(1, std::min(requested, kDirectSplitMax));
    const int U = std::max(a.sp[0].U, a.sp[1].U);
    return std::max(1, std::min((U + kDirectBlock - 1) / kDirectBlock, kDirectSplitMax));
}

int psi_splits(int64_t W, int requested) {
    if (requested > 0) return std::max(1, std::min(requested, kPsiParts));
    const int64_t tiles = (W + kSpmmTile - 1) / kSpmmTile;
    const int rs = (int)((256 + tiles - 1) / tiles);
    return std::max(1, std::min(rs, kPsiParts));
}

hipError_t launch_core(const KernelArgs &a, hipStream_t st, hipEvent_t *ev, const AuxStreams *aux);
hipError_t launch_chain(const KernelArgs &a, hipStream_t st, hipEvent_t *ev);

}  // namespace

hipError_t launch_eval(const KernelArgs &args, hipStream_t st, hipEvent_t *ev,
                       const AuxStreams *aux) {
    const int64_t W = args.W;
    if (W == 0) return hipSuccess;
    KernelArgs a = args;
    a.psi_nparts = psi_splits(W, a.cfg.spmm_rsplit);
    a.direct_split = direct_splits(a, a.cfg.direct_split);
    // stage the orbital derivatives of the fallback in LDS when they fit
    a.direct_stage_grad = sizeof(double) * (5 * (size_t)a.nmax * a.M) <= 96 * 1024 ? 1 : 0;
    if (!(a.max_degree && a.cfg.sort_walkers)) return launch_core(a, st, ev, aux);
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
    const hipError_t e = launch_core(b, st, ev, aux);
    if (e != hipSuccess) return e;
    k_sort_scatter<<<dim3((unsigned)((W * N * 4 + 255) / 256)), dim3(256), 0, st>>>(
        W, N, a.wk.perm, a.wk.sign_s, a.wk.logabs_s, a.wk.gl_s, a.wk.ws_s, a.sign_out, a.logabs_out,
        a.gl_out, a.wstatus);
    return hipGetLastError();
}

namespace {

// The table method.  With `aux` and cfg.overlap_fallback, the direct-LU
// fallback of the ill-conditioned pairs runs on the second stream: its list
// and ratios beside the table ratios (joined before the sparse products,
// which read every ratio), its derivative sums beside the derivative
// aggregation (joined before the outputs).  Otherwise everything runs in
// order on `st`.
hipError_t launch_core(const KernelArgs &a, hipStream_t st, hipEvent_t *ev, const AuxStreams *aux) {
    const int W = (int)a.W;
    const int n = a.nmax, M = a.M;
    const dim3 g2(2 * W), blk(kBlock);
    const bool ovl = aux && a.cfg.overlap_fallback && a.method != MDET_METHOD_SM_CHAIN;
    hipStream_t sf = ovl ? aux->s : st;  // the fallback's stream
    auto mark = [&](int k, bool end, hipStream_t s) {
        if (ev && ((a.ev_mask >> k) & 1u)) (void)hipEventRecord(ev[2 * k + (end ? 1 : 0)], s);
    };
    hipError_t err = hipSuccess;
    auto fork = [&](hipEvent_t e, hipStream_t from, hipStream_t to) {
        if (err == hipSuccess) err = hipEventRecord(e, from);
        if (err == hipSuccess) err = hipStreamWaitEvent(to, e, 0);
    };
    mark(0, false, st);
    const size_t prim_bytes = (size_t)(a.prim_dn != a.prim ? 2 : 1) * M * a.P * kPrimLdsBytes;
    const size_t lds_ref = sizeof(double) * (14 * (size_t)n * n + 2 * (2 * kMaxN + 2) +
                                             (size_t)a.N * (3 * kPowLd + 1)) +
                           sizeof(int) * (4 * (size_t)M + 2 * kMaxN) +
                           (prim_bytes <= kPrimLdsMax ? prim_bytes : 0);
    k_reference<<<dim3(W), blk, lds_ref, st>>>(a);
    mark(0, true, st);
    if (a.method == MDET_METHOD_SM_CHAIN) return launch_chain(a, st, ev);
    // beside the table-method kernels the fallback's grids are kept small: it
    // has their whole duration, and every block of a grid takes a CU slot
    const int cap_r = ovl ? 256 : 1024, cap_d = ovl ? 128 : 1024;
    const unsigned gscale = (unsigned)std::min<int64_t>(2 * (int64_t)W * a.direct_split, cap_r);
    auto fallback_ratios = [&]() {
        mark(2, false, sf);
        k_direct_list<<<dim3(1), dim3(1024), 0, sf>>>(a);
        launch_direct_n(a, sf, false, cap_r);
        k_direct_scale<<<dim3(gscale), blk, 0, sf>>>(a);
        mark(2, true, sf);
    };
    if (ovl) {
        fork(aux->ev[0], st, sf);
        fallback_ratios();
        if (err == hipSuccess) err = hipEventRecord(aux->ev[1], sf);
    }
    mark(1, false, st);
    const size_t lds_rat = sizeof(double) * ((size_t)n * M + n * n) + sizeof(int) * (M + n);
    if (a.wk.hi_stride > 0) k_ratios_hi<<<g2, blk, lds_rat, st>>>(a);
    k_ratios<<<g2, blk, lds_rat, st>>>(a);
    mark(1, true, st);
    if (ovl) {
        if (err == hipSuccess) err = hipStreamWaitEvent(st, aux->ev[1], 0);
    } else {
        fallback_ratios();
    }
    mark(3, false, st);
    const int tiles = (W + kSpmmTile - 1) / kSpmmTile;
    const dim3 gs((tiles + 7) / 8 * 8 * a.psi_nparts, 2), bs(64 * kSpmmWaves);
    if (a.precision == MDET_MIXED)
        k_spmm<float, kSpmmCols32, float><<<gs, bs, 0, st>>>(
            a, a.wk.R32, a.wk.R64, a.wk.uv32, a.C.rval32, a.C.cval32, a.C.rcol, a.C.crow, a.C.rseg32,
            a.C.cseg32, a.C.nch_r32, a.C.nch_c32, a.psi_nparts);
    else
        k_spmm<double, kSpmmCols64, double><<<gs, bs, 0, st>>>(
            a, a.wk.R64, a.wk.R64, a.wk.uv64, a.C.rval, a.C.cval, a.C.rcol, a.C.crow, a.C.rseg64,
            a.C.cseg64, a.C.nch_r64, a.C.nch_c64, a.psi_nparts);
    mark(3, true, st);
    if (ovl) {
        fork(aux->ev[2], st, sf);
        mark(5, false, sf);
        launch_direct_n(a, sf, true, cap_d);
        mark(5, true, sf);
        if (err == hipSuccess) err = hipEventRecord(aux->ev[3], sf);
    }
    mark(4, false, st);
    const size_t lds_der = sizeof(double) * (2 * (size_t)n * M + n * n + deriv_union_doubles(n, M)) +
                           sizeof(int) * (M + n);
    k_deriv<<<g2, blk, lds_der, st>>>(a);
    mark(4, true, st);
    if (ovl) {
        if (err == hipSuccess) err = hipStreamWaitEvent(st, aux->ev[3], 0);
    } else {
        mark(5, false, st);
        launch_direct_n(a, st, true);
        mark(5, true, st);
    }
    mark(6, false, st);
    k_finalize<<<dim3((unsigned)(((int64_t)W * 4 * a.N + kBlock - 1) / kBlock)), blk, 0, st>>>(a);
    mark(6, true, st);
    if (err != hipSuccess) return err;
    return hipGetLastError();
}

// Sherman-Morrison chain method: chain pieces, exponent shift, the sparse
// combination, derivative sums, outputs (event slots 0, 7, 3, 8, 6).
hipError_t launch_chain(const KernelArgs &a, hipStream_t st, hipEvent_t *ev) {
    const int W = (int)a.W;
    const dim3 g2(2 * W), blk(kBlock);
    auto mark = [&](int k, bool end) {
        if (ev && ((a.ev_mask >> k) & 1u)) (void)hipEventRecord(ev[2 * k + (end ? 1 : 0)], st);
    };
    const bool mixed = a.precision == MDET_MIXED;
    mark(7, false);
    launch_chain_pieces(a, st);
    mark(7, true);
    mark(3, false);
    const int tiles = (W + kSpmmTile - 1) / kSpmmTile;
    const dim3 gs((tiles + 7) / 8 * 8 * a.psi_nparts, 2), bs(64 * kSpmmWaves);
    if (mixed)
        k_spmm<float, kSpmmCols32, float><<<gs, bs, 0, st>>>(
            a, a.wk.R32, a.wk.R64, a.wk.uv32, a.C.rval32, a.C.cval32, a.C.rcol, a.C.crow, a.C.rseg32,
            a.C.cseg32, a.C.nch_r32, a.C.nch_c32, a.psi_nparts);
    else
        k_spmm<double, kSpmmCols64, double><<<gs, bs, 0, st>>>(
            a, a.wk.R64, a.wk.R64, a.wk.uv64, a.C.rval, a.C.cval, a.C.rcol, a.C.crow, a.C.rseg64,
            a.C.cseg64, a.C.nch_r64, a.C.nch_c64, a.psi_nparts);
    mark(3, true);
    mark(8, false);
    launch_chain_deriv(a, st);
    mark(8, true);
    mark(6, false);
    k_finalize<<<dim3((unsigned)(((int64_t)W * 4 * a.N + kBlock - 1) / kBlock)), blk, 0, st>>>(a);
    mark(6, true);
    return hipGetLastError();
}

}  // namespace

}  // namespace mdet
