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

__device__ __forceinline__ void load_excitation(const DetDesc &D, const double *T, int M,
                                                double *mat) {
    const int s = D.s;
    for (int a = 0; a < s; ++a)
        for (int b = 0; b < s; ++b) mat[a * s + b] = T[D.h[a] * M + D.p[b]];
}

__device__ __forceinline__ int delta_exponent(const DetDesc &D, const int *Ex, const int *occ0) {
    int dx = 0;
    for (int a = 0; a < D.s; ++a) dx += Ex[D.p[a]] - Ex[occ0[D.h[a]]];
    return dx;
}

__device__ __forceinline__ size_t rv_offset(const KernelArgs &a, int sp) {
    return sp == 0 ? 0 : (size_t)a.wk.Upad;
}

__device__ __forceinline__ size_t rv_stride(const KernelArgs &a) {
    return (size_t)a.wk.Upad + a.wk.Vpad;
}

}  // namespace

// ---------------------------------------------------------------------------
// K1+K2+K3: orbitals, scaled reference LU, inverse, refinement, table T, g0.
// One block per (walker, spin).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_reference(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, N = a.N, e0 = S.e0, tid = threadIdx.x;
    extern __shared__ double lds[];
    double *phi0 = lds;            // [n][M] scaled orbital values
    double *Aor = phi0 + n * M;    // [n][n] scaled reference
    double *LU = Aor + n * n;      // [n][n]
    double *Xs = LU + n * n;       // [n][n]
    double *Rm = Xs + n * n;       // [n][n]
    int *Ex = (int *)(Rm + n * n); // [M]
    __shared__ int piv[kMaxN];
    __shared__ int s_state;        // 0 ok, 2 singular
    __shared__ double colA[kMaxN], colX[kMaxN];

    double *phig = a.wk.phi + (size_t)w * N * 5 * M;
    const double *Rw = a.R + (size_t)w * N * 3;

    for (int idx = tid; idx < n * M; idx += kBlock) {
        const int e = idx / M, m = idx - e * M;
        const double *r = Rw + 3 * (e0 + e);
        double o[5];
        orbital5(a.prim, a.P, m, r[0], r[1], r[2], o);
        double *dst = phig + (size_t)(e0 + e) * 5 * M + m;
        for (int q = 0; q < 5; ++q) dst[q * M] = o[q];
        phi0[e * M + m] = o[0];
    }
    if (tid == 0) s_state = 0;
    __syncthreads();
    for (int m = tid; m < M; m += kBlock) {
        double mx = 0.0;
        for (int e = 0; e < n; ++e) mx = fmax(mx, fabs(phi0[e * M + m]));
        Ex[m] = expo(mx);
        a.wk.E[((size_t)w * 2 + sp) * M + m] = Ex[m];
    }
    __syncthreads();
    for (int idx = tid; idx < n * M; idx += kBlock) {
        const int e = idx / M, m = idx - e * M;
        const double sc = pow2(-Ex[m]);
        phi0[idx] *= sc;
        double *dst = phig + (size_t)(e0 + e) * 5 * M + m;
        for (int q = 0; q < 5; ++q) dst[q * M] *= sc;
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int e = idx / n, c = idx - e * n;
        const double v = phi0[e * M + S.occ0[c]];
        Aor[idx] = v;
        LU[idx] = v;
    }
    __syncthreads();
    // LU with partial pivoting: lane i of wave 0 scans row i
    for (int j = 0; j < n; ++j) {
        if (tid < 64) {
            double v = (tid >= j && tid < n) ? fabs(LU[tid * n + j]) : -1.0;
            int id = tid;
            for (int off = 32; off > 0; off >>= 1) {
                const double v2 = __shfl_xor(v, off, 64);
                const int i2 = __shfl_xor(id, off, 64);
                if (v2 > v || (v2 == v && i2 < id)) {
                    v = v2;
                    id = i2;
                }
            }
            if (tid == 0) {
                piv[j] = id;
                if (!(v > 0.0)) s_state = 2;
            }
        }
        __syncthreads();
        if (s_state) break;
        const int p = piv[j];
        if (p != j && tid < n) {
            const double t = LU[j * n + tid];
            LU[j * n + tid] = LU[p * n + tid];
            LU[p * n + tid] = t;
        }
        __syncthreads();
        if (tid > j && tid < n) {
            const double l = LU[tid * n + j] / LU[j * n + j];
            LU[tid * n + j] = l;
            for (int c = j + 1; c < n; ++c) LU[tid * n + c] -= l * LU[j * n + c];
        }
        __syncthreads();
    }
    const size_t ws = (size_t)w * 2 + sp;
    if (s_state) {
        if (tid == 0) {
            a.wk.flag[ws] = 2;
            a.wk.logdet0[ws] = 0.0;
            a.wk.sign0[ws] = 1.0;
        }
        return;
    }
    // inverse: thread k solves A x = e_k using the factors
    if (tid < n) {
        const int k = tid;
        for (int i = 0; i < n; ++i) Xs[i * n + k] = (i == k) ? 1.0 : 0.0;
        for (int j = 0; j < n; ++j) {
            const int p = piv[j];
            if (p != j) {
                const double t = Xs[j * n + k];
                Xs[j * n + k] = Xs[p * n + k];
                Xs[p * n + k] = t;
            }
        }
        for (int i = 0; i < n; ++i) {
            double s = Xs[i * n + k];
            for (int j = 0; j < i; ++j) s -= LU[i * n + j] * Xs[j * n + k];
            Xs[i * n + k] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = Xs[i * n + k];
            for (int j = i + 1; j < n; ++j) s -= LU[i * n + j] * Xs[j * n + k];
            Xs[i * n + k] = s / LU[i * n + i];
        }
    }
    if (tid == 0) {
        double la = 0.0, sg = 1.0;
        for (int j = 0; j < n; ++j) {
            const double d = LU[j * n + j];
            la += log(fabs(d));
            if (d < 0) sg = -sg;
            if (piv[j] != j) sg = -sg;
        }
        int sx = 0;
        for (int c = 0; c < n; ++c) sx += Ex[S.occ0[c]];
        a.wk.logdet0[ws] = la + (double)sx * 0.69314718055994530942;
        a.wk.sign0[ws] = sg;
    }
    __syncthreads();
    // one residual-correction step: X <- X + X (I - A X)
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int i = idx / n, j = idx - i * n;
        double s = (i == j) ? 1.0 : 0.0;
        for (int k = 0; k < n; ++k) s -= Aor[i * n + k] * Xs[k * n + j];
        Rm[idx] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int i = idx / n, j = idx - i * n;
        double s = Xs[idx];
        for (int k = 0; k < n; ++k) s += Xs[i * n + k] * Rm[k * n + j];
        LU[idx] = s;  // refined inverse
    }
    __syncthreads();
    double *X = LU;
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
        double na = 0.0, nx = 0.0;
        for (int c = 0; c < n; ++c) {
            na = fmax(na, colA[c]);
            nx = fmax(nx, colX[c]);
        }
        const double kappa = na * nx;
        a.wk.flag[ws] = (kappa <= a.kappa_max) ? 0 : 1;  // NaN -> fallback
    }
    double *Xg = a.wk.X + ws * a.nmax * a.nmax;
    for (int idx = tid; idx < n * n; idx += kBlock) Xg[idx] = X[idx];
    double *Tg = a.wk.T + ws * a.nmax * M;
    for (int idx = tid; idx < n * M; idx += kBlock) {
        const int c = idx / M, m = idx - c * M;
        double s = 0.0;
        for (int e = 0; e < n; ++e) s += X[c * n + e] * phi0[e * M + m];
        Tg[idx] = s;
    }
    for (int idx = tid; idx < 4 * n; idx += kBlock) {
        const int e = idx >> 2, q = idx & 3;
        const double *g = phig + (size_t)(e0 + e) * 5 * M + (size_t)(1 + q) * M;
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += X[c * n + e] * g[S.occ0[c]];
        a.wk.g0[((size_t)w * N + e0 + e) * 4 + q] = s;
    }
}

// ---------------------------------------------------------------------------
// K4: ratios R_d / 2^K of every distinct determinant (table method).
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
    double *R64 = a.wk.R64 + (size_t)w * rv_stride(a) + rv_offset(a, sp);
    int kmax = INT_MIN;
    for (int d = tid; d < S.U; d += kBlock) {
        const DetDesc D = S.desc[d];
        double r = 0.0;
        if (D.s <= dmax) {
            double mat[16];
            load_excitation(D, T, M, mat);
            r = (double)D.eps * small_det(mat, D.s);
            if (r != 0.0) kmax = max(kmax, expo(r) + delta_exponent(D, Ex, occ0));
        }
        R64[d] = r;
    }
    int K = block_max_int(kmax, red);
    if (K == INT_MIN) K = 0;
    if (tid == 0) a.wk.K[ws] = K;
    float *R32 = a.wk.R32 + (size_t)w * rv_stride(a) + rv_offset(a, sp);
    for (int d = tid; d < S.U; d += kBlock) {
        const DetDesc D = S.desc[d];
        const double r = ldexp(R64[d], delta_exponent(D, Ex, occ0) - K);
        if (a.precision == MDET_MIXED) R32[d] = (float)r;
        else R64[d] = r;
    }
}

// ---------------------------------------------------------------------------
// Direct-LU fallback: one wave per determinant, LU of the scaled S_d.
// ---------------------------------------------------------------------------
namespace {

// Builds S_d (slot order) into Sm[n][n] for determinant D, lanes over rows.
// Returns the wave-uniform (mantissa, exponent) of det S_d' (slot order,
// scaled columns) times eps; mant == 0 for an exactly singular matrix.  Also
// leaves the LU factors and pivots in Sm / piv for a later inverse.
__device__ void wave_lu_det(const DetDesc &D, const int *occ0, const double *phig, int e0,
                            int M, int n, int lane, double *Sm, int *piv, int *occ,
                            double &mant, int &ex) {
    if (lane < n) {
        int o = occ0[lane];
        for (int a = 0; a < D.s; ++a)
            if (D.h[a] == lane) o = D.p[a];
        occ[lane] = o;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < n)
        for (int c = 0; c < n; ++c) Sm[lane * n + c] = phig[(size_t)(e0 + lane) * 5 * M + occ[c]];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double m = (double)D.eps;
    int k = 0;
    bool sing = false;
    for (int j = 0; j < n; ++j) {
        double v = (lane >= j && lane < n) ? fabs(Sm[lane * n + j]) : -1.0;
        int id = lane;
        for (int off = 32; off > 0; off >>= 1) {
            const double v2 = __shfl_xor(v, off, 64);
            const int i2 = __shfl_xor(id, off, 64);
            if (v2 > v || (v2 == v && i2 < id)) {
                v = v2;
                id = i2;
            }
        }
        if (!(v > 0.0)) {
            sing = true;
            break;
        }
        if (lane == 0) piv[j] = id;
        if (id != j && lane < n) {
            const double t = Sm[j * n + lane];
            Sm[j * n + lane] = Sm[id * n + lane];
            Sm[id * n + lane] = t;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double dj = Sm[j * n + j];
        if (id != j) m = -m;
        m *= dj;
        int kk;
        m = frexp(m, &kk);
        k += kk;
        if (lane > j && lane < n) {
            const double l = Sm[lane * n + j] / dj;
            Sm[lane * n + j] = l;
            for (int c = j + 1; c < n; ++c) Sm[lane * n + c] -= l * Sm[j * n + c];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (sing) {
        mant = 0.0;
        ex = 0;
    } else {
        mant = m;
        ex = k;
    }
}

}  // namespace

__global__ void __launch_bounds__(kBlock) k_direct_ratios(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] == 0) return;
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    constexpr int kWaves = kBlock / 64;
    __shared__ double Sm[kWaves][kMaxN * kMaxN];
    __shared__ int piv[kWaves][kMaxN];
    __shared__ int occ[kWaves][kMaxN];
    __shared__ int occ0[kMaxN];
    __shared__ int red[kBlock];
    extern __shared__ double lds[];
    int *Ex = (int *)lds;
    for (int m = tid; m < M; m += kBlock) Ex[m] = a.wk.E[ws * M + m];
    for (int c = tid; c < n; c += kBlock) occ0[c] = S.occ0[c];
    __syncthreads();
    const double *phig = a.wk.phi + (size_t)w * a.N * 5 * M;
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    int kmax = INT_MIN;
    // pass 1: largest exponent
    for (int d = wave; d < S.U; d += kWaves) {
        const DetDesc D = S.desc[d];
        if (D.s > dmax) continue;
        double mant;
        int ex;
        wave_lu_det(D, occ0, phig, S.e0, M, n, lane, Sm[wave], piv[wave], occ[wave], mant, ex);
        if (mant != 0.0) {
            int sx = 0;
            for (int c = 0; c < n; ++c) sx += Ex[occ[wave][c]];
            kmax = max(kmax, ex + sx);
        }
    }
    int K = block_max_int(kmax, red);
    if (K == INT_MIN) K = 0;
    if (tid == 0) {
        a.wk.K[ws] = K;
        a.wk.logdet0[ws] = 0.0;
        a.wk.sign0[ws] = 1.0;
    }
    double *R64 = a.wk.R64 + (size_t)w * rv_stride(a) + rv_offset(a, sp);
    float *R32 = a.wk.R32 + (size_t)w * rv_stride(a) + rv_offset(a, sp);
    for (int d = wave; d < S.U; d += kWaves) {
        const DetDesc D = S.desc[d];
        double r = 0.0;
        if (D.s <= dmax) {
            double mant;
            int ex;
            wave_lu_det(D, occ0, phig, S.e0, M, n, lane, Sm[wave], piv[wave], occ[wave], mant, ex);
            int sx = 0;
            for (int c = 0; c < n; ++c) sx += Ex[occ[wave][c]];
            r = ldexp(mant, ex + sx - K);
        }
        if (lane == 0) {
            if (a.precision == MDET_MIXED) R32[d] = (float)r;
            else R64[d] = r;
        }
    }
    for (int idx = tid; idx < 4 * n; idx += kBlock)
        a.wk.g0[((size_t)w * a.N + S.e0 + (idx >> 2)) * 4 + (idx & 3)] = 0.0;
}

// ---------------------------------------------------------------------------
// K5: u = C R_dn, v = C^T R_up, psi = R_up . u   (one block per walker)
// ---------------------------------------------------------------------------
template <typename F>
__global__ void __launch_bounds__(kBlock) k_spmm(KernelArgs a, const F *R, F *uv, F *psi,
                                                  const F *rval, const F *cval) {
    const int w = blockIdx.x, tid = threadIdx.x;
    __shared__ F red[kBlock];
    const SparseDev C = a.C;
    const size_t st = rv_stride(a);
    const F *Rup = R + (size_t)w * st;
    const F *Rdn = Rup + a.wk.Upad;
    F *u = uv + (size_t)w * st;
    F *v = u + a.wk.Upad;
    F part = 0;
    for (int i = tid; i < C.U; i += kBlock) {
        F acc = 0;
        for (int k = C.rptr[i]; k < C.rptr[i + 1]; ++k) acc += rval[k] * Rdn[C.rcol[k]];
        u[i] = acc;
        part += Rup[i] * acc;
    }
    for (int j = tid; j < C.V; j += kBlock) {
        F acc = 0;
        for (int k = C.cptr[j]; k < C.cptr[j + 1]; ++k) acc += cval[k] * Rup[C.crow[k]];
        v[j] = acc;
    }
    const F s = block_sum<F>(part, red);
    if (tid == 0) psi[w] = s;
}

// ---------------------------------------------------------------------------
// K6: derivative aggregation (table method)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_deriv(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] != 0) return;
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, N = a.N, tid = threadIdx.x;
    extern __shared__ double lds[];
    double *T = lds;               // [n][M]
    double *X = T + n * M;         // [n][n]
    double *Gam = X + n * n;       // [M][n]
    double *Y = Gam + M * n;       // [M][n]
    double *Zc = Y + M * n;        // [n][n]
    int *Ex = (int *)(Zc + n * n); // [M]
    int *occ0 = Ex + M;            // [n]
    const double *Tg = a.wk.T + ws * a.nmax * M;
    for (int idx = tid; idx < n * M; idx += kBlock) T[idx] = Tg[idx];
    const double *Xg = a.wk.X + ws * a.nmax * a.nmax;
    for (int idx = tid; idx < n * n; idx += kBlock) X[idx] = Xg[idx];
    for (int m = tid; m < M; m += kBlock) Ex[m] = a.wk.E[ws * M + m];
    for (int c = tid; c < n; c += kBlock) occ0[c] = S.occ0[c];
    __syncthreads();
    const int K = a.wk.K[ws];
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const size_t off = (size_t)w * rv_stride(a) + rv_offset(a, sp);
    const bool mixed = a.precision == MDET_MIXED;
    for (int t = tid; t < n * M; t += kBlock) {
        const int c = t / M, m = t - c * M;
        double g = 0.0;
        for (int q = S.gptr[t]; q < S.gptr[t + 1]; ++q) {
            const uint32_t ent = S.gent[q];
            const int d = (int)(ent >> 8), ia = (ent >> 4) & 15, ib = ent & 15;
            const DetDesc D = S.desc[d];
            if (D.s > dmax) continue;
            double mat[16];
            load_excitation(D, T, M, mat);
            const double wt = mixed ? (double)a.wk.uv32[off + d] : a.wk.uv64[off + d];
            const double f = (double)D.eps * pow2(delta_exponent(D, Ex, occ0) - K);
            g += wt * f * cofactor(mat, D.s, ia, ib);
        }
        Gam[m * n + c] = g;
    }
    __syncthreads();
    for (int idx = tid; idx < M * n; idx += kBlock) {
        const int m = idx / n, e = idx - m * n;
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += Gam[m * n + c] * X[c * n + e];
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
    const double psi = mixed ? (double)a.wk.psi32[w] : a.wk.psi64[w];
    const double *phig = a.wk.phi + (size_t)w * N * 5 * M;
    for (int idx = tid; idx < 4 * n; idx += kBlock) {
        const int e = idx >> 2, q = idx & 3;
        const double *G = phig + (size_t)(S.e0 + e) * 5 * M + (size_t)(1 + q) * M;
        double s1 = 0.0, s2 = 0.0;
        for (int m = 0; m < M; ++m) s1 += G[m] * Y[m * n + e];
        for (int c = 0; c < n; ++c) s2 += G[occ0[c]] * Zc[c * n + e];
        const size_t o = ((size_t)w * N + S.e0 + e) * 4 + q;
        a.gl_out[o] = a.wk.g0[o] + (s1 - s2) / psi;
    }
}

// ---------------------------------------------------------------------------
// Direct-LU fallback for the derivatives: sum_d w_d R_d grad~D_d/D_d / psi.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_direct_deriv(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    if (a.wk.flag[ws] == 0) return;
    const SpinDev S = a.sp[sp];
    const int n = S.n, M = a.M, N = a.N, tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    constexpr int kWaves = kBlock / 64;
    __shared__ double Sm[kWaves][kMaxN * kMaxN];
    __shared__ double Xw[kWaves][kMaxN * kMaxN];
    __shared__ int piv[kWaves][kMaxN];
    __shared__ int occ[kWaves][kMaxN];
    __shared__ int occ0[kMaxN];
    __shared__ double part[kWaves][kMaxN * 4];
    extern __shared__ double lds[];
    int *Ex = (int *)lds;
    for (int m = tid; m < M; m += kBlock) Ex[m] = a.wk.E[ws * M + m];
    for (int c = tid; c < n; c += kBlock) occ0[c] = S.occ0[c];
    __syncthreads();
    const double *phig = a.wk.phi + (size_t)w * N * 5 * M;
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const int K = a.wk.K[ws];
    const size_t off = (size_t)w * rv_stride(a) + rv_offset(a, sp);
    const bool mixed = a.precision == MDET_MIXED;
    double acc[4] = {0, 0, 0, 0};
    for (int d = wave; d < S.U; d += kWaves) {
        const DetDesc D = S.desc[d];
        if (D.s > dmax) continue;
        double mant;
        int ex;
        wave_lu_det(D, occ0, phig, S.e0, M, n, lane, Sm[wave], piv[wave], occ[wave], mant, ex);
        if (mant == 0.0) continue;
        int sx = 0;
        for (int c = 0; c < n; ++c) sx += Ex[occ[wave][c]];
        const double r = ldexp(mant, ex + sx - K);
        const double wt = mixed ? (double)a.wk.uv32[off + d] : a.wk.uv64[off + d];
        double *LUm = Sm[wave];
        double *Xm = Xw[wave];
        if (lane < n) {  // column `lane` of S_d^-1
            const int k = lane;
            for (int i = 0; i < n; ++i) Xm[i * n + k] = (i == k) ? 1.0 : 0.0;
            for (int j = 0; j < n; ++j) {
                const int p = piv[wave][j];
                if (p != j) {
                    const double t = Xm[j * n + k];
                    Xm[j * n + k] = Xm[p * n + k];
                    Xm[p * n + k] = t;
                }
            }
            for (int i = 0; i < n; ++i) {
                double s = Xm[i * n + k];
                for (int j = 0; j < i; ++j) s -= LUm[i * n + j] * Xm[j * n + k];
                Xm[i * n + k] = s;
            }
            for (int i = n - 1; i >= 0; --i) {
                double s = Xm[i * n + k];
                for (int j = i + 1; j < n; ++j) s -= LUm[i * n + j] * Xm[j * n + k];
                Xm[i * n + k] = s / LUm[i * n + i];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < n) {
            const int e = lane;
            for (int q = 0; q < 4; ++q) {
                const double *G = phig + (size_t)(S.e0 + e) * 5 * M + (size_t)(1 + q) * M;
                double s = 0.0;
                for (int c = 0; c < n; ++c) s += Xm[c * n + e] * G[occ[wave][c]];
                acc[q] += wt * r * s;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lane < n)
        for (int q = 0; q < 4; ++q) part[wave][lane * 4 + q] = acc[q];
    __syncthreads();
    const double psi = mixed ? (double)a.wk.psi32[w] : a.wk.psi64[w];
    for (int idx = tid; idx < 4 * n; idx += kBlock) {
        double s = 0.0;
        for (int v = 0; v < kWaves; ++v) s += part[v][idx];
        a.gl_out[((size_t)w * N + S.e0) * 4 + idx] = s / psi;
    }
}

// ---------------------------------------------------------------------------
// Outputs: sign, ln|Psi|, status; nodes get zero derivatives.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_finalize(KernelArgs a) {
    const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (w >= a.W) return;
    const bool mixed = a.precision == MDET_MIXED;
    const double psi = mixed ? (double)a.wk.psi32[w] : a.wk.psi64[w];
    const int f0 = a.wk.flag[2 * w], f1 = a.wk.flag[2 * w + 1];
    const bool node = !(psi != 0.0) || !isfinite(psi);
    if (node) {
        a.sign_out[w] = 0.0;
        a.logabs_out[w] = -INFINITY;
        for (int t = 0; t < 4 * a.N; ++t) a.gl_out[w * 4 * a.N + t] = 0.0;
        if (a.wstatus) a.wstatus[w] = MDET_W_NODE;
        return;
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

hipError_t launch_eval(const KernelArgs &a, hipStream_t st, hipEvent_t *ev) {
    const int W = (int)a.W;
    if (W == 0) return hipSuccess;
    const int n = a.nmax, M = a.M;
    const dim3 g2(2 * W), blk(kBlock);
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    size_t lds_ref = sizeof(double) * ((size_t)n * M + 4 * n * n) + sizeof(int) * M;
    k_reference<<<g2, blk, lds_ref, st>>>(a);
    mark(1);
    size_t lds_rat = sizeof(double) * (size_t)n * M + sizeof(int) * (M + n);
    k_ratios<<<g2, blk, lds_rat, st>>>(a);
    mark(2);
    k_direct_ratios<<<g2, blk, sizeof(int) * M, st>>>(a);
    mark(3);
    if (a.precision == MDET_MIXED)
        k_spmm<float><<<dim3(W), blk, 0, st>>>(a, a.wk.R32, a.wk.uv32, a.wk.psi32, a.C.rval32,
                                               a.C.cval32);
    else
        k_spmm<double><<<dim3(W), blk, 0, st>>>(a, a.wk.R64, a.wk.uv64, a.wk.psi64, a.C.rval,
                                                a.C.cval);
    mark(4);
    size_t lds_der = sizeof(double) * ((size_t)n * M + 2 * n * n + 2 * (size_t)M * n) +
                     sizeof(int) * (M + n);
    k_deriv<<<g2, blk, lds_der, st>>>(a);
    mark(5);
    k_direct_deriv<<<g2, blk, sizeof(int) * M, st>>>(a);
    mark(6);
    k_finalize<<<dim3((W + kBlock - 1) / kBlock), blk, 0, st>>>(a);
    mark(7);
    return hipGetLastError();
}

}  // namespace mdet
