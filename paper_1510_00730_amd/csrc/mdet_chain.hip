// HIP kernels of the Sherman-Morrison chain method (Sec. 2.2-2.3), the
// paper's own way of evaluating the distinct spin determinants, offered beside
// the table method: chain pieces, the exponent shift of their determinants
// and the derivative sums over the stored per-determinant ratios.

#include "mdet_device.h"

#include <climits>

namespace mdet {

namespace {

// ---------------------------------------------------------------------------
// The paper's own method (Sec. 2.2-2.3): a Sherman-Morrison chain over the
// distinct determinants in the sorted order of Eq. (comp).  One block per
// (walker, spin) stages that spin's scaled orbitals in LDS; each of its waves
// takes pieces of sm_chunk consecutive determinants: it factorises the first
// one, then reaches every next determinant by column substitutions on the
// inverse held in LDS.  Per determinant it writes the determinant as mantissa
// and exponent (like the direct-LU fallback) and the ratios
// grad~_e D / D = sum_c X[c][e] grad~phi_{col_c}(r_e).
// The inverse lives in a zero-padded 16 x 16 LDS tile, so every loop runs to
// 16 without per-step guards and vectors reach the lanes through LDS
// broadcasts (few scalar instructions).  Lane c < 16 owns row c of the
// products, lane 16 g + e updates column e of rows g, g + 4, g + 8, g + 12,
// lane 4 e + q forms the derivative ratio (e, q).
// ---------------------------------------------------------------------------
constexpr int kSmWaves = 8;
constexpr int kSmLd = kMaxN + 1;  // LDS row pitch of the inverse tile

// FP64 lane broadcast from a wave-uniform lane index
__device__ __forceinline__ double readlane_d(double v, int l) {
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Orbital planes staged per block: all five (values and derivatives) when
// they fit in 96 KB, else the values only (derivatives then read from HBM).
__host__ __device__ __forceinline__ int sm_planes(int nmax, int M) {
    return 5 * (size_t)nmax * M * sizeof(double) <= 96 * 1024 ? 5 : 1;
}
// LDS doubles of one chain wave: inverse tile, update factors, Gauss-Jordan
// scratch (the column orbitals stay in a register per lane)
constexpr int kSmWaveDoubles = kMaxN * kSmLd + kMaxN + 2 * kMaxN + 2;
__host__ __device__ __forceinline__ size_t sm_block_doubles(int nmax, int M) {
    return (size_t)sm_planes(nmax, M) * nmax * M + (M + 1) / 2 + (size_t)kSmWaves * kSmWaveDoubles;
}

// In-place Gauss-Jordan inversion with partial pivoting of the n x n matrix
// held in the zero-padded 16 x 16 LDS tile T (row e, column c at e * kSmLd + c)
// by the whole wave, four tile entries per lane, rows never exchanged: column
// j's pivot is the unused row with the largest |entry| (lowest row on ties).
// On return T holds the inverse, T[c][e] = (A^-1)[c][e], and det A = mant 2^ex
// (sign in mant).  pr_of / j_of: the wave's 16-int LDS scratch each (pivot row
// of column j, column pivoted by row e).  Returns false on a zero, infinite or
// NaN pivot.  The padding stays zero throughout.
__device__ bool tile_gauss_jordan(int n, int lane, double *T, int *pr_of, int *j_of,
                                  double &mant_out, int &ex_out) {
    uint32_t used = 0;
    double mant = 1.0;
    int ex = 0;
    for (int j = 0; j < n; ++j) {
        double v = -1.0;
        if (lane < n && !((used >> lane) & 1u)) {
            v = fabs(T[lane * kSmLd + j]);
            if (v != v) v = INFINITY;  // NaN: pick it, then fail below
        }
        int id = lane;
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {  // arg max over lanes 0..15
            const double ov = __shfl_xor(v, off, 64);
            const int oid = __shfl_xor(id, off, 64);
            if (ov > v || (ov == v && oid < id)) {
                v = ov;
                id = oid;
            }
        }
        const double best = readlane_d(v, 0);
        const int pr = __builtin_amdgcn_readlane(id, 0);
        if (!(best > 0.0) || !(best < INFINITY)) return false;
        used |= 1u << pr;
        if (lane == 0) {
            pr_of[j] = pr;
            j_of[pr] = j;
        }
        const double piv = T[pr * kSmLd + j];
        mant *= piv;
        int kk;
        mant = frexp(mant, &kk);
        ex += kk;
        const double rp = 1.0 / piv;
        double nv[4];
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
            const int t = lane + 64 * t4, i = t >> 4, c = t & 15;
            const double a_ic = T[i * kSmLd + c], a_pc = T[pr * kSmLd + c], a_ij = T[i * kSmLd + j];
            if (i == pr) nv[t4] = (c == j) ? rp : a_pc * rp;
            else nv[t4] = (c == j) ? -a_ij * rp : a_ic - a_ij * (a_pc * rp);
        }
        wave_lds_sync();
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
            const int t = lane + 64 * t4;
            T[(t >> 4) * kSmLd + (t & 15)] = nv[t4];
        }
        wave_lds_sync();
    }
    // the sweep leaves A^-1[c][e] at row pr_of[c], column j_of[e]: permute
    double tv[4];
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4) {
        const int t = lane + 64 * t4;
        tv[t4] = T[(t >> 4) * kSmLd + (t & 15)];
    }
    wave_lds_sync();
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4) {
        const int t = lane + 64 * t4, i = t >> 4, c = t & 15;
        if (i < n && c < n) T[j_of[i] * kSmLd + pr_of[c]] = tv[t4];
    }
    // det A = det(permutation j -> pr_of[j]) prod pivots
    int inv = 0;
    if (lane < n) {
        const int pa = pr_of[lane];
        for (int b = lane + 1; b < n; ++b) inv += pa > pr_of[b] ? 1 : 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) inv += __shfl_xor(inv, off, 64);
    wave_lds_sync();
    mant_out = (inv & 1) ? -mant : mant;
    ex_out = ex;
    return true;
}

template <typename F>
__global__ void __launch_bounds__(64 * kSmWaves) k_sm_chain(KernelArgs a, F *smg) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1, tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const SpinDev &S = a.sp[sp];
    const int n = S.n, M = a.M, nmax = a.nmax;
    const int planes = sm_planes(nmax, M);
    const size_t ws = (size_t)w * 2 + sp;
    extern __shared__ double lds[];
    double *Pst = lds;                                   // [planes][n][M] scaled orbitals
    int *Ex = (int *)(Pst + (size_t)planes * nmax * M);  // [M] column exponents
    double *Xs = (double *)Ex + (M + 1) / 2 + (size_t)wv * kSmWaveDoubles;  // X[c][e] at c*kSmLd+e
    double *fv = Xs + kMaxN * kSmLd;                     // [16] update factors
    double *sc = fv + kMaxN;                             // Gauss-Jordan scratch
    const double *Pg = a.wk.phi + ((size_t)w * a.N + S.e0) * 5 * M;  // [e][5][M] unscaled
    for (int m = tid; m < M; m += 64 * kSmWaves) Ex[m] = a.wk.E[ws * M + m];
    __syncthreads();
    for (int i = tid; i < planes * n * M; i += 64 * kSmWaves) {
        const int q = i / (n * M), r = i - q * (n * M), e = r / M, m = r - e * M;
        Pst[i] = ldexp(Pg[((size_t)e * 5 + q) * M + m], -Ex[m]);
    }
    __syncthreads();
    const double thr = a.sm_threshold;
    const int dmax = a.max_degree ? (int)a.max_degree[w] : 1 << 20;
    const int L = a.sm_chunk, npieces = (S.U + L - 1) / L;
    const int C4 = 4 * nmax;
    F *gout = smg + ws * (size_t)a.wk.Umax * C4;
    const int ge = lane & 15, gg = lane >> 4;      // update role: column ge, rows gg + 4 j
    const int de = min(lane >> 2, max(n - 1, 0));  // derivative role: electron (clamped)
    const int dq = 1 + (lane & 3);
    int kmax = INT_MIN;
    unsigned long long nsub = 0, ninv = 0, nfail = 0, nstart = 0;

    for (int piece = wv; piece < npieces; piece += kSmWaves) {
        const int p0 = piece * L, p1 = min(p0 + L, S.U);
        int colv = 0;          // lane c < n: orbital in column slot c
        double mant = 0.0;     // det of the scaled matrix = mant 2^ex (sign in mant)
        int ex = 0, esum = 0;  // esum: sum of the column exponents of the current columns
        bool have = false;

        // factorise the determinant at chain position pos from scratch
        auto restart = [&](int pos) {
            const int occ_l = lane < n ? (int)S.sm_occ[(size_t)pos * n + lane] : 0;
            // the scaled Slater matrix into the tile, zero beyond n
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                const int t = lane + 64 * t4, e = t >> 4, c = t & 15;
                const int m = __shfl(occ_l, c, 64);
                const int ec = max(min(e, n - 1), 0);  // in range whatever the tile row
                Xs[e * kSmLd + c] = (e < n && c < n) ? Pst[ec * M + m] : 0.0;
            }
            int es = lane < n ? Ex[occ_l] : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) es += __shfl_xor(es, off, 64);
            colv = occ_l;
            esum = es;
            wave_lds_sync();
            have = tile_gauss_jordan(n, lane, Xs, (int *)sc, (int *)sc + kMaxN, mant, ex);
            wave_lds_sync();
        };

        // one column substitution h -> p; false if |ratio| < thr
        auto substitute = [&](int h, int p) -> bool {
            const uint64_t hb = __ballot(lane < n && colv == h);
            if (hb == 0) return false;  // not reached for a consistent list
            const int k = __builtin_amdgcn_readfirstlane(__builtin_ctzll(hb));
            // phi_p at the electrons, read as broadcasts from the staged orbitals
            // (electron index clamped: the tile's columns beyond n are zero)
            double w0 = 0.0, w1 = 0.0;  // lane c < 16: (X phi_p)[c]
            if (lane < kMaxN) {
#pragma unroll
                for (int e = 0; e < kMaxN; e += 2) {
                    w0 += Xs[lane * kSmLd + e] * Pst[min(e, n - 1) * M + p];
                    w1 += Xs[lane * kSmLd + e + 1] * Pst[min(e + 1, n - 1) * M + p];
                }
            }
            const double wc = w0 + w1;
            const double r = readlane_d(wc, k);
            if (!(fabs(r) >= thr)) return false;
            // X <- X - (X u)(row k of X) / r with X u = X phi_p - e_k
            if (lane < kMaxN) fv[lane] = (wc - (lane == k ? 1.0 : 0.0)) / r;
            const double xk = Xs[k * kSmLd + ge];
            wave_lds_sync();
#pragma unroll
            for (int j = 0; j < kMaxN / 4; ++j) {
                const int c = gg + 4 * j;
                Xs[c * kSmLd + ge] -= fv[c] * xk;
            }
            // the sorting permutation changes parity once per other column between h and p
            const int lo = min(h, p), hi = max(h, p);
            const uint64_t between = __ballot(lane < n && lane != k && colv > lo && colv < hi);
            mant *= (__popcll(between) & 1) ? -r : r;
            int kk;
            mant = frexp(mant, &kk);
            ex += kk;
            esum += Ex[p] - Ex[h];
            if (lane == k) colv = p;
            wave_lds_sync();
            return true;
        };

        for (int win = p0; win < p1; win += 64) {
            // per-determinant lists of the next (up to) 64 positions, one per lane
            const int pl = win + lane;
            const bool in = pl < p1;
            const int exec_l = in ? S.sm_exec[pl] : 0;
            const int off_l = in ? S.sm_off[pl] : 0;
            const int offn_l = in ? S.sm_off[pl + 1] : 0;
            const int deg_l = in ? (int)S.desc[exec_l].s : 0;
            const int wend = min(win + 64, p1);
            for (int pos = win; pos < wend; ++pos) {
                const int j = pos - win;
                bool fresh = pos == p0 || !have;  // factorise this determinant from scratch
                if (!fresh) {
                    const int s0 = __builtin_amdgcn_readlane(off_l, j);
                    const int ns = __builtin_amdgcn_readlane(offn_l, j) - s0;
                    const uint32_t pr_l = lane < ns ? S.sm_sub[s0 + lane] : 0u;
                    uint32_t todo = ns >= 32 ? 0xffffffffu : ((1u << ns) - 1u);
                    while (todo) {
                        uint32_t left = todo;
                        int done = 0;
                        for (uint32_t bits = todo; bits; bits &= bits - 1) {
                            const int i = __builtin_ctz(bits);
                            const uint32_t pr = __builtin_amdgcn_readlane(pr_l, i);
                            if (substitute((int)(pr & 0xffffu), (int)(pr >> 16))) {
                                left &= ~(1u << i);
                                ++done;
                                ++nsub;
                            } else {
                                ++nfail;
                            }
                        }
                        todo = left;
                        if (todo && done == 0) {  // no progress: factorise from scratch
                            fresh = true;
                            break;
                        }
                    }
                }
                if (fresh) {
                    restart(pos);
                    if (pos == p0) ++nstart;
                    else ++ninv;
                }
                const int d = __builtin_amdgcn_readlane(exec_l, j);
                const bool keep = have && __builtin_amdgcn_readlane(deg_l, j) <= dmax;
                if (lane < 4 * n) {
                    double t0 = 0.0, t1 = 0.0;
                    if (planes == 5) {
                        const double *G = Pst + ((size_t)dq * n + de) * M;
#pragma unroll
                        for (int c = 0; c < kMaxN; c += 2) {
                            t0 += Xs[c * kSmLd + de] * G[__builtin_amdgcn_readlane(colv, c)];
                            t1 += Xs[(c + 1) * kSmLd + de] *
                                  G[__builtin_amdgcn_readlane(colv, c + 1)];
                        }
                    } else {
                        const double *G = Pg + ((size_t)de * 5 + dq) * M;
#pragma unroll
                        for (int c = 0; c < kMaxN; c += 2) {
                            const int m0 = __builtin_amdgcn_readlane(colv, c);
                            const int m1 = __builtin_amdgcn_readlane(colv, c + 1);
                            t0 += Xs[c * kSmLd + de] * ldexp(G[m0], -Ex[m0]);
                            t1 += Xs[(c + 1) * kSmLd + de] * ldexp(G[m1], -Ex[m1]);
                        }
                    }
                    gout[(size_t)d * C4 + lane] = keep ? (F)(t0 + t1) : (F)0;
                }
                if (lane == 0) {
                    const size_t o = rv_index(a, sp, d, w);
                    a.wk.R64[o] = keep ? mant : 0.0;
                    a.wk.Rexp[o] = keep ? ex + esum : INT_MIN;
                }
                if (keep && mant != 0.0) kmax = max(kmax, ex + esum);
            }
        }
    }
    if (lane == 0) {
        if (kmax != INT_MIN) atomicMax(&a.wk.Kmax[ws], kmax);
        atomicAdd(&a.wk.smstat[0], nsub);
        atomicAdd(&a.wk.smstat[1], ninv);
        atomicAdd(&a.wk.smstat[2], nfail);
        atomicAdd(&a.wk.smstat[3], nstart);
    }
}

// shift the chain's determinants by the (walker, spin) maximum exponent:
// one block per (walker, spin)
__global__ void __launch_bounds__(kBlock) k_sm_scale(KernelArgs a) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1;
    const size_t ws = (size_t)w * 2 + sp;
    int K = a.wk.Kmax[ws];
    if (K == INT_MIN) K = 0;
    if (threadIdx.x == 0) {
        a.wk.K[ws] = K;
        a.wk.logdet0[ws] = 0.0;
        a.wk.sign0[ws] = 1.0;
        a.wk.flag[ws] = 0;
    }
    for (int d = threadIdx.x; d < a.sp[sp].U; d += kBlock) {
        const size_t o = rv_index(a, sp, d, w);
        const int e = a.wk.Rexp[o];
        const double r = (e == INT_MIN) ? 0.0 : ldexp(a.wk.R64[o], e - K);
        a.wk.R64[o] = r;
        if (a.precision == MDET_MIXED) a.wk.R32[o] = (float)r;
    }
}

// grad~_e Psi / Psi = sum_d R_d w_d (grad~_e D_d / D_d) / psi with w = u (up)
// or v (down), the FP64 ratios R_d, and psi = R_up.u, the psi of ln|Psi|
// (the quotient times the returned Psi is the numerator itself): one block
// per (walker, spin); thread t
// reads component t mod 4n of determinants t / 4n + k (256 / 4n), so each
// pass reads a contiguous run of the stored ratios.
template <typename F>
__global__ void __launch_bounds__(kBlock) k_sm_deriv(KernelArgs a, const double *R, const F *uv,
                                                     const F *smg) {
    const int w = blockIdx.x >> 1, sp = blockIdx.x & 1, tid = threadIdx.x;
    const SpinDev &S = a.sp[sp];
    const int n = S.n, cn = 4 * n, C4 = 4 * a.nmax;
    if (cn == 0) return;
    const size_t ws = (size_t)w * 2 + sp;
    const int per = kBlock / cn;
    __shared__ double red[kBlock];
    double s = 0.0;
    if (tid < per * cn) {
        const int k = tid % cn;
        const F *g = smg + ws * (size_t)a.wk.Umax * C4;
        for (int d = tid / cn; d < S.U; d += per) {
            const size_t o = rv_index(a, sp, d, w);
            s += (R[o] * (double)uv[o]) * (double)g[(size_t)d * C4 + k];
        }
    }
    red[tid] = s;
    __syncthreads();
    if (tid < cn) {
        double t = 0.0;
        for (int j = 0; j < per; ++j) t += red[j * cn + tid];
        const double psi = psi_value(a, w, 0);  // the psi of ln|Psi|
        a.gl_out[((size_t)w * a.N + S.e0) * 4 + tid] = t / psi;
    }
}

}  // namespace

void launch_chain_pieces(const KernelArgs &a, hipStream_t st) {
    const dim3 g2(2 * (unsigned)a.W);
    const size_t lds = sizeof(double) * sm_block_doubles(a.nmax, a.M);
    if (a.precision == MDET_MIXED)
        k_sm_chain<float><<<g2, dim3(64 * kSmWaves), lds, st>>>(a, a.wk.smg32);
    else
        k_sm_chain<double><<<g2, dim3(64 * kSmWaves), lds, st>>>(a, a.wk.smg64);
    k_sm_scale<<<g2, dim3(kBlock), 0, st>>>(a);
}

void launch_chain_deriv(const KernelArgs &a, hipStream_t st) {
    const dim3 g2(2 * (unsigned)a.W);
    if (a.precision == MDET_MIXED)
        k_sm_deriv<float><<<g2, dim3(kBlock), 0, st>>>(a, a.wk.R64, a.wk.uv32, a.wk.smg32);
    else
        k_sm_deriv<double><<<g2, dim3(kBlock), 0, st>>>(a, a.wk.R64, a.wk.uv64, a.wk.smg64);
}

}  // namespace mdet
