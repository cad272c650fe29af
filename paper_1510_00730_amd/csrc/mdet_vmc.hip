// Variational Monte Carlo step and learned (MLP) Metropolis proposal for gfx950.
//
//  * Philox-4x32-10 counter-based random numbers (Salmon et al., SC'11) for
//    the move noise and the acceptance uniforms.
//  * VMC step: proposal (Gaussian, drift-diffusion, or the MLP), evaluation
//    of Psi at the proposed positions by the multideterminant path, exact
//    Metropolis-Hastings acceptance in logs, local energy of a point nucleus.
//  * MLP 3N -> H -> H -> 4N (tanh): per-electron move mean and log step.
//    Its dense layers are FP32 matrix products on the matrix cores
//    (v_mfma_f32_16x16x4_f32), forward and backward; Adam updates.
//  * The training objective is the expected squared jump distance with the
//    exact acceptance; its gradient is assembled per walker in FP64 and fed
//    back through both MLP evaluations (at R and at R').

#include "mdet_internal.h"

#include <math.h>

namespace mdet {

namespace {

constexpr int kVBlock = 256;

// ------------------------------------------------------------- Philox-4x32-10
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// two 32-bit words -> double in (0, 1) from 52 bits (m + 1/2 is exact)
__device__ __forceinline__ double unit52(uint32_t a, uint32_t b) {
    const uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
    return ((double)m + 0.5) * 0x1p-52;
}

}  // namespace

// pair i of (seed, stream, step): kind 0 = two uniforms, 1 = two normals
__global__ void __launch_bounds__(kVBlock) k_philox(uint64_t seed, uint64_t stream_id, uint64_t step,
                                                    int64_t n, int kind, double *out) {
    const int64_t i = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (2 * i >= n) return;
    const U4 x = philox10(U4{(uint32_t)i, (uint32_t)stream_id, (uint32_t)step, (uint32_t)(step >> 32)},
                          (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = unit52(x.x, x.y), u2 = unit52(x.z, x.w);
    double a = u1, b = u2;
    if (kind == 1) {
        const double r = sqrt(-2.0 * log(u1));
        const double t = 2.0 * M_PI * u2;
        a = r * cos(t);
        b = r * sin(t);
    }
    out[2 * i] = a;
    if (2 * i + 1 < n) out[2 * i + 1] = b;
}

// ------------------------------------------------------------------- VMC step
// proposal 0: R' = R + step xi; proposal 1: R' = R + step F + sqrt(step) xi
__global__ void __launch_bounds__(kVBlock) k_vmc_propose(int64_t W, int N, int proposal, double step,
                                                         const double *R, const double *gl,
                                                         const double *xi, double *Rp) {
    const int64_t t = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (t >= W * N * 3) return;
    const int64_t we = t / 3;
    const int ax = (int)(t - we * 3);
    double r = R[t];
    if (proposal == 0) r += step * xi[t];
    else r += step * gl[we * 4 + ax] + sqrt(step) * xi[t];
    Rp[t] = r;
}

namespace {

__device__ double local_energy_w(const double *Rw, const double *glw, int N, double Z) {
    double kin = 0.0, ven = 0.0, vee = 0.0;
    for (int e = 0; e < N; ++e) {
        kin += glw[4 * e + 3];
        const double x = Rw[3 * e], y = Rw[3 * e + 1], z = Rw[3 * e + 2];
        ven += 1.0 / sqrt(x * x + y * y + z * z);
        for (int f = e + 1; f < N; ++f) {
            const double dx = x - Rw[3 * f], dy = y - Rw[3 * f + 1], dz = z - Rw[3 * f + 2];
            vee += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
    return -0.5 * kin - Z * ven + vee;
}

// ln q(B | A) of the MLP proposal, per walker, from the head outputs at A
__device__ double mlp_log_q(const double *B, const double *A, const float *o, int N) {
    double s = 0.0;
    for (int e = 0; e < N; ++e) {
        double ls = (double)o[3 * N + e];
        ls = fmin(fmax(ls, kMlpLogSigMin), kMlpLogSigMax);
        const double inv = exp(-2.0 * ls);
        double d2 = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            const double d = B[3 * e + ax] - A[3 * e + ax] - (double)o[3 * e + ax];
            d2 += d * d;
        }
        s += -0.5 * d2 * inv - 3.0 * ls;
    }
    return s;
}

}  // namespace

// Metropolis-Hastings test, in-place update of the walker state, local energy.
// o1 / o2 (MLP proposal only): network outputs at R and at R'.
__global__ void __launch_bounds__(kVBlock) k_vmc_accept(int64_t W, int N, int proposal, double step,
                                                        double Z, double *R, double *sign,
                                                        double *logabs, double *gl,
                                                        const double *Rp, const double *signp,
                                                        const double *logabsp, const double *glp,
                                                        const double *uniform, const float *o1,
                                                        const float *o2, double *elocal,
                                                        int32_t *accepted, int fixed_node) {
    const int64_t w = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (w >= W) return;
    const int n3 = 3 * N, n4 = 4 * N;
    double *Rw = R + w * n3;
    const double *Rpw = Rp + w * n3;
    bool ok;
    if (signp[w] == 0.0) {
        ok = false;  // never move onto a node
    } else if (fixed_node && signp[w] != sign[w]) {
        ok = false;  // never cross a node (diffusion Monte Carlo)
    } else if (sign[w] == 0.0) {
        ok = true;   // leave a node whatever the ratio
    } else {
        double ell = 2.0 * (logabsp[w] - logabs[w]);
        if (proposal == 1) {
            double f2 = 0.0, r2 = 0.0;
            for (int e = 0; e < N; ++e)
                for (int ax = 0; ax < 3; ++ax) {
                    const double fw = Rpw[3 * e + ax] - Rw[3 * e + ax] - step * gl[w * n4 + 4 * e + ax];
                    const double rv = Rw[3 * e + ax] - Rpw[3 * e + ax] - step * glp[w * n4 + 4 * e + ax];
                    f2 += fw * fw;
                    r2 += rv * rv;
                }
            ell += (f2 - r2) / (2.0 * step);
        } else if (proposal == 2) {
            ell += mlp_log_q(Rw, Rpw, o2 + w * n4, N) - mlp_log_q(Rpw, Rw, o1 + w * n4, N);
        }
        ok = log(uniform[w]) < ell;
    }
    if (ok) {
        for (int t = 0; t < n3; ++t) Rw[t] = Rpw[t];
        for (int t = 0; t < n4; ++t) gl[w * n4 + t] = glp[w * n4 + t];
        sign[w] = signp[w];
        logabs[w] = logabsp[w];
    }
    accepted[w] = ok ? 1 : 0;
    elocal[w] = (sign[w] == 0.0) ? NAN : local_energy_w(Rw, gl + w * n4, N, Z);
}

// ------------------------------------------------------------------- MLP GEMM
// C[m][n] (+)= sum_k A[m*a_rs + k*a_cs] * B[k*b_rs + n*b_cs] (+ bias[n]),
// optional tanh, FP32 on the matrix cores: one wave per 16 x 16 tile of C,
// v_mfma_f32_16x16x4_f32 (lane l holds A[l%16][l/16] and B[l/16][l%16] of each
// 16x4 / 4x16 step; the 16x16 result sits as C[4(l/16)+i][l%16], i = 0..3).
__global__ void __launch_bounds__(256) k_gemm_f32(int M, int Nn, int K, const float *A, int a_rs,
                                                  int a_cs, const float *B, int b_rs, int b_cs,
                                                  float *C, int c_rs, const float *bias, int act,
                                                  int accumulate) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_n = (Nn + 15) / 16;
    const int tile = blockIdx.x * 4 + wv;
    const int m0 = (tile / tiles_n) * 16, n0 = (tile % tiles_n) * 16;
    if (m0 >= M) return;
    const int li = lane & 15, lk = lane >> 4;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const int am = m0 + li, bn = n0 + li;
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + lk;
        const float av = (am < M && k < K) ? A[(size_t)am * a_rs + (size_t)k * a_cs] : 0.f;
        const float bv = (bn < Nn && k < K) ? B[(size_t)k * b_rs + (size_t)bn * b_cs] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    const int cn = n0 + li;
    if (cn >= Nn) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int cm = m0 + 4 * lk + i;
        if (cm >= M) continue;
        float v = acc[i];
        float *dst = C + (size_t)cm * c_rs + cn;
        if (accumulate) v += *dst;
        if (bias) v += bias[cn];
        if (act == 1) v = tanhf(v);
        *dst = v;
    }
}

// dz = dh * (1 - h^2) in place
__global__ void __launch_bounds__(kVBlock) k_tanh_back(int64_t n, const float *h, float *d) {
    const int64_t t = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (t < n) d[t] *= 1.f - h[t] * h[t];
}

// db[j] (+)= sum_b dz[b][j], fixed order (one thread per column)
__global__ void __launch_bounds__(kVBlock) k_colsum(int B, int Nn, const float *dz, float *db,
                                                    int accumulate) {
    const int j = blockIdx.x * kVBlock + threadIdx.x;
    if (j >= Nn) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dz[(size_t)b * Nn + j];
    db[j] = accumulate ? db[j] + s : s;
}

// R' = R + mu(R) + sigma(R) xi (FP64 positions, FP32 network outputs)
__global__ void __launch_bounds__(kVBlock) k_mlp_propose(int64_t W, int N, const double *R,
                                                         const float *o, const double *xi,
                                                         double *Rp) {
    const int64_t t = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (t >= W * N * 3) return;
    const int64_t w = t / (3 * N);
    const int r = (int)(t - w * 3 * N), e = r / 3;
    const float *ow = o + w * 4 * N;
    double ls = fmin(fmax((double)ow[3 * N + e], kMlpLogSigMin), kMlpLogSigMax);
    Rp[t] = R[t] + (double)ow[r] + exp(ls) * xi[t];
}

// weight of electron e's squared jump: 1, or 1 / (|r_e|^2 + jref^2)
__device__ __forceinline__ double jump_weight(const double *r, double jref) {
    return jref > 0.0 ? 1.0 / (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + jref * jref) : 1.0;
}

// Coulomb potential energy of one configuration, point nucleus of charge Z at
// the origin: V = -Z sum_e 1/|r_e| + sum_{e<f} 1/|r_e - r_f|; with dV (not
// null) also its gradient dV[3e + ax].
__device__ double coulomb_v(int N, double Z, const double *r, double *dV) {
    double v = 0.0;
    for (int e = 0; e < N; ++e) {
        const double *re = r + 3 * e;
        const double d2 = re[0] * re[0] + re[1] * re[1] + re[2] * re[2];
        const double id = 1.0 / sqrt(d2);
        v -= Z * id;
        if (dV) {
            const double c = Z * id * id * id;
            for (int ax = 0; ax < 3; ++ax) dV[3 * e + ax] = c * re[ax];
        }
    }
    for (int e = 0; e < N; ++e)
        for (int f = e + 1; f < N; ++f) {
            double d[3], d2 = 0.0;
            for (int ax = 0; ax < 3; ++ax) {
                d[ax] = r[3 * e + ax] - r[3 * f + ax];
                d2 += d[ax] * d[ax];
            }
            const double id = 1.0 / sqrt(d2);
            v += id;
            if (dV) {
                const double c = id * id * id;
                for (int ax = 0; ax < 3; ++ax) {
                    dV[3 * e + ax] -= c * d[ax];
                    dV[3 * f + ax] += c * d[ax];
                }
            }
        }
    return v;
}

// Per-walker part of the training objective J = A jump (loss = -mean J),
// jump = sum_e c_e |r'_e - r_e|^2 (objective 0, c_e = jump_weight) or
// (V(R') - V(R))^2 (objective 1, the squared change of the potential energy):
// writes the output gradient of the evaluation at R' (dO2, FP32), the direct
// gradient w.r.t. R' (gRp, FP64), g_ell and the walker's J.
__global__ void __launch_bounds__(kVBlock) k_esjd_head(int64_t W, int N, const double *R,
                                                       const double *Rp, const double *xi,
                                                       const double *logabsR, const double *signp,
                                                       const double *logabsp, const double *glp,
                                                       const float *o1, const float *o2, float *dO2,
                                                       double *gRp, double *gell, double *Jw,
                                                       double jref, int objective, double Z) {
    const int64_t w = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (w >= W) return;
    const int n3 = 3 * N, n4 = 4 * N;
    const double *Rw = R + w * n3, *Rpw = Rp + w * n3, *xw = xi + w * n3;
    const float *a1 = o1 + w * n4, *a2 = o2 + w * n4;
    double lq_fwd = 0.0, lq_rev = 0.0, jump = 0.0;
    for (int e = 0; e < N; ++e) {
        const double ls = fmin(fmax((double)a1[n3 + e], kMlpLogSigMin), kMlpLogSigMax);
        const double ls2 = fmin(fmax((double)a2[n3 + e], kMlpLogSigMin), kMlpLogSigMax);
        const double inv2 = exp(-2.0 * ls2);
        double x2 = 0.0, d2 = 0.0, j2 = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            x2 += xw[3 * e + ax] * xw[3 * e + ax];
            const double d = Rw[3 * e + ax] - Rpw[3 * e + ax] - (double)a2[3 * e + ax];
            d2 += d * d;
            const double j = Rpw[3 * e + ax] - Rw[3 * e + ax];
            j2 += j * j;
        }
        jump += jump_weight(Rw + 3 * e, jref) * j2;
        lq_fwd += -0.5 * x2 - 3.0 * ls;
        lq_rev += -0.5 * d2 * inv2 - 3.0 * ls2;
    }
    // potential-energy objective: the gradient of V at R' goes to gRp first
    // (scaled below), so no per-walker array beyond gRp is needed
    double dv = 0.0;
    if (objective == 1) {
        dv = coulomb_v(N, Z, Rpw, gRp + w * n3) - coulomb_v(N, Z, Rw, nullptr);
        jump = dv * dv;
    }
    const bool node = signp[w] == 0.0;
    const double ell = node ? -INFINITY : 2.0 * (logabsp[w] - logabsR[w]) + lq_rev - lq_fwd;
    const double A = node ? 0.0 : (ell < 0.0 ? exp(ell) : 1.0);
    const double gJ = -1.0 / (double)W;
    const double ge = (ell < 0.0) ? gJ * A * jump : 0.0;
    Jw[w] = A * jump;
    gell[w] = ge;
    for (int e = 0; e < N; ++e) {
        const double raw2 = (double)a2[n3 + e];
        const double ls2 = fmin(fmax(raw2, kMlpLogSigMin), kMlpLogSigMax);
        const bool in2 = raw2 > kMlpLogSigMin && raw2 < kMlpLogSigMax;
        const double inv2 = exp(-2.0 * ls2);
        const double ce = jump_weight(Rw + 3 * e, jref);
        double d2 = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            const double d = Rw[3 * e + ax] - Rpw[3 * e + ax] - (double)a2[3 * e + ax];
            d2 += d * d;
            const double dj = objective == 1 ? 2.0 * dv * gRp[w * n3 + 3 * e + ax]
                                             : 2.0 * ce * (Rpw[3 * e + ax] - Rw[3 * e + ax]);
            const double g = gJ * A * dj +
                             ge * (2.0 * glp[w * n4 + 4 * e + ax] + d * inv2);
            gRp[w * n3 + 3 * e + ax] = g;
            dO2[w * n4 + 3 * e + ax] = (float)(ge * d * inv2);
        }
        dO2[w * n4 + n3 + e] = in2 ? (float)(ge * (d2 * inv2 - 3.0)) : 0.f;
    }
}

// Chain rule through R' = R + mu + sigma xi: output gradient of the
// evaluation at R (dO1) from gRp + the input gradient of the second pass.
__global__ void __launch_bounds__(kVBlock) k_esjd_chain(int64_t W, int N, const double *xi,
                                                        const float *o1, const double *gRp,
                                                        const float *dX2, const double *gell,
                                                        float *dO1) {
    const int64_t w = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (w >= W) return;
    const int n3 = 3 * N, n4 = 4 * N;
    const float *a1 = o1 + w * n4;
    for (int e = 0; e < N; ++e) {
        const double raw = (double)a1[n3 + e];
        const double ls = fmin(fmax(raw, kMlpLogSigMin), kMlpLogSigMax);
        const bool in1 = raw > kMlpLogSigMin && raw < kMlpLogSigMax;
        const double sg = exp(ls);
        double gls = 3.0 * gell[w];
        for (int ax = 0; ax < 3; ++ax) {
            const int64_t t = w * n3 + 3 * e + ax;
            const double g = gRp[t] + (double)dX2[t];
            dO1[w * n4 + 3 * e + ax] = (float)g;
            gls += g * sg * xi[t];
        }
        dO1[w * n4 + n3 + e] = in1 ? (float)gls : 0.f;
    }
}

// fixed-order block sum of J into out[0] = -mean J (one block)
__global__ void __launch_bounds__(1024) k_esjd_loss(int64_t W, const double *Jw, double *out) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int64_t w = threadIdx.x; w < W; w += 1024) s += Jw[w];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 512; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = -red[0] / (double)W;
}

// x_in (FP64) -> FP32 network input
__global__ void __launch_bounds__(kVBlock) k_to_f32(int64_t n, const double *x, float *y) {
    const int64_t t = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (t < n) y[t] = (float)x[t];
}

__global__ void __launch_bounds__(kVBlock) k_adam(int64_t n, float *p, const float *g, float *m,
                                                  float *v, float lr, float b1, float b2, float eps,
                                                  float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * kVBlock + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// ------------------------------------------------------------------ launchers
namespace {
inline dim3 g1(int64_t n) { return dim3((unsigned)((n + kVBlock - 1) / kVBlock)); }
}  // namespace

void launch_philox(uint64_t seed, uint64_t stream_id, uint64_t step, int64_t n, int kind,
                   double *out, hipStream_t st) {
    k_philox<<<g1((n + 1) / 2), dim3(kVBlock), 0, st>>>(seed, stream_id, step, n, kind, out);
}

void launch_vmc_propose(int64_t W, int N, int proposal, double step, const double *R,
                        const double *gl, const double *xi, double *Rp, hipStream_t st) {
    k_vmc_propose<<<g1(W * N * 3), dim3(kVBlock), 0, st>>>(W, N, proposal, step, R, gl, xi, Rp);
}

void launch_vmc_accept(int64_t W, int N, int proposal, double step, double Z, double *R,
                       double *sign, double *logabs, double *gl, const double *Rp,
                       const double *signp, const double *logabsp, const double *glp,
                       const double *uniform, const float *o1, const float *o2, double *elocal,
                       int32_t *accepted, int fixed_node, hipStream_t st) {
    k_vmc_accept<<<g1(W), dim3(kVBlock), 0, st>>>(W, N, proposal, step, Z, R, sign, logabs, gl,
                                                   Rp, signp, logabsp, glp, uniform, o1, o2,
                                                   elocal, accepted, fixed_node);
}

void launch_gemm_f32(int M, int Nn, int K, const float *A, int a_rs, int a_cs, const float *B,
                     int b_rs, int b_cs, float *C, int c_rs, const float *bias, int act,
                     int accumulate, hipStream_t st) {
    const int tiles = ((M + 15) / 16) * ((Nn + 15) / 16);
    k_gemm_f32<<<dim3((tiles + 3) / 4), dim3(256), 0, st>>>(M, Nn, K, A, a_rs, a_cs, B, b_rs, b_cs,
                                                           C, c_rs, bias, act, accumulate);
}

void launch_mlp_forward(const MlpShape &s, const float *params, int64_t Bn, const float *X,
                        float *h1, float *h2, float *O, hipStream_t st) {
    const int B = (int)Bn;
    const float *W1 = params, *b1 = W1 + s.n_in * s.n_hid;
    const float *W2 = b1 + s.n_hid, *b2 = W2 + s.n_hid * s.n_hid;
    const float *W3 = b2 + s.n_hid, *b3 = W3 + s.n_hid * s.n_out;
    launch_gemm_f32(B, s.n_hid, s.n_in, X, s.n_in, 1, W1, s.n_hid, 1, h1, s.n_hid, b1, 1, 0, st);
    launch_gemm_f32(B, s.n_hid, s.n_hid, h1, s.n_hid, 1, W2, s.n_hid, 1, h2, s.n_hid, b2, 1, 0, st);
    launch_gemm_f32(B, s.n_out, s.n_hid, h2, s.n_hid, 1, W3, s.n_out, 1, O, s.n_out, b3, 0, 0, st);
}

void launch_mlp_backward(const MlpShape &s, const float *params, int64_t Bn, const float *X,
                         const float *h1, const float *h2, const float *dO, float *dparams,
                         int accumulate, float *dX, float *work_h1, float *work_h2,
                         hipStream_t st) {
    const int B = (int)Bn;
    const float *W1 = params, *b1 = W1 + s.n_in * s.n_hid;
    const float *W2 = b1 + s.n_hid, *b2 = W2 + s.n_hid * s.n_hid;
    const float *W3 = b2 + s.n_hid;
    float *dW1 = dparams, *db1 = dW1 + s.n_in * s.n_hid;
    float *dW2 = db1 + s.n_hid, *db2 = dW2 + s.n_hid * s.n_hid;
    float *dW3 = db2 + s.n_hid, *db3 = dW3 + s.n_hid * s.n_out;
    (void)b1;
    (void)b2;
    // layer 3: dW3 = h2^T dO, db3 = sum dO, dh2 = dO W3^T
    launch_gemm_f32(s.n_hid, s.n_out, B, h2, 1, s.n_hid, dO, s.n_out, 1, dW3, s.n_out, nullptr, 0,
                    accumulate, st);
    k_colsum<<<g1(s.n_out), dim3(kVBlock), 0, st>>>(B, s.n_out, dO, db3, accumulate);
    launch_gemm_f32(B, s.n_hid, s.n_out, dO, s.n_out, 1, W3, 1, s.n_out, work_h2, s.n_hid, nullptr,
                    0, 0, st);
    k_tanh_back<<<g1((int64_t)B * s.n_hid), dim3(kVBlock), 0, st>>>((int64_t)B * s.n_hid, h2, work_h2);
    // layer 2
    launch_gemm_f32(s.n_hid, s.n_hid, B, h1, 1, s.n_hid, work_h2, s.n_hid, 1, dW2, s.n_hid, nullptr,
                    0, accumulate, st);
    k_colsum<<<g1(s.n_hid), dim3(kVBlock), 0, st>>>(B, s.n_hid, work_h2, db2, accumulate);
    launch_gemm_f32(B, s.n_hid, s.n_hid, work_h2, s.n_hid, 1, W2, 1, s.n_hid, work_h1, s.n_hid,
                    nullptr, 0, 0, st);
    k_tanh_back<<<g1((int64_t)B * s.n_hid), dim3(kVBlock), 0, st>>>((int64_t)B * s.n_hid, h1, work_h1);
    // layer 1
    launch_gemm_f32(s.n_in, s.n_hid, B, X, 1, s.n_in, work_h1, s.n_hid, 1, dW1, s.n_hid, nullptr, 0,
                    accumulate, st);
    k_colsum<<<g1(s.n_hid), dim3(kVBlock), 0, st>>>(B, s.n_hid, work_h1, db1, accumulate);
    if (dX)
        launch_gemm_f32(B, s.n_in, s.n_hid, work_h1, s.n_hid, 1, W1, 1, s.n_hid, dX, s.n_in, nullptr,
                        0, 0, st);
}

void launch_to_f32(int64_t n, const double *x, float *y, hipStream_t st) {
    k_to_f32<<<g1(n), dim3(kVBlock), 0, st>>>(n, x, y);
}

void launch_mlp_propose(int64_t W, int N, const double *R, const float *o, const double *xi,
                        double *Rp, hipStream_t st) {
    k_mlp_propose<<<g1(W * N * 3), dim3(kVBlock), 0, st>>>(W, N, R, o, xi, Rp);
}

void launch_esjd_head(int64_t W, int N, const double *R, const double *Rp, const double *xi,
                      const double *logabsR, const double *signp, const double *logabsp,
                      const double *glp, const float *o1, const float *o2, float *dO2,
                      double *gRp, double *gell, double *Jw, double jump_ref, int objective,
                      double Z, hipStream_t st) {
    k_esjd_head<<<g1(W), dim3(kVBlock), 0, st>>>(W, N, R, Rp, xi, logabsR, signp, logabsp, glp, o1,
                                                  o2, dO2, gRp, gell, Jw, jump_ref, objective, Z);
}

void launch_esjd_chain(int64_t W, int N, const double *xi, const float *o1, const double *gRp,
                       const float *dX2, const double *gell, float *dO1, hipStream_t st) {
    k_esjd_chain<<<g1(W), dim3(kVBlock), 0, st>>>(W, N, xi, o1, gRp, dX2, gell, dO1);
}

void launch_esjd_loss(int64_t W, const double *Jw, double *out, hipStream_t st) {
    k_esjd_loss<<<dim3(1), dim3(1024), 0, st>>>(W, Jw, out);
}

void launch_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1,
                 float b2, float eps, int t, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    k_adam<<<g1(n), dim3(kVBlock), 0, st>>>(n, p, g, m, v, lr, b1, b2, eps, c1, c2);
}

}  // namespace mdet
