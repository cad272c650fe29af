// Device helpers shared by the kernels of libmdet (table method, direct-LU
// fallback and the Sherman-Morrison chain).  Internal, not part of the ABI.
#pragma once

#include <math.h>

#include "mdet_internal.h"

namespace mdet {

namespace {

constexpr int kBlock = 256;                // threads of the one-block-per-(walker, spin) kernels
constexpr int kMaxN = MDET_MAX_SPIN_ELEC;  // largest electron count of one spin

// Offsets of the walker-major vectors R, u, v: entry d of spin sp for walker
// w sits at w * (Upad + Vpad) + (sp ? Upad : 0) + d.
__device__ __forceinline__ size_t rv_index(const KernelArgs &a, int sp, int d, int w) {
    return (size_t)w * (size_t)(a.wk.Upad + a.wk.Vpad) + (sp ? (size_t)a.wk.Upad : 0) + d;
}

// psi of walker w formed by spin sp: psi_up = sum_i R_up[i] u[i] (sp 0) or
// psi_dn = sum_j R_dn[j] v[j] (sp 1), with the FP64 ratios and the stored
// weights u, v -- equal in exact arithmetic; each matches the derivative
// aggregate of its spin (same ratios and weights), so that in mixed precision
// the rounding of the weights is not amplified by a large reference term.
// The row-split partial sums of the sparse combination are added in a fixed
// order; all kPsiParts slots are loaded at once (indices clamped to the used
// ones) so that the loads are in flight together.
__device__ __forceinline__ double psi_value(const KernelArgs &a, int w, int sp) {
    const double *p = a.wk.psi64 + ((size_t)w * 2 + sp) * kPsiParts;
    const int np = a.psi_nparts, last = np > 0 ? np - 1 : 0;
    double v[kPsiParts];
#pragma unroll
    for (int k = 0; k < kPsiParts; ++k) v[k] = p[k < np ? k : last];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kPsiParts; ++k)
        if (k < np) s += v[k];
    return s;
}

// LDS hand-off between the lanes of one wave (no block barrier)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place Gauss-Jordan inversion with partial pivoting of an n x n matrix
// A by the first 16 lanes of one wave, lane i holding row i in r[].  Rows are
// never exchanged: the pivot of column j is the unused lane with the largest
// |entry| (lowest lane on ties), and the lane that pivots column c ends up
// holding row c of A^-1 with column plane[j] in slot j.  The pivot search and
// the pivot row go through the wave's LDS scratch sc (at least 2 kMaxN + 1
// doubles).  The inverse is written to Xo (LDS, row-major, leading dimension
// ldx); det A = mant 2^ex (mant signed).  Returns false on an exactly zero,
// infinite or NaN pivot.
__device__ __forceinline__ bool lane_gj_core(int n, int lane, double (&r)[kMaxN], double *Xo,
                                             int ldx, double *sc, double &mant_out, int &ex_out) {
    double *cand = sc, *prow = sc + kMaxN;  // |candidates| per lane, normalised pivot row
    int pc = -1;
    int plane[kMaxN];
    double mant = 1.0;
    int ex = 0;
#pragma unroll
    for (int j = 0; j < kMaxN; ++j) {
        if (j >= n) break;
        if (lane < kMaxN) {
            double v = (pc < 0 && lane < n) ? fabs(r[j]) : -1.0;
            if (v != v) v = INFINITY;  // NaN: pick it, then fail below
            cand[lane] = v;
        }
        wave_lds_sync();
        double best = cand[0];
        int id = 0;
#pragma unroll
        for (int l = 1; l < kMaxN; ++l) {
            const double v = cand[l];
            if (v > best) {
                best = v;
                id = l;
            }
        }
        id = __builtin_amdgcn_readfirstlane(id);
        if (!(best > 0.0) || !(best < INFINITY)) return false;
        plane[j] = id;
        const double f = r[j];
        if (lane == id) {
            const double rinv = 1.0 / f;
            pc = j;
            r[j] = 1.0;
#pragma unroll
            for (int k = 0; k < kMaxN; ++k) {
                r[k] *= rinv;
                if (k < n) prow[k] = r[k];
            }
            prow[kMaxN] = f;
        }
        wave_lds_sync();
        const double piv = prow[kMaxN];
        mant *= piv;
        int kk;
        mant = frexp(mant, &kk);
        ex += kk;
        if (lane != id) {
            r[j] = 0.0;
#pragma unroll
            for (int k = 0; k < kMaxN; ++k)
                if (k < n) r[k] -= f * prow[k];
        }
        wave_lds_sync();  // cand / prow are rewritten by the next step
    }
    // det A = det(Q) prod piv, Q the permutation j -> plane[j]
    int inv = 0;
#pragma unroll
    for (int i = 0; i < kMaxN; ++i)
#pragma unroll
        for (int j = i + 1; j < kMaxN; ++j)
            if (j < n && plane[i] > plane[j]) ++inv;
    mant_out = (inv & 1) ? -mant : mant;
    ex_out = ex;
    if (pc >= 0) {
#pragma unroll
        for (int j = 0; j < kMaxN; ++j)
            if (j < n) Xo[pc * ldx + plane[j]] = r[j];
    }
    return true;
}

}  // namespace

}  // namespace mdet
