// Internal types shared by the host pre-processing and the HIP kernels of
// libmdet.  Not part of the public ABI (include/mdet.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mdet.h"

namespace mdet {

// One Gaussian primitive of a molecular orbital: coef * x^a y^b z^c exp(-alpha r^2).
struct Prim {
    double alpha;
    double coef;
    int32_t a, b, c, pad;
};

// Excitation of a distinct spin determinant relative to the reference one
// (the "table method" view of Sec. 5): the s occupied slots h[0..s) of the
// reference (positions in its ascending occupied list, ascending) are
// replaced in place by the particles p[0..s) (orbital indices, ascending);
// eps is the sign of the permutation that sorts the substituted list.
struct DetDesc {
    uint8_t s;
    int8_t eps;
    uint8_t h[4];
    uint8_t pad[2];
    uint16_t p[4];
};
static_assert(sizeof(DetDesc) == 16, "DetDesc layout");

// Degrees up to kFastDegree keep their holes and particles in DetDesc and
// have closed-form or register minors; a determinant of degree
// kFastDegree < s <= MDET_MAX_DEGREE keeps them in a DetDescHi (same meaning,
// up to eight of each), and its s x s minor is inverted by a separate kernel.
constexpr int kFastDegree = 4;
struct DetDescHi {
    uint8_t h[MDET_MAX_DEGREE];
    uint16_t p[MDET_MAX_DEGREE];
    uint8_t pad[8];
};
static_assert(sizeof(DetDescHi) == 32, "DetDescHi layout");

// Capacity (doubles) of the LDS staging buffer that holds the scaled
// adjugates of one chunk of determinants during the derivative aggregation.
constexpr int kAdjChunk = 3072;
// Threads of the derivative-aggregation block.
constexpr int kBlockThreads = 256;
// Largest number of determinants in one such chunk (three per thread).
constexpr int kAdjChunkDets = 768;
// Staged entries one thread adds per chunk (its targets' lists), and the
// padding of a thread's list.
constexpr int kGent = 16;
constexpr uint32_t kGentNone = 0xFFFFFFFFu;
// Sparse combination: a tile of 64 walkers (one per lane) stages the
// gathered vector in LDS by chunks of kSpmmCols64 (FP64) or kSpmmCols32
// (FP32) entries, 130 KB either way (row pitch 65).
constexpr int kSpmmTile = 64;
constexpr int kSpmmCols64 = 250;
constexpr int kSpmmCols32 = 500;

// Device view of one spin channel of the expansion.
struct SpinDev {
    int32_t n;            // electrons of this spin
    int32_t e0;           // first electron index of this spin
    int32_t U;            // distinct determinants
    int32_t nchunk;       // adjugate chunks
    int32_t deg_end[MDET_MAX_DEGREE + 1];  // execution-order end of degree <= d
    const int32_t *occ0;  // [n] reference occupied orbitals, ascending
    const DetDesc *desc;  // [U] in execution order (ascending degree)
    // determinants of degree above kFastDegree: execution indices
    // deg_end[kFastDegree] .. U-1, their holes and particles, and the offset
    // of each one's s*s cofactors in the (walker, spin) high-degree buffer
    const DetDescHi *desc_hi;  // [U - deg_end[kFastDegree]]
    const int32_t *hi_off;     // [U - deg_end[kFastDegree] + 1]
    const int32_t *adj_off;    // [U+1] first adjugate slot of each determinant (sum of s^2)
    const int32_t *chunk_det;  // [nchunk+1] determinant range of each chunk
    // [nchunk][kBlockThreads][kGent] per chunk and thread, the staged slots
    // the thread adds: chunk-local slot | target t << 16 (t = c*M + m), sorted
    // by target; kGentNone pads
    const uint32_t *gent;
    // Sherman-Morrison chain (Sec. 2.2): the distinct determinants in the
    // sorted order of Eq. (comp), position i -> execution index sm_exec[i]
    const int32_t *sm_exec;    // [U]
    const uint16_t *sm_occ;    // [U][n] occupied orbitals, ascending
    const int32_t *sm_off;     // [U+1] substitutions from position i-1 to i:
    const uint32_t *sm_sub;    //   sm_sub[sm_off[i] .. sm_off[i+1]), hole | particle << 16,
                               //   holes ascending paired with particles ascending
};

// Device view of the sparse coefficient matrix in execution indices.  The
// CSR rows (and CSC columns) are cut into segments by chunks of gathered
// entries: seg[c*U + i] is the first entry of row i whose column lies in
// chunk c (seg[nch*U + i] = end of row i).  One set per chunk width.
struct SparseDev {
    int32_t U, V;
    int64_t Z;
    int32_t nch_r64, nch_c64, nch_r32, nch_c32;
    const int32_t *rptr;   // [U+1] CSR (rows = up determinants)
    const int32_t *rcol;   // [Z]
    const double *rval;    // [Z]
    const int32_t *rseg64, *rseg32;  // [(nch+1)*U]
    const int32_t *cptr;   // [V+1] CSC (columns = down determinants)
    const int32_t *crow;   // [Z]
    const double *cval;    // [Z]
    const float *rval32, *cval32;  // the coefficients rounded to FP32 (mixed precision)
    const int32_t *cseg64, *cseg32;  // [(nch+1)*V]
    // end of the entries of row i (column j) whose column (row) determinant
    // has degree <= d: rdeg[i*(MDET_MAX_DEGREE+1) + d]
    const int32_t *rdeg, *cdeg;
};

// Per-call work buffers (device), sized for W walkers.
struct Work {
    int64_t W;
    int64_t Wld;       // leading dimension (walkers) of the walker-minor vectors
    int32_t M, N, nmax, Upad, Vpad;
    double *phi;       // [W][N][5][M] orbitals and derivatives (unscaled; column m of spin
                       // sigma is used as phi * 2^-E[sigma][m])
    int32_t *E;        // [W][2][M] per-spin column exponents
    double *X;         // [W][2][nmax*nmax] inverse of the scaled reference
    double *g0;        // [W][N][4] grad~ D0 / D0
    double *logdet0;   // [W][2]
    double *sign0;     // [W][2]
    int32_t *flag;     // [W][2] 0 table method, 1 ill-conditioned, 2 singular
    int32_t *K;        // [W][2] exponent shift of the ratio vectors
    double *R64;       // [W][Upad+Vpad] walker-major: R_up then R_dn
    float *R32;        // [W][Upad+Vpad]
    double *uv64;      // [W][Upad+Vpad] u (up part) then v (down part)
    float *uv32;       // [W][Upad+Vpad]
    double *psi64;     // [W][2][kPsiParts] partial sums of psi_up = R_up.u (FP64 ratios)
                       // and psi_dn = R_dn.v, FP64 in both precisions
    // R64 holds the shifted FP64 ratios in both precisions (R32 their FP32
    // copy in mixed precision, the vector the sparse products gather)
    int32_t *Rexp;     // [W][Upad+Vpad] direct-LU fallback: exponents of the determinants
    int32_t *Kmax;     // [W][2] direct-LU fallback: largest exponent (integer max)
    double *dpart;     // [W][kDirectSplitMax][N][4] direct-LU fallback: derivative partial sums
    int64_t hi_stride; // doubles of the high-degree cofactor buffer per (walker, spin)
    double *adjhi;     // [W][2][hi_stride] cofactors of the determinants of degree above
                       // kFastDegree (null when there are none)
    int32_t *dcount;   // [1] direct-LU fallback: number of listed (walker, spin) pairs
    int32_t *dlist;    // [2W] direct-LU fallback: listed pairs, w * 2 + spin (any order)
    // uneven batches: walkers sorted by maximum degree
    int32_t *perm;     // [W] sorted position -> caller's walker
    double *Rs;        // [W][N][3] positions in sorted order
    int8_t *mds;       // [W] maximum degrees in sorted order
    double *sign_s, *logabs_s, *gl_s;  // sorted-order outputs
    int32_t *ws_s;
    // Sherman-Morrison chain method
    int32_t Umax;      // max(U, V): determinant stride of the ratio derivatives
    double *smg64;     // [W][2][Umax][4 nmax] grad~_e D / D per determinant (FP64 runs)
    float *smg32;      // same storage, FP32 (mixed-precision runs)
    unsigned long long *smstat;  // [4] substitutions, recomputations, rejected attempts, chunk starts
};

// Size of the static device scratch of the allocation-free evaluation
// (mdet_eval_walkers_noalloc), and the device address of that array on
// `device` (looked up on the first call, with `device` current; later calls
// return the same address).
constexpr size_t kNoallocBytes = (size_t)MDET_NOALLOC_SCRATCH_BYTES;
hipError_t noalloc_scratch(int device, void **ptr);

// Largest number of blocks per (walker, spin) of the direct-LU fallback.
constexpr int kDirectSplitMax = 8;

// Launch parameters chosen per context (mdet_autotune) or by default.
struct LaunchCfg {
    int32_t spmm_rsplit;   // row splits per 64-walker tile of the sparse product (0 = auto)
    int32_t direct_split;  // determinant slices per flagged (walker, spin) of the direct-LU
                           // fallback (0 = one determinant per thread, at most kDirectSplitMax)
    int32_t sort_walkers;  // uneven batches: sort walkers by maximum degree
    int32_t overlap_fallback;  // run the direct-LU fallback on a second stream, concurrently
                               // with the table-method kernels (needs AuxStreams)
};

// A second stream and four events (no timing) owned by the context, for the
// fallback kernels that run beside the table method: ev[0] after the
// reference kernel, ev[1] after the fallback ratios, ev[2] after the sparse
// products, ev[3] after the fallback derivatives.
struct AuxStreams {
    hipStream_t s;
    hipEvent_t ev[4];
};

// Row splits of the sparse combination per walker tile (partial psi sums).
constexpr int kPsiParts = 16;

struct KernelArgs {
    int32_t n_up, n_dn, N, M, P, nmax;
    double kappa_max;
    const Prim *prim;         // [M][P] orbitals of the up electrons (and of all, if one set)
    const Prim *prim_dn;      // [M][P] orbitals of the down electrons (== prim for one set)
    SpinDev sp[2];
    SparseDev C;
    Work wk;
    int64_t W;
    const double *R;          // [W][N][3]
    const int8_t *max_degree; // [W] or null
    int32_t precision;
    int32_t psi_nparts;       // row splits used by the sparse combination
    int32_t direct_split;     // determinant slices per listed pair of the direct-LU fallback
    int32_t direct_stage_grad;  // fallback stages orbital derivatives in LDS (else reads HBM)
    LaunchCfg cfg;
    int32_t method;           // MDET_METHOD_TABLE or MDET_METHOD_SM_CHAIN
    double sm_threshold;      // chain: smallest accepted |ratio| of one substitution
    int32_t sm_chunk;         // chain: determinants per independently started chain piece
    uint32_t ev_mask;         // kernels whose events are recorded (timing)
    double *sign_out, *logabs_out, *gl_out;
    int32_t *wstatus;
};

// Number of kernels of one evaluation (for per-kernel timing).
constexpr int kNumKernels = 9;
const char *kernel_name(int k);
// Bit k set: kernel slot k runs (and has its events recorded) in `method`.
uint32_t kernels_of_method(int method);

// Launch the whole evaluation on `stream`; returns hipSuccess or the first
// error.  If `events` is not null, events[2k] and events[2k + 1] are recorded
// on the stream before and after kernel k (k < kNumKernels).
hipError_t launch_eval(const KernelArgs &a, hipStream_t stream, hipEvent_t *events,
                       const AuxStreams *aux = nullptr);
// Sherman-Morrison chain method (its own source file): the chain pieces with
// the exponent shift, and the derivative sums after the sparse combination.
void launch_chain_pieces(const KernelArgs &a, hipStream_t stream);
void launch_chain_deriv(const KernelArgs &a, hipStream_t stream);

// ---------------------------------------------------------------- VMC and MLP
constexpr double kMlpLogSigMin = -4.6051701859880914;  // ln 0.01
constexpr double kMlpLogSigMax = 0.69314718055994531;  // ln 2

struct MlpShape {
    int n_in, n_hid, n_out;
    int64_t n_params() const {
        return (int64_t)n_in * n_hid + n_hid + (int64_t)n_hid * n_hid + n_hid +
               (int64_t)n_hid * n_out + n_out;
    }
};

void launch_philox(uint64_t seed, uint64_t stream_id, uint64_t step, int64_t n, int kind,
                   double *out, hipStream_t st);
void launch_vmc_propose(int64_t W, int N, int proposal, double step, const double *R,
                        const double *gl, const double *xi, double *Rp, hipStream_t st);
void launch_vmc_accept(int64_t W, int N, int proposal, double step, double Z, double *R,
                       double *sign, double *logabs, double *gl, const double *Rp,
                       const double *signp, const double *logabsp, const double *glp,
                       const double *uniform, const float *o1, const float *o2, double *elocal,
                       int32_t *accepted, int fixed_node, hipStream_t st);
void launch_gemm_f32(int M, int Nn, int K, const float *A, int a_rs, int a_cs, const float *B,
                     int b_rs, int b_cs, float *C, int c_rs, const float *bias, int act,
                     int accumulate, hipStream_t st);
void launch_mlp_forward(const MlpShape &s, const float *params, int64_t B, const float *X,
                        float *h1, float *h2, float *O, hipStream_t st);
void launch_mlp_backward(const MlpShape &s, const float *params, int64_t B, const float *X,
                         const float *h1, const float *h2, const float *dO, float *dparams,
                         int accumulate, float *dX, float *work_h1, float *work_h2,
                         hipStream_t st);
void launch_to_f32(int64_t n, const double *x, float *y, hipStream_t st);
void launch_mlp_propose(int64_t W, int N, const double *R, const float *o, const double *xi,
                        double *Rp, hipStream_t st);
void launch_esjd_head(int64_t W, int N, const double *R, const double *Rp, const double *xi,
                      const double *logabsR, const double *signp, const double *logabsp,
                      const double *glp, const float *o1, const float *o2, float *dO2,
                      double *gRp, double *gell, double *Jw, double jump_ref, int objective,
                      double Z, hipStream_t st);
void launch_esjd_chain(int64_t W, int N, const double *xi, const float *o1, const double *gRp,
                       const float *dX2, const double *gell, float *dO1, hipStream_t st);
void launch_esjd_loss(int64_t W, const double *Jw, double *out, hipStream_t st);
void launch_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1,
                 float b2, float eps, int t, hipStream_t st);

// ------------------------------------------------------------ Jastrow and DMC
struct JastrowParams {
    double b_ee;  // electron-electron Pade denominator
    double a_en;  // electron-nucleus amplitude (-Z: nuclear cusp; 0: no term)
    double b_en;  // electron-nucleus Pade denominator
};

// DMC work buffers (device), W walkers
struct DmcWork {
    double *cum;     // [W] cumulative branching weights
    int32_t *src;    // [W] selected walker of each new slot
    double *R, *sign, *logabs, *gl, *elocal;  // gathered state
};

void launch_jastrow(int64_t W, int N, int n_up, const JastrowParams &p, const double *R,
                    double *logabs, double *gl, hipStream_t st);
void launch_dmc_save(int64_t W, const double *elocal, double *e_old, hipStream_t st);
void launch_dmc_branch(int64_t W, int N, double tau, double e_trial, double comb_u,
                       const double *e_old, const int32_t *accepted, DmcWork &d, double *R,
                       double *sign, double *logabs, double *gl, double *elocal, double *weight,
                       double *sums, hipStream_t st);

}  // namespace mdet
