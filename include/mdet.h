/*
 * mdet.h -- C ABI of libmdet: multideterminant wavefunction values, gradients
 * and Laplacians for batches of QMC walkers on an AMD Instinct MI355X (gfx950).
 *
 * The wavefunction is a CI expansion over products of spin determinants,
 *     Psi(R) = sum_k c_k det S_up[k](R_up) det S_dn[k](R_dn)       (Eq. (1))
 * evaluated through its bilinear form over the distinct spin determinants,
 *     Psi = D_up^T C D_dn                                             (Eq. (main))
 * with, for every electron e, the four-vector grad~_e = [d/dx, d/dy, d/dz,
 * Laplacian] of Sec. 2.3 (Eq. (nabla)).
 *
 * Conventions shared by every call:
 *  - Electrons 0..n_up-1 are spin up, n_up..n_up+n_dn-1 spin down; n_up >= n_dn
 *    (Sec. 2.4 fixes this convention).
 *  - [S]_{e,c} = phi_{o_c}(r_e): rows are electrons, columns are the occupied
 *    orbitals of the determinant in ascending orbital order (Eq. (1)).
 *  - A spin determinant is n_int 64-bit words; bit b of word w set means
 *    orbital 64*w+b (0-based) is occupied (Sec. 2.1, "Encoding"); n_int must be
 *    ceil(n_mo/64).
 *  - Host arrays are copied; the caller keeps ownership.  Device pointers are
 *    caller-owned, contiguous, 8-byte aligned and on the context's device.
 *  - Every call returns MDET_OK (0) or a negative status; the message of the
 *    last failing call is available from mdet_last_error.  No C++ exception
 *    crosses this boundary.  Argument errors are reported before any device
 *    work is queued; device faults surface as MDET_EHIP.
 *  - A context is bound to one device and is not thread-safe.  Calls that
 *    take a stream queue work on it and return without synchronising.
 */
#ifndef MDET_H
#define MDET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdet_ctx mdet_ctx;
typedef int32_t mdet_status;

enum {
    MDET_OK = 0,
    MDET_EINVAL = -1,      /* null pointer or negative/zero size where not allowed  */
    MDET_EDIM = -2,        /* sizes inconsistent with earlier calls or limits        */
    MDET_EPOPCOUNT = -3,   /* a determinant without exactly n_sigma set bits         */
    MDET_EORBITAL = -4,    /* a bit >= n_mo, or n_int != ceil(n_mo/64)              */
    MDET_EDUPLICATE = -5,  /* the same (det_up, det_dn) product given twice          */
    MDET_ESPIN = -6,       /* n_up < n_dn                                            */
    MDET_ENOMEM = -7,      /* device or host allocation failed                       */
    MDET_EHIP = -8,        /* a HIP runtime call failed                              */
    MDET_ESTATE = -9,      /* call order violated (e.g. eval before set_expansion)   */
    MDET_EDEGREE = -10     /* excitation degree above MDET_MAX_DEGREE                */
};

enum { MDET_FP64 = 0, MDET_MIXED = 1 };

/* Largest excitation degree (holes = particles) of a spin determinant relative
 * to the reference spin determinant that set_expansion accepts. */
#define MDET_MAX_DEGREE 4
/* Largest number of electrons of one spin. */
#define MDET_MAX_SPIN_ELEC 16
/* Largest number of orbitals. */
#define MDET_MAX_MO 512

/* Per-walker status codes written by mdet_eval_walkers. */
enum {
    MDET_W_OK = 0,        /* table method on the reference determinant         */
    MDET_W_FALLBACK = 1,  /* reference ill-conditioned: direct LU per det used */
    MDET_W_NODE = 2       /* Psi == 0: sign 0, logabs -inf, derivatives 0      */
};

/* Create a context on HIP device `hip_device` (sets it current).  *out is
 * owned by the caller and released with mdet_destroy.  hip_device == -1 makes
 * a host-only context: set_expansion pre-processes and get_indexing /
 * get_stats work, nothing touches a GPU, and eval_walkers returns
 * MDET_ESTATE. */
mdet_status mdet_create(mdet_ctx **out, int32_t hip_device);

/* Free every device and host buffer of the context.  Waits for the device. */
void mdet_destroy(mdet_ctx *ctx);

/* Message of the last failing call on this context ("" if none).  The string
 * lives until the next call on the context. */
const char *mdet_last_error(const mdet_ctx *ctx);

/*
 * Molecular orbitals (the Phi arrays of Sec. 2): orbital m is
 *   phi_m(r) = sum_{p<n_prim} coef[m][p] x^a y^b z^c exp(-alpha[m][p] |r|^2)
 * with (a,b,c) = pow_abc[m][p][0..2] (each 0..4), all centred at the origin.
 * Padding primitives have coef 0.  Gradients and Laplacians are analytic.
 * Layouts: pow_abc int32 [n_mo][n_prim][3], alpha/coef double [n_mo][n_prim],
 * host memory, copied.  1 <= n_mo <= MDET_MAX_MO, 1 <= n_prim <= 16, alpha > 0.
 * Calling it again replaces the orbitals (and drops the expansion).
 */
mdet_status mdet_init_orbitals(mdet_ctx *ctx, int32_t n_mo, int32_t n_prim,
                               const int32_t *pow_abc, const double *alpha,
                               const double *coef);

/*
 * CI expansion (Eq. (1)) and its one-time pre-processing (Sec. 2.1):
 * encoding check, xor-key sort and duplicate removal of each spin list,
 * binary search of every product, column-major ordering of the sparse C,
 * plus the excitation analysis of every distinct spin determinant against
 * the reference (the spin determinants of the product with the largest |c_k|,
 * the earliest one on ties).
 * det_up, det_dn: uint64 [n_det][n_int] host; c: double [n_det] host.
 * Requires mdet_init_orbitals first.  Errors: MDET_ESPIN, MDET_EORBITAL,
 * MDET_EPOPCOUNT, MDET_EDUPLICATE, MDET_EDEGREE, MDET_EDIM (n_dn < 1,
 * n_up > MDET_MAX_SPIN_ELEC, n_up > n_mo, n_up * n_mo > 8192, or n_det
 * outside 1..2^30-1).
 * Synchronous.
 */
mdet_status mdet_set_expansion(mdet_ctx *ctx, int32_t n_up, int32_t n_dn, int32_t n_int,
                               int64_t n_det, const uint64_t *det_up,
                               const uint64_t *det_dn, const double *c);

/*
 * The indexing produced by set_expansion, bit for bit (Sec. 2.1):
 *  - uniq_up [U][n_int], uniq_dn [V][n_int]: the distinct spin determinants in
 *    ascending order of the key omega = xor of the words read as unsigned
 *    (Eq. (comp)); ties on omega are broken by comparing the words from the
 *    last to the first as unsigned integers;
 *  - row_i, col_j, val, src_pos [n_det]: the sparse C in coordinate form sorted
 *    by the 0-based key U*j + i (column by column), src_pos = the input
 *    position k of each entry;
 *  - ref_up, ref_dn: indices (in the uniq lists) of the reference determinants.
 * Every output pointer is host memory and may be NULL (then skipped).
 */
mdet_status mdet_get_indexing(const mdet_ctx *ctx, int64_t *n_uniq_up, int64_t *n_uniq_dn,
                              uint64_t *uniq_up, uint64_t *uniq_dn, int32_t *row_i,
                              int32_t *col_j, double *val, int64_t *src_pos,
                              int64_t *ref_up, int64_t *ref_dn);

/*
 * The hot path: for n_walk walkers, sign(Psi), ln|Psi| and grad~_e Psi / Psi
 * for every electron (the 4 x N array of Sec. 2.3).
 *  R_dev        double [n_walk][n_up+n_dn][3], device.
 *  precision    MDET_FP64: every step in FP64.  MDET_MIXED: the sparse
 *               combination over the n_det products (u = C R_dn, v = C^T R_up,
 *               psi) in FP32 with FP32 accumulation; LU, table, ratios and
 *               derivative aggregation stay FP64.
 *  max_degree_dev  int8 [n_walk] device or NULL: walker w keeps only products
 *               whose two spin determinants both have excitation degree
 *               <= max_degree[w] relative to the reference (uneven batches).
 *  sign_dev     double [n_walk] device: +1, -1, or 0 at a node.
 *  logabs_dev   double [n_walk] device: ln|Psi| (-inf at a node).
 *  gl_dev       double [n_walk][n_up+n_dn][4] device: [dx, dy, dz, lap] Psi/Psi.
 *  wstatus_dev  int32 [n_walk] device or NULL: MDET_W_* per walker.
 *  hip_stream   hipStream_t (NULL = default stream).
 * Asynchronous on hip_stream.  Library work buffers grow to the largest
 * n_walk seen and are reused; calls on one context must not overlap.
 */
mdet_status mdet_eval_walkers(mdet_ctx *ctx, int64_t n_walk, const double *R_dev,
                              int32_t precision, const int8_t *max_degree_dev,
                              double *sign_dev, double *logabs_dev, double *gl_dev,
                              int32_t *wstatus_dev, void *hip_stream);

/*
 * Reference-conditioning threshold: a (walker, spin) whose reference matrix A
 * has ||A||_1 ||A^-1||_1 above kappa_max (or a zero pivot) is evaluated by the
 * direct-LU fallback instead of the table method.  Default 3e4 -- the
 * analogue of the paper's 1e-3 ratio rule for its update chain (Sec. 2.2):
 * rounding errors of the table method grow with this condition number.
 */
mdet_status mdet_set_fallback_threshold(mdet_ctx *ctx, double kappa_max);

typedef struct {
    int64_t n_det, n_uniq_up, n_uniq_dn;
    int32_t n_up, n_dn, n_mo, n_prim, n_int;
    int64_t ref_up, ref_dn;
    int64_t n_by_degree_up[MDET_MAX_DEGREE + 1];
    int64_t n_by_degree_dn[MDET_MAX_DEGREE + 1];
    int64_t workspace_bytes;      /* device bytes held for walker buffers */
    int64_t expansion_bytes;      /* device bytes held for the expansion  */
    double preprocess_seconds;    /* host time of the last set_expansion  */
} mdet_stats;

/* Shapes and sizes of the loaded expansion. */
mdet_status mdet_get_stats(const mdet_ctx *ctx, mdet_stats *out);

/*
 * Per-kernel timing.  With enable != 0, every later mdet_eval_walkers call
 * records HIP events on its own stream around each of its kernels; the
 * accumulated times are reset by this call.  Timing adds one event record
 * per kernel and one wait on the previous call's last event per call.
 */
mdet_status mdet_set_profiling(mdet_ctx *ctx, int32_t enable);

/*
 * Accumulated kernel times (milliseconds, summed over the profiled calls,
 * host arrays of `capacity` entries, each nullable), the kernel names
 * (static strings) and counts.  Waits for the last profiled call.
 */
mdet_status mdet_get_kernel_times(mdet_ctx *ctx, int32_t capacity, double *ms_total,
                                  const char **names, int32_t *n_kernels, int64_t *n_calls);

#ifdef __cplusplus
}
#endif
#endif /* MDET_H */
