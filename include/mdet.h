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
    MDET_EDEGREE = -10     /* table-method evaluation of an expansion with an
                              excitation degree above MDET_MAX_DEGREE               */
};

enum { MDET_FP64 = 0, MDET_MIXED = 1 };

/* Largest excitation degree (holes = particles) of a spin determinant relative
 * to the reference spin determinant that the table method evaluates (the
 * degree mix of the paper's CIPSI expansions reaches 6-8, Sec. 4, Table 4),
 * and the largest per-walker degree limit.  Degrees up to 4 have closed-form
 * or in-register minors; degrees 5-8 take an s x s Gauss-Jordan inversion in
 * a separate kernel.  set_expansion accepts any degree; an expansion holding
 * a higher degree is evaluated by MDET_METHOD_SM_CHAIN only (the chain
 * substitutes columns between consecutive determinants and has no degree
 * limit), without per-walker degree limits. */
#define MDET_MAX_DEGREE 8
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
 * Separate orbitals for the down electrons (Eq. (1) uses one common set; the
 * paper notes that two sets are a direct generalisation, Sec. 2): the
 * matrices of the down determinants take phi_j^dn(r_i).  Same layout and
 * limits as mdet_init_orbitals, with that call's n_mo and n_prim.  Keeps the
 * expansion; a later mdet_init_orbitals returns to one common set.
 * Synchronous (waits for the device).
 */
mdet_status mdet_init_orbitals_dn(mdet_ctx *ctx, const int32_t *pow_abc, const double *alpha,
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
 * MDET_EPOPCOUNT, MDET_EDUPLICATE, MDET_EDIM (n_dn < 1,
 * n_up > MDET_MAX_SPIN_ELEC, n_up > n_mo, n_up * n_mo > 6144 (the per-walker tables
 * of the derivative kernel must fit in LDS), or n_det
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
 * Norm-based truncation of the expansion (Sec. 3, the improved truncation
 * scheme): with N = sum_k c_k^2, the contribution of a distinct spin
 * determinant is N_i^up = (sum of c_k^2 over the products holding it) / N
 * (likewise N_j^dn); sum_i N_i^up = sum_j N_j^dn = 1.  Product k is kept iff
 * N^up of its up determinant > eps_up and N^dn of its down determinant >
 * eps_dn (a determinant at or below its threshold is removed with every
 * product holding it).  Sums run over k in input order, in FP64.
 * det_up, det_dn uint64 [n_det][n_int], c double [n_det], host, read only.
 * Outputs (host, nullable): keep uint8 [n_det] (1 = kept); n_kept = kept
 * products; n_up_kept, n_dn_kept = distinct spin determinants among them.
 * No context needed.  Errors: MDET_EINVAL (null input, eps < 0 or NaN, all
 * c zero), MDET_EDIM (n_int < 1 or n_det < 1).  Synchronous.
 */
mdet_status mdet_norm_truncation(int32_t n_int, int64_t n_det, const uint64_t *det_up,
                                 const uint64_t *det_dn, const double *c, double eps_up,
                                 double eps_dn, uint8_t *keep, int64_t *n_kept,
                                 int64_t *n_up_kept, int64_t *n_dn_kept);

/*
 * The hot path: for n_walk walkers, sign(Psi), ln|Psi| and grad~_e Psi / Psi
 * for every electron (the 4 x N array of Sec. 2.3).
 *  R_dev        double [n_walk][n_up+n_dn][3], device.
 *  precision    MDET_FP64: every step in FP64.  MDET_MIXED: the vectors of
 *               the sparse combination over the n_det products (R_up, R_dn,
 *               u = C R_dn, v = C^T R_up) are stored and moved in FP32, C and
 *               every accumulation (u, v, psi) in FP64; LU, table, ratios and
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
 * Errors: MDET_EDEGREE when the expansion holds an excitation degree above
 * MDET_MAX_DEGREE and the method is the table method; MDET_EINVAL for
 * max_degree_dev with such an expansion.
 */
mdet_status mdet_eval_walkers(mdet_ctx *ctx, int64_t n_walk, const double *R_dev,
                              int32_t precision, const int8_t *max_degree_dev,
                              double *sign_dev, double *logabs_dev, double *gl_dev,
                              int32_t *wstatus_dev, void *hip_stream);

/*
 * Allocation-free variant of mdet_eval_walkers, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, outputs, asynchrony,
 * methods and errors as mdet_eval_walkers; the per-call work buffers come
 * from a static device array of MDET_NOALLOC_SCRATCH_BYTES per GPU (held by
 * every GPU the library runs on until the process ends) instead of the
 * context's grow-only buffers, and the call makes no hipMalloc, hipFree or
 * other allocating call (no timing events are recorded, and the chain
 * method's counters are not kept).  The scratch holds the orbital table of
 * every walker and the ratio and weight vectors of the sparse combination,
 * about W * (40 N M + 28 (U + V)) bytes; a call that needs more than
 * MDET_NOALLOC_SCRATCH_BYTES returns MDET_EDIM (with the size in the message)
 * before queueing anything.  All calls on one GPU share that GPU's array:
 * every kernel clears what it reads before it is written, but calls that
 * overlap on one GPU (two streams, two contexts or two threads) race.
 */
#define MDET_NOALLOC_SCRATCH_BYTES (64ull << 20)
mdet_status mdet_eval_walkers_noalloc(mdet_ctx *ctx, int64_t n_walk, const double *R_dev,
                                      int32_t precision, const int8_t *max_degree_dev,
                                      double *sign_dev, double *logabs_dev, double *gl_dev,
                                      int32_t *wstatus_dev, void *hip_stream);

/*
 * Reference-conditioning threshold of one precision: a (walker, spin) whose
 * scaled reference matrix A has ||A||_1 ||A^-1||_1 above kappa_max (or a zero
 * pivot) is evaluated by the direct-LU fallback instead of the table method
 * -- the analogue of the paper's 1e-3 ratio rule for its update chain
 * (Sec. 2.2): the rounding error of the table method grows with this
 * condition number (measured on 4096 walkers of the 1e5-product workload:
 * scaled derivative error up to 5e-11 below 3e4, 1e-8 to 3e-7 between 3e4
 * and 1e7, 1e-4 above), so each precision's threshold follows its error
 * bound (1e-10 in FP64, 1e-5 in mixed precision).  The defaults are
 * calibrated on that workload's orbitals; on other inputs the same kappa_1
 * can leave a larger derivative error (the same workload with its orbitals
 * in drawn order, FP64 at 3e4: Psi within 1.2e-11 everywhere, but the
 * derivatives of 1.8 % of the walkers above 1e-10, the largest 1.6e-8; at
 * 1e3, 99.6 % of the walkers fall back and one of the 180 worst stays
 * above it, at 1.04e-10), and such inputs need a lower threshold.
 *  precision  MDET_FP64, MDET_MIXED, or -1 for both.
 *  kappa_max  > 0; defaults MDET_KAPPA_FP64_DEFAULT and MDET_KAPPA_MIXED_DEFAULT.
 * Takes effect at the next evaluation; captured steps (mdet_eval_graph) are
 * dropped and re-captured.  Errors: MDET_EINVAL.
 */
#define MDET_KAPPA_FP64_DEFAULT 3e4
#define MDET_KAPPA_MIXED_DEFAULT 1e6
mdet_status mdet_set_fallback_threshold(mdet_ctx *ctx, int32_t precision, double kappa_max);

/* Evaluation methods of mdet_eval_walkers. */
enum { MDET_METHOD_TABLE = 0, MDET_METHOD_SM_CHAIN = 1 };

/*
 * Select how the spin determinants are evaluated (Sec. 2.2 against Sec. 5).
 *  MDET_METHOD_TABLE     (default) ratios from the table X Phi' of the
 *                        reference, with the direct-LU fallback above.
 *  MDET_METHOD_SM_CHAIN  the paper's chain: the distinct determinants in the
 *                        sorted order of Eq. (comp), each reached from the
 *                        previous one by Sherman-Morrison column substitutions
 *                        (Eq. (sherman)) on its inverse.  A substitution whose
 *                        determinant ratio has |r| < sm_threshold is postponed
 *                        and retried after the others; a retry pass that
 *                        completes none of the postponed ones restarts the
 *                        determinant from an O(n^3) factorisation.  The list
 *                        is cut into pieces of sm_chunk determinants that run
 *                        in parallel, each started by a factorisation.
 *                        grad~_e D / D comes from the current inverse
 *                        (Sec. 2.3) and is stored per determinant
 *                        (8 or 4 bytes x 4 n per determinant and walker,
 *                        FP64 or mixed precision).  Walker status is always
 *                        MDET_W_OK or MDET_W_NODE.
 *  sm_threshold  > 0 (the paper uses 1e-3); ignored for the table method.
 *  sm_chunk      >= 1 determinants per chain piece; ignored for the table.
 * Returns MDET_EINVAL for an unknown method or out-of-range parameter.
 */
mdet_status mdet_set_method(mdet_ctx *ctx, int32_t method, double sm_threshold,
                            int32_t sm_chunk);

/*
 * Counters of the last MDET_METHOD_SM_CHAIN evaluation on this context,
 * summed over walkers and both spins: out[0] column substitutions done,
 * out[1] factorisations forced by the retry rule or a singular predecessor,
 * out[2] postponed substitution attempts, out[3] chain pieces started by a
 * factorisation.  Synchronises the device.  Zeros if no chain evaluation ran.
 */
mdet_status mdet_get_sm_counters(mdet_ctx *ctx, int64_t *out4);

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
 * As mdet_set_profiling, timing only the kernels whose bit is set in mask
 * (bit k = kernel k of mdet_get_kernel_times); mask 0 turns timing off.
 * Fewer events per call leave less recording work on the stream.
 */
mdet_status mdet_set_profiling_mask(mdet_ctx *ctx, uint32_t mask);

/*
 * Accumulated kernel times (milliseconds, summed over the profiled calls,
 * host arrays of `capacity` entries, each nullable), the kernel names
 * (static strings) and counts.  Waits for the last profiled call.
 */
mdet_status mdet_get_kernel_times(mdet_ctx *ctx, int32_t capacity, double *ms_total,
                                  const char **names, int32_t *n_kernels, int64_t *n_calls);

/* ------------------------------------------------------------------------
 * Variational Monte Carlo and the learned proposal.  A Monte Carlo step
 * moves all electrons of a walker and computes Psi, its derivatives and the
 * local energy (the step of Sec. 4).
 * ------------------------------------------------------------------------ */

enum { MDET_PROP_GAUSSIAN = 0, MDET_PROP_DRIFT = 1, MDET_PROP_MLP = 2 };
enum { MDET_RNG_UNIFORM = 0, MDET_RNG_NORMAL = 1 };

/*
 * Slater-Jastrow trial function.  The paper treats the Jastrow prefactor by
 * standard O(N^2) techniques and leaves it out of its algorithm (Sec. 1);
 * here it multiplies the expansion: Psi_T = exp(J) Psi with
 *   J = sum_{i<j} a_ij r_ij / (1 + b_ee r_ij) + sum_i a_en r_i / (1 + b_en r_i),
 * a_ij = 1/2 for electrons of opposite spin, 1/4 for equal spin (the
 * electron-electron cusp conditions); a_en = -Z gives the cusp at a nucleus
 * of charge Z at the origin, a_en = 0 drops the term.  When enabled, every
 * evaluation (mdet_eval_walkers, mdet_eval_graph, the VMC and DMC steps)
 * returns ln|Psi_T|, grad ln Psi_T and lap Psi_T / Psi_T instead of the
 * expansion's values; the sign is unchanged.  Exactly coincident electrons
 * give non-finite Laplacians.  b_ee, b_en >= 0 and finite.
 */
mdet_status mdet_set_jastrow(mdet_ctx *ctx, int32_t enable, double b_ee, double a_en,
                             double b_en);

/*
 * One fixed-node diffusion Monte Carlo step for n_walk walkers (all device
 * pointers, updated in place; the walker state is consistent on entry and
 * on exit):
 *  1. drift-diffusion move R' = R + tau grad ln|Psi(R)| + sqrt(tau) xi
 *     (noise_dev [W][N][3] standard normals) with the Metropolis-Hastings
 *     test of mdet_vmc_step (uniform_dev [W]); a move onto a node or across
 *     one (sign of Psi changes) is rejected;
 *  2. branching weight w <- w exp(-tau ((E_L(R) + E_L(R_new)) / 2 - e_trial)),
 *     0 for a walker whose local energy is not finite; elocal_dev [W] holds
 *     E_L at the walker's position on entry and is updated;
 *  3. sums_dev [4] (device) receives, before the population is redrawn,
 *     sum w, sum w E_L, sum w^2 and the number of accepted moves;
 *  4. the population is redrawn at fixed size by the comb: new walker j is
 *     a copy of the first walker i whose cumulative weight exceeds
 *     (j + comb_u) sum w / n_walk (comb_u in [0, 1)); every copy carries
 *     weight 1 in weight_dev [W].  If every weight is zero nothing is
 *     redrawn.
 * Z = nuclear_charge (point nucleus at the origin, as mdet_vmc_step).
 * Deterministic for given random numbers.  Asynchronous on hip_stream.
 */
mdet_status mdet_dmc_step(mdet_ctx *ctx, int64_t n_walk, double tau, double e_trial,
                          double nuclear_charge, int32_t precision, double *R_dev,
                          double *sign_dev, double *logabs_dev, double *gl_dev, double *elocal_dev,
                          double *weight_dev, const double *noise_dev, const double *uniform_dev,
                          double comb_u, double *sums_dev, int32_t *accepted_dev,
                          void *hip_stream);

/*
 * Philox-4x32-10 counter-based random numbers (Salmon et al., SC'11).
 * Element pair i is drawn from counter (i, stream_id, step_lo, step_hi) under
 * key (seed_lo, seed_hi); its 4 outputs give two doubles in (0,1) from 52 bits
 * each, u = (x0 2^20 + (x1 >> 12) + 1/2) 2^-52, returned as is (kind
 * MDET_RNG_UNIFORM) or through Box-Muller (MDET_RNG_NORMAL).  out_dev: double
 * [n], device.  Asynchronous on hip_stream.
 */
mdet_status mdet_rng_fill(mdet_ctx *ctx, uint64_t seed, uint64_t stream_id, uint64_t step,
                          int64_t n, int32_t kind, double *out_dev, void *hip_stream);

/*
 * One VMC step for n_walk walkers (all device pointers, updated in place):
 *  proposal  MDET_PROP_GAUSSIAN: R' = R + step xi;  MDET_PROP_DRIFT:
 *            R' = R + step grad ln|Psi(R)| + sqrt(step) xi;  MDET_PROP_MLP:
 *            R' = R + mu(R) + sigma(R) xi with the network of mdet_mlp_forward
 *            (mlp_params, n_hidden; inputs the 3N coordinates, outputs the 3N
 *            move means and N log steps clamped to [ln 0.01, ln 2]).
 *  Acceptance: u < |Psi(R')/Psi(R)|^2 q(R|R')/q(R'|R) (exact Metropolis-
 *            Hastings, computed in logs; never onto a node of Psi).
 *  R_dev [W][N][3], sign/logabs [W], gl [W][N][4]: walker state, consistent on
 *            entry (from mdet_eval_walkers) and on exit.
 *  noise_dev [W][N][3] standard normals, uniform_dev [W] in (0,1) (e.g. from
 *            mdet_rng_fill).
 *  elocal_dev [W]: E_L = -1/2 sum_e lap_e Psi/Psi - Z sum_e 1/|r_e|
 *            + sum_{e<f} 1/|r_e - r_f| at the walker's position after the
 *            step (Z = nuclear_charge at the origin); accepted_dev [W]: 0/1.
 */
mdet_status mdet_vmc_step(mdet_ctx *ctx, int64_t n_walk, int32_t proposal, double step,
                          const float *mlp_params, int32_t n_hidden, double *R_dev,
                          double *sign_dev, double *logabs_dev, double *gl_dev,
                          const double *noise_dev, const double *uniform_dev,
                          double nuclear_charge, int32_t precision, double *elocal_dev,
                          int32_t *accepted_dev, void *hip_stream);

/*
 * The proposal network, FP32, on device: x -> tanh(x W1 + b1) -> tanh(. W2 +
 * b2) -> . W3 + b3.  params: [W1 (n_in x n_hidden), b1, W2 (n_hidden x
 * n_hidden), b2, W3 (n_hidden x n_out), b3], row-major, contiguous.
 * X [batch][n_in] -> Y [batch][n_out].  The dense layers run on the matrix
 * cores.
 */
mdet_status mdet_mlp_forward(mdet_ctx *ctx, int32_t n_in, int32_t n_hidden, int32_t n_out,
                             const float *params, int64_t batch, const float *X, float *Y,
                             void *hip_stream);

/* Gradient of sum(dY * Y(X)) w.r.t. the parameters (dparams, same layout,
 * overwritten) and, if dX is not null, w.r.t. the inputs. */
mdet_status mdet_mlp_backward(mdet_ctx *ctx, int32_t n_in, int32_t n_hidden, int32_t n_out,
                              const float *params, int64_t batch, const float *X, const float *dY,
                              float *dparams, float *dX, void *hip_stream);

/* One bias-corrected Adam step (t = 1-based step count) on n parameters. */
mdet_status mdet_mlp_adam(mdet_ctx *ctx, int64_t n, float *params, const float *grads, float *m,
                          float *v, int32_t t, float lr, float beta1, float beta2, float eps,
                          void *hip_stream);

/*
 * One training step of the proposal network on walker samples R_dev
 * [W][N][3] with move noise noise_dev [W][N][3]: maximises the expected jump
 * of a statistic with the exact acceptance,
 *   loss = -mean_w A_w jump_w,  R' = R + mu(R) + sigma(R) xi,
 *   A = min(1, |Psi(R')/Psi(R)|^2 q(R|R')/q(R'|R)),
 * with, for objective MDET_OBJ_JUMP, jump = sum_e c_e |r'_e - r_e|^2 (c_e = 1
 * when jump_ref <= 0, the plain squared jump distance; c_e = 1 / (|r_e|^2 +
 * jump_ref^2) otherwise, each electron's jump relative to its distance from
 * the nucleus), and for MDET_OBJ_POTENTIAL, jump = (V(R') - V(R))^2 with V the
 * Coulomb potential energy of the electrons around a point nucleus of charge
 * nuclear_charge at the origin (the part of the local energy a move changes
 * most, so decorrelating V targets the local energy's autocorrelation);
 * differentiating through both network evaluations, through ln|Psi(R')|
 * (grad ln|Psi| from the multideterminant path) and through q; then one Adam
 * step (beta 0.9/0.999, eps 1e-8).  loss_dev: double [1]; grad_dev: float
 * [n_params] or null (gradient before the update).
 */
enum { MDET_OBJ_JUMP = 0, MDET_OBJ_POTENTIAL = 1 };
mdet_status mdet_mlp_train_step(mdet_ctx *ctx, int64_t n_walk, int32_t n_hidden, float *params,
                                float *adam_m, float *adam_v, int32_t t, float lr,
                                const double *R_dev, const double *noise_dev, int32_t precision,
                                double jump_ref, int32_t objective, double nuclear_charge,
                                double *loss_dev, float *grad_dev, void *hip_stream);

/* ------------------------------------------------------------------------
 * Launch configuration, captured steps and tuning.
 * ------------------------------------------------------------------------ */

/*
 * Launch parameters: spmm_row_splits = row splits per 64-walker tile of the
 * sparse combination (0 = derived from the batch, 1..16); direct_split =
 * determinant slices (thread blocks) per flagged (walker, spin) of the
 * direct-LU fallback (0 = one determinant per thread up to 8 slices, 1..8);
 * sort_walkers = with a max_degree array, evaluate the walkers in ascending
 * order of their maximum degree, so that each tile of the sparse combination
 * touches only the determinants its walkers reach; overlap_fallback = run the
 * direct-LU fallback of the ill-conditioned (walker, spin) pairs on a second
 * stream of the context, beside the table-method kernels (its ratios beside
 * the table ratios, its derivative sums beside the derivative aggregation;
 * joined before the kernels that read them; also inside captured graphs).
 * FP64 results are bitwise reproducible for a fixed configuration (the
 * summation grouping depends on the splits; the overlap does not change
 * results).  Default (0, 0, 1, 0).  Setting it drops captured graphs and the
 * configurations mdet_autotune remembered.
 */
mdet_status mdet_set_launch_config(mdet_ctx *ctx, int32_t spmm_row_splits, int32_t direct_split,
                                   int32_t sort_walkers, int32_t overlap_fallback);
mdet_status mdet_get_launch_config(const mdet_ctx *ctx, int32_t *spmm_row_splits,
                                   int32_t *direct_split, int32_t *sort_walkers,
                                   int32_t *overlap_fallback);

/*
 * Same contract as mdet_eval_walkers, but the whole step (every kernel) is
 * captured once into a HIP graph per distinct argument set (n_walk,
 * precision, every pointer, stream; up to 8 cached, least recently used
 * evicted) and replayed with one graph launch per call.  Inputs may change
 * between calls, pointers may not (a new pointer set is captured anew).
 * A NULL stream is replaced by a blocking stream owned by the context.
 */
mdet_status mdet_eval_graph(mdet_ctx *ctx, int64_t n_walk, const double *R_dev, int32_t precision,
                            const int8_t *max_degree_dev, double *sign_dev, double *logabs_dev,
                            double *gl_dev, int32_t *wstatus_dev, void *hip_stream);

typedef struct {
    int32_t spmm_row_splits, direct_split, sort_walkers, overlap_fallback, n_candidates;
    double best_ms;     /* mean time per evaluation of the chosen configuration */
    double default_ms;  /* the same for the first candidate (auto splits)      */
} mdet_tune_result;

/*
 * Time every candidate launch configuration (row splits {auto, 4, 8, 16} x
 * fallback splits {auto, 4, 8} x fallback overlap {on, off} x walker sorting
 * {on, off} when max_degree_dev is given) on n_rep evaluations of the given
 * walkers and report the fastest in *out (nullable).  The context remembers
 * it for this shape -- (n_walk, precision, with or without per-walker degree
 * limits), up to 32 shapes -- and later evaluations of that shape use it;
 * other shapes keep the configuration of mdet_set_launch_config.
 * Synchronous.
 */
mdet_status mdet_autotune(mdet_ctx *ctx, int64_t n_walk, const double *R_dev, int32_t precision,
                          const int8_t *max_degree_dev, int32_t n_rep, mdet_tune_result *out);

#ifdef __cplusplus
}
#endif
#endif /* MDET_H */
