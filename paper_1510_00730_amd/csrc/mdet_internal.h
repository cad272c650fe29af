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

// Device view of one spin channel of the expansion.
struct SpinDev {
    int32_t n;            // electrons of this spin
    int32_t e0;           // first electron index of this spin
    int32_t U;            // distinct determinants
    int32_t pad;
    const int32_t *occ0;  // [n] reference occupied orbitals, ascending
    const DetDesc *desc;  // [U] in execution order (ascending degree)
    const int32_t *gptr;  // [n*M+1] aggregation lists, target t = c*M + m
    const uint32_t *gent; // entries: d_exec << 8 | a << 4 | b
};

// Device view of the sparse coefficient matrix in execution indices.
struct SparseDev {
    int32_t U, V;
    int64_t Z;
    const int32_t *rptr;   // [U+1] CSR (rows = up determinants)
    const int32_t *rcol;   // [Z]
    const double *rval;    // [Z]
    const float *rval32;   // [Z]
    const int32_t *cptr;   // [V+1] CSC (columns = down determinants)
    const int32_t *crow;   // [Z]
    const double *cval;    // [Z]
    const float *cval32;   // [Z]
};

// Per-call work buffers (device), sized for W walkers.
struct Work {
    int64_t W;
    int32_t M, N, nmax, Upad, Vpad;
    double *phi;       // [W][N][5][M] orbitals and derivatives, column-scaled
    int32_t *E;        // [W][2][M] per-spin column exponents
    double *X;         // [W][2][nmax*nmax] inverse of the scaled reference
    double *T;         // [W][2][nmax][M] table A^-1 Phi (scaled)
    double *g0;        // [W][N][4] grad~ D0 / D0
    double *logdet0;   // [W][2]
    double *sign0;     // [W][2]
    int32_t *flag;     // [W][2] 0 table method, 1 ill-conditioned, 2 singular
    int32_t *K;        // [W][2] exponent shift of the ratio vectors
    double *R64;       // [W][Upad+Vpad]
    float *R32;        // [W][Upad+Vpad]
    double *uv64;      // [W][Upad+Vpad]  u (up part) then v (down part)
    float *uv32;       // [W][Upad+Vpad]
    double *psi64;     // [W]
    float *psi32;      // [W]
};

struct KernelArgs {
    int32_t n_up, n_dn, N, M, P, nmax;
    double kappa_max;
    const Prim *prim;         // [M][P]
    SpinDev sp[2];
    SparseDev C;
    Work wk;
    int64_t W;
    const double *R;          // [W][N][3]
    const int8_t *max_degree; // [W] or null
    int32_t precision;
    double *sign_out, *logabs_out, *gl_out;
    int32_t *wstatus;
};

// Number of kernels of one evaluation (for per-kernel timing).
constexpr int kNumKernels = 7;
const char *kernel_name(int k);

// Launch the whole evaluation on `stream`; returns hipSuccess or the first
// error.  If `events` is not null, events[0..kNumKernels] are recorded on the
// stream before the first kernel and after each kernel.
hipError_t launch_eval(const KernelArgs &a, hipStream_t stream, hipEvent_t *events);

}  // namespace mdet
