// Global coarse-grid correction of the Schwarz preconditioner (Section 3,
// eq. (3.5)-(3.8)): A_C is inverted densely on the device and applied as a
// dense matrix-vector product.
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstdint>

namespace asmx {

// M = 0 except the scattered 3x3 blocks of the block CSR (rp, ci, vals) of
// nbr block rows; Minv = I.  n = 3 nbr.
hipError_t launch_dense_init(int nbr, const int32_t *rp, const int32_t *ci, const double *vals, double *M,
                             double *Minv, hipStream_t s);
// Minv <- M^-1 by Gauss-Jordan elimination with partial pivoting (M is
// destroyed; fcol: n doubles of scratch).  A zero or non-finite pivot
// writes its column to *bad (which must hold -1 before).
hipError_t launch_gauss_jordan(int n, double *M, double *Minv, double *fcol, int *bad, hipStream_t s);
// y = Minv x (n x n, row-major).
hipError_t launch_dense_gemv(int n, const double *Minv, const double *x, double *y, hipStream_t s);
// z[3c+q] += xc[3 cvar[c] + q] for every cell c < N (prolongation R_C^T).
hipError_t launch_prolong_add(int N, const int32_t *cvar, const double *xc, double *z, hipStream_t s);

}  // namespace asmx
