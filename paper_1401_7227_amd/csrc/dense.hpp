// Dense kernels: the global coarse-grid correction of the Schwarz
// preconditioner (Section 3, eq. (3.5)-(3.8)) and exact local solves
// (Section 5).  Each small matrix is inverted on the device by Gauss-Jordan
// elimination with partial pivoting and applied as a dense product.
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstdint>

#include "plan.hpp"

namespace asmx {

// ---------------------------------------------------------------- one matrix
// M = 0 except the scattered 3x3 blocks of the block CSR (rp, ci, vals) of
// nbr block rows; Minv = I.  n = 3 nbr.
hipError_t launch_dense_init(int nbr, const int32_t *rp, const int32_t *ci, const double *vals, double *M,
                             double *Minv, hipStream_t s);
// Minv <- M^-1 (M is destroyed; fcol: n doubles of scratch).  A zero or
// non-finite pivot writes its column to *bad (which must hold -1 before).
hipError_t launch_gauss_jordan(int n, double *M, double *Minv, double *fcol, int *bad, hipStream_t s);
// y = Minv x (n x n, row-major).
hipError_t launch_dense_gemv(int n, const double *Minv, const double *x, double *y, hipStream_t s);
// z[3c+q] += xc[3 cvar[c] + q] for every cell c < N (prolongation R_C^T).
hipError_t launch_prolong_add(int N, const int32_t *cvar, const double *xc, double *z, hipStream_t s);

// ---------------------------------------------------------------- one matrix per subdomain
// The local matrices of all subdomains, each of order 3 sub[s].n, stored
// row-major from doff[s], rows and columns in the subdomain's forward sweep
// order (lpos: per extended row, its position in that order).
struct DenseLocal {
  int32_t nsub;
  const SubDesc *sub;
  const int64_t *doff;
  const int32_t *lpos;
  const int32_t *psub;  // per global position: its subdomain
  const int32_t *pout;  // per global position: owned cell (restricted output) or -1
  const int32_t *pbpos; // per global position: backward position of the row
  double *M, *Minv;
  double *fcol;         // 3 ext rows of scratch
  int *bad;             // per subdomain, -1 or the failing column
};
// M = the assembled A_i (CSR arp/aci/aval of the factorisation plan,
// permuted to sweep order), Minv = I, bad = -1.
hipError_t launch_local_dense_init(const DenseLocal &d, const int32_t *arp, const int32_t *aci, const double *aval,
                                   int max_n3, hipStream_t s);
hipError_t launch_local_gauss_jordan(const DenseLocal &d, int max_n3, hipStream_t s);
// Local solves of all subdomains on the gathered right-hand sides rs
// (forward order); results go to z (owned fine rows, restricted combine) or
// to yx at backward positions (additive combine).
hipError_t launch_local_dense_apply(const DenseLocal &d, int64_t npos, const double *rs, bool restricted, double *z,
                                    double *yx, hipStream_t s);

}  // namespace asmx
