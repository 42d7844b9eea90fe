// Device-side data layout shared by the host setup and the HIP kernels.
//
// A preconditioner is a set of subdomains; subdomain s owns "extended rows"
// ext_off .. ext_off+n-1 (its fine cells, then its coarse rows), stored in a
// global CSR (entries sorted by local column) from which the factors are
// computed, and re-laid out per level step for the triangular solves.
#pragma once
#include <cstdint>

namespace asmx {

// Rows of one level-schedule step.  All rows of a step share one level, so
// they can be processed concurrently; consecutive steps are separated by a
// workgroup barrier.
//   mode 0: one thread per row; entries stored ELL-style, slot (k, j) of
//           the step's rows in structure-of-arrays order (coalesced).
//   mode 1: one 64-wide wavefront per row; entries of each row contiguous,
//           located by a per-step relative row pointer.
struct Step {
  int32_t pos;    // first position in the step row list
  int32_t nrows;  // rows in the step
  int32_t width;  // mode 0: max entries per row
  int32_t eoff;   // first block slot of the step's entries
  int32_t mode;   // 0 or 1
  int32_t rptr;   // mode 1: offset of the relative row pointer (nrows+1)
  int32_t fp32;   // 1 if the step's blocks are held in single precision
  int32_t pad;
};

struct SubDesc {
  int32_t ext_off;    // first extended row (global)
  int32_t n;          // rows of A_i
  int32_t nfine;      // fine rows of A_i
  int32_t fstep0, fstep1;  // forward steps [fstep0, fstep1)
  int32_t bstep0, bstep1;  // backward steps
  int32_t pad;
};

// Pointers handed to the apply / factor kernels.
struct DevPlan {
  int32_t nsub;
  const SubDesc *sub;
  const Step *fstep, *bstep;
  const int32_t *frow, *brow;    // local row of each step position
  const int32_t *fcol, *bcol;    // local column of each block slot, -1 pad
  const int32_t *frptr, *brptr;  // mode-1 relative row pointers
  const double *fval, *bval;     // block values (FP64 steps)
  const float *fval32, *bval32;  // block values (FP32 steps)
  const double *bdinv;           // D^-1 per backward position, SoA per step
  const float *bdinv32;
  const int32_t *rhs_src;        // per ext row: cell >= 0, or -(1+coarse row)
  const int32_t *out_cell;       // per ext row: cell written by a restricted
                                 // combine, -1 if none
  double *yext;                  // 3 doubles per ext row (work vector)
  const double *crhs;            // 3 doubles per coarse row (lumped rhs)
  // factorisation
  const int32_t *arp;            // per ext row: first CSR entry (global)
  const int32_t *aci;            // per entry: local column
  const int32_t *adiag;          // per ext row: CSR entry of the diagonal
  const int32_t *tptr;           // per entry: first update pair
  const int32_t *tdst, *tsrc;    // update pairs: a[dst] -= L * a[src]
  double *fact;                  // CSR values being factorised
};

}  // namespace asmx
