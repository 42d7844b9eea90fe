// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstddef>
#include <cstdint>

#include "plan.hpp"

namespace asmx {

// Sliced ELL layout of A: slices of 64 block rows (one wavefront); slice s
// holds groups sptr[s]..sptr[s+1]-1, group g holds one block per row of the
// slice: cols[g*64 + lane], block entry e at vals[(g*9 + e)*64 + lane].
struct SellDev {
  int32_t N = 0, nslices = 0, ngroups = 0;
  int32_t *sptr = nullptr;   // [nslices+1]
  int32_t *cols = nullptr;   // [ngroups*64]
  int32_t *src = nullptr;    // [ngroups*64] CSR entry feeding each slot, -1 pad
  double *vals = nullptr;    // [ngroups*9*64]
};

constexpr int kReduceBlocks = 1024;  // partial-sum blocks of the Krylov kernels
constexpr int kMaxRestart = 32;

hipError_t launch_sell_fill(const SellDev &A, const double *csr_vals, hipStream_t s);
hipError_t launch_spmv(const SellDev &A, const double *x, double *y, hipStream_t s);
// r = b - A x; partial[kReduceBlocks-sized region] receives per-block sums of r.r
hipError_t launch_residual(const SellDev &A, const double *x, const double *b, double *r,
                           double *partial, int *nblocks_out, hipStream_t s);

hipError_t launch_gather_sum9(int ndst, const int32_t *ptr, const int32_t *idx,
                              const double *srcA, int32_t nA, const double *srcB, double *dst,
                              hipStream_t s);
// lanes (1, 2, 4, 8 or 16) threads share each destination.
hipError_t launch_gather_sum3(int ndst, int lanes, const int32_t *ptr, const int32_t *idx, const double *src,
                              const double *scale, double *dst, hipStream_t s);

// Level-scheduled block ILU(0) of every subdomain; singular pivots reported
// through *bad as (subdomain << 32 | local row), minimum over all.
hipError_t launch_ilu_factor(const DevPlan &p, unsigned long long *bad, hipStream_t s);
// Copy factor blocks from CSR into the step layouts (FP64 and FP32 targets).
hipError_t launch_relayout(int nslots, const int32_t *src, const int32_t *base,
                           const int32_t *stride, const uint8_t *to32, const double *fact,
                           double *out64, float *out32, hipStream_t s);
// z = B^-1 (scale * r) over all subdomains: owned rows of a restricted
// combine go straight into z; values needed by the additive combine are in
// the plan's global work vector.
// Forward right-hand sides of all subdomains in sweep order (p.rs).
hipError_t launch_gather_rhs(int npos, const ApplyPlan &p, const double *r, const double *scale, hipStream_t s);
hipError_t launch_ilu_apply(const ApplyPlan &p, double *z, hipStream_t s);
hipError_t launch_additive_combine(int N, const int32_t *cptr, const int32_t *cidx,
                                   const double *yext, double *z, hipStream_t s);

// Krylov kernels (n = scalar length).
// U columns (stride ldu, even) and w must be 16-byte aligned.
hipError_t launch_multidot(int64_t n, int nv, const double *U, int64_t ldu, const double *w,
                           double *partial, int *nblocks_out, hipStream_t s);
hipError_t launch_reduce_cols(int nblocks, int ncols, const double *partial, double *out,
                              hipStream_t s);
// After multidot of column j: H[j*ldh + i] = scale[i]*d[i] (i<=j), coef[i] =
// H[j*ldh+i]*scale[i], wnorm = sqrt(d[nv]).
hipError_t launch_finalize_dots(int nv, const double *d, const double *scale, double *Hcol,
                                double *coef, double *wnorm, hipStream_t s);
hipError_t launch_update(int64_t n, int nv, const double *U, int64_t ldu, const double *coef,
                         const double *w, double *unew, double *partial, int *nblocks_out,
                         hipStream_t s);
// hn = sqrt(nrm2[0]); *hout = hn; *scale_out = hn > 0 ? 1/hn : 0.
// h = sqrt(*nrm2) into hcol[nv], 1/h into *scale_out; if pub is not NULL,
// hcol[0..nv] and *wnorm are also written to pub[0..nv+1] (pinned host).
hipError_t launch_finalize_norm(int nv, const double *nrm2, double *hcol, double *scale_out, const double *wnorm,
                                double *pub, hipStream_t s);
hipError_t launch_lincomb(int64_t n, int nv, const double *U, int64_t ldu, const double *coef,
                          double *out, hipStream_t s);
hipError_t launch_axpy(int64_t n, const double *z, double *x, hipStream_t s);

hipError_t launch_check_finite(int64_t n, const double *v, int *flag, hipStream_t s);
hipError_t launch_norm2(int64_t n, const double *v, double *partial, int *nblocks_out, hipStream_t s);
hipError_t launch_scale_copy(int64_t n, const double *r, const double *scale, double *z, hipStream_t s);

// ---------------------------------------------------------------- batches
// One system of a batched solve: what the batched kernels read (device
// table, one entry per system).  Vectors are the system's own workspace.
struct BatchSys {
  int64_t n, ldu;
  double *U, *w, *z, *t, *partial, *dvec, *H, *scale, *coef, *misc;
  double *pub;          // pinned (device view): published Hessenberg columns
  const double *coefh;  // pinned (device view): [0] = k, [1..k] = solution coefficients
  const double *b;
  double *x;
  int32_t N, nlog;
  const int32_t *sptr, *cols;
  const double *vals;
  int32_t kind, restricted, npos, nsub;
  ApplyPlan ap;
  int32_t c1n, c1lanes, c2n, c2lanes;
  const int32_t *c1ptr, *c1idx, *c2ptr, *c2idx;
  double *PA, *PNF;
  const int32_t *cptr, *cidx;
};

// Blocks of one batched launch: block b works for system sys[k] when
// start[k] <= b < start[k+1] (local block b - start[k]); n segments.
struct BatchSeg {
  const int32_t *start, *sys;
  int32_t n, total;
};

// Blocks each kernel gives one system (the same as a single-system launch,
// so batched and single results are identical).
enum BatchKernel {
  kBkC1, kBkC2, kBkRhs, kBkApply, kBkCombine, kBkCopy, kBkSpmv, kBkRed, kBkVec, kBkOne, kBkCount
};
int batch_blocks(BatchKernel k, const BatchSys &s);

// In every batched launcher, `col` selects the input of the preconditioner
// (basis column col with its scale, or t unscaled when col < 0).
hipError_t launch_batch_precond(const BatchSys *tab, const BatchSeg *seg, int col, hipStream_t s);
hipError_t launch_batch_spmv(const BatchSys *tab, const BatchSeg &seg, bool residual, hipStream_t s);
hipError_t launch_batch_multidot(const BatchSys *tab, const BatchSeg &seg, int nv, hipStream_t s);
// src 0: partial sums of the CGS kernels, 1: of the residual SpMV.
hipError_t launch_batch_reduce(const BatchSys *tab, const BatchSeg &seg, int ncols, bool dots, int src, hipStream_t s);
hipError_t launch_batch_finalize_dots(const BatchSys *tab, const BatchSeg &seg, int j, int ldh, hipStream_t s);
hipError_t launch_batch_update(const BatchSys *tab, const BatchSeg &seg, int nv, int ldh, hipStream_t s);
// j >= 0: step j (norm of the new basis vector, column published at
// pub + j*pub_stride); j < 0: true residual norm (beta published at pub[-1]).
hipError_t launch_batch_finalize_norm(const BatchSys *tab, const BatchSeg &seg, int j, int ldh, int pub_stride,
                                      hipStream_t s);
hipError_t launch_batch_lincomb(const BatchSys *tab, const BatchSeg &seg, hipStream_t s);
hipError_t launch_batch_axpy(const BatchSys *tab, const BatchSeg &seg, hipStream_t s);

}  // namespace asmx
