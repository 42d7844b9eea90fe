// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstddef>
#include <cstdint>

#include "plan.hpp"
#include "asm.h"

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

constexpr int kReduceBlocks = 1024;     // partial-sum blocks of the Krylov kernels (default)
constexpr int kMaxReduceBlocks = 4096;  // largest choice of the tuner (buffers are sized for it)
constexpr int kMaxRestart = 32;
// Doubles of a system's partial-sum buffer for N block rows: the Krylov
// kernels' (restart + 2 columns of at most kMaxReduceBlocks blocks) or the
// residual SpMV's (one per 256-row block, rounded up to 8).
inline int64_t partial_doubles(int64_t N) {
  const int64_t krylov = (int64_t)kMaxReduceBlocks * (kMaxRestart + 2);
  const int64_t resid = ((N + 255) / 256 + 7) / 8 * 8;
  return krylov > resid ? krylov : resid;
}

// The launchers of the kernels an Arnoldi step runs take an optional skip
// flag (device): a kernel whose flag is set returns at once.  A restart
// cycle captured as one graph sets it when the cycle ends on the device.

hipError_t launch_sell_fill(const SellDev &A, const double *csr_vals, hipStream_t s);
// rows: block rows per thread (1, 2 or 4; the same results, a tuning choice).
hipError_t launch_spmv(const SellDev &A, const double *x, double *y, hipStream_t s, const int *skip = nullptr,
                       int rows = 1);
// r = b - A x; partial[kReduceBlocks-sized region] receives per-block sums of r.r
hipError_t launch_residual(const SellDev &A, const double *x, const double *b, double *r,
                           double *partial, int *nblocks_out, hipStream_t s);

hipError_t launch_gather_sum9(int ndst, const int32_t *ptr, const int32_t *idx,
                              const double *srcA, int32_t nA, const double *srcB, double *dst,
                              hipStream_t s);
// dst[d] = scale * sum of src over idx[ptr[d] .. ptr[d+1]) (3 doubles per
// entry).  Destinations [0, n1) take lanes1 threads each, [n1, n) lanes2
// (powers of two, 1 .. 64).
hipError_t launch_gather_sum3(int n1, int lanes1, int n, int lanes2, const int32_t *ptr, const int32_t *idx,
                              const double *src, const double *scale, double *dst, hipStream_t s,
                              const int *skip = nullptr);
// Blocks of 256 threads of that launch.
inline int gather_sum3_blocks(int n1, int lanes1, int n, int lanes2) {
  return (int)(((int64_t)n1 * lanes1 + 255) / 256 + ((int64_t)(n - n1) * lanes2 + 255) / 256);
}

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
// Forward right-hand sides of all subdomains in sweep order (p.rs), for
// the dense local solves.
hipError_t launch_gather_rhs(int npos, const ApplyPlan &p, const double *r, const double *scale, hipStream_t s);
// Lumped inputs of the coarse rows (p.crs) from the near/far atom sums.
hipError_t launch_coarse_rhs(const ApplyPlan &p, hipStream_t s, const int *skip = nullptr);
// Both sweeps; the forward sweep gathers its inputs from r (times *scale,
// if scale is not NULL) and p.crs.
hipError_t launch_ilu_apply(const ApplyPlan &p, const double *r, const double *scale, double *z, hipStream_t s,
                            const int *skip = nullptr);
hipError_t launch_additive_combine(int N, const int32_t *cptr, const int32_t *cidx,
                                   const double *yext, double *z, hipStream_t s, const int *skip = nullptr);

// Krylov kernels (n = scalar length).
// U columns (stride ldu, even) and w must be 16-byte aligned.
// max_blocks: the partial-sum block count (at most kMaxReduceBlocks; a
// tuning choice that decides the summation order).
hipError_t launch_multidot(int64_t n, int nv, const double *U, int64_t ldu, const double *w,
                           double *partial, int *nblocks_out, hipStream_t s, const int *skip = nullptr,
                           int max_blocks = kReduceBlocks);
hipError_t launch_reduce_cols(int nblocks, int ncols, const double *partial, double *out,
                              hipStream_t s, const int *skip = nullptr);
// unew = w - sum_{i<nv} (scale[i] d[i]) scale[i] U_i, d the reduced
// projections of the step; per-block partial sums of ||unew||^2.
hipError_t launch_update(int64_t n, int nv, const double *U, int64_t ldu, const double *d,
                         const double *scale, const double *w, double *unew, double *partial,
                         int *nblocks_out, hipStream_t s, const int *skip = nullptr,
                         int max_blocks = kReduceBlocks);
// One block: h = sqrt(sum of partial[0..nblocks)) into hcol[nv], 1/h (0 if
// h = 0) into *scale_out, hcol[i] = scale[i]*d[i] for i < nv; if pub is not
// NULL, hcol[0..nv] and sqrt(d[nv]) are also written to pub[0..nv+1].
hipError_t launch_norm_finalize(int nblocks, const double *partial, int nv, const double *d, const double *scale,
                                double *hcol, double *scale_out, double *pub, hipStream_t s,
                                const int *skip = nullptr);
hipError_t launch_lincomb(int64_t n, int nv, const double *U, int64_t ldu, const double *coef,
                          double *out, hipStream_t s);
hipError_t launch_axpy(int64_t n, const double *z, double *x, hipStream_t s);

hipError_t launch_check_finite(int64_t n, const double *v, int *flag, hipStream_t s);
// p[0 .. n) = v.
hipError_t launch_fill(int64_t n, double v, double *p, hipStream_t s);
hipError_t launch_fill(int64_t n, int v, int *p, hipStream_t s);

// The fixed device array of the no-allocation solve (asm_solve_noalloc):
// its address on the current device, looked up on the first call per device.
constexpr size_t kNoAllocScratchBytes = (size_t)ASM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(void **out);

// ---------------------------------------------------------------- device-side restart cycles
// State of a restart cycle that runs on the device (a captured graph): done
// is the step kernels' skip flag, k the steps taken, kmax the steps allowed
// (written by the host before each cycle), use_tol / tol the stopping test
// on the residual estimate |g_k|.
struct CycleState {
  int done, k, kmax, use_tol;
  double tol;
};
// done = 0, k = 0, g[0] = *beta.
hipError_t launch_cycle_start(CycleState *st, double *g, const double *beta, hipStream_t s);
// Givens step j: rotates column j of H (leading dimension ld) by the
// earlier rotations, forms rotation j, updates g, sets k = j+1 and done on a
// breakdown (h_{j+1,j} <= 1e-14 ||w||, ||w||^2 = d[j+1]), on |g_{j+1}| <= tol
// or at kmax steps.  Does nothing once done is set.
hipError_t launch_givens(int j, int ld, double *H, double *cs, double *sn, double *g, const double *d,
                         CycleState *st, hipStream_t s);
// y from the rotated H and g (k = st->k rows), coef[i] = y[i] * scale[i].
hipError_t launch_cycle_end(int ld, const double *H, const double *g, const double *scale, double *coef,
                            const CycleState *st, hipStream_t s);
// out = sum_{i < st->k} coef[i] U_i.
hipError_t launch_lincomb_dev(int64_t n, const CycleState *st, const double *U, int64_t ldu, const double *coef,
                              double *out, hipStream_t s);
// pub[0] = k, pub[1] = *beta, pub[2] = |g_k| (pinned host memory).
hipError_t launch_cycle_publish(const CycleState *st, const double *g, const double *beta, double *pub,
                                hipStream_t s);
hipError_t launch_norm2(int64_t n, const double *v, double *partial, int *nblocks_out, hipStream_t s);
hipError_t launch_scale_copy(int64_t n, const double *r, const double *scale, double *z, hipStream_t s,
                             const int *skip = nullptr);

// ---------------------------------------------------------------- batches
// One system of a batched solve: what the batched kernels read (device
// table, one entry per system).  Vectors are the system's own workspace.
struct BatchSys {
  int64_t n, ldu;
  int32_t red_blocks, pad_;  // partial-sum blocks of the Krylov kernels (the system's tuned choice)
  double *U, *w, *z, *t, *partial, *dvec, *H, *scale, *misc;
  double *pub;          // pinned (device view): published Hessenberg columns
  const double *coefh;  // pinned (device view): [0] = k, [1..k] = solution coefficients
  const double *b;
  double *x;
  int32_t N, nlog;
  const int32_t *sptr, *cols;
  const double *vals;
  int32_t kind, restricted, npos, nsub;
  ApplyPlan ap;
  int32_t c1n, c1n1, c1lanes, c1lanes2, c2n, c2n1, c2lanes, c2lanes2;
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
  kBkC1, kBkC2, kBkCrs, kBkApply, kBkCombine, kBkCopy, kBkSpmv, kBkRed, kBkVec, kBkOne, kBkCount
};
int batch_blocks(BatchKernel k, const BatchSys &s);

// In every batched launcher, `col` selects the input of the preconditioner
// (basis column col with its scale, or t unscaled when col < 0).
hipError_t launch_batch_precond(const BatchSys *tab, const BatchSeg *seg, int col, hipStream_t s);
hipError_t launch_batch_spmv(const BatchSys *tab, const BatchSeg &seg, bool residual, hipStream_t s);
hipError_t launch_batch_multidot(const BatchSys *tab, const BatchSeg &seg, int nv, hipStream_t s);
// src 0: partial sums of the CGS kernels, 1: of the residual SpMV.
hipError_t launch_batch_reduce(const BatchSys *tab, const BatchSeg &seg, int ncols, bool dots, int src, hipStream_t s);
hipError_t launch_batch_update(const BatchSys *tab, const BatchSeg &seg, int nv, int ldh, hipStream_t s);
// Reduces the partial sums (src as for launch_batch_reduce) and finalises:
// j >= 0: step j (norm of the new basis vector, column published at
// pub + j*pub_stride); j < 0: true residual norm (beta published at pub[-1]).
hipError_t launch_batch_norm_finalize(const BatchSys *tab, const BatchSeg &seg, int j, int ldh, int pub_stride,
                                      int src, hipStream_t s);
hipError_t launch_batch_lincomb(const BatchSys *tab, const BatchSeg &seg, hipStream_t s);
hipError_t launch_batch_axpy(const BatchSys *tab, const BatchSeg &seg, hipStream_t s);

}  // namespace asmx
