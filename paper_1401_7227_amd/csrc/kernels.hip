// gfx950 kernels of the Schwarz-preconditioned GMRES solve.
//
// Everything on this path is HBM- or latency-bound (3x3 blocks are not a
// dense contraction), so the kernels are written for coalesced streaming
// with 64-wide wavefronts; no matrix cores are used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <mutex>
#include <utility>

#include "kernels.hpp"

namespace asmx {

namespace {

constexpr int kWave = 64;

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on
// XCD b % 8).  Remap so that each XCD walks a contiguous range of logical
// blocks: neighbouring rows then share that XCD's L2.  The grid is launched
// with 8 * ceil(nlogical / 8) blocks; logical indices >= nlogical are idle.
__device__ inline int xcd_logical_block(int nlogical, int b) {
  const int per = (nlogical + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

inline int xcd_grid(int nlogical) { return ((nlogical + 7) >> 3) << 3; }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Cross-lane moves inside the VALU (DPP), no LDS traffic.  CTRL is a DPP
// control: quad_perm 0xB1 (lanes xor 1), 0x4E (xor 2), 0x141 row half
// mirror (lane i <-> 7-i within 8), 0x140 row mirror (i <-> 15-i within 16).
// Every source lane of these controls is inside the same row of 16 lanes,
// so no lane reads outside the row (bound_ctrl set: no old value needed).
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp32(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_any(double v) { return dpp64<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ float dpp_any(float v) { return dpp32<CTRL>(v); }

// Sum over each group of 4 lanes (every lane of the group gets it); all
// lanes of the wave must be active.
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
  v += dpp_any<0xB1>(v);
  v += dpp_any<0x4E>(v);
  return v;
}

// Fixed-order block reduction (deterministic): wave butterflies, then the
// per-wave sums in wave order.  Result valid in thread 0.
template <int NT>
__device__ inline double block_sum(double v, double *lds) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) s += lds[i];
  }
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- SpMV
__global__ __launch_bounds__(256) void sell_fill_kernel(int nslots, const int32_t *__restrict__ src,
                                                        const double *__restrict__ csr,
                                                        double *__restrict__ vals) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  const int g = t >> 6, lane = t & 63;
  const int e = src[t];
#pragma unroll
  for (int q = 0; q < 9; ++q) vals[((size_t)g * 9 + q) * 64 + lane] = (e >= 0) ? csr[(size_t)e * 9 + q] : 0.0;
}

// y = A x, or (RESID) y = b - A x with per-block partial sums of y.y.
// One thread per block row; the 64 lanes of a wave cover one slice.
// Streaming loads: the matrix of the SpMV and the Krylov basis are read
// once per step and do not fit the caches, so they are loaded
// non-temporally (measured: SpMV and CGS kernels 4-9% faster).
typedef double d2v_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream2(const double2 *p) {
  const d2v_nt v = __builtin_nontemporal_load(reinterpret_cast<const d2v_nt *>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ double ld_stream(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int32_t ld_stream(const int32_t *p) { return __builtin_nontemporal_load(p); }

template <bool RESID>
__device__ __forceinline__ void spmv_body(int bid, int N, int nlogical, const int32_t *__restrict__ sptr,
                                          const int32_t *__restrict__ cols, const double *__restrict__ vals,
                                          const double *__restrict__ x, const double *__restrict__ b,
                                          double *__restrict__ y, double *__restrict__ partial, double *red) {
  const int lb = xcd_logical_block(nlogical, bid);
  double nrm = 0.0;
  const int row = lb * 256 + (int)threadIdx.x;
  if (lb < nlogical && row < N) {
    const int slice = row >> 6, lane = row & 63;
    const int g0 = sptr[slice], g1 = sptr[slice + 1];
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    for (int g = g0; g < g1; ++g) {
      const int c = ld_stream(cols + (size_t)g * 64 + lane);
      const double *v = vals + (size_t)g * 576 + lane;
      const double x0 = x[3 * (size_t)c], x1 = x[3 * (size_t)c + 1], x2 = x[3 * (size_t)c + 2];
      y0 += ld_stream(v) * x0 + ld_stream(v + 64) * x1 + ld_stream(v + 128) * x2;
      y1 += ld_stream(v + 192) * x0 + ld_stream(v + 256) * x1 + ld_stream(v + 320) * x2;
      y2 += ld_stream(v + 384) * x0 + ld_stream(v + 448) * x1 + ld_stream(v + 512) * x2;
    }
    if (RESID) {
      y0 = b[3 * (size_t)row] - y0;
      y1 = b[3 * (size_t)row + 1] - y1;
      y2 = b[3 * (size_t)row + 2] - y2;
      nrm = y0 * y0 + y1 * y1 + y2 * y2;
    }
    y[3 * (size_t)row] = y0;
    y[3 * (size_t)row + 1] = y1;
    y[3 * (size_t)row + 2] = y2;
  }
  if (RESID) {
    const double s = block_sum<256>(nrm, red);
    if (threadIdx.x == 0) partial[bid] = s;
  }
}

// R block rows per thread: thread t of logical block lb takes rows
// lb*256*R + k*256 + t, k < R (independent sums, more loads in flight per
// thread); every row's sum runs in the same order whatever R.
template <int R>
__global__ __launch_bounds__(256) void spmv_rows_kernel(int N, int nlogical, const int32_t *__restrict__ sptr,
                                                        const int32_t *__restrict__ cols,
                                                        const double *__restrict__ vals,
                                                        const double *__restrict__ x, double *__restrict__ y,
                                                        const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  const int lb = xcd_logical_block(nlogical, blockIdx.x);
  if (lb >= nlogical) return;
  int row[R], g0[R], g1[R];
  double a[R][3];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    row[k] = (lb * R + k) * 256 + (int)threadIdx.x;
    const int sl = (row[k] < N ? row[k] : 0) >> 6;
    g0[k] = row[k] < N ? sptr[sl] : 0;
    g1[k] = row[k] < N ? sptr[sl + 1] : 0;
    a[k][0] = a[k][1] = a[k][2] = 0.0;
  }
  int gmax = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) gmax = max(gmax, g1[k] - g0[k]);
  for (int q = 0; q < gmax; ++q) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (q < g1[k] - g0[k]) {
        const int g = g0[k] + q, lane = row[k] & 63;
        const int c = ld_stream(cols + (size_t)g * 64 + lane);
        const double *v = vals + (size_t)g * 576 + lane;
        const double x0 = x[3 * (size_t)c], x1 = x[3 * (size_t)c + 1], x2 = x[3 * (size_t)c + 2];
        a[k][0] += ld_stream(v) * x0 + ld_stream(v + 64) * x1 + ld_stream(v + 128) * x2;
        a[k][1] += ld_stream(v + 192) * x0 + ld_stream(v + 256) * x1 + ld_stream(v + 320) * x2;
        a[k][2] += ld_stream(v + 384) * x0 + ld_stream(v + 448) * x1 + ld_stream(v + 512) * x2;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (row[k] < N) {
      y[3 * (size_t)row[k]] = a[k][0];
      y[3 * (size_t)row[k] + 1] = a[k][1];
      y[3 * (size_t)row[k] + 2] = a[k][2];
    }
}

template <bool RESID>
__global__ __launch_bounds__(256) void spmv_kernel(int N, int nlogical, const int32_t *__restrict__ sptr,
                                                   const int32_t *__restrict__ cols,
                                                   const double *__restrict__ vals,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ b, double *__restrict__ y,
                                                   double *__restrict__ partial,
                                                   const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  __shared__ double red[4];
  spmv_body<RESID>(blockIdx.x, N, nlogical, sptr, cols, vals, x, b, y, partial, red);
}

// ---------------------------------------------------------------- gathers
__global__ __launch_bounds__(256) void gather_sum9_kernel(int ndst, const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ idx,
                                                          const double *__restrict__ srcA, int32_t nA,
                                                          const double *__restrict__ srcB,
                                                          double *__restrict__ dst) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= ndst) return;
  double acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  for (int t = ptr[d]; t < ptr[d + 1]; ++t) {
    const int sidx = idx[t];
    const double *p = (sidx < nA) ? srcA + (size_t)sidx * 9 : srcB + (size_t)(sidx - nA) * 9;
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] += p[q];
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) dst[(size_t)d * 9 + q] = acc[q];
}

// dst[d] = scale * sum of src over idx[ptr[d] .. ptr[d+1]), 3 doubles per
// entry.  Destinations [0, n1) take G1 lanes each and [n1, ndst) G2 lanes
// (powers of two up to 64), so that a segment of a few wide sums does not
// wait on lanes sized for many narrow ones.  The lanes of a destination
// combine their partial sums in a fixed butterfly order (deterministic).
// The first segment's blocks come first, so each block serves one segment.
__device__ __forceinline__ void gather_sum3_body(int bid, int n1, int G1, int ndst, int G2,
                                                 const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                 const double *__restrict__ src, const double *__restrict__ scale,
                                                 double *__restrict__ dst) {
  const int b1 = (int)(((int64_t)n1 * G1 + 255) / 256);
  const bool first = bid < b1;
  const int G = first ? G1 : G2;
  const int gid = (first ? bid : bid - b1) * 256 + (int)threadIdx.x;
  const int lg = 31 - __clz(G);
  int d = gid >> lg;
  const int lane = gid & (G - 1);
  if (first) {
    if (d >= n1) d = ndst;  // idle tail of the first segment
  } else {
    d += n1;
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (d < ndst) {
    for (int t = ptr[d] + lane; t < ptr[d + 1]; t += G) {
      const size_t q = (size_t)idx[t] * 3;
      a0 += src[q];
      a1 += src[q + 1];
      a2 += src[q + 2];
    }
  }
  for (int off = G / 2; off >= 1; off >>= 1) {
    a0 += __shfl_xor(a0, off, G);
    a1 += __shfl_xor(a1, off, G);
    a2 += __shfl_xor(a2, off, G);
  }
  if (d < ndst && lane == 0) {
    const double s = scale ? *scale : 1.0;
    dst[(size_t)d * 3] = s * a0;
    dst[(size_t)d * 3 + 1] = s * a1;
    dst[(size_t)d * 3 + 2] = s * a2;
  }
}

__global__ __launch_bounds__(256) void gather_sum3_kernel(int n1, int G1, int ndst, int G2,
                                                          const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ idx,
                                                          const double *__restrict__ src,
                                                          const double *__restrict__ scale,
                                                          double *__restrict__ dst,
                                                          const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  gather_sum3_body(blockIdx.x, n1, G1, ndst, G2, ptr, idx, src, scale, dst);
}

// ---------------------------------------------------------------- 3x3 block math
// Inverse by elimination with partial pivoting on [M | I]; returns false if a
// pivot column is exactly zero or the result is not finite.
__device__ inline bool invert3(const double *m, double *out) {
  double a[3][3], b[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      a[i][j] = m[3 * i + j];
      b[i][j] = (i == j) ? 1.0 : 0.0;
    }
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int p = c;
    double best = fabs(a[c][c]);
#pragma unroll
    for (int r = c + 1; r < 3; ++r) {
      const double v = fabs(a[r][c]);
      if (v > best) { best = v; p = r; }
    }
    ok = ok && (best > 0.0);
    if (p != c) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double t = a[c][j]; a[c][j] = a[p][j]; a[p][j] = t;
        t = b[c][j]; b[c][j] = b[p][j]; b[p][j] = t;
      }
    }
    const double inv = 1.0 / a[c][c];
#pragma unroll
    for (int j = 0; j < 3; ++j) { a[c][j] *= inv; b[c][j] *= inv; }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
#pragma unroll
      for (int j = 0; j < 3; ++j) { a[r][j] -= f * a[c][j]; b[r][j] -= f * b[c][j]; }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      out[3 * i + j] = b[i][j];
      ok = ok && isfinite(b[i][j]);
    }
  return ok;
}

__device__ inline void mat3mul(const double *x, const double *y, double *out) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      out[3 * i + j] = x[3 * i] * y[j] + x[3 * i + 1] * y[3 + j] + x[3 * i + 2] * y[6 + j];
}

// ---------------------------------------------------------------- ILU(0) factorisation
// One workgroup per subdomain, forward level steps in order; each row does
// the row-wise elimination of block ILU(0): for each lower entry (ascending)
// L = a_ik D_k^-1, then a_ij -= L U_kj over the precomputed update pairs;
// finally its pivot is inverted in place.
__global__ __launch_bounds__(256) void ilu_factor_kernel(DevPlan p, unsigned long long *bad) {
  const SubDesc sd = p.sub[blockIdx.x];
  for (int si = sd.fstep0; si < sd.fstep1; ++si) {
    const Step st = p.fstep[si];
    for (int j = threadIdx.x; j < st.nrows; j += blockDim.x) {
      const int u = p.frow[st.pos + j];
      const int gi = sd.ext_off + u;
      const int e0 = p.arp[gi], e1 = p.arp[gi + 1];
      for (int e = e0; e < e1; ++e) {
        const int k = p.aci[e];
        if (k >= u) break;
        double L[9], a[9], dk[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) { a[q] = p.fact[(size_t)e * 9 + q]; dk[q] = p.fact[(size_t)p.adiag[sd.ext_off + k] * 9 + q]; }
        mat3mul(a, dk, L);
#pragma unroll
        for (int q = 0; q < 9; ++q) p.fact[(size_t)e * 9 + q] = L[q];
        for (int t = p.tptr[e]; t < p.tptr[e + 1]; ++t) {
          const size_t dd = (size_t)p.tdst[t] * 9, ss = (size_t)p.tsrc[t] * 9;
          double uk[9], prod[9];
#pragma unroll
          for (int q = 0; q < 9; ++q) uk[q] = p.fact[ss + q];
          mat3mul(L, uk, prod);
#pragma unroll
          for (int q = 0; q < 9; ++q) p.fact[dd + q] -= prod[q];
        }
      }
      double d[9], dinv[9];
      const size_t de = (size_t)p.adiag[gi] * 9;
#pragma unroll
      for (int q = 0; q < 9; ++q) d[q] = p.fact[de + q];
      if (!invert3(d, dinv)) {
        atomicMin(bad, ((unsigned long long)blockIdx.x << 32) | (unsigned)u);
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) p.fact[de + q] = dinv[q];
    }
    __threadfence_block();
    __syncthreads();
  }
}

// Copies factor blocks into their record slots.  kind bit 0: FP32
// destination; bit 1: "granule" layout of a short-row section, where
// stride packs the section's entry count S (low 16 bits) and the entry q
// (high 16 bits): components are grouped in 16-byte granules (2 doubles
// or 4 floats) stored plane by plane, granule g of entry q at
// [g*W*S + W*q], the ninth component at [8*S + q] (W values per granule);
// otherwise component c goes to base + c*stride.
__global__ __launch_bounds__(256) void relayout_kernel(int nslots, const int32_t *__restrict__ src,
                                                       const int32_t *__restrict__ base,
                                                       const int32_t *__restrict__ stride,
                                                       const uint8_t *__restrict__ kind,
                                                       const double *__restrict__ fact,
                                                       double *__restrict__ out64,
                                                       float *__restrict__ out32) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  const int e = src[t];
  const size_t b0 = (size_t)base[t];
  const int k = kind ? kind[t] : 0;
  const bool f32 = k & 1;
  const int st = stride[t];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    size_t off;
    if (k & 2) {
      const int S = st & 0xffff, q = (int)((unsigned)st >> 16), W = f32 ? 4 : 2;
      off = (c < 8) ? b0 + (size_t)(c / W) * W * S + (size_t)W * q + c % W : b0 + 8 * (size_t)S + q;
    } else {
      off = b0 + (size_t)c * st;
    }
    const double v = (e >= 0) ? fact[(size_t)e * 9 + c] : 0.0;
    if (f32) out32[off] = (float)v;
    else out64[off] = v;
  }
}

// ---------------------------------------------------------------- ILU(0) apply
// One workgroup per subdomain runs its forward sweep y = L^-1 R_i r and
// backward sweep x = U^-1 y (D^-1 applied per row).  Every level step is a
// contiguous record (see RecStep) that the streaming waves copy from HBM,
// together with the step's row inputs (forward: gathered from r and the
// coarse rows' lumped inputs; backward: the forward results), straight into
// one of kRecBufs LDS buffers (gfx950's buffer loads to LDS: the data goes
// from memory to LDS without passing through registers): step s is
// computed from buffer s % kRecBufs while the records of the next
// kRecBufs - 1 steps are on their way.  The computing waves touch global
// memory only to store results: vector values live in an LDS slot pool, and
// values without a slot are reloaded into LDS by "fill" steps.
constexpr int kRecU4 = kRecBytes / 16;
constexpr int kRounds = (kRecU4 + 255) / 256;  // 1 KiB chunk loads per streaming wave and record
static_assert(kRecChunk == 64 * 16, "a chunk is one wave's 16-byte load");
static_assert(kMaxStepRows <= 8 * kInRowsPerLoad, "row inputs: two loads of 32 rows per streaming wave");

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
#ifndef ASM_SWEEP_COMPUTE_WAVES
#define ASM_SWEEP_COMPUTE_WAVES 8
#endif
constexpr int kConsumerThreads = 64 * ASM_SWEEP_COMPUTE_WAVES;  // computing waves of the sweep
constexpr int kSweepThreads = kConsumerThreads + 256;           // plus four streaming waves

// Explicit address spaces: LDS reads must never become generic (flat)
// accesses, whose completion is tracked together with global memory.
#define ASMX_LDS __attribute__((address_space(3)))
#define ASMX_GLB __attribute__((address_space(1)))
typedef ASMX_LDS double lds_double;
typedef const ASMX_LDS double lds_cdouble;
typedef const ASMX_GLB double glb_cdouble;
typedef ASMX_GLB double glb_double;
typedef ASMX_LDS void lds_void;
typedef const ASMX_GLB void glb_cvoid;

// Global memory by its own address space.  A pointer the kernel reads from
// memory (the batched launches take their plans from a table) is generic
// to the compiler, and a generic (flat) access is counted with the LDS
// accesses too: every wait for the LDS stores before a barrier would then
// also wait for the record loads in flight.
template <typename T>
__device__ __forceinline__ const ASMX_GLB T *glb(const T *p) {
  return (const ASMX_GLB T *)p;
}
template <typename T>
__device__ __forceinline__ ASMX_GLB T *glb(T *p) {
  return (ASMX_GLB T *)p;
}
// A small plan struct read word by word through a global pointer.
template <typename T>
__device__ __forceinline__ T ld_glb(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  T v;
  const ASMX_GLB int32_t *q = (const ASMX_GLB int32_t *)p;
  int32_t *o = reinterpret_cast<int32_t *>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = q[i];
  return v;
}

template <typename T>
__device__ __forceinline__ void block9(const T *v, int S, T (&b)[9]) {
#pragma unroll
  for (int e = 0; e < 9; ++e) b[e] = v[e * S];
}

// Block q of a short-row section in the granule layout (see relayout_kernel):
// 16-byte reads, five per FP64 block, three per FP32 block.
__device__ __forceinline__ void granule9(const double *sec, int S, int q, double (&b)[9]) {
  const double2 *g = reinterpret_cast<const double2 *>(sec);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double2 v = g[u * S + q];
    b[2 * u] = v.x;
    b[2 * u + 1] = v.y;
  }
  b[8] = sec[8 * S + q];
}
__device__ __forceinline__ void granule9(const float *sec, int S, int q, float (&b)[9]) {
  const float4 *g = reinterpret_cast<const float4 *>(sec);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const float4 v = g[u * S + q];
    b[4 * u] = v.x;
    b[4 * u + 1] = v.y;
    b[4 * u + 2] = v.z;
    b[4 * u + 3] = v.w;
  }
  b[8] = sec[8 * S + q];
}

struct SweepLds {
  u32x4 buf[kRecBufs][kRecU4];     // record of step s (read), of the next steps (arriving)
  double vec[3 * kVecSlots];       // vector slot pool (top kFillSlots: reloaded values)
  double part[4];                  // partial sum of a split row
  int32_t src[3][kMaxStepRows];    // gathering: input sources of three records (record k in slot k % 3)
  u32x4 trash[64];                 // destination of the loads that carry nothing
};
static_assert(sizeof(SweepLds) <= 160 * 1024, "the sweep's LDS must fit one CU");

// A record row's header (see RecHead): the result's LDS slot (-1: none),
// flags, entry count, and the index word (forward: the row's backward
// position; backward: the output cell or -1).
struct RowHead {
  int slot, flags, cnt, idx;
};
__device__ __forceinline__ RowHead row_head(int2 m) {
  RowHead r;
  const unsigned w = (unsigned)m.x;
  const int sl = (int)(w & 0xffff);
  r.slot = sl == kRecNoSlot ? -1 : sl;
  r.flags = (int)((w >> 16) & 3);
  r.cnt = (int)(w >> 18);
  r.idx = m.y;
  return r;
}

// Short rows of one section: four threads per row.  Thread r of a row
// takes the row's entries r and r+4 (jagged diagonals), the four partial
// sums are combined inside the quad (DPP), and thread r < 3 finishes
// component r of the result.  Sections with more rows than a quarter of
// the threads take several passes; waves without a row in a pass skip it.  tid, nthr: this thread among the nthr (a multiple of 64)
// threads given to the section; j0: first step row of the section; n: its rows; q0,
// q1: the starts of this thread's diagonals r and r+4 (in the section's
// values and in its dependency slots at slots_off alike); dinv rows of the
// section start at index doff of a plane of dstride rows; sc: the basis
// scale of the forward inputs flagged as cell values.
// The critical path is kept to two LDS round trips per pass: the row's
// header, dependency slots, input, D^-1 row and its first entry's block
// are read together (the block unconditionally: a thread without that
// entry reads some other word of LDS and its product is discarded), then
// the dependency values.
template <bool FWD, typename T>
__device__ __forceinline__ void short_rows(const char *recp, SweepLds &L, double *__restrict__ yx,
                                           double *__restrict__ z, int tid, int nthr, int spos, int j0, int n, int q0,
                                           int q1, int nslots, int slots_off, int vals_off, int dinv_off, int dstride,
                                           int doff, int in_off, double sc) {
  const int rows_per_pass = nthr / 4;
  lds_cdouble *vec = (lds_cdouble *)L.vec;
  const int r = tid & 3;
  const char *rows = recp + kRecHead;
  const T *vals = reinterpret_cast<const T *>(recp + vals_off);
  const ASMX_LDS uint16_t *sl = (const ASMX_LDS uint16_t *)(recp + slots_off);
  const int qmax = max(nslots - 1, 0);
  const double *inb = reinterpret_cast<const double *>(recp + in_off);
  const int rc = r < 3 ? r : 2;
  for (int i0 = 0; i0 < n; i0 += rows_per_pass) {
    if (i0 + ((tid & ~63) >> 2) >= n) break;  // no row of this wave in the pass (uniform)
    const int i = i0 + (tid >> 2);
    const bool act = i < n;
    const int ia = act ? i : 0;
    const int j = j0 + ia;
    const RowHead m = row_head(*reinterpret_cast<const int2 *>(rows + kRecRowBytes * j));
    // the dependency slot of entry r (any word of the array for a thread
    // without that entry: its product is discarded)
    const int da = sl[min(q0 + ia, qmax)];
    T a0, a1, a2, e0 = 0, e1 = 0, e2 = 0;
    double x = 0.0;
    if (FWD) {
      x = inb[4 * j + rc + (rc >> 1)];
      a1 = a2 = 0;
    } else {
      a0 = (T)inb[4 * j]; a1 = (T)inb[4 * j + 1]; a2 = (T)inb[4 * j + 3];
      const T *dv = reinterpret_cast<const T *>(recp + dinv_off) + doff + ia + 3 * rc * dstride;
      e0 = dv[0]; e1 = dv[dstride]; e2 = dv[2 * dstride];
    }
    T b[9];
    granule9(vals, nslots, q0 + ia, b);
    const int cnt = act ? m.cnt : 0;
    if (FWD) a0 = (T)((m.flags & 2) ? sc * x : x);  // a cell value of r times the basis scale
    const bool has0 = r < cnt;
    const int d0 = has0 ? da : 0;
    const T u0 = (T)vec[3 * d0], u1 = (T)vec[3 * d0 + 1], u2 = (T)vec[3 * d0 + 2];
    const T t0 = b[0] * u0 + b[1] * u1 + b[2] * u2;
    const T t1 = b[3] * u0 + b[4] * u1 + b[5] * u2;
    const T t2 = b[6] * u0 + b[7] * u1 + b[8] * u2;
    T s0 = has0 ? t0 : (T)0, s1 = has0 ? t1 : (T)0, s2 = has0 ? t2 : (T)0;
    if (r + 4 < cnt) {
      const int d1 = sl[q1 + i];
      T c[9];
      granule9(vals, nslots, q1 + i, c);
      const T v0 = (T)vec[3 * d1], v1 = (T)vec[3 * d1 + 1], v2 = (T)vec[3 * d1 + 2];
      s0 += c[0] * v0 + c[1] * v1 + c[2] * v2;
      s1 += c[3] * v0 + c[4] * v1 + c[5] * v2;
      s2 += c[6] * v0 + c[7] * v1 + c[8] * v2;
    }
    s0 = quad_sum(s0);
    s1 = quad_sum(s1);
    s2 = quad_sum(s2);
    if (act && r < 3) {
      T o;
      if (FWD) {
        o = a0 - (r == 0 ? s0 : (r == 1 ? s1 : s2));
      } else {
        o = e0 * (a0 - s0) + e1 * (a1 - s1) + e2 * (a2 - s2);
      }
      const double od = (double)o;
      if (m.slot >= 0) ((lds_double *)L.vec)[3 * m.slot + r] = od;
      if (m.flags & 1) glb(yx)[3 * (size_t)(FWD ? m.idx : spos + j) + r] = od;
      if (!FWD && m.idx >= 0) glb(z)[3 * (size_t)m.idx + r] = od;
    }
  }
}

// Long rows (FP64): sixteen threads (one DPP row) per row, striding over
// its entries, nthr / 16 rows at a time; the partial sums are combined inside
// the sixteen threads (DPP), and the first of them finishes the row.
// Pieces of a split row carry their partial sum in LDS.  The row's header,
// input and D^-1 are read before the entries, so that they are not on the
// critical path after the reduction.
constexpr int kLongLanes = 16;
template <bool FWD>
__device__ __forceinline__ void long_rows(const char *recp, SweepLds &L, double *__restrict__ yx,
                                          double *__restrict__ z, int tid, int nthr, int spos, int j0, int n,
                                          int piece, int deps_off, int rptr_off, int vals_off, int dinv_off,
                                          int dstride, int doff, int in_off, double sc) {
  const int groups = nthr / kLongLanes;
  const int lane = tid % kLongLanes, grp = tid / kLongLanes;
  lds_cdouble *vec = (lds_cdouble *)L.vec;
  const int32_t *deps = reinterpret_cast<const int32_t *>(recp + deps_off);
  const int32_t *rptr = reinterpret_cast<const int32_t *>(recp + rptr_off);
  const double *vals = reinterpret_cast<const double *>(recp + vals_off);
  // the loop bound is the same for all sixteen threads of a row, and the
  // DPP reductions stay inside them
  for (int i = grp; i < n; i += groups) {
    const int j = j0 + i;
    const RowHead m = row_head(*reinterpret_cast<const int2 *>(recp + kRecHead + kRecRowBytes * j));
    const int e0 = rptr[i], e1 = rptr[i + 1];
    double a0, a1, a2;
    if (piece == kPieceMiddle || piece == kPieceLast) {
      a0 = L.part[0]; a1 = L.part[1]; a2 = L.part[2];
    } else {
      const double *inp = reinterpret_cast<const double *>(recp + in_off) + 4 * j;
      a0 = inp[0]; a1 = inp[1]; a2 = inp[3];
    }
    double dv[9] = {};
    if (!FWD && (piece == kPieceWhole || piece == kPieceLast)) {
      const double *dp = reinterpret_cast<const double *>(recp + dinv_off) + doff + i;
#pragma unroll
      for (int e = 0; e < 9; ++e) dv[e] = dp[e * dstride];
    }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = e0 + lane; q < e1; q += kLongLanes) {
      const int d = deps[q];
      const double *b = vals + 9 * q;
      const double y0 = vec[3 * d], y1 = vec[3 * d + 1], y2 = vec[3 * d + 2];
      s0 += b[0] * y0 + b[1] * y1 + b[2] * y2;
      s1 += b[3] * y0 + b[4] * y1 + b[5] * y2;
      s2 += b[6] * y0 + b[7] * y1 + b[8] * y2;
    }
    // sums over the sixteen threads: quads, then halves, then the row
    s0 = quad_sum(s0); s1 = quad_sum(s1); s2 = quad_sum(s2);
    s0 += dpp64<0x141>(s0); s1 += dpp64<0x141>(s1); s2 += dpp64<0x141>(s2);
    s0 += dpp64<0x140>(s0); s1 += dpp64<0x140>(s1); s2 += dpp64<0x140>(s2);
    if (lane == 0) {
      if (FWD && (m.flags & 2) && !(piece == kPieceMiddle || piece == kPieceLast)) {
        a0 = sc * a0; a1 = sc * a1; a2 = sc * a2;
      }
      a0 -= s0; a1 -= s1; a2 -= s2;
      if (piece == kPieceFirst || piece == kPieceMiddle) {
        L.part[0] = a0; L.part[1] = a1; L.part[2] = a2;
      } else {
        if (!FWD) {
          const double x0 = dv[0] * a0 + dv[1] * a1 + dv[2] * a2;
          const double x1 = dv[3] * a0 + dv[4] * a1 + dv[5] * a2;
          const double x2 = dv[6] * a0 + dv[7] * a1 + dv[8] * a2;
          a0 = x0; a1 = x1; a2 = x2;
        }
        lds_double *w = (lds_double *)L.vec;
        if (m.slot >= 0) { w[3 * m.slot] = a0; w[3 * m.slot + 1] = a1; w[3 * m.slot + 2] = a2; }
        if (m.flags & 1) {
          glb_double *g = glb(yx) + 3 * (size_t)(FWD ? m.idx : spos + j);
          g[0] = a0; g[1] = a1; g[2] = a2;
        }
        if (!FWD && m.idx >= 0) {
          glb_double *g = glb(z) + 3 * (size_t)m.idx;
          g[0] = a0; g[1] = a1; g[2] = a2;
        }
      }
    }
  }
}

// Fill step: reloads values of the next step that have no LDS slot of
// their own from the global vector (stored before an earlier barrier).
__device__ __forceinline__ void fill_values(const RecHead &h, const char *recp, SweepLds &L,
                                            const double *__restrict__ yx) {
  const ASMX_LDS int32_t *fl = (const ASMX_LDS int32_t *)(recp + h.fill);
  lds_double *w = (lds_double *)L.vec;
  for (int q = threadIdx.x; q < h.nfill; q += kConsumerThreads) {
    const int gpos = fl[2 * q], slot = fl[2 * q + 1];
    glb_cdouble *src = (glb_cdouble *)yx + 3 * (size_t)gpos;
    const double v0 = src[0], v1 = src[1], v2 = src[2];
    w[3 * slot] = v0; w[3 * slot + 1] = v1; w[3 * slot + 2] = v2;
  }
}

// The sweep runs with wave-specialised roles.  The first
// ASM_SWEEP_COMPUTE_WAVES waves compute the steps; the last four waves
// only stream.  Both roles execute the same sequence of barriers.
//
// Streaming, per step s (every load goes straight to LDS; three record
// buffers shown, kRecBufs in general):
//   1. the step four ahead, s+4, is read from record s's head (in LDS
//      since the last barrier); gathering, its rows' input sources are
//      loaded into one of three source slots;
//   2. record s+2 is loaded into buffer (s+2) % 3, which step s-1 has left,
//      and its rows' inputs behind it (gathering: through the sources
//      loaded two steps earlier);
//   3. each streaming wave waits until record s+1 and (gathering) the
//      sources of record s+3 have landed (loads complete in issue order)
//      and joins the barrier that starts step s+1.
// Every streaming wave issues the same number of loads per step whatever
// the record's length (chunks past a record's end, and the loads of
// records past the sweep's end, go to a trash area), so the wait count is
// a compile-time constant; no load of the streaming waves writes a
// register.

// Where the streaming waves take a sweep's row inputs from.  Backward: the
// forward results, contiguous at the step's positions (src).  Forward
// (gather): the input of forward position q is sc * r[3c + k] for a fine
// row of cell c (fsrc[q] = c) or the lumped input crs[3j + k] of coarse row
// j (fsrc[q] = -(1 + j)): the restriction R_i r of Section 4 read straight
// from r, with no gathered copy in between.  The computing waves apply sc
// to the rows flagged as cell values.
struct SweepIn {
  const double *src;
  const int32_t *fsrc;
  const double *r, *crs;
};

// An LDS array of the sweep's shared struct by its own address space.
__device__ __forceinline__ ASMX_LDS u32x4 *lds(u32x4 *p) { return (ASMX_LDS u32x4 *)p; }
__device__ __forceinline__ ASMX_LDS int32_t *lds(int32_t *p) { return (ASMX_LDS int32_t *)p; }

// Wave-uniform copy of a step descriptor held in LDS (a record's head).
__device__ __forceinline__ RecStep desc_lds(const RecStep *p) {
  const ASMX_LDS int32_t *q = (const ASMX_LDS int32_t *)p;
  RecStep d;
  d.rec = __builtin_amdgcn_readfirstlane(q[0]);
  d.len = __builtin_amdgcn_readfirstlane(q[1]);
  d.pos = __builtin_amdgcn_readfirstlane(q[2]);
  d.nrows = __builtin_amdgcn_readfirstlane(q[3]);
  return d;
}

// Cache policy of the record loads: non-temporal (gfx950 cache-policy
// bit); records are read once per application.
constexpr int kNontemporalAux = 2;

// The streaming waves address memory through buffer resources built per
// step in scalar registers: a load's per-lane offset is a constant of the
// lane and its per-load offset a scalar, so issuing a load costs no vector
// instructions (the streaming waves share their SIMDs with computing waves,
// and every vector instruction of theirs delays a step).  Raw resource (no
// stride, no swizzle) over nbytes at p, gfx9 data-format word.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t buf_rsrc(const void *p, int nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, nbytes, 0x00020000);
}
// A value every lane holds, in a scalar register (the compiler may form a
// clamp of scalars with a vector instruction; a buffer resource built from
// a vector register would need a loop over distinct values).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A pointer every lane holds, in scalar registers (a plan read through a
// generic pointer arrives in vector registers).
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v), hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return reinterpret_cast<T *>(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ RecStep uniform_step(const RecStep &d) {
  RecStep u;
  u.rec = __builtin_amdgcn_readfirstlane(d.rec);
  u.len = __builtin_amdgcn_readfirstlane(d.len);
  u.pos = __builtin_amdgcn_readfirstlane(d.pos);
  u.nrows = __builtin_amdgcn_readfirstlane(d.nrows);
  return u;
}

// Per-lane byte offsets of the streaming loads.
struct LaneOff {
  unsigned rec;  // 16 * lane: record chunks
  unsigned src;  // 4 * lane: input sources
  unsigned in;   // backward inputs: 24 * (lane >> 1) + 8 * (lane & 1)
  int row, odd;  // forward inputs: lane >> 1, lane & 1
};

// Loads record d (live: a step of the sweep) into LDS buffer dst: chunk i
// of streaming wave w holds 16-byte words i*256 + w*64 .. +63.  Each chunk
// has a resource of its own that ends with the record, so lanes past the
// end fetch nothing (whatever they write lands in the rest of the record's
// last chunk, before the inputs); chunks wholly past the end, and every
// chunk of a dead record, have an empty resource and go to the trash area.
__device__ __forceinline__ void dma_record(const RecStep &d, bool live, const u32x4 *rec, ASMX_LDS u32x4 *dst,
                                           ASMX_LDS u32x4 *trash, int w, const LaneOff &lo) {
  // bytes of the record from this wave's first chunk on (integer
  // arithmetic only: every chunk's range and destination follow from it)
  const int rb = live ? 16 * (d.len - 64 * w) : 0;
  const u32x4 *r0 = rec + d.rec + 64 * w;
#pragma unroll
  for (int i = 0; i < kRounds; ++i) {
    const int nb = uniform(min(max(rb - 4096 * i, 0), 1024));
    __builtin_amdgcn_raw_ptr_buffer_load_lds(buf_rsrc(r0 + 256 * i, nb),
                                             (lds_void *)(nb > 0 ? dst + (i * 256 + w * 64) : trash), 16, lo.rec, 0, 0,
                                             kNontemporalAux);
  }
}

// Gathering: the input sources of record d's rows (fsrc at its positions)
// into a source slot; streaming wave w loads entries 64w .. 64w+63 (lanes
// past the step's rows fetch nothing).
__device__ __forceinline__ void dma_sources(const RecStep &d, bool live, const int32_t *fsrc, ASMX_LDS int32_t *dst,
                                            ASMX_LDS u32x4 *trash, int w, const LaneOff &lo) {
  const int nb = uniform(live ? min(max(4 * (d.nrows - 64 * w), 0), 256) : 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(buf_rsrc(fsrc + d.pos + 64 * w, nb),
                                           nb > 0 ? (lds_void *)(dst + 64 * w) : (lds_void *)trash, 4, lo.src, 0, 0, 0);
}

// Row inputs: load k of a record covers rows 32k .. 32k+31 (streaming wave
// w issues loads k = w and k = w + 4); lane l carries doubles (0, 1) of
// row 32k + (l >> 1) if l is even, doubles (1, 2) if odd, so row j's input
// lands as 32 bytes at kInRowBytes * j, component c at double 4j + c +
// (c >> 1).  Rows past the record's end: the gathering repeats the last
// row; the backward loads' resources end with the step's rows.
template <bool G>
__device__ __forceinline__ void dma_inputs(const RecStep &d, bool live, const ASMX_LDS int32_t *srcs,
                                           const SweepIn &in, ASMX_LDS u32x4 *dst, ASMX_LDS u32x4 *trash, int w,
                                           const LaneOff &lo) {
  ASMX_LDS char *area = reinterpret_cast<ASMX_LDS char *>(dst) + rec_in_offset((int64_t)d.len * 16);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int k = w + 4 * q;
    if constexpr (G) {
      const bool on = live && d.nrows > kInRowsPerLoad * k;  // scalar
      ASMX_LDS char *dl = on ? area + k * (kInRowsPerLoad * kInRowBytes) : reinterpret_cast<ASMX_LDS char *>(trash);
      // a dead load reads row 0 of r (its source slot may hold anything)
      int c = srcs[min(kInRowsPerLoad * k + lo.row, max(d.nrows, 1) - 1)];
      c = on ? c : 0;
      const double *p = c >= 0 ? in.r + 3 * (size_t)c : in.crs + 3 * (size_t)(-c - 1);
      __builtin_amdgcn_global_load_lds((glb_cvoid *)(p + lo.odd), (lds_void *)dl, 16, 0, 0);
    } else {
      const int r0 = kInRowsPerLoad * k;
      const int nb = uniform(live ? min(max(24 * (d.nrows - r0), 0), 24 * kInRowsPerLoad) : 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(buf_rsrc(in.src + 3 * ((size_t)d.pos + r0), nb),
                                               nb > 0 ? (lds_void *)(area + k * (kInRowsPerLoad * kInRowBytes))
                                                      : (lds_void *)trash,
                                               16, lo.in, 0, 0, 0);
    }
  }
}

// vmcnt(n) alone (the other counters at their maximum), gfx9 encoding.
constexpr int vmcnt_imm(int n) { return (n & 15) | (((n >> 4) & 3) << 14) | (7 << 4) | (15 << 8); }

// Loads of one streaming step after (and including) the record loads.
constexpr int kRecordLoads = kRounds + 2;
// Loads that may still be in flight at the end of step s, when the record
// of step s+1 and (gathering) the input sources of record s + kRecBufs,
// issued first in step s-1, must have landed.  Gathering, a step issues
// one source load and then a record's loads: with three buffers record s+1
// came last in step s-1, so only step s's own loads may be in flight; with
// four, step s-1's record loads may be too.  Without sources (backward),
// the records of steps s+2 .. s + kRecBufs - 1 may be.
template <bool G>
constexpr int step_wait() {
  static_assert(kRecBufs == 3 || kRecBufs == 4, "three or four record buffers");
  return G ? (kRecBufs == 3 ? kRecordLoads + 1 : 2 * kRecordLoads + 1) : (kRecBufs - 2) * kRecordLoads;
}
// Barriers before a sweep's first step (the computing waves match them).
constexpr int kOpenBarriers = kRecBufs;

// Keeps the compiler from moving memory operations across this point.
__device__ __forceinline__ void mem_order() { __asm__ __volatile__("" ::: "memory"); }

// Streaming waves of one sweep.  Step s (after the barrier that ends step
// s-1, which frees buffer (s-1) % kRecBufs) issues, in this order: the
// input sources of record s + kRecBufs + 1 (its descriptor read from the
// head of record s), then record s + kRecBufs - 1 with its inputs (gathered
// through the sources loaded two steps earlier).  Source slots are reused
// only after a barrier has followed the last gather that read them.
template <bool G>
__device__ __forceinline__ void producer_sweep(const RecStep *__restrict__ steps, int S,
                                               const u32x4 *__restrict__ rec_in, const SweepIn &in_v, SweepLds &L) {
  if (S == 0) return;
  constexpr int NB = kRecBufs;
  const int t = threadIdx.x - kConsumerThreads, l = t & 63;
  // the wave index, pointers and step descriptors in scalar registers, so
  // that every resource, LDS address and per-load offset below is scalar
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const LaneOff lo{16u * l, 4u * l, 24u * (l >> 1) + 8u * (l & 1), l >> 1, l & 1};
  const u32x4 *rec = uniform_ptr(rec_in);
  const SweepIn in{uniform_ptr(in_v.src), uniform_ptr(in_v.fsrc), uniform_ptr(in_v.r), uniform_ptr(in_v.crs)};
  ASMX_LDS u32x4 *trash = lds(L.trash);
  RecStep dd[NB + 1];  // steps 0 .. NB (the last step for those past it)
#pragma unroll
  for (int k = 0; k <= NB; ++k) dd[k] = uniform_step(ld_glb(steps + min(k, S - 1)));
  // sources of records 0, 1 and 2, visible to all streaming waves after the
  // sweep's first barrier
  if constexpr (G) {
#pragma unroll
    for (int k = 0; k < 3; ++k) dma_sources(dd[k], k < S, in.fsrc, lds(L.src[k]), trash, w, lo);
  }
  mem_order();
  __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
  __builtin_amdgcn_s_barrier();
  // records 0 .. NB-2; the sources of records 3 .. NB into the slots just read
#pragma unroll
  for (int k = 0; k + 1 < NB; ++k) {
    mem_order();
    dma_record(dd[k], k < S, rec, lds(L.buf[k]), trash, w, lo);
    dma_inputs<G>(dd[k], k < S, lds(L.src[k % 3]), in, lds(L.buf[k]), trash, w, lo);
    if (k + 3 <= NB) {
      mem_order();
      __builtin_amdgcn_s_barrier();
      mem_order();
      if constexpr (G) dma_sources(dd[k + 3], k + 3 < S, in.fsrc, lds(L.src[k % 3]), trash, w, lo);
    }
  }
  mem_order();
  // record 0 and the sources of record NB-1 landed
  __builtin_amdgcn_s_waitcnt(vmcnt_imm(step_wait<G>()));
  __builtin_amdgcn_s_barrier();
  RecStep da = dd[NB - 1], db = dd[NB];  // the records loaded at steps s and s+1
  for (int s = 0; s < S; ++s) {
    mem_order();
    const RecStep dn = desc_lds(&reinterpret_cast<const RecHead *>(L.buf[s % NB])->ahead);
    if constexpr (G) dma_sources(dn, s + NB + 1 < S, in.fsrc, lds(L.src[(s + NB + 1) % 3]), trash, w, lo);
    mem_order();
    const bool live = s + NB - 1 < S;
    ASMX_LDS u32x4 *dst = lds(L.buf[(s + NB - 1) % NB]);
    dma_record(da, live, rec, dst, trash, w, lo);
    dma_inputs<G>(da, live, lds(L.src[(s + NB - 1) % 3]), in, dst, trash, w, lo);
    mem_order();
    da = db;
    db = dn;
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(step_wait<G>()));
    __builtin_amdgcn_s_barrier();
  }
  mem_order();
  // the loads of the records past the end (trash) complete before the
  // next sweep starts; matches the computing waves' final barrier
  __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
  __builtin_amdgcn_s_barrier();
}

// Computing iteration for step s: step s from LDS (or the reloads of a
// fill step), results stored at once.
template <bool FWD>
__device__ __forceinline__ void cons_iter(int s, SweepLds &L, double *__restrict__ yx, double *__restrict__ z,
                                          double sc) {
  const char *recp = reinterpret_cast<const char *>(L.buf[s % kRecBufs]);
  const RecHead *hp = reinterpret_cast<const RecHead *>(recp);
  const RecHead h = *hp;
  // this thread's diagonal starts, read with the head
  const int r = threadIdx.x & 3;
  const int q32a = hp->koff32[r], q32b = hp->koff32[r + 4], q64a = hp->koff64[r], q64b = hp->koff64[r + 4];
  const int nlong = h.nrows - h.n32 - h.n64, nshort = h.n32 + h.n64;
  // a step with both kinds runs them side by side: the long rows on the
  // last waves (four rows per wave, at most half of the waves), the short
  // rows on the others
  const int wlong = nlong == 0 ? 0 : (nshort == 0 ? kConsumerThreads / 64 : min(kConsumerThreads / 128, (nlong + 3) / 4));
  const int tshort = kConsumerThreads - 64 * wlong;
  const int tid = (int)threadIdx.x;
  // a step holding both short sections runs them side by side when the
  // FP32 rows fit one pass on fewer waves than the short rows have: the
  // FP32 rows on the first waves, the FP64 rows on the rest
  const int w32 = (h.n32 + 15) / 16;
  const bool side = h.n32 > 0 && h.n64 > 0 && 64 * w32 < tshort;
  const int t32 = side ? 64 * w32 : tshort;
  if (tid < tshort) {
    if (h.n32 > 0 && tid < t32)
      short_rows<FWD, float>(recp, L, yx, z, tid, t32, h.pos, 0, h.n32, q32a, q32b, h.nslots32, h.slots32, h.vals32,
                             h.dinv32, h.n32, 0, h.in, sc);
    if (h.n64 > 0 && (!side || tid >= t32))
      short_rows<FWD, double>(recp, L, yx, z, side ? tid - t32 : tid, side ? tshort - t32 : tshort, h.pos, h.n32,
                              h.n64, q64a, q64b, h.nslots64, h.slots64, h.vals64, h.dinv64, h.n64 + nlong, 0, h.in,
                              sc);
  } else {
    long_rows<FWD>(recp, L, yx, z, tid - tshort, kConsumerThreads - tshort, h.pos, nshort, nlong, h.piece, h.ldeps, h.lrptr,
                   h.lvals, h.dinv64, h.n64 + nlong, h.n64, h.in, sc);
  }
  if (h.nfill > 0) fill_values(h, recp, L, yx);
  __syncthreads();
}

template <bool FWD>
__device__ __forceinline__ void consumer_sweep(int S, SweepLds &L, double *__restrict__ yx, double *__restrict__ z,
                                               double sc) {
  if (S == 0) return;
  // the streaming waves' opening barriers (sources of the first records,
  // source slots freed, the first record landed)
  for (int k = 0; k < kOpenBarriers; ++k) __syncthreads();
  for (int s = 0; s < S; ++s) cons_iter<FWD>(s, L, yx, z, sc);
  __syncthreads();  // matches the streaming waves' final barrier
}

__device__ __forceinline__ void ilu_apply_body(const ApplyPlan &p, int sub, const double *__restrict__ r,
                                               const double *__restrict__ scale, double *__restrict__ z,
                                               SweepLds &L) {
  const SubDesc sd = ld_glb(p.sub + sub);
  const u32x4 *rec = reinterpret_cast<const u32x4 *>(p.rec);
  // the step counts bound loops of barriers: wave-uniform values, held in
  // scalar registers whatever address space the plan was read through, so
  // that the compiler treats the loops as uniform control flow
  const int rf0 = __builtin_amdgcn_readfirstlane(sd.rf0), rb0 = __builtin_amdgcn_readfirstlane(sd.rb0);
  const int nf = __builtin_amdgcn_readfirstlane(sd.rf1) - rf0, nb = __builtin_amdgcn_readfirstlane(sd.rb1) - rb0;
  if (threadIdx.x < kConsumerThreads) {
    consumer_sweep<true>(nf, L, p.yx, z, scale ? *glb(scale) : 1.0);
    consumer_sweep<false>(nb, L, p.yx, z, 1.0);
  } else {
    const SweepIn fin{nullptr, p.fsrc, r, p.crs};
    const SweepIn bin{p.yx, nullptr, nullptr, nullptr};
    producer_sweep<true>(p.fstep + rf0, nf, rec, fin, L);
    producer_sweep<false>(p.bstep + rb0, nb, rec, bin, L);
  }
}

__global__ __launch_bounds__(kSweepThreads, 1) void ilu_apply_kernel(ApplyPlan p, const double *__restrict__ r,
                                                                     const double *__restrict__ scale,
                                                                     double *__restrict__ z,
                                                                     const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  __shared__ SweepLds L;
  ilu_apply_body(p, blockIdx.x, r, scale, z, L);
}

// Forward right-hand sides in sweep order, for the dense local solves (the
// ILU sweeps gather their own): the restriction R_i r of every subdomain.
// Fine rows gather r (times the basis scale); a coarse row sums its near/far
// atoms' lumped residuals (App. B, eq. (B.2)).  Sweep order
// walks a subdomain's level planes, so consecutive positions touch cells far
// apart in r while a few consecutive blocks share cache lines: the launches
// give each XCD a contiguous range of blocks, so those lines stay in one L2.
__device__ __forceinline__ void gather_rhs_body(int bid, int npos, const int32_t *__restrict__ fsrc,
                                                const double *__restrict__ r, const double *__restrict__ scale,
                                                const int32_t *__restrict__ cptr3, const int32_t *__restrict__ cidx3,
                                                const double *__restrict__ pnf, double *__restrict__ rs) {
  const int q = bid * 256 + (int)threadIdx.x;
  if (q >= npos) return;
  const int src = fsrc[q];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (src >= 0) {
    const double sc = scale ? *scale : 1.0;
    a0 = sc * r[3 * (size_t)src]; a1 = sc * r[3 * (size_t)src + 1]; a2 = sc * r[3 * (size_t)src + 2];
  } else {
    const int c = -src - 1;
    for (int t = cptr3[c]; t < cptr3[c + 1]; ++t) {
      const double *p = pnf + 3 * (size_t)cidx3[t];
      a0 += p[0]; a1 += p[1]; a2 += p[2];
    }
  }
  rs[3 * (size_t)q] = a0; rs[3 * (size_t)q + 1] = a1; rs[3 * (size_t)q + 2] = a2;
}

__global__ __launch_bounds__(256) void gather_rhs_kernel(int npos, const int32_t *__restrict__ fsrc,
                                                         const double *__restrict__ r,
                                                         const double *__restrict__ scale,
                                                         const int32_t *__restrict__ cptr3,
                                                         const int32_t *__restrict__ cidx3,
                                                         const double *__restrict__ pnf, double *__restrict__ rs) {
  gather_rhs_body(xcd_logical_block((npos + 255) / 256, blockIdx.x), npos, fsrc, r, scale, cptr3, cidx3, pnf, rs);
}

// Lumped input of each coarse row: the sum of its near/far atoms' lumped
// residuals (App. B, eq. (B.2)), in the order the gather above sums them.
__device__ __forceinline__ void coarse_rhs_body(int bid, int ncoarse, const int32_t *__restrict__ cptr3,
                                                const int32_t *__restrict__ cidx3, const double *__restrict__ pnf,
                                                double *__restrict__ crs) {
  const int c = bid * 256 + (int)threadIdx.x;
  if (c >= ncoarse) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int t = cptr3[c]; t < cptr3[c + 1]; ++t) {
    const double *p = pnf + 3 * (size_t)cidx3[t];
    a0 += p[0]; a1 += p[1]; a2 += p[2];
  }
  crs[3 * (size_t)c] = a0; crs[3 * (size_t)c + 1] = a1; crs[3 * (size_t)c + 2] = a2;
}

__global__ __launch_bounds__(256) void coarse_rhs_kernel(int ncoarse, const int32_t *__restrict__ cptr3,
                                                         const int32_t *__restrict__ cidx3,
                                                         const double *__restrict__ pnf, double *__restrict__ crs,
                                                         const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  coarse_rhs_body(blockIdx.x, ncoarse, cptr3, cidx3, pnf, crs);
}

__device__ __forceinline__ void additive_combine_body(int bid, int N, const int32_t *__restrict__ cptr,
                                                      const int32_t *__restrict__ cidx,
                                                      const double *__restrict__ yext, double *__restrict__ z) {
  const int c = bid * 256 + (int)threadIdx.x;
  if (c >= N) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int t = cptr[c]; t < cptr[c + 1]; ++t) {
    const size_t q = (size_t)cidx[t] * 3;
    a0 += yext[q]; a1 += yext[q + 1]; a2 += yext[q + 2];
  }
  z[3 * (size_t)c] = a0; z[3 * (size_t)c + 1] = a1; z[3 * (size_t)c + 2] = a2;
}

__global__ __launch_bounds__(256) void additive_combine_kernel(int N, const int32_t *__restrict__ cptr,
                                                               const int32_t *__restrict__ cidx,
                                                               const double *__restrict__ yext,
                                                               double *__restrict__ z,
                                                               const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  additive_combine_body(blockIdx.x, N, cptr, cidx, yext, z);
}

// ---------------------------------------------------------------- Krylov
// partial[b*(NV+1) + i] = sum over the block's elements of U_i . w (i < NV),
// partial[b*(NV+1) + NV] = w . w.
// Krylov vectors are processed two doubles per thread (16-byte loads); an
// odd last element is handled by thread 0 of block 0.
template <int NV>
__device__ __forceinline__ void multidot_body(int bid, int nblk, int64_t n, const double *__restrict__ U, int64_t ldu,
                                              const double *__restrict__ w, double *__restrict__ partial,
                                              double *red) {
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  const int64_t n2 = n / 2;
  const double2 *w2 = reinterpret_cast<const double2 *>(w);
  for (int64_t e = (int64_t)bid * 256 + threadIdx.x; e < n2; e += (int64_t)nblk * 256) {
    const double2 we = w2[e];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double2 u = ld_stream2(reinterpret_cast<const double2 *>(U + i * ldu) + e);
      acc[i] += u.x * we.x + u.y * we.y;
    }
    acc[NV] += we.x * we.x + we.y * we.y;
  }
  if ((n & 1) && bid == 0 && threadIdx.x == 0) {
    const double we = w[n - 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += U[i * ldu + n - 1] * we;
    acc[NV] += we * we;
  }
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int i = 0; i <= NV; ++i) {
    const double v = wave_sum(acc[i]);
    if (lane == 0) red[wv * (NV + 1) + i] = v;
  }
  __syncthreads();
  if (threadIdx.x <= NV) {
    const double s = red[threadIdx.x] + red[(NV + 1) + threadIdx.x] + red[2 * (NV + 1) + threadIdx.x] +
                     red[3 * (NV + 1) + threadIdx.x];
    partial[(size_t)bid * (NV + 1) + threadIdx.x] = s;
  }
}

template <int NV>
__global__ __launch_bounds__(256) void multidot_kernel(int64_t n, const double *__restrict__ U, int64_t ldu,
                                                       const double *__restrict__ w,
                                                       double *__restrict__ partial,
                                                       const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  __shared__ double red[4 * (NV + 1)];
  multidot_body<NV>(blockIdx.x, gridDim.x, n, U, ldu, w, partial, red);
}

// out[c] = sum_b partial[b*ncols + c], fixed order: one workgroup per column.
__device__ __forceinline__ void reduce_cols_body(int c, int nblocks, int ncols, const double *__restrict__ partial,
                                                 double *__restrict__ out, double *red) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[(size_t)b * ncols + c];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) out[c] = s;
}

__global__ __launch_bounds__(256) void reduce_cols_kernel(int nblocks, int ncols, const double *__restrict__ partial,
                                                          double *__restrict__ out,
                                                          const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  __shared__ double red[4];
  reduce_cols_body(blockIdx.x, nblocks, ncols, partial, out, red);
}

// unew = w - sum_i c_i U_i and per-block partial sums of ||unew||^2.  The
// basis is stored unnormalised (v_i = scale_i U_i) and d[i] = U_i . w, so
// the Hessenberg entry is h_i = scale_i d_i and c_i = h_i scale_i.
template <int NV>
__device__ __forceinline__ void update_body(int bid, int nblk, int64_t n, const double *__restrict__ U, int64_t ldu,
                                            const double *__restrict__ d, const double *__restrict__ scale,
                                            const double *__restrict__ w, double *__restrict__ unew,
                                            double *__restrict__ partial, double *red) {
  double cs[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) cs[i] = (scale[i] * d[i]) * scale[i];
  double nrm = 0.0;
  const int64_t n2 = n / 2;
  const double2 *w2 = reinterpret_cast<const double2 *>(w);
  double2 *o2 = reinterpret_cast<double2 *>(unew);
  for (int64_t e = (int64_t)bid * 256 + threadIdx.x; e < n2; e += (int64_t)nblk * 256) {
    double2 a = w2[e];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double2 u = ld_stream2(reinterpret_cast<const double2 *>(U + i * ldu) + e);
      a.x -= cs[i] * u.x;
      a.y -= cs[i] * u.y;
    }
    o2[e] = a;
    nrm += a.x * a.x + a.y * a.y;
  }
  if ((n & 1) && bid == 0 && threadIdx.x == 0) {
    double a = w[n - 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) a -= cs[i] * U[i * ldu + n - 1];
    unew[n - 1] = a;
    nrm += a * a;
  }
  const double s = block_sum<256>(nrm, red);
  if (threadIdx.x == 0) partial[bid] = s;
}

template <int NV>
__global__ __launch_bounds__(256) void update_kernel(int64_t n, const double *__restrict__ U, int64_t ldu,
                                                     const double *__restrict__ d, const double *__restrict__ scale,
                                                     const double *__restrict__ w, double *__restrict__ unew,
                                                     double *__restrict__ partial,
                                                     const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  __shared__ double red[4];
  update_body<NV>(blockIdx.x, gridDim.x, n, U, ldu, d, scale, w, unew, partial, red);
}

// One block of 256 threads: h = sqrt(sum of partial[0 .. nblocks)) (the
// partial sums in the order of reduce_cols_body) into hcol[nv] and 1/h
// into scale_out; for i < nv, hcol[i] = scale[i] * d[i] (the projections
// of the step).  If pub is not NULL, hcol[0..nv] and sqrt(d[nv]) (the norm
// of w before the projections) are also written to pub[0..nv+1].
__device__ __forceinline__ void norm_finalize_body(int nblocks, const double *__restrict__ partial, int nv,
                                                   const double *__restrict__ d, const double *__restrict__ scale,
                                                   double *__restrict__ hcol, double *__restrict__ scale_out,
                                                   double *__restrict__ pub, double *red) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[b];
  s = block_sum<256>(s, red);
  for (int q = threadIdx.x; q < nv; q += 256) {
    const double h = scale[q] * d[q];
    hcol[q] = h;
    if (pub) pub[q] = h;
  }
  if (threadIdx.x == 0) {
    const double h = sqrt(s);
    hcol[nv] = h;
    *scale_out = (h > 0.0) ? 1.0 / h : 0.0;
    if (pub) {
      pub[nv] = h;
      pub[nv + 1] = sqrt(d[nv]);
    }
  }
}

__global__ __launch_bounds__(256) void norm_finalize_kernel(int nblocks, const double *__restrict__ partial, int nv,
                                                            const double *__restrict__ d,
                                                            const double *__restrict__ scale,
                                                            double *__restrict__ hcol, double *__restrict__ scale_out,
                                                            double *__restrict__ pub,
                                                            const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  __shared__ double red[4];
  norm_finalize_body(nblocks, partial, nv, d, scale, hcol, scale_out, pub, red);
}

__device__ __forceinline__ void lincomb_body(int bid, int nblk, int64_t n, int nv, const double *__restrict__ U,
                                             int64_t ldu, const double *__restrict__ coef, double *__restrict__ out,
                                             double *cs) {
  for (int i = threadIdx.x; i < nv; i += blockDim.x) cs[i] = coef[i];
  __syncthreads();
  for (int64_t e = (int64_t)bid * 256 + threadIdx.x; e < n; e += (int64_t)nblk * 256) {
    double a = 0.0;
    for (int i = 0; i < nv; ++i) a += cs[i] * U[i * ldu + e];
    out[e] = a;
  }
}

__global__ __launch_bounds__(256) void lincomb_kernel(int64_t n, int nv, const double *__restrict__ U, int64_t ldu,
                                                      const double *__restrict__ coef, double *__restrict__ out) {
  __shared__ double cs[kMaxRestart + 1];
  lincomb_body(blockIdx.x, gridDim.x, n, nv, U, ldu, coef, out, cs);
}

__device__ __forceinline__ void axpy_body(int bid, int nblk, int64_t n, const double *__restrict__ z,
                                          double *__restrict__ x) {
  for (int64_t e = (int64_t)bid * 256 + threadIdx.x; e < n; e += (int64_t)nblk * 256) x[e] += z[e];
}

__global__ __launch_bounds__(256) void axpy_kernel(int64_t n, const double *__restrict__ z, double *__restrict__ x) {
  axpy_body(blockIdx.x, gridDim.x, n, z, x);
}

__global__ __launch_bounds__(256) void check_finite_kernel(int64_t n, const double *__restrict__ v, int *__restrict__ flag) {
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) bad |= !isfinite(v[e]);
  if (bad) atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void norm2_kernel(int64_t n, const double *__restrict__ v, double *__restrict__ partial) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) s += v[e] * v[e];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__device__ __forceinline__ void scale_copy_body(int bid, int nblk, int64_t n, const double *__restrict__ r,
                                                const double *__restrict__ scale, double *__restrict__ z) {
  const double s = scale ? *scale : 1.0;
  for (int64_t e = (int64_t)bid * 256 + threadIdx.x; e < n; e += (int64_t)nblk * 256) z[e] = s * r[e];
}

__global__ __launch_bounds__(256) void scale_copy_kernel(int64_t n, const double *__restrict__ r, const double *__restrict__ scale,
                                                         double *__restrict__ z,
                                                         const int *__restrict__ skip) {
  if (skip && *skip) return;  // a graph-mode cycle that has ended
  scale_copy_body(blockIdx.x, gridDim.x, n, r, scale, z);
}

// p[0 .. n) = v (also a flag cleared without a memset node).
template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(int64_t n, T v, T *__restrict__ p) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p[e] = v;
}

// Device memory of the no-allocation solve: one fixed array per device,
// reserved when the code object is loaded on that device and kept until the
// process ends.  Host code never passes the symbol itself to a kernel (on
// the host it is only a stand-in); it passes the device address looked up
// once per device by noalloc_scratch().
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

// ---------------------------------------------------------------- batches
// A batched launch covers several independent systems; each block finds
// its system by binary search over the segment starts and runs the same
// body, with the same local block numbering, as a single-system launch.
struct SegPos {
  int sys, lb, nb;
};
__device__ __forceinline__ SegPos seg_find(const BatchSeg &g, int b = blockIdx.x) {
  int lo = 0, hi = g.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return {g.sys[lo], b - g.start[lo], g.start[lo + 1] - g.start[lo]};
}

// preconditioner input of a system: basis column col (scaled) or t
__device__ __forceinline__ const double *prec_in(const BatchSys &S, int col, const double *&scale) {
  if (col >= 0) {
    scale = S.scale + col;
    return S.U + (size_t)col * S.ldu;
  }
  scale = nullptr;
  return S.t;
}

__global__ __launch_bounds__(256) void batch_c1_kernel(const BatchSys *__restrict__ tab, BatchSeg g, int col) {
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  const double *scale;
  const double *r = prec_in(S, col, scale);
  gather_sum3_body(p.lb, S.c1n1, S.c1lanes, S.c1n, S.c1lanes2, S.c1ptr, S.c1idx, r, scale, S.PA);
}

__global__ __launch_bounds__(256) void batch_c2_kernel(const BatchSys *__restrict__ tab, BatchSeg g) {
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  gather_sum3_body(p.lb, S.c2n1, S.c2lanes, S.c2n, S.c2lanes2, S.c2ptr, S.c2idx, S.PA, nullptr, S.PNF);
}

__global__ __launch_bounds__(256) void batch_crs_kernel(const BatchSys *__restrict__ tab, BatchSeg g) {
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  coarse_rhs_body(p.lb, S.ap.ncoarse, S.ap.cptr3, S.ap.cidx3, S.ap.pnf, S.ap.crs);
}

__global__ __launch_bounds__(kSweepThreads, 1) void batch_apply_kernel(const BatchSys *__restrict__ tab, BatchSeg g,
                                                                       int col) {
  __shared__ SweepLds L;
  // the system and its subdomain are the same for the whole workgroup:
  // scalar registers keep the plan's fields out of the vector budget
  const SegPos p = seg_find(g);
  const int sys = __builtin_amdgcn_readfirstlane(p.sys), lb = __builtin_amdgcn_readfirstlane(p.lb);
  const BatchSys &S = tab[sys];
  const ApplyPlan ap = S.ap;
  const double *scale;
  const double *r = prec_in(S, col, scale);
  ilu_apply_body(ap, lb, r, scale, S.z, L);
}

__global__ __launch_bounds__(256) void batch_combine_kernel(const BatchSys *__restrict__ tab, BatchSeg g) {
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  additive_combine_body(p.lb, S.N, S.cptr, S.cidx, S.ap.yx, S.z);
}

__global__ __launch_bounds__(256) void batch_copy_kernel(const BatchSys *__restrict__ tab, BatchSeg g, int col) {
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  const double *scale;
  const double *r = prec_in(S, col, scale);
  scale_copy_body(p.lb, p.nb, S.n, r, scale, S.z);
}

template <bool RESID>
__global__ __launch_bounds__(256) void batch_spmv_kernel(const BatchSys *__restrict__ tab, BatchSeg g) {
  __shared__ double red[4];
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  if (RESID) spmv_body<true>(p.lb, S.N, S.nlog, S.sptr, S.cols, S.vals, S.x, S.b, S.U, S.partial, red);
  else spmv_body<false>(p.lb, S.N, S.nlog, S.sptr, S.cols, S.vals, S.z, nullptr, S.w, nullptr, red);
}

template <int NV>
__global__ __launch_bounds__(256) void batch_multidot_kernel(const BatchSys *__restrict__ tab, BatchSeg g) {
  __shared__ double red[4 * (NV + 1)];
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  multidot_body<NV>(p.lb, p.nb, S.n, S.U, S.ldu, S.w, S.partial, red);
}

// One block per system reduces its ncols columns in turn (the same sums, in
// the same order, as one block per column) from the partial sums of the
// system's reduction blocks (src 0: CGS kernels, 1: residual SpMV); dots:
// into dvec, else into misc[2].
__device__ __forceinline__ int red_blocks(const BatchSys &S, int src) {
  if (src == 1) return (((int)((S.N + 255) / 256) + 7) >> 3) << 3;
  const int64_t b = (S.n / 2 + 255) / 256;
  return (int)(b < 1 ? 1 : (b > S.red_blocks ? S.red_blocks : b));
}

__global__ __launch_bounds__(256) void batch_reduce_kernel(const BatchSys *__restrict__ tab, BatchSeg g, int ncols,
                                                           int dots, int src) {
  __shared__ double sh[4];
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  const int nb = red_blocks(S, src);
  for (int c = 0; c < ncols; ++c) reduce_cols_body(c, nb, ncols, S.partial, dots ? S.dvec : S.misc + 2, sh);
}

template <int NV>
__global__ __launch_bounds__(256) void batch_update_kernel(const BatchSys *__restrict__ tab, BatchSeg g, int ldh) {
  __shared__ double red[4];
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  update_body<NV>(p.lb, p.nb, S.n, S.U, S.ldu, S.dvec, S.scale, S.w, S.U + (size_t)NV * S.ldu, S.partial, red);
}

// One block per system: the norm of the new basis vector of step j from the
// partial sums of the update kernel (src 0), or for j < 0 the true residual
// norm from those of the residual SpMV (src 1): beta into misc[1], 1/beta
// into scale[0], beta to the host at pub[-1].
__global__ __launch_bounds__(256) void batch_norm_finalize_kernel(const BatchSys *__restrict__ tab, BatchSeg g, int j,
                                                                  int ldh, int pub_stride, int src) {
  __shared__ double red[4];
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  const int nb = red_blocks(S, src);
  if (j >= 0) {
    norm_finalize_body(nb, S.partial, j + 1, S.dvec, S.scale, S.H + (size_t)j * ldh, S.scale + j + 1,
                       S.pub + (size_t)j * pub_stride, red);
  } else {
    norm_finalize_body(nb, S.partial, 0, nullptr, nullptr, S.misc + 1, S.scale, nullptr, red);
    if (threadIdx.x == 0) S.pub[-1] = S.misc[1];
  }
}

__global__ __launch_bounds__(256) void batch_lincomb_kernel(const BatchSys *__restrict__ tab, BatchSeg g) {
  __shared__ double cs[kMaxRestart + 1];
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  const int k = (int)S.coefh[0];
  lincomb_body(p.lb, p.nb, S.n, k, S.U, S.ldu, S.coefh + 1, S.t, cs);
}

__global__ __launch_bounds__(256) void batch_axpy_kernel(const BatchSys *__restrict__ tab, BatchSeg g) {
  const SegPos p = seg_find(g);
  const BatchSys &S = tab[p.sys];
  axpy_body(p.lb, p.nb, S.n, S.z, S.x);
}

// ---------------------------------------------------------------- device-side restart cycles
// The host loop's Givens and triangular-solve arithmetic, one thread, for a
// cycle that runs without the host.
__global__ void cycle_start_kernel(CycleState *st, double *g, const double *beta) {
  if (threadIdx.x != 0) return;
  st->done = 0;
  st->k = 0;
  g[0] = *beta;
}

__global__ void givens_kernel(int j, int ld, double *H, double *cs, double *sn, double *g, const double *d,
                              CycleState *st) {
  if (threadIdx.x != 0 || st->done) return;
  double *col = H + (size_t)j * ld;
  const double hn = col[j + 1];
  const double w0 = sqrt(d[j + 1]);
  for (int i = 0; i < j; ++i) {
    const double a = col[i], c = col[i + 1];
    col[i] = cs[i] * a + sn[i] * c;
    col[i + 1] = -sn[i] * a + cs[i] * c;
  }
  const double rho = hypot(col[j], col[j + 1]);
  if (rho == 0.0) {
    cs[j] = 1.0;
    sn[j] = 0.0;
  } else {
    cs[j] = col[j] / rho;
    sn[j] = col[j + 1] / rho;
  }
  col[j] = rho;
  col[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  st->k = j + 1;
  if (hn <= 1e-14 * w0 || (st->use_tol && fabs(g[j + 1]) <= st->tol) || j + 1 >= st->kmax) st->done = 1;
}

__global__ void cycle_end_kernel(int ld, const double *H, const double *g, const double *scale, double *coef,
                                 const CycleState *st) {
  __shared__ double y[kMaxRestart];  // indexed dynamically: LDS, not private (scratch) memory
  if (threadIdx.x != 0) return;
  const int k = st->k;
  for (int i = k - 1; i >= 0; --i) {
    double acc = g[i];
    for (int c = i + 1; c < k; ++c) acc -= H[(size_t)c * ld + i] * y[c];
    y[i] = acc / H[(size_t)i * ld + i];
  }
  for (int i = 0; i < k; ++i) coef[i] = y[i] * scale[i];
}

__global__ __launch_bounds__(256) void lincomb_dev_kernel(int64_t n, const CycleState *__restrict__ st,
                                                          const double *__restrict__ U, int64_t ldu,
                                                          const double *__restrict__ coef, double *__restrict__ out) {
  __shared__ double cs[kMaxRestart + 1];
  lincomb_body(blockIdx.x, gridDim.x, n, st->k, U, ldu, coef, out, cs);
}

__global__ void cycle_publish_kernel(const CycleState *st, const double *g, const double *beta, double *pub) {
  if (threadIdx.x != 0) return;
  const int k = st->k;
  pub[0] = (double)k;
  pub[1] = *beta;
  pub[2] = fabs(g[k]);
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_cycle_start(CycleState *st, double *g, const double *beta, hipStream_t s) {
  cycle_start_kernel<<<1, 64, 0, s>>>(st, g, beta);
  return hipGetLastError();
}

hipError_t launch_givens(int j, int ld, double *H, double *cs, double *sn, double *g, const double *d,
                         CycleState *st, hipStream_t s) {
  givens_kernel<<<1, 64, 0, s>>>(j, ld, H, cs, sn, g, d, st);
  return hipGetLastError();
}

hipError_t launch_cycle_end(int ld, const double *H, const double *g, const double *scale, double *coef,
                            const CycleState *st, hipStream_t s) {
  cycle_end_kernel<<<1, 64, 0, s>>>(ld, H, g, scale, coef, st);
  return hipGetLastError();
}

hipError_t launch_lincomb_dev(int64_t n, const CycleState *st, const double *U, int64_t ldu, const double *coef,
                              double *out, hipStream_t s) {
  const int grid = std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  lincomb_dev_kernel<<<grid, 256, 0, s>>>(n, st, U, ldu, coef, out);
  return hipGetLastError();
}

hipError_t launch_cycle_publish(const CycleState *st, const double *g, const double *beta, double *pub,
                                hipStream_t s) {
  cycle_publish_kernel<<<1, 64, 0, s>>>(st, g, beta, pub);
  return hipGetLastError();
}
hipError_t launch_sell_fill(const SellDev &A, const double *csr_vals, hipStream_t s) {
  const int nslots = A.ngroups * 64;
  if (nslots == 0) return hipSuccess;
  sell_fill_kernel<<<blocks_for(nslots, 256), 256, 0, s>>>(nslots, A.src, csr_vals, A.vals);
  return hipGetLastError();
}

hipError_t launch_spmv(const SellDev &A, const double *x, double *y, hipStream_t s, const int *skip, int rows) {
  if (rows == 2 || rows == 4) {
    const int nlog = blocks_for(A.N, 256 * rows);
    if (rows == 2)
      spmv_rows_kernel<2><<<xcd_grid(nlog), 256, 0, s>>>(A.N, nlog, A.sptr, A.cols, A.vals, x, y, skip);
    else
      spmv_rows_kernel<4><<<xcd_grid(nlog), 256, 0, s>>>(A.N, nlog, A.sptr, A.cols, A.vals, x, y, skip);
    return hipGetLastError();
  }
  const int nlog = blocks_for(A.N, 256);
  spmv_kernel<false><<<xcd_grid(nlog), 256, 0, s>>>(A.N, nlog, A.sptr, A.cols, A.vals, x, nullptr, y, nullptr, skip);
  return hipGetLastError();
}

hipError_t launch_residual(const SellDev &A, const double *x, const double *b, double *r, double *partial,
                           int *nblocks_out, hipStream_t s) {
  const int nlog = blocks_for(A.N, 256);
  const int grid = xcd_grid(nlog);
  spmv_kernel<true><<<grid, 256, 0, s>>>(A.N, nlog, A.sptr, A.cols, A.vals, x, b, r, partial, nullptr);
  *nblocks_out = grid;
  return hipGetLastError();
}

hipError_t launch_gather_sum9(int ndst, const int32_t *ptr, const int32_t *idx, const double *srcA, int32_t nA,
                              const double *srcB, double *dst, hipStream_t s) {
  if (ndst == 0) return hipSuccess;
  gather_sum9_kernel<<<blocks_for(ndst, 256), 256, 0, s>>>(ndst, ptr, idx, srcA, nA, srcB, dst);
  return hipGetLastError();
}

static bool lanes_ok(int g) { return g >= 1 && g <= 64 && (g & (g - 1)) == 0; }

hipError_t launch_gather_sum3(int n1, int lanes1, int n, int lanes2, const int32_t *ptr, const int32_t *idx,
                              const double *src, const double *scale, double *dst, hipStream_t s, const int *skip) {
  if (n == 0) return hipSuccess;
  if (n1 < 0 || n1 > n || !lanes_ok(lanes1) || !lanes_ok(lanes2)) return hipErrorInvalidValue;
  gather_sum3_kernel<<<gather_sum3_blocks(n1, lanes1, n, lanes2), 256, 0, s>>>(n1, lanes1, n, lanes2, ptr, idx,
                                                                                src, scale, dst, skip);
  return hipGetLastError();
}

hipError_t launch_ilu_factor(const DevPlan &p, unsigned long long *bad, hipStream_t s) {
  if (p.nsub == 0) return hipSuccess;
  ilu_factor_kernel<<<p.nsub, 256, 0, s>>>(p, bad);
  return hipGetLastError();
}

hipError_t launch_relayout(int nslots, const int32_t *src, const int32_t *base, const int32_t *stride,
                           const uint8_t *to32, const double *fact, double *out64, float *out32, hipStream_t s) {
  if (nslots == 0) return hipSuccess;
  relayout_kernel<<<blocks_for(nslots, 256), 256, 0, s>>>(nslots, src, base, stride, to32, fact, out64, out32);
  return hipGetLastError();
}

hipError_t launch_gather_rhs(int npos, const ApplyPlan &p, const double *r, const double *scale, hipStream_t s) {
  if (npos == 0) return hipSuccess;
  gather_rhs_kernel<<<xcd_grid(blocks_for(npos, 256)), 256, 0, s>>>(npos, p.fsrc, r, scale, p.cptr3, p.cidx3, p.pnf, p.rs);
  return hipGetLastError();
}

hipError_t launch_coarse_rhs(const ApplyPlan &p, hipStream_t s, const int *skip) {
  if (p.ncoarse == 0) return hipSuccess;
  coarse_rhs_kernel<<<blocks_for(p.ncoarse, 256), 256, 0, s>>>(p.ncoarse, p.cptr3, p.cidx3, p.pnf, p.crs, skip);
  return hipGetLastError();
}

hipError_t launch_ilu_apply(const ApplyPlan &p, const double *r, const double *scale, double *z, hipStream_t s,
                            const int *skip) {
  if (p.nsub == 0) return hipSuccess;
  ilu_apply_kernel<<<p.nsub, kSweepThreads, 0, s>>>(p, r, scale, z, skip);
  return hipGetLastError();
}

hipError_t launch_additive_combine(int N, const int32_t *cptr, const int32_t *cidx, const double *yext, double *z,
                                   hipStream_t s, const int *skip) {
  additive_combine_kernel<<<blocks_for(N, 256), 256, 0, s>>>(N, cptr, cidx, yext, z, skip);
  return hipGetLastError();
}

template <int NV>
static void multidot_launch(int64_t n, const double *U, int64_t ldu, const double *w, double *partial, int grid,
                            hipStream_t s, const int *skip) {
  multidot_kernel<NV><<<grid, 256, 0, s>>>(n, U, ldu, w, partial, skip);
}

template <int... Is>
static bool multidot_dispatch(int nv, int64_t n, const double *U, int64_t ldu, const double *w, double *partial,
                              int grid, hipStream_t s, const int *skip, std::integer_sequence<int, Is...>) {
  bool done = false;
  ((nv == Is + 1 ? (multidot_launch<Is + 1>(n, U, ldu, w, partial, grid, s, skip), done = true) : false), ...);
  return done;
}

hipError_t launch_multidot(int64_t n, int nv, const double *U, int64_t ldu, const double *w, double *partial,
                           int *nblocks_out, hipStream_t s, const int *skip, int max_blocks) {
  if (max_blocks < 1 || max_blocks > kMaxReduceBlocks) return hipErrorInvalidValue;
  const int grid = std::min<int64_t>(max_blocks, std::max<int64_t>(1, (n / 2 + 255) / 256));
  if (nv < 1 || nv > 32) return hipErrorInvalidValue;
  multidot_dispatch(nv, n, U, ldu, w, partial, grid, s, skip, std::make_integer_sequence<int, 32>{});
  *nblocks_out = grid;
  return hipGetLastError();
}

hipError_t launch_reduce_cols(int nblocks, int ncols, const double *partial, double *out, hipStream_t s,
                              const int *skip) {
  reduce_cols_kernel<<<ncols, 256, 0, s>>>(nblocks, ncols, partial, out, skip);
  return hipGetLastError();
}

template <int NV>
static void update_launch(int64_t n, const double *U, int64_t ldu, const double *d, const double *scale,
                          const double *w, double *unew, double *partial, int grid, hipStream_t s,
                          const int *skip) {
  update_kernel<NV><<<grid, 256, 0, s>>>(n, U, ldu, d, scale, w, unew, partial, skip);
}

template <int... Is>
static bool update_dispatch(int nv, int64_t n, const double *U, int64_t ldu, const double *d, const double *scale,
                            const double *w, double *unew, double *partial, int grid, hipStream_t s,
                            const int *skip, std::integer_sequence<int, Is...>) {
  bool done = false;
  ((nv == Is + 1 ? (update_launch<Is + 1>(n, U, ldu, d, scale, w, unew, partial, grid, s, skip), done = true)
                 : false),
   ...);
  return done;
}

hipError_t launch_update(int64_t n, int nv, const double *U, int64_t ldu, const double *d, const double *scale,
                         const double *w, double *unew, double *partial, int *nblocks_out, hipStream_t s,
                         const int *skip, int max_blocks) {
  if (max_blocks < 1 || max_blocks > kMaxReduceBlocks) return hipErrorInvalidValue;
  const int grid = std::min<int64_t>(max_blocks, std::max<int64_t>(1, (n / 2 + 255) / 256));
  if (nv < 1 || nv > kMaxRestart) return hipErrorInvalidValue;
  update_dispatch(nv, n, U, ldu, d, scale, w, unew, partial, grid, s, skip,
                  std::make_integer_sequence<int, kMaxRestart>{});
  *nblocks_out = grid;
  return hipGetLastError();
}

hipError_t launch_norm_finalize(int nblocks, const double *partial, int nv, const double *d, const double *scale,
                                double *hcol, double *scale_out, double *pub, hipStream_t s, const int *skip) {
  norm_finalize_kernel<<<1, 256, 0, s>>>(nblocks, partial, nv, d, scale, hcol, scale_out, pub, skip);
  return hipGetLastError();
}

hipError_t launch_lincomb(int64_t n, int nv, const double *U, int64_t ldu, const double *coef, double *out,
                          hipStream_t s) {
  const int grid = std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  lincomb_kernel<<<grid, 256, 0, s>>>(n, nv, U, ldu, coef, out);
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, const double *z, double *x, hipStream_t s) {
  const int grid = std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  axpy_kernel<<<grid, 256, 0, s>>>(n, z, x);
  return hipGetLastError();
}

hipError_t launch_check_finite(int64_t n, const double *v, int *flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int grid = std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  check_finite_kernel<<<grid, 256, 0, s>>>(n, v, flag);
  return hipGetLastError();
}

hipError_t launch_norm2(int64_t n, const double *v, double *partial, int *nblocks_out, hipStream_t s) {
  const int grid = std::min<int64_t>(kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  norm2_kernel<<<grid, 256, 0, s>>>(n, v, partial);
  *nblocks_out = grid;
  return hipGetLastError();
}

int batch_blocks(BatchKernel k, const BatchSys &s) {
  const int64_t n = s.n;
  switch (k) {
    case kBkC1: return s.c1n > 0 ? gather_sum3_blocks(s.c1n1, s.c1lanes, s.c1n, s.c1lanes2) : 0;
    case kBkC2: return s.c2n > 0 ? gather_sum3_blocks(s.c2n1, s.c2lanes, s.c2n, s.c2lanes2) : 0;
    case kBkCrs: return blocks_for(s.ap.ncoarse, 256);
    case kBkApply: return s.nsub;
    case kBkCombine: return blocks_for(s.N, 256);
    case kBkCopy: return (int)std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
    case kBkSpmv: return xcd_grid(blocks_for(s.N, 256));
    case kBkRed: return (int)std::min<int64_t>(s.red_blocks, std::max<int64_t>(1, (n / 2 + 255) / 256));
    case kBkVec: return (int)std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
    case kBkOne: return 1;
    default: return 0;
  }
}

hipError_t launch_batch_precond(const BatchSys *tab, const BatchSeg *seg, int col, hipStream_t s) {
  // seg[k] for every BatchKernel k (empty segments launch nothing)
  if (seg[kBkCopy].total > 0) batch_copy_kernel<<<seg[kBkCopy].total, 256, 0, s>>>(tab, seg[kBkCopy], col);
  if (seg[kBkC1].total > 0) batch_c1_kernel<<<seg[kBkC1].total, 256, 0, s>>>(tab, seg[kBkC1], col);
  if (seg[kBkC2].total > 0) batch_c2_kernel<<<seg[kBkC2].total, 256, 0, s>>>(tab, seg[kBkC2]);
  if (seg[kBkCrs].total > 0) batch_crs_kernel<<<seg[kBkCrs].total, 256, 0, s>>>(tab, seg[kBkCrs]);
  if (seg[kBkApply].total > 0)
    batch_apply_kernel<<<seg[kBkApply].total, kSweepThreads, 0, s>>>(tab, seg[kBkApply], col);
  if (seg[kBkCombine].total > 0) batch_combine_kernel<<<seg[kBkCombine].total, 256, 0, s>>>(tab, seg[kBkCombine]);
  return hipGetLastError();
}

hipError_t launch_batch_spmv(const BatchSys *tab, const BatchSeg &seg, bool residual, hipStream_t s) {
  if (seg.total == 0) return hipSuccess;
  if (residual) batch_spmv_kernel<true><<<seg.total, 256, 0, s>>>(tab, seg);
  else batch_spmv_kernel<false><<<seg.total, 256, 0, s>>>(tab, seg);
  return hipGetLastError();
}

template <int NV>
static void batch_multidot_launch(const BatchSys *tab, const BatchSeg &seg, hipStream_t s) {
  batch_multidot_kernel<NV><<<seg.total, 256, 0, s>>>(tab, seg);
}
template <int... Is>
static void batch_multidot_dispatch(int nv, const BatchSys *tab, const BatchSeg &seg, hipStream_t s,
                                    std::integer_sequence<int, Is...>) {
  ((nv == Is + 1 ? (batch_multidot_launch<Is + 1>(tab, seg, s), 0) : 0), ...);
}
hipError_t launch_batch_multidot(const BatchSys *tab, const BatchSeg &seg, int nv, hipStream_t s) {
  if (nv < 1 || nv > kMaxRestart) return hipErrorInvalidValue;
  if (seg.total == 0) return hipSuccess;
  batch_multidot_dispatch(nv, tab, seg, s, std::make_integer_sequence<int, kMaxRestart>{});
  return hipGetLastError();
}

template <int NV>
static void batch_update_launch(const BatchSys *tab, const BatchSeg &seg, int ldh, hipStream_t s) {
  batch_update_kernel<NV><<<seg.total, 256, 0, s>>>(tab, seg, ldh);
}
template <int... Is>
static void batch_update_dispatch(int nv, const BatchSys *tab, const BatchSeg &seg, int ldh, hipStream_t s,
                                  std::integer_sequence<int, Is...>) {
  ((nv == Is + 1 ? (batch_update_launch<Is + 1>(tab, seg, ldh, s), 0) : 0), ...);
}
hipError_t launch_batch_update(const BatchSys *tab, const BatchSeg &seg, int nv, int ldh, hipStream_t s) {
  if (nv < 1 || nv > kMaxRestart) return hipErrorInvalidValue;
  if (seg.total == 0) return hipSuccess;
  batch_update_dispatch(nv, tab, seg, ldh, s, std::make_integer_sequence<int, kMaxRestart>{});
  return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchSys *tab, const BatchSeg &seg, int ncols, bool dots, int src, hipStream_t s) {
  if (seg.total == 0) return hipSuccess;
  batch_reduce_kernel<<<seg.total, 256, 0, s>>>(tab, seg, ncols, dots ? 1 : 0, src);
  return hipGetLastError();
}

hipError_t launch_batch_norm_finalize(const BatchSys *tab, const BatchSeg &seg, int j, int ldh, int pub_stride,
                                      int src, hipStream_t s) {
  if (seg.total == 0) return hipSuccess;
  batch_norm_finalize_kernel<<<seg.total, 256, 0, s>>>(tab, seg, j, ldh, pub_stride, src);
  return hipGetLastError();
}

hipError_t launch_batch_lincomb(const BatchSys *tab, const BatchSeg &seg, hipStream_t s) {
  if (seg.total == 0) return hipSuccess;
  batch_lincomb_kernel<<<seg.total, 256, 0, s>>>(tab, seg);
  return hipGetLastError();
}

hipError_t launch_batch_axpy(const BatchSys *tab, const BatchSeg &seg, hipStream_t s) {
  if (seg.total == 0) return hipSuccess;
  batch_axpy_kernel<<<seg.total, 256, 0, s>>>(tab, seg);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double *p, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int grid = std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  fill_kernel<double><<<grid, 256, 0, s>>>(n, v, p);
  return hipGetLastError();
}
hipError_t launch_fill(int64_t n, int v, int *p, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int grid = std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  fill_kernel<int><<<grid, 256, 0, s>>>(n, v, p);
  return hipGetLastError();
}

hipError_t noalloc_scratch(void **out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  static std::mutex mu;
  static void *ptr[kMaxDevices] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    // with this device current: its own copy of the array
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return hipSuccess;
}

hipError_t launch_scale_copy(int64_t n, const double *r, const double *scale, double *z, hipStream_t s,
                             const int *skip) {
  const int grid = std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  scale_copy_kernel<<<grid, 256, 0, s>>>(n, r, scale, z, skip);
  return hipGetLastError();
}

}  // namespace asmx
