// gfx950 kernels of the Schwarz-preconditioned GMRES solve.
//
// Everything on this path is HBM- or latency-bound (3x3 blocks are not a
// dense contraction), so the kernels are written for coalesced streaming
// with 64-wide wavefronts; no matrix cores are used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <utility>

#include "kernels.hpp"

namespace asmx {

namespace {

constexpr int kWave = 64;

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on
// XCD b % 8).  Remap so that each XCD walks a contiguous range of logical
// blocks: neighbouring rows then share that XCD's L2.  The grid is launched
// with 8 * ceil(nlogical / 8) blocks; logical indices >= nlogical are idle.
__device__ inline int xcd_logical_block(int nlogical) {
  const int per = (nlogical + 7) >> 3;
  const int b = blockIdx.x;
  return (b & 7) * per + (b >> 3);
}

inline int xcd_grid(int nlogical) { return ((nlogical + 7) >> 3) << 3; }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
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
template <bool RESID>
__global__ __launch_bounds__(256) void spmv_kernel(int N, int nlogical, const int32_t *__restrict__ sptr,
                                                   const int32_t *__restrict__ cols,
                                                   const double *__restrict__ vals,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ b, double *__restrict__ y,
                                                   double *__restrict__ partial) {
  __shared__ double red[4];
  const int lb = xcd_logical_block(nlogical);
  double nrm = 0.0;
  const int row = lb * 256 + (int)threadIdx.x;
  if (lb < nlogical && row < N) {
    const int slice = row >> 6, lane = row & 63;
    const int g0 = sptr[slice], g1 = sptr[slice + 1];
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    for (int g = g0; g < g1; ++g) {
      const int c = cols[(size_t)g * 64 + lane];
      const double *v = vals + (size_t)g * 576 + lane;
      const double x0 = x[3 * (size_t)c], x1 = x[3 * (size_t)c + 1], x2 = x[3 * (size_t)c + 2];
      y0 += v[0] * x0 + v[64] * x1 + v[128] * x2;
      y1 += v[192] * x0 + v[256] * x1 + v[320] * x2;
      y2 += v[384] * x0 + v[448] * x1 + v[512] * x2;
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
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
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

__global__ __launch_bounds__(256) void gather_sum3_kernel(int ndst, const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ idx,
                                                          const double *__restrict__ src,
                                                          const double *__restrict__ scale,
                                                          double *__restrict__ dst) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= ndst) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int t = ptr[d]; t < ptr[d + 1]; ++t) {
    const size_t q = (size_t)idx[t] * 3;
    a0 += src[q];
    a1 += src[q + 1];
    a2 += src[q + 2];
  }
  const double s = scale ? *scale : 1.0;
  dst[(size_t)d * 3] = s * a0;
  dst[(size_t)d * 3 + 1] = s * a1;
  dst[(size_t)d * 3 + 2] = s * a2;
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

__global__ __launch_bounds__(256) void relayout_kernel(int nslots, const int32_t *__restrict__ src,
                                                       const int32_t *__restrict__ base,
                                                       const int32_t *__restrict__ stride,
                                                       const uint8_t *__restrict__ to32,
                                                       const double *__restrict__ fact,
                                                       double *__restrict__ out64,
                                                       float *__restrict__ out32) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  const int e = src[t];
  const size_t b0 = (size_t)base[t];
  const size_t st = (size_t)stride[t];
  const bool f32 = to32 && to32[t];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double v = (e >= 0) ? fact[(size_t)e * 9 + q] : 0.0;
    if (f32) out32[b0 + q * st] = (float)v;
    else out64[b0 + q * st] = v;
  }
}

// ---------------------------------------------------------------- ILU(0) apply
// acc -= B y for a block stored with component stride S (FP64 or FP32).
template <typename T>
__device__ inline void sub_block(const T *__restrict__ B, size_t S, double y0, double y1, double y2,
                                 double &a0, double &a1, double &a2) {
  a0 -= (double)B[0] * y0 + (double)B[S] * y1 + (double)B[2 * S] * y2;
  a1 -= (double)B[3 * S] * y0 + (double)B[4 * S] * y1 + (double)B[5 * S] * y2;
  a2 -= (double)B[6 * S] * y0 + (double)B[7 * S] * y1 + (double)B[8 * S] * y2;
}

// Single-precision variant: the row's arithmetic runs in FP32.
__device__ inline void sub_block32(const float *__restrict__ B, size_t S, float y0, float y1, float y2,
                                   float &a0, float &a1, float &a2) {
  a0 -= B[0] * y0 + B[S] * y1 + B[2 * S] * y2;
  a1 -= B[3 * S] * y0 + B[4 * S] * y1 + B[5 * S] * y2;
  a2 -= B[6 * S] * y0 + B[7 * S] * y1 + B[8 * S] * y2;
}

// Rows of one step of a sweep.  FWD: y_u = rhs_u - sum L_uk y_k.
// !FWD: x_u = D_u^-1 (y_u - sum U_uj x_j), written over y_u.
template <bool FWD>
__device__ inline void sweep_step(const DevPlan &p, const SubDesc &sd, const Step &st, double *__restrict__ Y,
                                  const double *__restrict__ r, double sc, double *__restrict__ z,
                                  int restricted) {
  const int32_t *rowl = FWD ? p.frow : p.brow;
  const int32_t *coll = FWD ? p.fcol : p.bcol;
  const double *val = FWD ? p.fval : p.bval;
  const float *val32 = FWD ? p.fval32 : p.bval32;
  const size_t S = (size_t)st.nrows;
  if (st.mode == 0) {
    for (int j = threadIdx.x; j < st.nrows; j += blockDim.x) {
      const int u = rowl[st.pos + j];
      double a0, a1, a2;
      if (FWD) {
        const int src = p.rhs_src[sd.ext_off + u];
        if (src >= 0) {
          a0 = sc * r[3 * (size_t)src]; a1 = sc * r[3 * (size_t)src + 1]; a2 = sc * r[3 * (size_t)src + 2];
        } else {
          const double *q = p.crhs + 3 * (size_t)(-src - 1);
          a0 = q[0]; a1 = q[1]; a2 = q[2];
        }
      } else {
        a0 = Y[3 * u]; a1 = Y[3 * u + 1]; a2 = Y[3 * u + 2];
      }
      if (st.fp32) {
        float f0 = (float)a0, f1 = (float)a1, f2 = (float)a2;
        for (int k = 0; k < st.width; ++k) {
          const size_t slot = (size_t)st.eoff + (size_t)k * S + j;
          const int c = coll[slot];
          if (c < 0) continue;
          sub_block32(val32 + (size_t)st.eoff * 9 + (size_t)k * 9 * S + j, S, (float)Y[3 * c],
                      (float)Y[3 * c + 1], (float)Y[3 * c + 2], f0, f1, f2);
        }
        if (!FWD) {
          const float *D = p.bdinv32 + (size_t)st.pos * 9 + j;
          const float x0 = D[0] * f0 + D[S] * f1 + D[2 * S] * f2;
          const float x1 = D[3 * S] * f0 + D[4 * S] * f1 + D[5 * S] * f2;
          const float x2 = D[6 * S] * f0 + D[7 * S] * f1 + D[8 * S] * f2;
          f0 = x0; f1 = x1; f2 = x2;
        }
        a0 = f0; a1 = f1; a2 = f2;
      } else {
        for (int k = 0; k < st.width; ++k) {
          const size_t slot = (size_t)st.eoff + (size_t)k * S + j;
          const int c = coll[slot];
          if (c < 0) continue;
          sub_block<double>(val + (size_t)st.eoff * 9 + (size_t)k * 9 * S + j, S, Y[3 * c], Y[3 * c + 1],
                            Y[3 * c + 2], a0, a1, a2);
        }
        if (!FWD) {
          const double *D = p.bdinv + (size_t)st.pos * 9 + j;
          const double x0 = D[0] * a0 + D[S] * a1 + D[2 * S] * a2;
          const double x1 = D[3 * S] * a0 + D[4 * S] * a1 + D[5 * S] * a2;
          const double x2 = D[6 * S] * a0 + D[7 * S] * a1 + D[8 * S] * a2;
          a0 = x0; a1 = x1; a2 = x2;
        }
      }
      Y[3 * u] = a0; Y[3 * u + 1] = a1; Y[3 * u + 2] = a2;
      if (!FWD && restricted) {
        const int cell = p.out_cell[sd.ext_off + u];
        if (cell >= 0) {
          z[3 * (size_t)cell] = a0; z[3 * (size_t)cell + 1] = a1; z[3 * (size_t)cell + 2] = a2;
        }
      }
    }
  } else {
    // one wavefront per (long) row; lanes stride over its entries
    const int32_t *rp = (FWD ? p.frptr : p.brptr) + st.rptr;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    for (int j = wv; j < st.nrows; j += nw) {
      const int u = rowl[st.pos + j];
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int t = rp[j] + lane; t < rp[j + 1]; t += kWave) {
        const size_t slot = (size_t)st.eoff + t;
        const int c = coll[slot];
        if (st.fp32) sub_block<float>(val32 + slot * 9, 1, Y[3 * c], Y[3 * c + 1], Y[3 * c + 2], s0, s1, s2);
        else sub_block<double>(val + slot * 9, 1, Y[3 * c], Y[3 * c + 1], Y[3 * c + 2], s0, s1, s2);
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      if (lane == 0) {
        double a0, a1, a2;
        if (FWD) {
          const int src = p.rhs_src[sd.ext_off + u];
          if (src >= 0) {
            a0 = sc * r[3 * (size_t)src]; a1 = sc * r[3 * (size_t)src + 1]; a2 = sc * r[3 * (size_t)src + 2];
          } else {
            const double *q = p.crhs + 3 * (size_t)(-src - 1);
            a0 = q[0]; a1 = q[1]; a2 = q[2];
          }
        } else {
          a0 = Y[3 * u]; a1 = Y[3 * u + 1]; a2 = Y[3 * u + 2];
        }
        a0 += s0; a1 += s1; a2 += s2;
        if (!FWD) {
          double x0, x1, x2;
          if (st.fp32) {
            const float *D = p.bdinv32 + (size_t)st.pos * 9 + j;
            x0 = D[0] * a0 + D[S] * a1 + D[2 * S] * a2;
            x1 = D[3 * S] * a0 + D[4 * S] * a1 + D[5 * S] * a2;
            x2 = D[6 * S] * a0 + D[7 * S] * a1 + D[8 * S] * a2;
          } else {
            const double *D = p.bdinv + (size_t)st.pos * 9 + j;
            x0 = D[0] * a0 + D[S] * a1 + D[2 * S] * a2;
            x1 = D[3 * S] * a0 + D[4 * S] * a1 + D[5 * S] * a2;
            x2 = D[6 * S] * a0 + D[7 * S] * a1 + D[8 * S] * a2;
          }
          a0 = x0; a1 = x1; a2 = x2;
        }
        Y[3 * u] = a0; Y[3 * u + 1] = a1; Y[3 * u + 2] = a2;
        if (!FWD && restricted) {
          const int cell = p.out_cell[sd.ext_off + u];
          if (cell >= 0) {
            z[3 * (size_t)cell] = a0; z[3 * (size_t)cell + 1] = a1; z[3 * (size_t)cell + 2] = a2;
          }
        }
      }
    }
  }
}

// One workgroup per subdomain: gather (R_i), forward sweep, backward sweep,
// restricted write-back, all inside the workgroup with barriers between
// level steps.
__global__ __launch_bounds__(256) void ilu_apply_kernel(DevPlan p, const double *__restrict__ r,
                                                        const double *__restrict__ scale,
                                                        double *__restrict__ z, int restricted) {
  const SubDesc sd = p.sub[blockIdx.x];
  double *Y = p.yext + 3 * (size_t)sd.ext_off;
  const double sc = scale ? *scale : 1.0;
  for (int si = sd.fstep0; si < sd.fstep1; ++si) {
    const Step st = p.fstep[si];
    sweep_step<true>(p, sd, st, Y, r, sc, z, restricted);
    __threadfence_block();
    __syncthreads();
  }
  for (int si = sd.bstep0; si < sd.bstep1; ++si) {
    const Step st = p.bstep[si];
    sweep_step<false>(p, sd, st, Y, r, sc, z, restricted);
    __threadfence_block();
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void additive_combine_kernel(int N, const int32_t *__restrict__ cptr,
                                                               const int32_t *__restrict__ cidx,
                                                               const double *__restrict__ yext,
                                                               double *__restrict__ z) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int t = cptr[c]; t < cptr[c + 1]; ++t) {
    const size_t q = (size_t)cidx[t] * 3;
    a0 += yext[q]; a1 += yext[q + 1]; a2 += yext[q + 2];
  }
  z[3 * (size_t)c] = a0; z[3 * (size_t)c + 1] = a1; z[3 * (size_t)c + 2] = a2;
}

// ---------------------------------------------------------------- Krylov
// partial[b*(NV+1) + i] = sum over the block's elements of U_i . w (i < NV),
// partial[b*(NV+1) + NV] = w . w.
template <int NV>
__global__ __launch_bounds__(256) void multidot_kernel(int64_t n, const double *__restrict__ U, int64_t ldu,
                                                       const double *__restrict__ w,
                                                       double *__restrict__ partial) {
  __shared__ double red[4 * (NV + 1)];
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const double we = w[e];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += U[i * ldu + e] * we;
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
    partial[(size_t)blockIdx.x * (NV + 1) + threadIdx.x] = s;
  }
}

// out[c] = sum_b partial[b*ncols + c], fixed order: one workgroup per column.
__global__ __launch_bounds__(256) void reduce_cols_kernel(int nblocks, int ncols, const double *__restrict__ partial,
                                                          double *__restrict__ out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[(size_t)b * ncols + c];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) out[c] = s;
}

__global__ void finalize_dots_kernel(int nv, const double *__restrict__ d, const double *__restrict__ scale,
                                     double *__restrict__ Hcol, double *__restrict__ coef,
                                     double *__restrict__ wnorm) {
  const int i = threadIdx.x;
  if (i < nv) {
    const double h = scale[i] * d[i];
    Hcol[i] = h;
    coef[i] = h * scale[i];
  }
  if (i == 0) *wnorm = sqrt(d[nv]);
}

__global__ __launch_bounds__(256) void update_kernel(int64_t n, int nv, const double *__restrict__ U, int64_t ldu,
                                                     const double *__restrict__ coef,
                                                     const double *__restrict__ w, double *__restrict__ unew,
                                                     double *__restrict__ partial) {
  __shared__ double cs[kMaxRestart + 1];
  __shared__ double red[4];
  for (int i = threadIdx.x; i < nv; i += blockDim.x) cs[i] = coef[i];
  __syncthreads();
  double nrm = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double a = w[e];
    for (int i = 0; i < nv; ++i) a -= cs[i] * U[i * ldu + e];
    unew[e] = a;
    nrm += a * a;
  }
  const double s = block_sum<256>(nrm, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void finalize_norm_kernel(const double *__restrict__ nrm2, double *__restrict__ hout,
                                     double *__restrict__ scale_out) {
  if (threadIdx.x == 0) {
    const double h = sqrt(nrm2[0]);
    *hout = h;
    *scale_out = (h > 0.0) ? 1.0 / h : 0.0;
  }
}

__global__ __launch_bounds__(256) void lincomb_kernel(int64_t n, int nv, const double *__restrict__ U, int64_t ldu,
                                                      const double *__restrict__ coef, double *__restrict__ out) {
  __shared__ double cs[kMaxRestart + 1];
  for (int i = threadIdx.x; i < nv; i += blockDim.x) cs[i] = coef[i];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double a = 0.0;
    for (int i = 0; i < nv; ++i) a += cs[i] * U[i * ldu + e];
    out[e] = a;
  }
}

__global__ __launch_bounds__(256) void axpy_kernel(int64_t n, const double *__restrict__ z, double *__restrict__ x) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) x[e] += z[e];
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

__global__ __launch_bounds__(256) void scale_copy_kernel(int64_t n, const double *__restrict__ r, const double *__restrict__ scale,
                                                         double *__restrict__ z) {
  const double s = scale ? *scale : 1.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) z[e] = s * r[e];
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_sell_fill(const SellDev &A, const double *csr_vals, hipStream_t s) {
  const int nslots = A.ngroups * 64;
  if (nslots == 0) return hipSuccess;
  sell_fill_kernel<<<blocks_for(nslots, 256), 256, 0, s>>>(nslots, A.src, csr_vals, A.vals);
  return hipGetLastError();
}

hipError_t launch_spmv(const SellDev &A, const double *x, double *y, hipStream_t s) {
  const int nlog = blocks_for(A.N, 256);
  spmv_kernel<false><<<xcd_grid(nlog), 256, 0, s>>>(A.N, nlog, A.sptr, A.cols, A.vals, x, nullptr, y, nullptr);
  return hipGetLastError();
}

hipError_t launch_residual(const SellDev &A, const double *x, const double *b, double *r, double *partial,
                           int *nblocks_out, hipStream_t s) {
  const int nlog = blocks_for(A.N, 256);
  const int grid = xcd_grid(nlog);
  spmv_kernel<true><<<grid, 256, 0, s>>>(A.N, nlog, A.sptr, A.cols, A.vals, x, b, r, partial);
  *nblocks_out = grid;
  return hipGetLastError();
}

hipError_t launch_gather_sum9(int ndst, const int32_t *ptr, const int32_t *idx, const double *srcA, int32_t nA,
                              const double *srcB, double *dst, hipStream_t s) {
  if (ndst == 0) return hipSuccess;
  gather_sum9_kernel<<<blocks_for(ndst, 256), 256, 0, s>>>(ndst, ptr, idx, srcA, nA, srcB, dst);
  return hipGetLastError();
}

hipError_t launch_gather_sum3(int ndst, const int32_t *ptr, const int32_t *idx, const double *src,
                              const double *scale, double *dst, hipStream_t s) {
  if (ndst == 0) return hipSuccess;
  gather_sum3_kernel<<<blocks_for(ndst, 256), 256, 0, s>>>(ndst, ptr, idx, src, scale, dst);
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

hipError_t launch_ilu_apply(const DevPlan &p, const double *r, const double *scale, double *z, int restricted,
                            bool, hipStream_t s) {
  if (p.nsub == 0) return hipSuccess;
  ilu_apply_kernel<<<p.nsub, 256, 0, s>>>(p, r, scale, z, restricted);
  return hipGetLastError();
}

hipError_t launch_additive_combine(int N, const int32_t *cptr, const int32_t *cidx, const double *yext, double *z,
                                   hipStream_t s) {
  additive_combine_kernel<<<blocks_for(N, 256), 256, 0, s>>>(N, cptr, cidx, yext, z);
  return hipGetLastError();
}

template <int NV>
static void multidot_launch(int64_t n, const double *U, int64_t ldu, const double *w, double *partial, int grid,
                            hipStream_t s) {
  multidot_kernel<NV><<<grid, 256, 0, s>>>(n, U, ldu, w, partial);
}

template <int... Is>
static bool multidot_dispatch(int nv, int64_t n, const double *U, int64_t ldu, const double *w, double *partial,
                              int grid, hipStream_t s, std::integer_sequence<int, Is...>) {
  bool done = false;
  ((nv == Is + 1 ? (multidot_launch<Is + 1>(n, U, ldu, w, partial, grid, s), done = true) : false), ...);
  return done;
}

hipError_t launch_multidot(int64_t n, int nv, const double *U, int64_t ldu, const double *w, double *partial,
                           int *nblocks_out, hipStream_t s) {
  const int grid = std::min<int64_t>(kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  if (nv < 1 || nv > 32) return hipErrorInvalidValue;
  multidot_dispatch(nv, n, U, ldu, w, partial, grid, s, std::make_integer_sequence<int, 32>{});
  *nblocks_out = grid;
  return hipGetLastError();
}

hipError_t launch_reduce_cols(int nblocks, int ncols, const double *partial, double *out, hipStream_t s) {
  reduce_cols_kernel<<<ncols, 256, 0, s>>>(nblocks, ncols, partial, out);
  return hipGetLastError();
}

hipError_t launch_finalize_dots(int nv, const double *d, const double *scale, double *Hcol, double *coef,
                                double *wnorm, hipStream_t s) {
  finalize_dots_kernel<<<1, 64, 0, s>>>(nv, d, scale, Hcol, coef, wnorm);
  return hipGetLastError();
}

hipError_t launch_update(int64_t n, int nv, const double *U, int64_t ldu, const double *coef, const double *w,
                         double *unew, double *partial, int *nblocks_out, hipStream_t s) {
  const int grid = std::min<int64_t>(kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  update_kernel<<<grid, 256, 0, s>>>(n, nv, U, ldu, coef, w, unew, partial);
  *nblocks_out = grid;
  return hipGetLastError();
}

hipError_t launch_finalize_norm(const double *nrm2, double *hout, double *scale_out, hipStream_t s) {
  finalize_norm_kernel<<<1, 64, 0, s>>>(nrm2, hout, scale_out);
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

hipError_t launch_scale_copy(int64_t n, const double *r, const double *scale, double *z, hipStream_t s) {
  const int grid = std::min<int64_t>(4 * kReduceBlocks, std::max<int64_t>(1, (n + 255) / 256));
  scale_copy_kernel<<<grid, 256, 0, s>>>(n, r, scale, z);
  return hipGetLastError();
}

}  // namespace asmx
