// Dense kernels of the global coarse-grid correction (Section 3, eq. (3.5)-
// (3.8)) and of exact local solves (Section 5).  The matrices are small (at
// most a few thousand unknowns), so each is inverted once per numeric setup
// and each application is one dense matrix-vector product.
#include <hip/hip_runtime.h>

#include "dense.hpp"

namespace asmx {
namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------- Gauss-Jordan steps
// Step k on one matrix of order n, one block: pivot row = largest |M[i][k]|,
// i >= k (ties: the lower row); rows k and p swapped in M and Minv; row k
// scaled by the pivot's inverse; fcol receives column k (0 on row k).
__device__ void gj_pivot_body(int n, int k, double *__restrict__ M, double *__restrict__ Minv,
                              double *__restrict__ fcol, int *__restrict__ bad) {
  __shared__ double sv[kThreads];
  __shared__ int si[kThreads];
  const int t = threadIdx.x;
  double best = -1.0;
  int bi = n;
  for (int i = k + t; i < n; i += kThreads) {
    const double v = fabs(M[(int64_t)i * n + k]);
    if (v > best) {  // rows visited in increasing order: ties keep the lower row
      best = v;
      bi = i;
    }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      const double ov = sv[t + w];
      const int oi = si[t + w];
      if (ov > sv[t] || (ov == sv[t] && oi < si[t])) {
        sv[t] = ov;
        si[t] = oi;
      }
    }
    __syncthreads();
  }
  const int p = si[0];
  const double pv = (p < n) ? M[(int64_t)p * n + k] : 0.0;
  if (!(fabs(pv) > 0.0) || !isfinite(pv)) {
    if (t == 0 && *bad < 0) *bad = k;
    for (int i = t; i < n; i += kThreads) fcol[i] = 0.0;  // leave the matrices as they are
    return;
  }
  if (p != k)
    for (int j = t; j < n; j += kThreads) {
      const double a = M[(int64_t)k * n + j], b = M[(int64_t)p * n + j];
      M[(int64_t)k * n + j] = b;
      M[(int64_t)p * n + j] = a;
      const double c = Minv[(int64_t)k * n + j], d = Minv[(int64_t)p * n + j];
      Minv[(int64_t)k * n + j] = d;
      Minv[(int64_t)p * n + j] = c;
    }
  __syncthreads();
  const double inv = 1.0 / pv;
  for (int j = t; j < n; j += kThreads) {
    M[(int64_t)k * n + j] = (j == k) ? 1.0 : M[(int64_t)k * n + j] * inv;
    Minv[(int64_t)k * n + j] *= inv;
  }
  __syncthreads();
  for (int i = t; i < n; i += kThreads) fcol[i] = (i == k) ? 0.0 : M[(int64_t)i * n + k];
}

// Step k, row i: row i -= fcol[i] * row k in M (columns >= k; row k is
// zero left of column k) and in Minv (all columns); jj indexes M's columns
// then Minv's.
__device__ __forceinline__ void gj_elim_body(int n, int k, int i, int jj, double *__restrict__ M,
                                             double *__restrict__ Minv, const double *__restrict__ fcol) {
  const double f = fcol[i];
  if (i == k || f == 0.0) return;
  if (jj < n) {
    if (jj < k) return;
    M[(int64_t)i * n + jj] = (jj == k) ? 0.0 : M[(int64_t)i * n + jj] - f * M[(int64_t)k * n + jj];
  } else if (jj < 2 * n) {
    const int j = jj - n;
    Minv[(int64_t)i * n + j] -= f * Minv[(int64_t)k * n + j];
  }
}

// Dot product of one row with a vector by one wavefront; lanes take
// columns lane, lane+64, ...; a fixed shuffle tree combines them.
__device__ __forceinline__ double wave_row_dot(const double *__restrict__ a, const double *__restrict__ x, int n,
                                               int lane) {
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += a[j] * x[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// ---------------------------------------------------------------- one matrix
__global__ void dense_zero_kernel(int64_t nn, int n, double *__restrict__ M, double *__restrict__ Minv) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= nn) return;
  M[i] = 0.0;
  Minv[i] = (i / n == i % n) ? 1.0 : 0.0;
}

// One thread per block row: its 3x3 blocks into the dense matrix.
__global__ void dense_scatter_kernel(int nbr, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                     const double *__restrict__ vals, double *__restrict__ M) {
  const int u = blockIdx.x * kThreads + threadIdx.x;
  if (u >= nbr) return;
  const int64_t n = 3 * (int64_t)nbr;
  for (int e = rp[u]; e < rp[u + 1]; ++e) {
    const int v = ci[e];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M[(3 * u + i) * n + 3 * v + j] = vals[9 * (int64_t)e + 3 * i + j];
  }
}

__global__ __launch_bounds__(kThreads) void gj_pivot_kernel(int n, int k, double *M, double *Minv, double *fcol,
                                                            int *bad) {
  gj_pivot_body(n, k, M, Minv, fcol, bad);
}

__global__ __launch_bounds__(kThreads) void gj_elim_kernel(int n, int k, double *M, double *Minv,
                                                           const double *fcol) {
  gj_elim_body(n, k, blockIdx.y, blockIdx.x * kThreads + threadIdx.x, M, Minv, fcol);
}

__global__ __launch_bounds__(kThreads) void dense_gemv_kernel(int n, const double *__restrict__ A,
                                                              const double *__restrict__ x, double *__restrict__ y) {
  const int row = blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= n) return;
  const double s = wave_row_dot(A + (int64_t)row * n, x, n, lane);
  if (lane == 0) y[row] = s;
}

__global__ void prolong_add_kernel(int N, const int32_t *__restrict__ cvar, const double *__restrict__ xc,
                                   double *__restrict__ z) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= N) return;
  const int b = cvar[c];
  z[3 * (int64_t)c] += xc[3 * b];
  z[3 * (int64_t)c + 1] += xc[3 * b + 1];
  z[3 * (int64_t)c + 2] += xc[3 * b + 2];
}

// ---------------------------------------------------------------- one matrix per subdomain
// grid (blocks over the largest matrix, nsub): zero M, identity Minv.
__global__ void local_zero_kernel(DenseLocal d) {
  const int s = blockIdx.y;
  const int n = 3 * d.sub[s].n;
  const int64_t nn = (int64_t)n * n;
  double *M = d.M + d.doff[s], *Minv = d.Minv + d.doff[s];
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < nn; i += (int64_t)gridDim.x * kThreads) {
    M[i] = 0.0;
    Minv[i] = (i / n == i % n) ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) d.bad[s] = -1;
}

// grid (rows, nsub): the blocks of each row of A_i into M at sweep positions.
__global__ void local_scatter_kernel(DenseLocal d, const int32_t *__restrict__ arp, const int32_t *__restrict__ aci,
                                     const double *__restrict__ aval) {
  const int s = blockIdx.y;
  const SubDesc sd = d.sub[s];
  const int u = blockIdx.x * kThreads + threadIdx.x;
  if (u >= sd.n) return;
  const int64_t n = 3 * (int64_t)sd.n;
  double *M = d.M + d.doff[s];
  const int pu = d.lpos[sd.ext_off + u];
  for (int e = arp[sd.ext_off + u]; e < arp[sd.ext_off + u + 1]; ++e) {
    const int pv = d.lpos[sd.ext_off + aci[e]];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M[(3 * pu + i) * n + 3 * pv + j] = aval[9 * (int64_t)e + 3 * i + j];
  }
}

__global__ __launch_bounds__(kThreads) void local_gj_pivot_kernel(DenseLocal d, int k) {
  const int s = blockIdx.x;
  const SubDesc sd = d.sub[s];
  const int n = 3 * sd.n;
  if (k >= n) return;
  gj_pivot_body(n, k, d.M + d.doff[s], d.Minv + d.doff[s], d.fcol + 3 * (int64_t)sd.ext_off, d.bad + s);
}

__global__ __launch_bounds__(kThreads) void local_gj_elim_kernel(DenseLocal d, int k) {
  const int s = blockIdx.z;
  const SubDesc sd = d.sub[s];
  const int n = 3 * sd.n;
  const int i = blockIdx.y;
  if (k >= n || i >= n) return;
  gj_elim_body(n, k, i, blockIdx.x * kThreads + threadIdx.x, d.M + d.doff[s], d.Minv + d.doff[s],
               d.fcol + 3 * (int64_t)sd.ext_off);
}

// One wavefront per scalar row (3 per position): x_i = A_i^-1 rs_i, written
// to z for owned fine rows (restricted) or to yx at the row's backward
// position (additive).
__global__ __launch_bounds__(kThreads) void local_apply_kernel(DenseLocal d, int64_t nrows,
                                                               const double *__restrict__ rs, int restricted,
                                                               double *__restrict__ z, double *__restrict__ yx) {
  const int64_t row = blockIdx.x * (int64_t)(kThreads / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= nrows) return;
  const int64_t pos = row / 3;
  const int comp = (int)(row % 3);
  const int s = d.psub[pos];
  const SubDesc sd = d.sub[s];
  const int n = 3 * sd.n;
  const int64_t lr = 3 * (pos - sd.ext_off) + comp;
  const double v = wave_row_dot(d.Minv + d.doff[s] + lr * n, rs + 3 * (int64_t)sd.ext_off, n, lane);
  if (lane != 0) return;
  if (restricted) {
    const int c = d.pout[pos];
    if (c >= 0) z[3 * (int64_t)c + comp] = v;
  } else {
    yx[3 * (int64_t)d.pbpos[pos] + comp] = v;
  }
}

}  // namespace

hipError_t launch_dense_init(int nbr, const int32_t *rp, const int32_t *ci, const double *vals, double *M,
                             double *Minv, hipStream_t s) {
  const int n = 3 * nbr;
  const int64_t nn = (int64_t)n * n;
  if (nn == 0) return hipSuccess;
  dense_zero_kernel<<<(unsigned)((nn + kThreads - 1) / kThreads), kThreads, 0, s>>>(nn, n, M, Minv);
  dense_scatter_kernel<<<(nbr + kThreads - 1) / kThreads, kThreads, 0, s>>>(nbr, rp, ci, vals, M);
  return hipGetLastError();
}

hipError_t launch_gauss_jordan(int n, double *M, double *Minv, double *fcol, int *bad, hipStream_t s) {
  const dim3 eg((2 * n + kThreads - 1) / kThreads, n);
  for (int k = 0; k < n; ++k) {
    gj_pivot_kernel<<<1, kThreads, 0, s>>>(n, k, M, Minv, fcol, bad);
    gj_elim_kernel<<<eg, kThreads, 0, s>>>(n, k, M, Minv, fcol);
  }
  return hipGetLastError();
}

hipError_t launch_dense_gemv(int n, const double *Minv, const double *x, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  dense_gemv_kernel<<<(n + kThreads / 64 - 1) / (kThreads / 64), kThreads, 0, s>>>(n, Minv, x, y);
  return hipGetLastError();
}

hipError_t launch_prolong_add(int N, const int32_t *cvar, const double *xc, double *z, hipStream_t s) {
  if (N == 0) return hipSuccess;
  prolong_add_kernel<<<(N + kThreads - 1) / kThreads, kThreads, 0, s>>>(N, cvar, xc, z);
  return hipGetLastError();
}

hipError_t launch_local_dense_init(const DenseLocal &d, const int32_t *arp, const int32_t *aci, const double *aval,
                                   int max_n3, hipStream_t s) {
  if (d.nsub == 0 || max_n3 == 0) return hipSuccess;
  const int64_t nn = (int64_t)max_n3 * max_n3;
  const unsigned bx = (unsigned)std::min<int64_t>((nn + kThreads - 1) / kThreads, 4096);
  local_zero_kernel<<<dim3(bx, d.nsub), kThreads, 0, s>>>(d);
  local_scatter_kernel<<<dim3((max_n3 / 3 + kThreads - 1) / kThreads, d.nsub), kThreads, 0, s>>>(d, arp, aci, aval);
  return hipGetLastError();
}

hipError_t launch_local_gauss_jordan(const DenseLocal &d, int max_n3, hipStream_t s) {
  const dim3 eg((2 * max_n3 + kThreads - 1) / kThreads, max_n3, d.nsub);
  for (int k = 0; k < max_n3; ++k) {
    local_gj_pivot_kernel<<<d.nsub, kThreads, 0, s>>>(d, k);
    local_gj_elim_kernel<<<eg, kThreads, 0, s>>>(d, k);
  }
  return hipGetLastError();
}

hipError_t launch_local_dense_apply(const DenseLocal &d, int64_t npos, const double *rs, bool restricted, double *z,
                                    double *yx, hipStream_t s) {
  const int64_t nrows = 3 * npos;
  if (nrows == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((nrows + kThreads / 64 - 1) / (kThreads / 64));
  local_apply_kernel<<<blocks, kThreads, 0, s>>>(d, nrows, rs, restricted ? 1 : 0, z, yx);
  return hipGetLastError();
}

}  // namespace asmx
