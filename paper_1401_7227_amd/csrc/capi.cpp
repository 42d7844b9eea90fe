// C ABI: system and preconditioner handles, numeric setup on the device, and
// the restarted right-preconditioned GMRES driver.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/asm.h"
#include "kernels.hpp"
#include "setup.hpp"

namespace asmx {
namespace {

thread_local std::string g_err;

asm_status fail(asm_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define ASM_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(e_ == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP,                     \
                  std::string(#call) + ": " + hipGetErrorString(e_));                        \
  } while (0)

// Owner of device allocations; frees everything on destruction.
struct DevMem {
  std::vector<void *> ptrs;
  size_t bytes = 0;
  ~DevMem() { release(); }
  void release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
  template <typename T>
  hipError_t alloc(T **out, size_t n) {
    *out = nullptr;
    if (n == 0) n = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) return e;
    ptrs.push_back(p);
    bytes += n * sizeof(T);
    *out = static_cast<T *>(p);
    return hipSuccess;
  }
  template <typename T>
  hipError_t upload(T **out, const std::vector<T> &v, hipStream_t s) {
    hipError_t e = alloc(out, v.size());
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
  }
};

struct GatherDev {
  int32_t n = 0;
  int32_t lanes = 1;  // threads per destination (about the mean fan-in)
  int32_t *ptr = nullptr, *idx = nullptr;
};

hipError_t upload_gather(DevMem &m, GatherDev &g, const GatherList &h, hipStream_t s) {
  g.n = h.size();
  const double mean = g.n > 0 ? (double)h.idx.size() / g.n : 0.0;
  g.lanes = 1;
  while (g.lanes < 16 && g.lanes < mean) g.lanes *= 2;
  hipError_t e = m.upload(&g.ptr, h.ptr, s);
  if (e == hipSuccess) e = m.upload(&g.idx, h.idx, s);
  return e;
}

// HIP-event timing of solve phases (enabled per system).
struct Profiler {
  bool on = false;
  uint32_t mask = 0;  // phases timed (bit k = phase k)
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  struct Span {
    int phase;
    size_t a, b;
  };
  std::vector<Span> pend;
  int64_t launches[ASM_NPHASE] = {};
  double ms[ASM_NPHASE] = {};
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  // Records an event if the phase is timed; returns its pool index, or
  // SIZE_MAX when not timed.
  size_t mark(int phase, hipStream_t s) {
    if (!on || !(mask >> phase & 1u)) return SIZE_MAX;
    return record(s);
  }
  size_t record(hipStream_t s) {
    if (next == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return SIZE_MAX;
      pool.push_back(e);
    }
    const size_t i = next++;
    if (hipEventRecord(pool[i], s) != hipSuccess) return SIZE_MAX;
    return i;
  }
  void span(int phase, size_t a, hipStream_t s) {
    if (!on || a == SIZE_MAX) return;
    const size_t b = record(s);
    if (b != SIZE_MAX) pend.push_back({phase, a, b});
  }
  // Only after the stream has been synchronised.
  void flush() {
    for (const Span &p : pend) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, pool[p.a], pool[p.b]) == hipSuccess) {
        ms[p.phase] += t;
        launches[p.phase]++;
      }
    }
    pend.clear();
    next = 0;
  }
  void reset() {
    std::fill(launches, launches + ASM_NPHASE, 0);
    std::fill(ms, ms + ASM_NPHASE, 0.0);
  }
};

// Krylov workspace of a system, sized for one restart length.
struct Workspace {
  DevMem mem;
  int m = 0;
  double *U = nullptr;        // (m+1) columns of n (stride ldu) basis (unnormalised)
  int64_t ldu = 0;
  double *w = nullptr, *z = nullptr, *t = nullptr;
  double *partial = nullptr;  // kReduceBlocks x (kMaxRestart+2)
  double *dvec = nullptr;     // reduced dot products
  double *H = nullptr;        // (m+1) x m Hessenberg, column-major, ld m+1
  double *scale = nullptr;    // 1/||U_i||
  double *coef = nullptr;
  double *misc = nullptr;     // [0] wnorm, [1] beta, [2] scratch norm
  int *flag = nullptr;
  double *pinned = nullptr;   // host staging: scalars, then one published column per step
  double *pinned_dev = nullptr;  // the same memory as seen by kernels
  hipEvent_t step_done[kMaxRestart] = {};
  ~Workspace() {
    if (pinned) (void)hipHostFree(pinned);
    for (hipEvent_t e : step_done)
      if (e) (void)hipEventDestroy(e);
  }
};

// Pinned layout: [0, 16) scalars; column j of a cycle at kPubBase + j*kPubStride
// holds H(0..j+1, j) and then ||w|| (the breakdown reference).
constexpr int kPubBase = 16, kPubStride = kMaxRestart + 4;

}  // namespace
}  // namespace asmx

using namespace asmx;

struct asm_system_s {
  int device = 0;
  HostPattern pat;
  DevMem mem;
  int32_t *rp = nullptr, *ci = nullptr;
  double *vals = nullptr;  // CSR values (sources of the assembly)
  SellDev sell;
  Workspace ws;
  Profiler prof;
};

struct asm_precond_s {
  asm_system sys = nullptr;
  asm_precond_opts opts{};
  PlanHost plan;  // small host-side parts kept for export and messages
  DevMem mem;
  DevPlan dp{};     // factorisation
  ApplyPlan ap{};   // sweeps
  GatherDev l1, l2, asrc, c1, c2, c3;
  double *L1 = nullptr, *L2 = nullptr;  // lumped block values
  double *aval = nullptr;               // assembled A_i (CSR)
  double *PA = nullptr, *PNF = nullptr; // lumped residual sums
  void *recbuf = nullptr;               // sweep records
  int32_t *rl_src = nullptr, *rl_base = nullptr, *rl_stride = nullptr;
  uint8_t *rl_to32 = nullptr;
  int64_t rl_n = 0;
  int32_t *cptr = nullptr, *cidx = nullptr;
  unsigned long long *bad = nullptr;
  asm_precond_stats stats{};
};

namespace {

asm_status ensure_workspace(asm_system S, int m, hipStream_t s) {
  Workspace &W = S->ws;
  if (W.m >= m && W.U) return ASM_OK;
  W.mem.release();
  if (W.pinned) {
    (void)hipHostFree(W.pinned);
    W.pinned = nullptr;
  }
  const size_t n = 3 * (size_t)S->pat.N;
  W.ldu = (int64_t)((n + 1) & ~(size_t)1);  // even: 16-byte aligned columns
  ASM_HIP(W.mem.alloc(&W.U, (size_t)(m + 1) * W.ldu));
  ASM_HIP(W.mem.alloc(&W.w, n));
  ASM_HIP(W.mem.alloc(&W.z, n));
  ASM_HIP(W.mem.alloc(&W.t, n));
  ASM_HIP(W.mem.alloc(&W.partial, (size_t)kReduceBlocks * (kMaxRestart + 2) + 8 * (size_t)kReduceBlocks));
  ASM_HIP(W.mem.alloc(&W.dvec, kMaxRestart + 2));
  ASM_HIP(W.mem.alloc(&W.H, (size_t)(m + 1) * m));
  ASM_HIP(W.mem.alloc(&W.scale, m + 1));
  ASM_HIP(W.mem.alloc(&W.coef, m + 1));
  ASM_HIP(W.mem.alloc(&W.misc, 8));
  ASM_HIP(W.mem.alloc(&W.flag, 4));
  ASM_HIP(hipHostMalloc((void **)&W.pinned, sizeof(double) * (kPubBase + (size_t)kMaxRestart * kPubStride),
                        hipHostMallocCoherent));
  ASM_HIP(hipHostGetDevicePointer((void **)&W.pinned_dev, W.pinned, 0));
  for (hipEvent_t &e : W.step_done)
    if (!e) ASM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  W.m = m;
  (void)s;
  return ASM_OK;
}

// Non-finite check of a device vector (synchronises the stream).
asm_status any_nonfinite(asm_system S, const double *v, int64_t n, hipStream_t s, bool *out) {
  ASM_HIP(hipMemsetAsync(S->ws.flag, 0, sizeof(int), s));
  ASM_HIP(launch_check_finite(n, v, S->ws.flag, s));
  int h = 0;
  ASM_HIP(hipMemcpyAsync(&h, S->ws.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  ASM_HIP(hipStreamSynchronize(s));
  *out = (h != 0);
  return ASM_OK;
}

asm_status build_sell(asm_system S, hipStream_t s) {
  const HostPattern &P = S->pat;
  SellDev &A = S->sell;
  A.N = P.N;
  A.nslices = (P.N + 63) / 64;
  std::vector<int32_t> sptr(A.nslices + 1, 0);
  for (int sl = 0; sl < A.nslices; ++sl) {
    int w = 0;
    for (int r = sl * 64; r < std::min(P.N, sl * 64 + 64); ++r) w = std::max(w, P.rp[r + 1] - P.rp[r]);
    sptr[sl + 1] = sptr[sl] + w;
  }
  A.ngroups = sptr[A.nslices];
  std::vector<int32_t> cols((size_t)A.ngroups * 64), src((size_t)A.ngroups * 64);
  for (int sl = 0; sl < A.nslices; ++sl)
    for (int g = sptr[sl]; g < sptr[sl + 1]; ++g) {
      const int k = g - sptr[sl];
      for (int lane = 0; lane < 64; ++lane) {
        const int r = sl * 64 + lane;
        const size_t slot = (size_t)g * 64 + lane;
        if (r < P.N && k < P.rp[r + 1] - P.rp[r]) {
          cols[slot] = P.ci[P.rp[r] + k];
          src[slot] = P.rp[r] + k;
        } else {
          cols[slot] = (r < P.N) ? r : 0;  // padding reads a valid row
          src[slot] = -1;
        }
      }
    }
  ASM_HIP(S->mem.upload(&A.sptr, sptr, s));
  ASM_HIP(S->mem.upload(&A.cols, cols, s));
  ASM_HIP(S->mem.upload(&A.src, src, s));
  ASM_HIP(S->mem.alloc(&A.vals, (size_t)A.ngroups * 9 * 64));
  ASM_HIP(launch_sell_fill(A, S->vals, s));
  return ASM_OK;
}

// Assembly (lumped matrices, A_i values) and factorisation on the device.
asm_status numeric_setup(asm_precond pc, hipStream_t s) {
  asm_system S = pc->sys;
  const PlanHost &P = pc->plan;
  if (pc->l1.n > 0) {
    ASM_HIP(launch_gather_sum9(pc->l1.n, pc->l1.ptr, pc->l1.idx, S->vals, INT32_MAX, nullptr, pc->L1, s));
    ASM_HIP(launch_gather_sum9(pc->l2.n, pc->l2.ptr, pc->l2.idx, pc->L1, INT32_MAX, nullptr, pc->L2, s));
  }
  ASM_HIP(launch_gather_sum9(pc->asrc.n, pc->asrc.ptr, pc->asrc.idx, S->vals, (int32_t)S->pat.nnzb, pc->L2,
                             pc->aval, s));
  ASM_HIP(hipMemcpyAsync(pc->dp.fact, pc->aval, (size_t)P.total_entries * 9 * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  ASM_HIP(hipMemsetAsync(pc->bad, 0xff, sizeof(unsigned long long), s));
  ASM_HIP(launch_ilu_factor(pc->dp, pc->bad, s));
  ASM_HIP(launch_relayout((int)pc->rl_n, pc->rl_src, pc->rl_base, pc->rl_stride, pc->rl_to32, pc->dp.fact,
                          static_cast<double *>(pc->recbuf), static_cast<float *>(pc->recbuf), s));
  unsigned long long bad = 0;
  ASM_HIP(hipMemcpyAsync(&bad, pc->bad, sizeof bad, hipMemcpyDeviceToHost, s));
  ASM_HIP(hipStreamSynchronize(s));
  if (bad != ~0ull) {
    const int sub = (int)(bad >> 32), row = (int)(bad & 0xffffffffu);
    const SubDesc &d = P.sub[sub];
    const int cell = (row < d.nfine) ? P.rhs_src[d.ext_off + row] : -1;
    return fail(ASM_ERR_SINGULAR_PIVOT, "singular pivot in subdomain " + std::to_string(sub) + ", local block row " +
                                            std::to_string(row) + " (global cell " + std::to_string(cell) + ")");
  }
  return ASM_OK;
}

asm_status apply_precond(asm_precond pc, const double *r, const double *scale, double *z, hipStream_t s,
                         Profiler *prof = nullptr) {
  asm_system S = pc->sys;
  const int64_t n = 3 * (int64_t)S->pat.N;
  Profiler dummy;
  Profiler &pf = prof ? *prof : dummy;
  if (pc->opts.kind == ASM_KIND_NONE) {
    const size_t t0 = pf.mark(ASM_PHASE_OTHER, s);
    ASM_HIP(launch_scale_copy(n, r, scale, z, s));
    pf.span(ASM_PHASE_OTHER, t0, s);
    return ASM_OK;
  }
  const size_t t0 = pf.mark(ASM_PHASE_LUMP, s);
  if (pc->c1.n > 0) {
    ASM_HIP(launch_gather_sum3(pc->c1.n, pc->c1.lanes, pc->c1.ptr, pc->c1.idx, r, scale, pc->PA, s));
    ASM_HIP(launch_gather_sum3(pc->c2.n, pc->c2.lanes, pc->c2.ptr, pc->c2.idx, pc->PA, nullptr, pc->PNF, s));
  }
  ASM_HIP(launch_gather_rhs((int)pc->plan.total_pos, pc->ap, r, scale, s));
  pf.span(ASM_PHASE_LUMP, t0, s);
  const bool restricted = pc->opts.combine == ASM_COMBINE_RESTRICTED;
  const size_t t1 = pf.mark(ASM_PHASE_ILU_APPLY, s);
  ASM_HIP(launch_ilu_apply(pc->ap, z, s));
  pf.span(ASM_PHASE_ILU_APPLY, t1, s);
  if (!restricted) {
    const size_t t2 = pf.mark(ASM_PHASE_COMBINE, s);
    ASM_HIP(launch_additive_combine(S->pat.N, pc->cptr, pc->cidx, pc->ap.yx, z, s));
    pf.span(ASM_PHASE_COMBINE, t2, s);
  }
  return ASM_OK;
}

}  // namespace

extern "C" {

const char *asm_last_error(void) { return g_err.c_str(); }

asm_status asm_create_system(const asm_grid *grid, int32_t nb, int64_t nnzb, const int32_t *row_ptr_dev,
                             const int32_t *col_idx_dev, const double *vals_dev, hipStream_t stream,
                             asm_system *out) {
  g_err.clear();
  if (!out) return fail(ASM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!grid || !row_ptr_dev || !col_idx_dev || !vals_dev) return fail(ASM_ERR_INVALID, "NULL argument");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || (int64_t)grid->nx * grid->ny * grid->nz != nb)
    return fail(ASM_ERR_INVALID, "grid nx*ny*nz does not equal nb");
  if (nnzb < nb || nnzb >= ((int64_t)1 << 31) / 9) return fail(ASM_ERR_INVALID, "nnzb out of range");
  auto S = new (std::nothrow) asm_system_s();
  if (!S) return fail(ASM_ERR_OOM, "host allocation failed");
  auto cleanup = [&](asm_status st) {
    delete S;
    return st;
  };
  (void)hipGetDevice(&S->device);
  HostPattern &P = S->pat;
  P.nx = grid->nx; P.ny = grid->ny; P.nz = grid->nz; P.N = nb; P.nnzb = nnzb;
  P.rp.resize(nb + 1);
  P.ci.resize(nnzb);
  hipError_t e = hipMemcpyAsync(P.rp.data(), row_ptr_dev, (nb + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P.ci.data(), col_idx_dev, nnzb * sizeof(int32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return cleanup(fail(ASM_ERR_HIP, std::string("pattern copy: ") + hipGetErrorString(e)));
  if (P.rp[0] != 0 || P.rp[nb] != nnzb) return cleanup(fail(ASM_ERR_INVALID, "row_ptr must start at 0 and end at nnzb"));
  for (int r = 0; r < nb; ++r) {
    if (P.rp[r + 1] < P.rp[r]) return cleanup(fail(ASM_ERR_INVALID, "row_ptr not monotone at row " + std::to_string(r)));
    bool diag = false;
    for (int q = P.rp[r]; q < P.rp[r + 1]; ++q) {
      const int c = P.ci[q];
      if (c < 0 || c >= nb) return cleanup(fail(ASM_ERR_INVALID, "column out of range in row " + std::to_string(r)));
      if (q > P.rp[r] && P.ci[q - 1] >= c)
        return cleanup(fail(ASM_ERR_INVALID, "columns not strictly increasing in row " + std::to_string(r)));
      diag |= (c == r);
    }
    if (!diag) return cleanup(fail(ASM_ERR_INVALID, "missing diagonal block in row " + std::to_string(r)));
  }
  if ((e = S->mem.upload(&S->rp, P.rp, stream)) != hipSuccess ||
      (e = S->mem.upload(&S->ci, P.ci, stream)) != hipSuccess ||
      (e = S->mem.alloc(&S->vals, (size_t)nnzb * 9)) != hipSuccess)
    return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
  if ((e = hipMemcpyAsync(S->vals, vals_dev, (size_t)nnzb * 9 * sizeof(double), hipMemcpyDeviceToDevice, stream)) !=
      hipSuccess)
    return cleanup(fail(ASM_ERR_HIP, hipGetErrorString(e)));
  asm_status st = ensure_workspace(S, 1, stream);
  if (st != ASM_OK) return cleanup(st);
  bool bad = false;
  if ((st = any_nonfinite(S, S->vals, (int64_t)nnzb * 9, stream, &bad)) != ASM_OK) return cleanup(st);
  if (bad) return cleanup(fail(ASM_ERR_NONFINITE, "non-finite matrix value"));
  if ((st = build_sell(S, stream)) != ASM_OK) return cleanup(st);
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return cleanup(fail(ASM_ERR_HIP, hipGetErrorString(e)));
  *out = S;
  return ASM_OK;
}

asm_status asm_update_values(asm_system S, const double *vals_dev, hipStream_t stream) {
  g_err.clear();
  if (!S || !vals_dev) return fail(ASM_ERR_INVALID, "NULL argument");
  ASM_HIP(hipMemcpyAsync(S->vals, vals_dev, (size_t)S->pat.nnzb * 9 * sizeof(double), hipMemcpyDeviceToDevice,
                         stream));
  bool bad = false;
  asm_status st = any_nonfinite(S, S->vals, S->pat.nnzb * 9, stream, &bad);
  if (st != ASM_OK) return st;
  if (bad) return fail(ASM_ERR_NONFINITE, "non-finite matrix value");
  ASM_HIP(launch_sell_fill(S->sell, S->vals, stream));
  return ASM_OK;
}

asm_status asm_spmv(asm_system S, const double *x_dev, double *y_dev, hipStream_t stream) {
  g_err.clear();
  if (!S || !x_dev || !y_dev) return fail(ASM_ERR_INVALID, "NULL argument");
  ASM_HIP(launch_spmv(S->sell, x_dev, y_dev, stream));
  return ASM_OK;
}

asm_status asm_setup_precond(asm_system S, const asm_precond_opts *o, hipStream_t stream, asm_precond *out) {
  g_err.clear();
  if (!S || !o || !out) return fail(ASM_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (o->kind < ASM_KIND_NONE || o->kind > ASM_KIND_TWO_LEVEL) return fail(ASM_ERR_INVALID, "bad kind");
  if (o->combine != ASM_COMBINE_ADDITIVE && o->combine != ASM_COMBINE_RESTRICTED)
    return fail(ASM_ERR_INVALID, "bad combine");
  if (o->precision != ASM_PREC_FP64 && o->precision != ASM_PREC_FP32) return fail(ASM_ERR_INVALID, "bad precision");
  auto pc = new (std::nothrow) asm_precond_s();
  if (!pc) return fail(ASM_ERR_OOM, "host allocation failed");
  pc->sys = S;
  pc->opts = *o;
  if (o->kind == ASM_KIND_NONE) {
    *out = pc;
    return ASM_OK;
  }
  auto cleanup = [&](asm_status st) {
    delete pc;
    return st;
  };
  const HostPattern &A = S->pat;
  if (o->sx < 1 || o->sy < 1 || o->sx > A.nx || o->sy > A.ny || o->overlap < 0)
    return cleanup(fail(ASM_ERR_INVALID, "bad subdomain split or overlap"));
  if (o->kind == ASM_KIND_TWO_LEVEL)
    for (int d = 0; d < 3; ++d)
      if (o->near_box[d] < 1 || o->far_box[d] < 1) return cleanup(fail(ASM_ERR_INVALID, "bad coarsening box"));
  PlanHost &P = pc->plan;
  std::string err;
  asm_status st = build_plan(A, *o, P, err);
  if (st != ASM_OK) return cleanup(fail(st, err));
  DevMem &M = pc->mem;
  DevPlan &d = pc->dp;
  hipStream_t s = stream;
  auto up = [&](auto **dst, const auto &vec) { return M.upload(dst, vec, s); };
  hipError_t e = hipSuccess;
  SubDesc *dsub;
  int32_t *t32;
#define UP(dst, vec)                                                                           \
  if ((e = up(dst, vec)) != hipSuccess)                                                        \
    return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
  d.nsub = P.nsub;
  UP(&dsub, P.sub); d.sub = dsub;
  Step *dfst;
  UP(&dfst, P.fstep); d.fstep = dfst;
  UP(&t32, P.frow); d.frow = t32;
  UP(&t32, P.arp); d.arp = t32;
  UP(&t32, P.aci); d.aci = t32;
  UP(&t32, P.adiag); d.adiag = t32;
  UP(&t32, P.tptr); d.tptr = t32;
  UP(&t32, P.tdst); d.tdst = t32;
  UP(&t32, P.tsrc); d.tsrc = t32;
  UP(&pc->cptr, P.cptr);
  UP(&pc->cidx, P.cidx);
  UP(&pc->rl_src, P.rl.src);
  UP(&pc->rl_base, P.rl.base);
  UP(&pc->rl_stride, P.rl.stride);
  UP(&pc->rl_to32, P.rl.to32);
  pc->rl_n = (int64_t)P.rl.src.size();
  RecStep *drf, *drb;
  UP(&drf, P.rf);
  UP(&drb, P.rb);
  uint8_t *drec;
  UP(&drec, P.rec);
  UP(&t32, P.fsrc);
  ApplyPlan &ap = pc->ap;
  ap.nsub = P.nsub;
  ap.sub = dsub;
  ap.fstep = drf;
  ap.bstep = drb;
  ap.rec = drec;
  pc->recbuf = drec;
  ap.fsrc = t32;
#undef UP
  auto ALLOC = [&](auto **dst, size_t n) { return M.alloc(dst, n); };
  double *yx, *rs, *fact;
  if ((e = ALLOC(&yx, (size_t)P.total_pos * 3)) != hipSuccess ||
      (e = ALLOC(&rs, (size_t)P.total_pos * 3)) != hipSuccess ||
      (e = ALLOC(&fact, (size_t)P.total_entries * 9)) != hipSuccess ||
      (e = ALLOC(&pc->aval, (size_t)P.total_entries * 9)) != hipSuccess ||
      (e = ALLOC(&pc->bad, 1)) != hipSuccess)
    return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
  ap.yx = yx;
  ap.rs = rs;
  d.fact = fact;
  if ((e = upload_gather(M, pc->asrc, P.asm_src, s)) != hipSuccess)
    return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
  if (o->kind == ASM_KIND_TWO_LEVEL) {
    if ((e = upload_gather(M, pc->l1, P.l1, s)) != hipSuccess || (e = upload_gather(M, pc->l2, P.l2, s)) != hipSuccess ||
        (e = upload_gather(M, pc->c1, P.c1, s)) != hipSuccess || (e = upload_gather(M, pc->c2, P.c2, s)) != hipSuccess ||
        (e = upload_gather(M, pc->c3, P.c3, s)) != hipSuccess || (e = ALLOC(&pc->L1, (size_t)pc->l1.n * 9)) != hipSuccess ||
        (e = ALLOC(&pc->L2, (size_t)pc->l2.n * 9)) != hipSuccess ||
        (e = ALLOC(&pc->PA, (size_t)pc->c1.n * 3)) != hipSuccess ||
        (e = ALLOC(&pc->PNF, (size_t)pc->c2.n * 3)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
    ap.cptr3 = pc->c3.ptr;
    ap.cidx3 = pc->c3.idx;
    ap.pnf = pc->PNF;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return cleanup(fail(ASM_ERR_HIP, hipGetErrorString(e)));
  // keep only what export and error messages need on the host
  P.rl = RelayoutMap{};
  P.rec = std::vector<uint8_t>();
  P.frow = std::vector<int32_t>();
  P.fsrc = std::vector<int32_t>();
  P.tdst = std::vector<int32_t>();
  P.tsrc = std::vector<int32_t>();
  P.asm_src = GatherList{};
  P.l1 = GatherList{};
  P.l2 = GatherList{};
  st = numeric_setup(pc, s);
  if (st != ASM_OK) return cleanup(st);
  pc->stats.nsub = P.nsub;
  pc->stats.ext_rows = P.total_ext;
  pc->stats.coarse_rows = P.total_coarse;
  pc->stats.factor_blocks = P.total_entries;
  pc->stats.fine_row_blocks = P.fine_row_entries;
  pc->stats.max_levels = P.max_levels;
  pc->stats.device_bytes = (int64_t)M.bytes;
  pc->stats.sweep_steps = P.sweep_steps;
  pc->stats.reloaded_rows = P.lds_spilled_rows;
  *out = pc;
  return ASM_OK;
}

asm_status asm_refactor(asm_precond pc, hipStream_t stream) {
  g_err.clear();
  if (!pc) return fail(ASM_ERR_INVALID, "NULL argument");
  if (pc->opts.kind == ASM_KIND_NONE) return ASM_OK;
  return numeric_setup(pc, stream);
}

asm_status asm_precond_apply(asm_precond pc, const double *r_dev, double *z_dev, hipStream_t stream) {
  g_err.clear();
  if (!pc || !r_dev || !z_dev) return fail(ASM_ERR_INVALID, "NULL argument");
  return apply_precond(pc, r_dev, nullptr, z_dev, stream);
}

asm_status asm_precond_get_stats(asm_precond pc, asm_precond_stats *st) {
  g_err.clear();
  if (!pc || !st) return fail(ASM_ERR_INVALID, "NULL argument");
  *st = pc->stats;
  return ASM_OK;
}

asm_status asm_precond_export_sub(asm_precond pc, int32_t s, int32_t *n_out, int32_t *nnz_out, int32_t *rp_host,
                                  int32_t *ci_host, double *a_host, double *f_host, int32_t *label_host) {
  g_err.clear();
  if (!pc || pc->opts.kind == ASM_KIND_NONE) return fail(ASM_ERR_INVALID, "no subdomains");
  const PlanHost &P = pc->plan;
  if (s < 0 || s >= P.nsub) return fail(ASM_ERR_INVALID, "subdomain out of range");
  const SubDesc &d = P.sub[s];
  const int32_t e0 = P.arp[d.ext_off], e1 = P.arp[d.ext_off + d.n];
  if (n_out) *n_out = d.n;
  if (nnz_out) *nnz_out = e1 - e0;
  if (rp_host)
    for (int u = 0; u <= d.n; ++u) rp_host[u] = P.arp[d.ext_off + u] - e0;
  if (ci_host) std::copy(P.aci.begin() + e0, P.aci.begin() + e1, ci_host);
  if (a_host) ASM_HIP(hipMemcpy(a_host, pc->aval + (size_t)e0 * 9, (size_t)(e1 - e0) * 9 * sizeof(double), hipMemcpyDeviceToHost));
  if (f_host) ASM_HIP(hipMemcpy(f_host, pc->dp.fact + (size_t)e0 * 9, (size_t)(e1 - e0) * 9 * sizeof(double), hipMemcpyDeviceToHost));
  if (label_host) {
    const int N = pc->sys->pat.N;
    std::fill(label_host, label_host + N, -1);
    for (int u = 0; u < d.nfine; ++u) label_host[P.rhs_src[d.ext_off + u]] = u;
    // coarse rows: member near/far atoms -> fine atoms -> cells
    const int nNa_plus = (int)P.c2.size();
    (void)nNa_plus;
    for (int u = d.nfine; u < d.n; ++u) {
      const int q = -P.rhs_src[d.ext_off + u] - 1;
      for (int t = P.c3.ptr[q]; t < P.c3.ptr[q + 1]; ++t) {
        const int nf = P.c3.idx[t];
        for (int t2 = P.c2.ptr[nf]; t2 < P.c2.ptr[nf + 1]; ++t2) {
          const int a = P.c2.idx[t2];
          for (int t3 = P.c1.ptr[a]; t3 < P.c1.ptr[a + 1]; ++t3) label_host[P.c1.idx[t3]] = u;
        }
      }
    }
  }
  return ASM_OK;
}

asm_status asm_solve(asm_system S, asm_precond pc, const double *b, double *x, const asm_solve_opts *o,
                     hipStream_t s, asm_solve_info *info) {
  g_err.clear();
  if (!S || !pc || !b || !x || !o || !info) return fail(ASM_ERR_INVALID, "NULL argument");
  if (pc->sys != S) return fail(ASM_ERR_INVALID, "preconditioner belongs to another system");
  std::memset(info, 0, sizeof *info);
  const int m = o->restart;
  if (m < 1 || m > kMaxRestart || !(o->rtol >= 0.0) || o->max_iters < 1 || o->fixed_iters < 0)
    return fail(ASM_ERR_INVALID, "bad solver option");
  const int64_t n = 3 * (int64_t)S->pat.N;
  asm_status st = ensure_workspace(S, m, s);
  if (st != ASM_OK) return st;
  Workspace &W = S->ws;
  Profiler &pf = S->prof;
  bool bad = false;
  if ((st = any_nonfinite(S, b, n, s, &bad)) != ASM_OK) return st;
  if (!bad && (st = any_nonfinite(S, x, n, s, &bad)) != ASM_OK) return st;
  if (bad) return fail(ASM_ERR_NONFINITE, "non-finite b or x0");
  const int ld = m + 1;
  double *hp = W.pinned;
  int nb = 0;
  // ||b||
  ASM_HIP(launch_norm2(n, b, W.partial, &nb, s));
  ASM_HIP(launch_reduce_cols(nb, 1, W.partial, W.misc + 2, s));
  ASM_HIP(hipMemcpyAsync(hp, W.misc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  ASM_HIP(hipStreamSynchronize(s));
  const double bnorm = std::sqrt(hp[0]);
  if (bnorm == 0.0 && o->fixed_iters == 0) {
    ASM_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
    ASM_HIP(hipStreamSynchronize(s));
    return ASM_OK;
  }
  const double scl = bnorm > 0.0 ? bnorm : 1.0;
  const double tol = o->rtol * bnorm;
  auto true_residual = [&](double *beta) -> asm_status {
    int nbr = 0;
    const size_t t0 = pf.mark(ASM_PHASE_RESIDUAL, s);
    ASM_HIP(launch_residual(S->sell, x, b, W.U, W.partial, &nbr, s));
    pf.span(ASM_PHASE_RESIDUAL, t0, s);
    const size_t t1 = pf.mark(ASM_PHASE_OTHER, s);
    ASM_HIP(launch_reduce_cols(nbr, 1, W.partial, W.misc + 2, s));
    ASM_HIP(launch_finalize_norm(0, W.misc + 2, W.misc + 1, W.scale, nullptr, nullptr, s));
    pf.span(ASM_PHASE_OTHER, t1, s);
    ASM_HIP(hipMemcpyAsync(hp, W.misc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    ASM_HIP(hipStreamSynchronize(s));
    pf.flush();
    *beta = hp[0];
    return ASM_OK;
  };
  double beta = 0.0;
  if ((st = true_residual(&beta)) != ASM_OK) return st;
  info->rel_res_true = info->rel_res_est = beta / scl;
  if (o->fixed_iters == 0 && beta <= tol) return ASM_OK;
  const int limit = o->fixed_iters > 0 ? o->fixed_iters : o->max_iters;
  std::vector<double> H((size_t)ld * m), cs(m), sn(m), g(m + 1), y(m), sc(m + 1), coef(m + 1);
  auto Hh = [&](int i, int j) -> double & { return H[(size_t)j * ld + i]; };
  asm_status result = ASM_NOT_CONVERGED;
  // One Arnoldi step on the stream: z = B^-1 v_j, w = A z, CGS projections,
  // the new basis vector and its norm; the step's Hessenberg column is then
  // published to pinned memory and an event marks the step's end.
  auto enqueue_step = [&](int j) -> asm_status {
    const double *Uj = W.U + (size_t)j * W.ldu;
    asm_status e2 = apply_precond(pc, Uj, W.scale + j, W.z, s, &pf);
    if (e2 != ASM_OK) return e2;
    size_t t0 = pf.mark(ASM_PHASE_SPMV, s);
    ASM_HIP(launch_spmv(S->sell, W.z, W.w, s));
    pf.span(ASM_PHASE_SPMV, t0, s);
    int nbd = 0;
    t0 = pf.mark(ASM_PHASE_DOTS, s);
    ASM_HIP(launch_multidot(n, j + 1, W.U, W.ldu, W.w, W.partial, &nbd, s));
    pf.span(ASM_PHASE_DOTS, t0, s);
    t0 = pf.mark(ASM_PHASE_OTHER, s);
    ASM_HIP(launch_reduce_cols(nbd, j + 2, W.partial, W.dvec, s));
    ASM_HIP(launch_finalize_dots(j + 1, W.dvec, W.scale, W.H + (size_t)j * ld, W.coef, W.misc, s));
    pf.span(ASM_PHASE_OTHER, t0, s);
    int nbu = 0;
    t0 = pf.mark(ASM_PHASE_UPDATE, s);
    ASM_HIP(launch_update(n, j + 1, W.U, W.ldu, W.coef, W.w, W.U + (size_t)(j + 1) * W.ldu, W.partial, &nbu, s));
    pf.span(ASM_PHASE_UPDATE, t0, s);
    t0 = pf.mark(ASM_PHASE_OTHER, s);
    ASM_HIP(launch_reduce_cols(nbu, 1, W.partial, W.misc + 2, s));
    ASM_HIP(launch_finalize_norm(j + 1, W.misc + 2, W.H + (size_t)j * ld, W.scale + j + 1, W.misc,
                                 W.pinned_dev + kPubBase + (size_t)j * kPubStride, s));
    pf.span(ASM_PHASE_OTHER, t0, s);
    ASM_HIP(hipEventRecord(W.step_done[j], s));
    return ASM_OK;
  };
  while (true) {
    if (beta == 0.0) { result = ASM_OK; break; }
    info->cycles++;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    sc[0] = 1.0 / beta;
    // steps of this cycle: at most m, and never past the iteration limit
    const int kmax = std::min(m, limit - info->iters);
    int k = 0, queued = 0;
    if ((st = enqueue_step(0)) != ASM_OK) return st;
    queued = 1;
    for (int j = 0; j < kmax; ++j) {
      // keep the next step queued while step j's column is read back
      if (queued < kmax) {
        if ((st = enqueue_step(queued)) != ASM_OK) return st;
        ++queued;
      }
      ASM_HIP(hipEventSynchronize(W.step_done[j]));
      const double *col = hp + kPubBase + (size_t)j * kPubStride;
      for (int i = 0; i <= j + 1; ++i) Hh(i, j) = col[i];
      const double w0 = col[j + 2];
      const double hn = Hh(j + 1, j);
      sc[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
      // previous rotations, then a new one annihilating h_{j+1,j}
      for (int i = 0; i < j; ++i) {
        const double a = Hh(i, j), c = Hh(i + 1, j);
        Hh(i, j) = cs[i] * a + sn[i] * c;
        Hh(i + 1, j) = -sn[i] * a + cs[i] * c;
      }
      const double rho = std::hypot(Hh(j, j), Hh(j + 1, j));
      if (rho == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = Hh(j, j) / rho;
        sn[j] = Hh(j + 1, j) / rho;
      }
      Hh(j, j) = rho;
      Hh(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      info->rel_res_est = std::fabs(g[j + 1]) / scl;
      if (hn <= 1e-14 * w0) break;
      if (o->fixed_iters == 0 && std::fabs(g[j + 1]) <= tol) break;
    }
    info->iters += k;
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int j = i + 1; j < k; ++j) acc -= Hh(i, j) * y[j];
      y[i] = acc / Hh(i, i);
    }
    for (int i = 0; i < k; ++i) coef[i] = y[i] * sc[i];
    ASM_HIP(hipMemcpyAsync(W.coef, coef.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
    size_t t0 = pf.mark(ASM_PHASE_OTHER, s);
    ASM_HIP(launch_lincomb(n, k, W.U, W.ldu, W.coef, W.t, s));
    pf.span(ASM_PHASE_OTHER, t0, s);
    if ((st = apply_precond(pc, W.t, nullptr, W.z, s, &pf)) != ASM_OK) return st;
    t0 = pf.mark(ASM_PHASE_OTHER, s);
    ASM_HIP(launch_axpy(n, W.z, x, s));
    pf.span(ASM_PHASE_OTHER, t0, s);
    if ((st = true_residual(&beta)) != ASM_OK) return st;
    info->rel_res_true = beta / scl;
    if (o->fixed_iters > 0) {
      if (info->iters >= o->fixed_iters) { result = ASM_OK; break; }
    } else if (beta <= tol) {
      result = ASM_OK;
      break;
    }
    if (info->iters >= limit) { result = ASM_NOT_CONVERGED; break; }
  }
  ASM_HIP(hipStreamSynchronize(s));
  return result;
}

asm_status asm_solve_batch(int32_t count, const asm_system *systems, const asm_precond *preconds,
                           const double *const *b, double *const *x, const asm_solve_opts *o, hipStream_t s,
                           asm_solve_info *infos, int32_t *status) {
  g_err.clear();
  if (count < 1 || !systems || !preconds || !b || !x || !o || !infos || !status)
    return fail(ASM_ERR_INVALID, "NULL argument or empty batch");
  const int m = o->restart;
  if (m < 1 || m > kMaxRestart || !(o->rtol >= 0.0) || o->max_iters < 1 || o->fixed_iters < 0)
    return fail(ASM_ERR_INVALID, "bad solver option");
  for (int i = 0; i < count; ++i) {
    if (!systems[i] || !preconds[i] || !b[i] || !x[i]) return fail(ASM_ERR_INVALID, "NULL system, preconditioner or vector");
    if (preconds[i]->sys != systems[i]) return fail(ASM_ERR_INVALID, "preconditioner belongs to another system");
    for (int k = 0; k < i; ++k)
      if (systems[k] == systems[i]) return fail(ASM_ERR_INVALID, "a system appears twice in the batch");
  }
  asm_status st;
  for (int i = 0; i < count; ++i)
    if ((st = ensure_workspace(systems[i], m, s)) != ASM_OK) return st;
  const int ld = m + 1;
  // pinned area per system: [beta][m published columns][1 + m coefficients]
  const size_t region = 1 + (size_t)m * kPubStride + 1 + m;
  double *pin = nullptr, *pin_dev = nullptr;
  int32_t *segh = nullptr, *segd = nullptr;
  BatchSys *tabd = nullptr;
  struct Guard {
    double *&pin;
    int32_t *&segh, *&segd;
    BatchSys *&tabd;
    ~Guard() {
      if (pin) (void)hipHostFree(pin);
      if (segh) (void)hipHostFree(segh);
      if (segd) (void)hipFree(segd);
      if (tabd) (void)hipFree(tabd);
    }
  } guard{pin, segh, segd, tabd};
  ASM_HIP(hipHostMalloc((void **)&pin, sizeof(double) * (region * count + 16), hipHostMallocCoherent));
  ASM_HIP(hipHostGetDevicePointer((void **)&pin_dev, pin, 0));
  // per-system finiteness of b and x0, and ||b||
  for (int i = 0; i < count; ++i) {
    Workspace &W = systems[i]->ws;
    const int64_t n = 3 * (int64_t)systems[i]->pat.N;
    ASM_HIP(hipMemsetAsync(W.flag, 0, sizeof(int), s));
    ASM_HIP(launch_check_finite(n, b[i], W.flag, s));
    ASM_HIP(launch_check_finite(n, x[i], W.flag, s));
    int nb = 0;
    ASM_HIP(launch_norm2(n, b[i], W.partial, &nb, s));
    ASM_HIP(launch_reduce_cols(nb, 1, W.partial, W.misc + 2, s));
    ASM_HIP(hipMemcpyAsync(pin + region * i, W.misc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    ASM_HIP(hipMemcpyAsync(pin + region * i + 1, W.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  ASM_HIP(hipStreamSynchronize(s));
  std::vector<double> scl(count), tol(count), beta(count, 0.0);
  for (int i = 0; i < count; ++i) {
    int flag = 0;
    std::memcpy(&flag, pin + region * i + 1, sizeof(int));
    if (flag) return fail(ASM_ERR_NONFINITE, "non-finite b or x0 in batch entry " + std::to_string(i));
    const double bn = std::sqrt(pin[region * i]);
    scl[i] = bn > 0.0 ? bn : 1.0;
    tol[i] = o->rtol * bn;
    std::memset(&infos[i], 0, sizeof infos[i]);
    status[i] = ASM_NOT_CONVERGED;
  }
  // device table of the systems
  std::vector<BatchSys> tab(count);
  for (int i = 0; i < count; ++i) {
    asm_system S = systems[i];
    asm_precond pc = preconds[i];
    Workspace &W = S->ws;
    BatchSys &T = tab[i];
    std::memset(&T, 0, sizeof T);
    T.n = 3 * (int64_t)S->pat.N;
    T.ldu = W.ldu;
    T.U = W.U; T.w = W.w; T.z = W.z; T.t = W.t;
    T.partial = W.partial; T.dvec = W.dvec; T.H = W.H; T.scale = W.scale; T.coef = W.coef; T.misc = W.misc;
    T.pub = pin_dev + region * i + 1;
    T.coefh = pin_dev + region * i + 1 + (size_t)m * kPubStride;
    T.b = b[i];
    T.x = x[i];
    T.N = S->pat.N;
    T.nlog = (S->pat.N + 255) / 256;
    T.sptr = S->sell.sptr; T.cols = S->sell.cols; T.vals = S->sell.vals;
    T.kind = pc->opts.kind;
    T.restricted = pc->opts.combine == ASM_COMBINE_RESTRICTED;
    T.npos = (int32_t)pc->plan.total_pos;
    T.nsub = pc->ap.nsub;
    T.ap = pc->ap;
    T.c1n = pc->c1.n; T.c1lanes = pc->c1.lanes; T.c1ptr = pc->c1.ptr; T.c1idx = pc->c1.idx;
    T.c2n = pc->c2.n; T.c2lanes = pc->c2.lanes; T.c2ptr = pc->c2.ptr; T.c2idx = pc->c2.idx;
    T.PA = pc->PA; T.PNF = pc->PNF;
    T.cptr = pc->cptr; T.cidx = pc->cidx;
  }
  ASM_HIP(hipMalloc((void **)&tabd, sizeof(BatchSys) * count));
  ASM_HIP(hipMemcpyAsync(tabd, tab.data(), sizeof(BatchSys) * count, hipMemcpyHostToDevice, s));
  // Segment tables: one ring slot per launch group (a step, or a cycle
  // end), each holding the tables of every kernel kind for its systems.
  const int nslot = kMaxRestart + 4;
  const size_t slot_ints = (size_t)kBkCount * (2 * (size_t)count + 1);
  ASM_HIP(hipHostMalloc((void **)&segh, sizeof(int32_t) * slot_ints * nslot, hipHostMallocDefault));
  ASM_HIP(hipMalloc((void **)&segd, sizeof(int32_t) * slot_ints * nslot));
  int slot_next = 0;
  // Uploads the tables for the systems in `act`; fills seg[kBkCount].
  auto make_segs = [&](const std::vector<int> &act, BatchSeg *seg) -> asm_status {
    const int sl = slot_next;
    slot_next = (slot_next + 1) % nslot;
    int32_t *h = segh + slot_ints * sl, *d = segd + slot_ints * sl;
    const int na = (int)act.size();
    for (int k = 0; k < kBkCount; ++k) {
      int32_t *st0 = h + (size_t)k * (2 * count + 1), *sy = st0 + count + 1;
      int nseg = 0, tot = 0;
      for (int a = 0; a < na; ++a) {
        const BatchSys &T = tab[act[a]];
        int nb = batch_blocks((BatchKernel)k, T);
        if (k == kBkCopy && T.kind != ASM_KIND_NONE) nb = 0;
        if ((k == kBkC1 || k == kBkC2 || k == kBkRhs || k == kBkApply || k == kBkCombine) && T.kind == ASM_KIND_NONE) nb = 0;
        if (k == kBkCombine && T.restricted) nb = 0;
        if (nb <= 0) continue;
        st0[nseg] = tot;
        sy[nseg] = act[a];
        ++nseg;
        tot += nb;
      }
      st0[nseg] = tot;
      seg[k].start = d + (size_t)k * (2 * count + 1);
      seg[k].sys = seg[k].start + count + 1;
      seg[k].n = nseg;
      seg[k].total = tot;
    }
    ASM_HIP(hipMemcpyAsync(d, h, sizeof(int32_t) * slot_ints, hipMemcpyHostToDevice, s));
    return ASM_OK;
  };
  // the one-step-late readback needs the previous copy of a slot to have
  // run before the host rewrites it: ring slots are reused only after the
  // stream passed an event recorded after their last use
  std::vector<hipEvent_t> slot_ev(nslot, nullptr);
  struct EvGuard {
    std::vector<hipEvent_t> &v;
    ~EvGuard() {
      for (hipEvent_t e : v)
        if (e) (void)hipEventDestroy(e);
    }
  } evguard{slot_ev};
  for (hipEvent_t &e : slot_ev) ASM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  auto segs_for = [&](const std::vector<int> &act, BatchSeg *seg) -> asm_status {
    ASM_HIP(hipEventSynchronize(slot_ev[slot_next]));
    const int sl = slot_next;
    asm_status e2 = make_segs(act, seg);
    if (e2 != ASM_OK) return e2;
    (void)sl;
    return ASM_OK;
  };
  auto mark_slot = [&](int sl) -> asm_status {
    ASM_HIP(hipEventRecord(slot_ev[sl], s));
    return ASM_OK;
  };
  // true residuals of the systems in act (published as beta)
  auto residuals = [&](const std::vector<int> &act) -> asm_status {
    BatchSeg seg[kBkCount];
    const int sl = slot_next;
    asm_status e2 = segs_for(act, seg);
    if (e2 != ASM_OK) return e2;
    ASM_HIP(launch_batch_spmv(tabd, seg[kBkSpmv], true, s));
    ASM_HIP(launch_batch_reduce(tabd, seg[kBkOne], 1, false, 1, s));
    ASM_HIP(launch_batch_finalize_norm(tabd, seg[kBkOne], -1, ld, kPubStride, s));
    ASM_HIP(hipStreamSynchronize(s));
    (void)mark_slot(sl);
    for (int i : act) beta[i] = pin[region * i];
    return ASM_OK;
  };
  const int limit = o->fixed_iters > 0 ? o->fixed_iters : o->max_iters;
  std::vector<int> active;
  for (int i = 0; i < count; ++i) active.push_back(i);
  if ((st = residuals(active)) != ASM_OK) return st;
  {
    std::vector<int> keep;
    for (int i : active) {
      infos[i].rel_res_true = infos[i].rel_res_est = beta[i] / scl[i];
      if ((o->fixed_iters == 0 && beta[i] <= tol[i]) || beta[i] == 0.0) status[i] = ASM_OK;
      else keep.push_back(i);
    }
    active.swap(keep);
  }
  // host-side Arnoldi state per system
  std::vector<std::vector<double>> H(count), cs(count), sn(count), g(count), sc(count);
  std::vector<int> k(count, 0), kmax(count, 0);
  std::vector<char> in_cycle(count, 0);
  while (!active.empty()) {
    int K = 0;
    for (int i : active) {
      H[i].assign((size_t)ld * m, 0.0);
      cs[i].assign(m, 0.0);
      sn[i].assign(m, 0.0);
      g[i].assign(m + 1, 0.0);
      sc[i].assign(m + 1, 0.0);
      g[i][0] = beta[i];
      sc[i][0] = 1.0 / beta[i];
      k[i] = 0;
      kmax[i] = std::min(m, limit - infos[i].iters);
      in_cycle[i] = 1;
      infos[i].cycles++;
      K = std::max(K, kmax[i]);
    }
    std::vector<std::vector<int>> ran(K);  // systems that ran step j
    std::vector<int> ran_slot(K, 0);
    auto enqueue_step = [&](int j) -> asm_status {
      std::vector<int> act;
      for (int i : active)
        if (in_cycle[i] && kmax[i] > j) act.push_back(i);
      ran[j] = act;
      if (act.empty()) return ASM_OK;
      BatchSeg seg[kBkCount];
      const int sl = slot_next;
      asm_status e2 = segs_for(act, seg);
      if (e2 != ASM_OK) return e2;
      ran_slot[j] = sl;
      ASM_HIP(launch_batch_precond(tabd, seg, j, s));
      ASM_HIP(launch_batch_spmv(tabd, seg[kBkSpmv], false, s));
      ASM_HIP(launch_batch_multidot(tabd, seg[kBkRed], j + 1, s));
      ASM_HIP(launch_batch_reduce(tabd, seg[kBkOne], j + 2, true, 0, s));
      ASM_HIP(launch_batch_finalize_dots(tabd, seg[kBkOne], j, ld, s));
      ASM_HIP(launch_batch_update(tabd, seg[kBkRed], j + 1, ld, s));
      ASM_HIP(launch_batch_reduce(tabd, seg[kBkOne], 1, false, 0, s));
      ASM_HIP(launch_batch_finalize_norm(tabd, seg[kBkOne], j, ld, kPubStride, s));
      ASM_HIP(hipEventRecord(systems[0]->ws.step_done[j], s));
      return mark_slot(sl);
    };
    (void)ran_slot;
    if ((st = enqueue_step(0)) != ASM_OK) return st;
    for (int j = 0; j < K; ++j) {
      if (j + 1 < K && (st = enqueue_step(j + 1)) != ASM_OK) return st;
      if (ran[j].empty()) continue;
      ASM_HIP(hipEventSynchronize(systems[0]->ws.step_done[j]));
      for (int i : ran[j]) {
        if (!in_cycle[i]) continue;  // left the cycle at an earlier step; this step is discarded
        auto Hh = [&](int r, int c) -> double & { return H[i][(size_t)c * ld + r]; };
        const double *col = pin + region * i + 1 + (size_t)j * kPubStride;
        for (int r = 0; r <= j + 1; ++r) Hh(r, j) = col[r];
        const double w0 = col[j + 2];
        const double hn = Hh(j + 1, j);
        sc[i][j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
        for (int r = 0; r < j; ++r) {
          const double a = Hh(r, j), c = Hh(r + 1, j);
          Hh(r, j) = cs[i][r] * a + sn[i][r] * c;
          Hh(r + 1, j) = -sn[i][r] * a + cs[i][r] * c;
        }
        const double rho = std::hypot(Hh(j, j), Hh(j + 1, j));
        if (rho == 0.0) {
          cs[i][j] = 1.0;
          sn[i][j] = 0.0;
        } else {
          cs[i][j] = Hh(j, j) / rho;
          sn[i][j] = Hh(j + 1, j) / rho;
        }
        Hh(j, j) = rho;
        Hh(j + 1, j) = 0.0;
        g[i][j + 1] = -sn[i][j] * g[i][j];
        g[i][j] = cs[i][j] * g[i][j];
        k[i] = j + 1;
        infos[i].rel_res_est = std::fabs(g[i][j + 1]) / scl[i];
        if (hn <= 1e-14 * w0 || (o->fixed_iters == 0 && std::fabs(g[i][j + 1]) <= tol[i]) || k[i] >= kmax[i])
          in_cycle[i] = 0;
      }
    }
    // cycle end: x += B^-1 (V y) for every system of the cycle
    for (int i : active) {
      infos[i].iters += k[i];
      auto Hh = [&](int r, int c) -> double & { return H[i][(size_t)c * ld + r]; };
      std::vector<double> y(k[i]);
      for (int r = k[i] - 1; r >= 0; --r) {
        double acc = g[i][r];
        for (int c = r + 1; c < k[i]; ++c) acc -= Hh(r, c) * y[c];
        y[r] = acc / Hh(r, r);
      }
      double *coefh = pin + region * i + 1 + (size_t)m * kPubStride;
      coefh[0] = (double)k[i];
      for (int r = 0; r < k[i]; ++r) coefh[1 + r] = y[r] * sc[i][r];
    }
    {
      BatchSeg seg[kBkCount];
      const int sl = slot_next;
      if ((st = segs_for(active, seg)) != ASM_OK) return st;
      ASM_HIP(launch_batch_lincomb(tabd, seg[kBkVec], s));
      ASM_HIP(launch_batch_precond(tabd, seg, -1, s));
      ASM_HIP(launch_batch_axpy(tabd, seg[kBkVec], s));
      if ((st = mark_slot(sl)) != ASM_OK) return st;
    }
    if ((st = residuals(active)) != ASM_OK) return st;
    std::vector<int> keep;
    for (int i : active) {
      infos[i].rel_res_true = beta[i] / scl[i];
      if (o->fixed_iters > 0) {
        if (infos[i].iters >= o->fixed_iters) { status[i] = ASM_OK; continue; }
      } else if (beta[i] <= tol[i]) {
        status[i] = ASM_OK;
        continue;
      }
      if (infos[i].iters >= limit || beta[i] == 0.0) {
        status[i] = beta[i] == 0.0 ? ASM_OK : ASM_NOT_CONVERGED;
        continue;
      }
      keep.push_back(i);
    }
    active.swap(keep);
  }
  ASM_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i)
    if (status[i] != ASM_OK) return ASM_NOT_CONVERGED;
  return ASM_OK;
}

asm_status asm_profile_enable(asm_system S, int32_t phase_mask) {
  g_err.clear();
  if (!S) return fail(ASM_ERR_INVALID, "NULL argument");
  S->prof.on = (phase_mask != 0);
  S->prof.mask = (uint32_t)phase_mask;
  return ASM_OK;
}

asm_status asm_profile_read(asm_system S, asm_profile *out, int32_t reset) {
  g_err.clear();
  if (!S || !out) return fail(ASM_ERR_INVALID, "NULL argument");
  for (int k = 0; k < ASM_NPHASE; ++k) {
    out->launches[k] = S->prof.launches[k];
    out->ms[k] = S->prof.ms[k];
  }
  if (reset) S->prof.reset();
  return ASM_OK;
}

void asm_destroy_precond(asm_precond pc) { delete pc; }
void asm_destroy_system(asm_system S) { delete S; }

}  // extern "C"
