// C ABI: system and preconditioner handles, numeric setup on the device, and
// the restarted right-preconditioned GMRES driver.
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>

#include "handles.hpp"

namespace asmx {

thread_local std::string g_err;

namespace {
std::mutex g_alloc_mu;
Allocator g_allocator;
}  // namespace

Allocator current_allocator() {
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  return g_allocator;
}

asm_status ensure_workspace(asm_system S, int m, hipStream_t s) {
  Workspace &W = S->ws;
  if (W.m >= m && W.U) return ASM_OK;
  W.drop_graph();
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
  ASM_HIP(W.mem.alloc(&W.partial, (size_t)partial_doubles(S->pat.N)));
  ASM_HIP(W.mem.alloc(&W.dvec, kMaxRestart + 2));
  ASM_HIP(W.mem.alloc(&W.H, (size_t)(m + 1) * m));
  ASM_HIP(W.mem.alloc(&W.scale, m + 1));
  ASM_HIP(W.mem.alloc(&W.coef, m + 1));
  ASM_HIP(W.mem.alloc(&W.misc, 8));
  ASM_HIP(W.mem.alloc(&W.flag, 4));
  ASM_HIP(W.mem.alloc(&W.cst, 1));
  ASM_HIP(W.mem.alloc(&W.gcs, m + 1));
  ASM_HIP(W.mem.alloc(&W.gsn, m + 1));
  ASM_HIP(W.mem.alloc(&W.gg, m + 1));
  // scalars, published columns, then a cycle's solution coefficients
  ASM_HIP(hipHostMalloc((void **)&W.pinned,
                        sizeof(double) * (kPubBase + (size_t)kMaxRestart * kPubStride + kMaxRestart + 2),
                        hipHostMallocCoherent));
  ASM_HIP(hipHostGetDevicePointer((void **)&W.pinned_dev, W.pinned, 0));
  for (hipEvent_t &e : W.step_done)
    if (!e) ASM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  W.m = m;
  (void)s;
  return ASM_OK;
}

// ---------------------------------------------------------------- tuning
namespace {

struct TuneKey {
  int device, size_class, restart;
  bool operator<(const TuneKey &o) const {
    if (device != o.device) return device < o.device;
    if (size_class != o.size_class) return size_class < o.size_class;
    return restart < o.restart;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, Tuning> g_tune_cache;

int size_class(int64_t N) {
  int c = 0;
  while (((int64_t)1 << c) < N) ++c;
  return c;
}

bool tuning_enabled() {
  const char *e = std::getenv("ASM_TUNE");
  return !(e && e[0] == '0' && e[1] == 0);
}

// Device milliseconds per call of f (one untimed call first, then reps).
template <class F>
asm_status time_calls(F &&f, int reps, hipEvent_t e0, hipEvent_t e1, hipStream_t s, double *us) {
  ASM_HIP(f());
  ASM_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) ASM_HIP(f());
  ASM_HIP(hipEventRecord(e1, s));
  ASM_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  ASM_HIP(hipEventElapsedTime(&ms, e0, e1));
  *us = 1e3 * (double)ms / reps;
  return ASM_OK;
}

// Times every candidate on the system's own matrix and work arrays (which
// the solve then overwrites): the SpMV z -> w, and the Gram-Schmidt kernels
// (V^T w, its reduction, then the update and its norm) of one whole restart
// cycle, over 1, 2, ..., restart columns as the solve runs them (the best
// block count differs between few and many columns).  A candidate replaces
// the default only when it is at least 3% faster.
asm_status time_candidates(asm_system S, int m, hipStream_t s, Tuning *t) {
  Workspace &W = S->ws;
  const int64_t n = 3 * (int64_t)S->pat.N;
  ASM_HIP(launch_fill(n, 1.0, W.z, s));
  ASM_HIP(launch_fill((int64_t)(m + 1) * W.ldu, 1.0, W.U, s));
  ASM_HIP(launch_fill(m + 2, 0.0, W.dvec, s));
  ASM_HIP(launch_fill(m + 1, 0.0, W.scale, s));  // zero projections: the columns stay bounded
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ASM_HIP(hipEventCreate(&e0));
  hipError_t ec = hipEventCreate(&e1);
  if (ec != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ASM_ERR_HIP, hipGetErrorString(ec));
  }
  struct Ev {
    hipEvent_t a, b;
    ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } guard{e0, e1};
  static const int rows[3] = {1, 2, 4};
  static const int blocks[4] = {512, 1024, 2048, 4096};
  for (int k = 0; k < 3; ++k) {
    asm_status st = time_calls([&] { return launch_spmv(S->sell, W.z, W.w, s, nullptr, rows[k]); }, 6, e0, e1, s,
                               &t->spmv_us[k]);
    if (st != ASM_OK) return st;
  }
  for (int k = 0; k < 4; ++k) {
    auto pair = [&](int nv) -> hipError_t {
      int nb = 0;
      hipError_t e = launch_multidot(n, nv, W.U, W.ldu, W.w, W.partial, &nb, s, nullptr, blocks[k]);
      if (e == hipSuccess) e = launch_reduce_cols(nb, nv + 1, W.partial, W.dvec, s);
      if (e != hipSuccess) return e;
      return launch_update(n, nv, W.U, W.ldu, W.dvec, W.scale, W.w, W.U + (size_t)nv * W.ldu, W.partial, &nb, s,
                           nullptr, blocks[k]);
    };
    ASM_HIP(pair(1));  // untimed
    ASM_HIP(hipEventRecord(e0, s));
    for (int nv = 1; nv <= m; ++nv) ASM_HIP(pair(nv));
    ASM_HIP(hipEventRecord(e1, s));
    ASM_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    ASM_HIP(hipEventElapsedTime(&ms, e0, e1));
    t->krylov_us[k] = 1e3 * (double)ms / m;  // per step
  }
  t->spmv_rows = 1;
  double best = t->spmv_us[0];
  for (int k = 1; k < 3; ++k)
    if (t->spmv_us[k] < 0.97 * t->spmv_us[0] && t->spmv_us[k] < best) { best = t->spmv_us[k]; t->spmv_rows = rows[k]; }
  t->red_blocks = kReduceBlocks;
  best = t->krylov_us[1];
  for (int k = 0; k < 4; ++k)
    if (k != 1 && t->krylov_us[k] < 0.97 * t->krylov_us[1] && t->krylov_us[k] < best) {
      best = t->krylov_us[k];
      t->red_blocks = blocks[k];
    }
  return ASM_OK;
}

}  // namespace

asm_status ensure_tuned(asm_system S, int m, hipStream_t s) {
  Tuning &t = S->tune;
  if (t.source != ASM_TUNE_DEFAULT || !tuning_enabled()) return ASM_OK;
  const TuneKey key{S->device, size_class(S->pat.N), m};
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune_cache.find(key);
  if (it != g_tune_cache.end() && !t.retime) {
    t = it->second;
    t.source = ASM_TUNE_CACHED;
    return ASM_OK;
  }
  Tuning nt;
  asm_status st = time_candidates(S, m, s, &nt);
  if (st != ASM_OK) return st;
  nt.source = ASM_TUNE_TIMED;
  nt.restart = m;
  t = nt;
  g_tune_cache[key] = nt;
  return ASM_OK;
}

namespace {

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

// This handle's arrays of the global coarse correction.
hipError_t alloc_coarse_own(asm_precond pc) {
  DevMem &O = pc->mem;
  const size_t n = 3 * (size_t)pc->ncv, N3 = 3 * (size_t)pc->sys->pat.N;
  hipError_t e;
  if ((e = O.alloc(&pc->acv, (size_t)pc->casrc.n * 9)) != hipSuccess || (e = O.alloc(&pc->cM, n * n)) != hipSuccess ||
      (e = O.alloc(&pc->cMinv, n * n)) != hipSuccess || (e = O.alloc(&pc->cfcol, n)) != hipSuccess ||
      (e = O.alloc(&pc->crc, n)) != hipSuccess || (e = O.alloc(&pc->cxc, n)) != hipSuccess ||
      (e = O.alloc(&pc->cbad, 1)) != hipSuccess)
    return e;
  if (pc->opts.coarse == ASM_COARSE_TWO_STAGE &&
      ((e = O.alloc(&pc->crtmp, N3)) != hipSuccess || (e = O.alloc(&pc->cr2, N3)) != hipSuccess ||
       (e = O.alloc(&pc->cpart, (size_t)kReduceBlocks * 8)) != hipSuccess))
    return e;
  return hipSuccess;
}

// This handle's dense inverses of the exact local solves.
hipError_t alloc_exact_own(asm_precond pc, int64_t dense_elems, int64_t total_ext) {
  DevMem &O = pc->mem;
  hipError_t e;
  if ((e = O.alloc(&pc->xd.M, (size_t)dense_elems)) != hipSuccess ||
      (e = O.alloc(&pc->xd.Minv, (size_t)dense_elems)) != hipSuccess ||
      (e = O.alloc(&pc->xd.fcol, 3 * (size_t)total_ext)) != hipSuccess ||
      (e = O.alloc(&pc->xd.bad, (size_t)pc->xd.nsub)) != hipSuccess)
    return e;
  return hipSuccess;
}

// Assembly (lumped matrices, A_i values) and factorisation on the device.
asm_status numeric_setup(asm_precond pc, hipStream_t s) {
  asm_system S = pc->sys;
  const PlanHost &P = *pc->plan;
  if (pc->l1.n > 0) {
    ASM_HIP(launch_gather_sum9(pc->l1.n, pc->l1.ptr, pc->l1.idx, S->vals, INT32_MAX, nullptr, pc->L1, s));
    ASM_HIP(launch_gather_sum9(pc->l2.n, pc->l2.ptr, pc->l2.idx, pc->L1, INT32_MAX, nullptr, pc->L2, s));
  }
  ASM_HIP(launch_gather_sum9(pc->asrc.n, pc->asrc.ptr, pc->asrc.idx, S->vals, (int32_t)S->pat.nnzb, pc->L2,
                             pc->aval, s));
  ASM_HIP(hipMemcpyAsync(pc->dp.fact, pc->aval, (size_t)P.total_entries * 9 * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  ASM_HIP(hipMemsetAsync(pc->bad, 0xff, sizeof(unsigned long long), s));
  if (pc->opts.local == ASM_LOCAL_EXACT) {
    // dense inverse of every A_i (no incomplete factors are computed)
    ASM_HIP(launch_local_dense_init(pc->xd, pc->dp.arp, pc->dp.aci, pc->aval, pc->xmaxn3, s));
    ASM_HIP(launch_local_gauss_jordan(pc->xd, pc->xmaxn3, s));
    std::vector<int> xb(pc->xd.nsub);
    ASM_HIP(hipMemcpyAsync(xb.data(), pc->xd.bad, xb.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    ASM_HIP(hipStreamSynchronize(s));
    for (int sd = 0; sd < pc->xd.nsub; ++sd)
      if (xb[sd] >= 0)
        return fail(ASM_ERR_SINGULAR_PIVOT, "singular local matrix A_i of subdomain " + std::to_string(sd) +
                                                " (dense elimination, column " + std::to_string(xb[sd]) + ")");
  } else {
    ASM_HIP(launch_ilu_factor(pc->dp, pc->bad, s));
    ASM_HIP(launch_relayout((int)pc->rl_n, pc->rl_src, pc->rl_base, pc->rl_stride, pc->rl_to32, pc->dp.fact,
                            static_cast<double *>(pc->recbuf), static_cast<float *>(pc->recbuf), s));
  }
  if (pc->opts.coarse != ASM_COARSE_NONE) {
    // A_C = R_C A R_C^T (box sums of A's blocks), inverted densely
    ASM_HIP(launch_gather_sum9(pc->casrc.n, pc->casrc.ptr, pc->casrc.idx, S->vals, (int32_t)S->pat.nnzb, nullptr,
                               pc->acv, s));
    ASM_HIP(launch_dense_init(pc->ncv, pc->acp, pc->acc, pc->acv, pc->cM, pc->cMinv, s));
    ASM_HIP(hipMemsetAsync(pc->cbad, 0xff, sizeof(int), s));
    ASM_HIP(launch_gauss_jordan(3 * pc->ncv, pc->cM, pc->cMinv, pc->cfcol, pc->cbad, s));
    int cbad = -1;
    ASM_HIP(hipMemcpyAsync(&cbad, pc->cbad, sizeof cbad, hipMemcpyDeviceToHost, s));
    ASM_HIP(hipStreamSynchronize(s));
    if (cbad >= 0)
      return fail(ASM_ERR_SINGULAR_PIVOT, "singular coarse operator A_C at coarse row " + std::to_string(cbad / 3));
  }
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

}  // namespace

asm_status apply_precond(asm_precond pc, const double *r, const double *scale, double *z, hipStream_t s,
                         Profiler *prof, const int *skip) {
  asm_system S = pc->sys;
  const int64_t n = 3 * (int64_t)S->pat.N;
  Profiler dummy;
  Profiler &pf = prof ? *prof : dummy;
  if (pc->opts.kind == ASM_KIND_NONE) {
    const size_t t0 = pf.mark(ASM_PHASE_OTHER, s);
    ASM_HIP(launch_scale_copy(n, r, scale, z, s, skip));
    pf.span(ASM_PHASE_OTHER, t0, s);
    return ASM_OK;
  }
  const size_t t0 = pf.mark(ASM_PHASE_LUMP, s);
  if (pc->c1.n > 0) {
    ASM_HIP(launch_gather_sum3(pc->c1.n1, pc->c1.lanes, pc->c1.n, pc->c1.lanes2, pc->c1.ptr, pc->c1.idx, r, scale,
                               pc->PA, s, skip));
    ASM_HIP(launch_gather_sum3(pc->c2.n1, pc->c2.lanes, pc->c2.n, pc->c2.lanes2, pc->c2.ptr, pc->c2.idx, pc->PA,
                               nullptr, pc->PNF, s, skip));
  }
  // the ILU sweeps gather their fine inputs from r themselves; the dense
  // local solves take every subdomain's inputs gathered in sweep order
  if (pc->opts.local == ASM_LOCAL_EXACT)
    ASM_HIP(launch_gather_rhs((int)pc->plan->total_pos, pc->ap, r, scale, s));
  else
    ASM_HIP(launch_coarse_rhs(pc->ap, s, skip));
  pf.span(ASM_PHASE_LUMP, t0, s);
  const bool restricted = pc->opts.combine == ASM_COMBINE_RESTRICTED;
  const size_t t1 = pf.mark(ASM_PHASE_ILU_APPLY, s);
  if (pc->opts.local == ASM_LOCAL_EXACT)
    ASM_HIP(launch_local_dense_apply(pc->xd, (int64_t)pc->plan->total_pos, pc->ap.rs, restricted, z, pc->ap.yx, s));
  else
    ASM_HIP(launch_ilu_apply(pc->ap, r, scale, z, s, skip));
  pf.span(ASM_PHASE_ILU_APPLY, t1, s);
  if (!restricted) {
    const size_t t2 = pf.mark(ASM_PHASE_COMBINE, s);
    ASM_HIP(launch_additive_combine(S->pat.N, pc->cptr, pc->cidx, pc->ap.yx, z, s, skip));
    pf.span(ASM_PHASE_COMBINE, t2, s);
  }
  if (pc->opts.coarse != ASM_COARSE_NONE) {
    // z += R_C^T A_C^-1 R_C r (eq. (3.5)), or of the residual r - A z left
    // by the Schwarz part (eq. (3.8))
    const size_t t3 = pf.mark(ASM_PHASE_OTHER, s);
    const double *rr = r, *sc = scale;
    if (pc->opts.coarse == ASM_COARSE_TWO_STAGE) {
      if (scale) {
        ASM_HIP(launch_scale_copy(n, r, scale, pc->crtmp, s));
        rr = pc->crtmp;
      }
      int nb = 0;
      ASM_HIP(launch_residual(S->sell, z, rr, pc->cr2, pc->cpart, &nb, s));
      rr = pc->cr2;
      sc = nullptr;
    }
    ASM_HIP(launch_gather_sum3(pc->cbox.n1, pc->cbox.lanes, pc->cbox.n, pc->cbox.lanes2, pc->cbox.ptr, pc->cbox.idx,
                               rr, sc, pc->crc, s));
    ASM_HIP(launch_dense_gemv(3 * pc->ncv, pc->cMinv, pc->crc, pc->cxc, s));
    ASM_HIP(launch_prolong_add(S->pat.N, pc->cvar, pc->cxc, z, s));
    pf.span(ASM_PHASE_OTHER, t3, s);
  }
  return ASM_OK;
}

asm_status validate_pattern(const HostPattern &P) {
  const int nb = P.N;
  const int64_t nnzb = P.nnzb;
  if (P.rp[0] != 0 || P.rp[nb] != nnzb) return fail(ASM_ERR_INVALID, "row_ptr must start at 0 and end at nnzb");
  for (int r = 0; r < nb; ++r) {
    if (P.rp[r + 1] < P.rp[r]) return fail(ASM_ERR_INVALID, "row_ptr not monotone at row " + std::to_string(r));
    bool diag = false;
    for (int q = P.rp[r]; q < P.rp[r + 1]; ++q) {
      const int c = P.ci[q];
      if (c < 0 || c >= nb) return fail(ASM_ERR_INVALID, "column out of range in row " + std::to_string(r));
      if (q > P.rp[r] && P.ci[q - 1] >= c)
        return fail(ASM_ERR_INVALID, "columns not strictly increasing in row " + std::to_string(r));
      diag |= (c == r);
    }
    if (!diag) return fail(ASM_ERR_INVALID, "missing diagonal block in row " + std::to_string(r));
  }
  return ASM_OK;
}

asm_status check_precond_opts(const HostPattern &A, const asm_precond_opts *o) {
  if (o->kind < ASM_KIND_NONE || o->kind > ASM_KIND_TWO_LEVEL) return fail(ASM_ERR_INVALID, "bad kind");
  if (o->combine != ASM_COMBINE_ADDITIVE && o->combine != ASM_COMBINE_RESTRICTED)
    return fail(ASM_ERR_INVALID, "bad combine");
  if (o->precision != ASM_PREC_FP64 && o->precision != ASM_PREC_FP32) return fail(ASM_ERR_INVALID, "bad precision");
  if (o->field < ASM_FIELD_NEAR_FAR || o->field > ASM_FIELD_FAR) return fail(ASM_ERR_INVALID, "bad field");
  if (o->coarse < ASM_COARSE_NONE || o->coarse > ASM_COARSE_TWO_STAGE) return fail(ASM_ERR_INVALID, "bad coarse");
  if (o->local != ASM_LOCAL_ILU0 && o->local != ASM_LOCAL_EXACT) return fail(ASM_ERR_INVALID, "bad local solver");
  if (o->coarse != ASM_COARSE_NONE) {
    if (o->kind == ASM_KIND_NONE) return fail(ASM_ERR_INVALID, "a coarse correction needs a Schwarz preconditioner");
    for (int d = 0; d < 3; ++d)
      if (o->coarse_box[d] < 1) return fail(ASM_ERR_INVALID, "bad coarse box");
  }
  if (o->kind == ASM_KIND_NONE) return ASM_OK;
  if (o->sx < 1 || o->sy < 1 || o->sx > A.nx || o->sy > A.ny || o->overlap < 0)
    return fail(ASM_ERR_INVALID, "bad subdomain split or overlap");
  if (o->kind == ASM_KIND_TWO_LEVEL)
    for (int d = 0; d < 3; ++d)
      if (o->near_box[d] < 1 || o->far_box[d] < 1) return fail(ASM_ERR_INVALID, "bad coarsening box");
  return ASM_OK;
}

asm_status setup_from_plan(asm_system S, const asm_precond_opts *o, std::shared_ptr<PlanHost> plan,
                           hipStream_t stream, asm_precond *out) {
  *out = nullptr;
  std::unique_ptr<asm_precond_s> hold(new (std::nothrow) asm_precond_s());
  asm_precond pc = hold.get();
  if (!pc) return fail(ASM_ERR_OOM, "host allocation failed");
  pc->sys = S;
  pc->opts = *o;
  if (o->kind == ASM_KIND_NONE) {
    *out = hold.release();
    return ASM_OK;
  }
  auto cleanup = [](asm_status st) { return st; };  // hold frees the handle
  pc->plan = std::move(plan);
  pc->smem = std::make_shared<DevMem>();
  PlanHost &P = *pc->plan;
  asm_status st = ASM_OK;
  DevMem &M = *pc->smem;  // pattern-only arrays
  DevMem &O = pc->mem;    // records, factors and work vectors of this handle
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
  if ((e = O.upload(&drec, P.rec, s)) != hipSuccess)
    return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
  pc->rec_bytes = P.rec.size();
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
  auto ALLOC = [&](auto **dst, size_t n) { return O.alloc(dst, n); };
  // gathered inputs in sweep order: only the dense local solves read them
  const size_t nrs = o->local == ASM_LOCAL_EXACT ? (size_t)P.total_pos * 3 : 0;
  double *yx, *rs, *fact;
  if ((e = ALLOC(&yx, ((size_t)P.total_pos + kPosPad) * 3)) != hipSuccess || (e = ALLOC(&rs, nrs)) != hipSuccess ||
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
        (e = ALLOC(&pc->PNF, (size_t)pc->c2.n * 3)) != hipSuccess ||
        (e = ALLOC(&ap.crs, (size_t)pc->c3.n * 3)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
    ap.cptr3 = pc->c3.ptr;
    ap.cidx3 = pc->c3.idx;
    ap.pnf = pc->PNF;
    ap.ncoarse = pc->c3.n;
  }
  if (o->coarse != ASM_COARSE_NONE) {
    pc->ncv = P.ncv;
    if ((e = M.upload(&pc->cvar, P.cvar, s)) != hipSuccess || (e = upload_gather(M, pc->cbox, P.cbox_cells, s)) != hipSuccess ||
        (e = M.upload(&pc->acp, P.acp, s)) != hipSuccess || (e = M.upload(&pc->acc, P.acc, s)) != hipSuccess ||
        (e = upload_gather(M, pc->casrc, P.ac_src, s)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
    if ((e = alloc_coarse_own(pc)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
  }
  if (o->local == ASM_LOCAL_EXACT) {
    DenseLocal &x = pc->xd;
    x.nsub = P.nsub;
    x.sub = dsub;
    int64_t *doff;
    int32_t *lpos, *psub, *pout, *pbpos;
    if ((e = M.upload(&doff, P.xdoff, s)) != hipSuccess || (e = M.upload(&lpos, P.xlpos, s)) != hipSuccess ||
        (e = M.upload(&psub, P.xpsub, s)) != hipSuccess || (e = M.upload(&pout, P.xout, s)) != hipSuccess ||
        (e = M.upload(&pbpos, P.xbpos, s)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
    x.doff = doff; x.lpos = lpos; x.psub = psub; x.pout = pout; x.pbpos = pbpos;
    pc->xmaxn3 = P.xmaxn3;
    if ((e = alloc_exact_own(pc, P.xdoff[P.nsub], P.total_ext)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
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
  P.cvar = std::vector<int32_t>();
  P.cbox_cells = GatherList{};
  P.ac_src = GatherList{};
  P.xlpos = std::vector<int32_t>();
  P.xpsub = std::vector<int32_t>();
  P.xout = std::vector<int32_t>();
  P.xbpos = std::vector<int32_t>();
  st = numeric_setup(pc, s);
  if (st != ASM_OK) return cleanup(st);
  pc->stats.nsub = P.nsub;
  pc->stats.ext_rows = P.total_ext;
  pc->stats.coarse_rows = P.total_coarse;
  pc->stats.factor_blocks = P.total_entries;
  pc->stats.fine_row_blocks = P.fine_row_entries;
  pc->stats.max_levels = P.max_levels;
  pc->stats.device_bytes = (int64_t)(M.bytes + O.bytes);
  pc->stats.sweep_steps = P.sweep_steps;
  pc->stats.reloaded_rows = P.lds_spilled_rows;
  pc->stats.split_rows = P.split_rows;
  *out = hold.release();
  return ASM_OK;
}

}  // namespace asmx

using namespace asmx;

extern "C" {

const char *asm_last_error(void) { return g_err.c_str(); }

asm_status asm_create_system(const asm_grid *grid, int32_t nb, int64_t nnzb, const int32_t *row_ptr_dev,
                             const int32_t *col_idx_dev, const double *vals_dev, hipStream_t stream,
                             asm_system *out) {
  try {
    g_err.clear();
    if (!out) return fail(ASM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!grid || !row_ptr_dev || !col_idx_dev || !vals_dev) return fail(ASM_ERR_INVALID, "NULL argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || (int64_t)grid->nx * grid->ny * grid->nz != nb)
      return fail(ASM_ERR_INVALID, "grid nx*ny*nz does not equal nb");
    if (nnzb < nb || nnzb >= ((int64_t)1 << 31) / 9) return fail(ASM_ERR_INVALID, "nnzb out of range");
    std::unique_ptr<asm_system_s> hold(new (std::nothrow) asm_system_s());
    asm_system S = hold.get();
    if (!S) return fail(ASM_ERR_OOM, "host allocation failed");
    auto cleanup = [](asm_status st) { return st; };  // hold frees the handle
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
    asm_status vst = validate_pattern(P);
    if (vst != ASM_OK) return cleanup(vst);
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
    *out = hold.release();
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_update_values(asm_system S, const double *vals_dev, hipStream_t stream) {
  try {
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
  ASM_CATCH_ALL
}

asm_status asm_spmv(asm_system S, const double *x_dev, double *y_dev, hipStream_t stream) {
  try {
    g_err.clear();
    if (!S || !x_dev || !y_dev) return fail(ASM_ERR_INVALID, "NULL argument");
    ASM_HIP(launch_spmv(S->sell, x_dev, y_dev, stream, nullptr, S->tune.spmv_rows));
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_setup_precond(asm_system S, const asm_precond_opts *o, hipStream_t stream, asm_precond *out) {
  try {
    TraceRange range_("asm_setup_precond");
    g_err.clear();
    if (!S || !o || !out) return fail(ASM_ERR_INVALID, "NULL argument");
    *out = nullptr;
    asm_status st = check_precond_opts(S->pat, o);
    if (st != ASM_OK) return st;
    std::shared_ptr<PlanHost> plan;
    if (o->kind != ASM_KIND_NONE) {
      plan = std::make_shared<PlanHost>();
      std::string err;
      st = build_plan(S->pat, *o, *plan, err);
      if (st != ASM_OK) return fail(st, err);
    }
    return setup_from_plan(S, o, std::move(plan), stream, out);
  }
  ASM_CATCH_ALL
}

asm_status asm_refactor(asm_precond pc, hipStream_t stream) {
  try {
    TraceRange range_("asm_refactor");
    g_err.clear();
    if (!pc) return fail(ASM_ERR_INVALID, "NULL argument");
    if (pc->opts.kind == ASM_KIND_NONE) return ASM_OK;
    return numeric_setup(pc, stream);
  }
  ASM_CATCH_ALL
}

asm_status asm_precond_clone(asm_precond src, asm_system S, hipStream_t stream, asm_precond *out) {
  try {
    g_err.clear();
    if (!out) return fail(ASM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!src || !S) return fail(ASM_ERR_INVALID, "NULL argument");
    const HostPattern &A = S->pat, &B = src->sys->pat;
    if (A.nx != B.nx || A.ny != B.ny || A.nz != B.nz || A.nnzb != B.nnzb || A.rp != B.rp || A.ci != B.ci)
      return fail(ASM_ERR_INVALID, "the system's grid or block pattern differs from the source preconditioner's");
    std::unique_ptr<asm_precond_s> hold(new (std::nothrow) asm_precond_s());
    asm_precond pc = hold.get();
    if (!pc) return fail(ASM_ERR_OOM, "host allocation failed");
    pc->sys = S;
    pc->opts = src->opts;
    pc->stats = src->stats;
    if (src->opts.kind == ASM_KIND_NONE) {
      *out = hold.release();
      return ASM_OK;
    }
    auto cleanup = [](asm_status st) { return st; };  // hold frees the handle
    // pattern-only state is shared; everything holding values is this handle's
    pc->plan = src->plan;
    pc->smem = src->smem;
    pc->dp = src->dp;
    pc->ap = src->ap;
    pc->l1 = src->l1; pc->l2 = src->l2; pc->asrc = src->asrc;
    pc->c1 = src->c1; pc->c2 = src->c2; pc->c3 = src->c3;
    pc->rl_src = src->rl_src; pc->rl_base = src->rl_base; pc->rl_stride = src->rl_stride; pc->rl_to32 = src->rl_to32;
    pc->rl_n = src->rl_n;
    pc->cptr = src->cptr; pc->cidx = src->cidx;
    pc->rec_bytes = src->rec_bytes;
    const PlanHost &P = *pc->plan;
    DevMem &O = pc->mem;
    hipError_t e = hipSuccess;
    uint8_t *rec = nullptr;
    double *yx = nullptr, *rs = nullptr, *fact = nullptr;
    if ((e = O.alloc(&rec, pc->rec_bytes)) != hipSuccess || (e = O.alloc(&yx, ((size_t)P.total_pos + kPosPad) * 3)) != hipSuccess ||
        (e = O.alloc(&rs, pc->opts.local == ASM_LOCAL_EXACT ? (size_t)P.total_pos * 3 : 0)) != hipSuccess ||
        (e = O.alloc(&fact, (size_t)P.total_entries * 9)) != hipSuccess ||
        (e = O.alloc(&pc->aval, (size_t)P.total_entries * 9)) != hipSuccess || (e = O.alloc(&pc->bad, 1)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
    if (pc->opts.kind == ASM_KIND_TWO_LEVEL &&
        ((e = O.alloc(&pc->L1, (size_t)pc->l1.n * 9)) != hipSuccess ||
         (e = O.alloc(&pc->L2, (size_t)pc->l2.n * 9)) != hipSuccess ||
         (e = O.alloc(&pc->PA, (size_t)pc->c1.n * 3)) != hipSuccess ||
         (e = O.alloc(&pc->PNF, (size_t)pc->c2.n * 3)) != hipSuccess ||
         (e = O.alloc(&pc->ap.crs, (size_t)pc->c3.n * 3)) != hipSuccess))
      return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
    // the records carry the sweep's row headers and slots next to the factor
    // values; the values are rewritten by the numeric setup below
    if ((e = hipMemcpyAsync(rec, src->recbuf, pc->rec_bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
      return cleanup(fail(ASM_ERR_HIP, hipGetErrorString(e)));
    pc->recbuf = rec;
    pc->ap.rec = rec;
    pc->ap.yx = yx;
    pc->ap.rs = rs;
    pc->ap.pnf = pc->PNF;
    pc->dp.fact = fact;
    if (pc->opts.coarse != ASM_COARSE_NONE) {
      pc->ncv = src->ncv;
      pc->cvar = src->cvar;
      pc->cbox = src->cbox;
      pc->casrc = src->casrc;
      pc->acp = src->acp;
      pc->acc = src->acc;
      if ((e = alloc_coarse_own(pc)) != hipSuccess)
        return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
    }
    if (pc->opts.local == ASM_LOCAL_EXACT) {
      pc->xd = src->xd;
      pc->xmaxn3 = src->xmaxn3;
      if ((e = alloc_exact_own(pc, P.xdoff.back(), P.total_ext)) != hipSuccess)
        return cleanup(fail(e == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP, hipGetErrorString(e)));
    }
    pc->stats.device_bytes = (int64_t)(pc->smem->bytes + O.bytes);
    asm_status st = numeric_setup(pc, stream);
    if (st != ASM_OK) return cleanup(st);
    *out = hold.release();
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_precond_apply(asm_precond pc, const double *r_dev, double *z_dev, hipStream_t stream) {
  try {
    TraceRange range_("asm_precond_apply");
    g_err.clear();
    if (!pc || !r_dev || !z_dev) return fail(ASM_ERR_INVALID, "NULL argument");
    return apply_precond(pc, r_dev, nullptr, z_dev, stream);
  }
  ASM_CATCH_ALL
}

asm_status asm_precond_get_stats(asm_precond pc, asm_precond_stats *st) {
  try {
    g_err.clear();
    if (!pc || !st) return fail(ASM_ERR_INVALID, "NULL argument");
    *st = pc->stats;
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_precond_export_sub(asm_precond pc, int32_t s, int32_t *n_out, int32_t *nnz_out, int32_t *rp_host,
                                  int32_t *ci_host, double *a_host, double *f_host, int32_t *label_host) {
  try {
    g_err.clear();
    if (!pc || pc->opts.kind == ASM_KIND_NONE) return fail(ASM_ERR_INVALID, "no subdomains");
    const PlanHost &P = *pc->plan;
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
  ASM_CATCH_ALL
}

}  // extern "C"

namespace asmx {
namespace {

// The Krylov work arrays one solve uses: the system's own workspace
// (asm_solve), or parts of the library's fixed device array
// (asm_solve_noalloc).  Each step's last kernel writes the step's Hessenberg
// column to pub_dev + j*kPubStride.  With events (the workspace's pinned
// host memory, which pub_dev maps) the host reads it there one step late;
// without, it copies the column to the host buffer pub_host and waits for it.
struct KrylovView {
  double *U = nullptr;
  int64_t ldu = 0;
  double *w = nullptr, *z = nullptr, *t = nullptr, *partial = nullptr, *dvec = nullptr, *scale = nullptr,
         *coef = nullptr, *misc = nullptr;
  int *flag = nullptr;
  double *pub_dev = nullptr;   // kMaxRestart columns of kPubStride doubles
  double *pub_host = nullptr;  // host view of them
  double *host = nullptr;      // host staging of single scalars (pinned or not)
  double *coef_host = nullptr; // host staging of a cycle's solution coefficients
  const hipEvent_t *step_done = nullptr;  // per-step events: read columns one step late
};

// Doubles the no-allocation solve takes from the fixed array for restart m
// and n unknowns (each part 256-byte aligned).
int64_t noalloc_doubles(int m, int64_t n, int64_t *ldu) {
  auto up = [](int64_t v) { return (v + 31) & ~int64_t(31); };
  *ldu = (n + 1) & ~int64_t(1);
  return up((int64_t)(m + 1) * *ldu) + 3 * up(n) + up(partial_doubles(n / 3)) +
         5 * up(kMaxRestart + 2) + up((int64_t)kMaxRestart * kPubStride) + 32;
}

asm_status check_nonfinite(const KrylovView &W, const double *v, int64_t n, hipStream_t s, bool *out) {
  ASM_HIP(launch_fill(1, 0, W.flag, s));
  ASM_HIP(launch_check_finite(n, v, W.flag, s));
  int h = 0;
  ASM_HIP(hipMemcpyAsync(&h, W.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  ASM_HIP(hipStreamSynchronize(s));
  *out = (h != 0);
  return ASM_OK;
}

// Restarted right-preconditioned GMRES (see asm_solve in asm.h) on the work
// arrays of W.
asm_status gmres_run(asm_system S, asm_precond pc, const double *b, double *x, const asm_solve_opts *o,
                     hipStream_t s, asm_solve_info *info, const KrylovView &W, Profiler &pf) {
  const int m = o->restart;
  const int64_t n = 3 * (int64_t)S->pat.N;
  asm_status st;
  bool bad = false;
  if ((st = check_nonfinite(W, b, n, s, &bad)) != ASM_OK) return st;
  if (!bad && (st = check_nonfinite(W, x, n, s, &bad)) != ASM_OK) return st;
  if (bad) return fail(ASM_ERR_NONFINITE, "non-finite b or x0");
  const int ld = m + 1;
  double *hp = W.host;
  const bool ahead = W.step_done != nullptr;
  int nb = 0;
  // ||b||
  ASM_HIP(launch_norm2(n, b, W.partial, &nb, s));
  ASM_HIP(launch_reduce_cols(nb, 1, W.partial, W.misc + 2, s));
  ASM_HIP(hipMemcpyAsync(hp, W.misc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  ASM_HIP(hipStreamSynchronize(s));
  const double bnorm = std::sqrt(hp[0]);
  if (bnorm == 0.0 && o->fixed_iters == 0) {
    ASM_HIP(launch_fill(n, 0.0, x, s));
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
    ASM_HIP(launch_norm_finalize(nbr, W.partial, 0, nullptr, nullptr, W.misc + 1, W.scale, nullptr, s));
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
  // host-side Hessenberg matrix, rotations and coefficients (no heap)
  double H[(kMaxRestart + 1) * kMaxRestart], cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart],
      sc[kMaxRestart + 1], coef[kMaxRestart + 1];
  auto Hh = [&](int i, int j) -> double & { return H[(size_t)j * ld + i]; };
  asm_status result = ASM_NOT_CONVERGED;
  // One Arnoldi step on the stream: z = B^-1 v_j, w = A z, CGS projections,
  // the new basis vector and its norm; the step's Hessenberg column is then
  // published and (with events) an event marks the step's end.
  auto enqueue_step = [&](int j) -> asm_status {
    const double *Uj = W.U + (size_t)j * W.ldu;
    asm_status e2 = apply_precond(pc, Uj, W.scale + j, W.z, s, &pf);
    if (e2 != ASM_OK) return e2;
    size_t t0 = pf.mark(ASM_PHASE_SPMV, s);
    ASM_HIP(launch_spmv(S->sell, W.z, W.w, s, nullptr, S->tune.spmv_rows));
    pf.span(ASM_PHASE_SPMV, t0, s);
    int nbd = 0;
    t0 = pf.mark(ASM_PHASE_DOTS, s);
    ASM_HIP(launch_multidot(n, j + 1, W.U, W.ldu, W.w, W.partial, &nbd, s, nullptr, S->tune.red_blocks));
    pf.span(ASM_PHASE_DOTS, t0, s);
    t0 = pf.mark(ASM_PHASE_OTHER, s);
    ASM_HIP(launch_reduce_cols(nbd, j + 2, W.partial, W.dvec, s));
    pf.span(ASM_PHASE_OTHER, t0, s);
    int nbu = 0;
    t0 = pf.mark(ASM_PHASE_UPDATE, s);
    ASM_HIP(launch_update(n, j + 1, W.U, W.ldu, W.dvec, W.scale, W.w, W.U + (size_t)(j + 1) * W.ldu, W.partial,
                          &nbu, s, nullptr, S->tune.red_blocks));
    pf.span(ASM_PHASE_UPDATE, t0, s);
    t0 = pf.mark(ASM_PHASE_OTHER, s);
    // the Hessenberg column goes to the published area only (the host keeps H)
    ASM_HIP(launch_norm_finalize(nbu, W.partial, j + 1, W.dvec, W.scale, W.pub_dev + (size_t)j * kPubStride,
                                 W.scale + j + 1, W.pub_dev + (size_t)j * kPubStride, s));
    pf.span(ASM_PHASE_OTHER, t0, s);
    if (ahead) ASM_HIP(hipEventRecord(W.step_done[j], s));
    return ASM_OK;
  };
  // Residual estimate and its last one-step reduction factor: when the
  // estimate after the next step is predicted within 4 tol, the step after
  // it is not queued ahead (it would be wasted at convergence).
  double ratio = 1.0;
  while (true) {
    if (beta == 0.0) { result = ASM_OK; break; }
    info->cycles++;
    std::fill(g, g + m + 1, 0.0);
    g[0] = beta;
    sc[0] = 1.0 / beta;
    double est = beta;
    // steps of this cycle: at most m, and never past the iteration limit
    const int kmax = std::min(m, limit - info->iters);
    int k = 0, queued = 0;
    for (int j = 0; j < kmax; ++j) {
      // with events, keep the next step queued while step j's column is read
      const bool near_tol = o->fixed_iters == 0 && est * ratio <= 4.0 * tol;
      while (queued < kmax && queued <= j + (ahead && !near_tol ? 1 : 0)) {
        if ((st = enqueue_step(queued)) != ASM_OK) return st;
        ++queued;
      }
      const double *col = W.pub_host + (size_t)j * kPubStride;
      if (ahead) {
        ASM_HIP(hipEventSynchronize(W.step_done[j]));
      } else {
        ASM_HIP(hipMemcpyAsync(W.pub_host + (size_t)j * kPubStride, W.pub_dev + (size_t)j * kPubStride,
                               sizeof(double) * (j + 3), hipMemcpyDeviceToHost, s));
        ASM_HIP(hipStreamSynchronize(s));
      }
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
      ratio = est > 0.0 ? std::fabs(g[j + 1]) / est : 0.0;
      est = std::fabs(g[j + 1]);
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
    // coefficients to the device through their staging buffer (pinned: read
    // by the copy in stream order, not rewritten before the next cycle's
    // end; pageable: the stream is synchronised at once)
    std::copy(coef, coef + k, W.coef_host);
    ASM_HIP(hipMemcpyAsync(W.coef, W.coef_host, k * sizeof(double), hipMemcpyHostToDevice, s));
    if (!ahead) ASM_HIP(hipStreamSynchronize(s));
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

asm_status check_solve_args(asm_system S, asm_precond pc, const double *b, double *x, const asm_solve_opts *o,
                            asm_solve_info *info) {
  if (!S || !pc || !b || !x || !o || !info) return fail(ASM_ERR_INVALID, "NULL argument");
  if (pc->sys != S) return fail(ASM_ERR_INVALID, "preconditioner belongs to another system");
  std::memset(info, 0, sizeof *info);
  const int m = o->restart;
  if (m < 1 || m > kMaxRestart || !(o->rtol >= 0.0) || o->max_iters < 1 || o->fixed_iters < 0)
    return fail(ASM_ERR_INVALID, "bad solver option");
  return ASM_OK;
}

}  // namespace
}  // namespace asmx

extern "C" {

asm_status asm_solve(asm_system S, asm_precond pc, const double *b, double *x, const asm_solve_opts *o,
                     hipStream_t s, asm_solve_info *info) {
  try {
    TraceRange range_("asm_solve");
    g_err.clear();
    asm_status st = check_solve_args(S, pc, b, x, o, info);
    if (st != ASM_OK) return st;
    if ((st = ensure_workspace(S, o->restart, s)) != ASM_OK) return st;
    if ((st = ensure_tuned(S, o->restart, s)) != ASM_OK) return st;
    Workspace &W = S->ws;
    KrylovView v;
    v.U = W.U; v.ldu = W.ldu; v.w = W.w; v.z = W.z; v.t = W.t; v.partial = W.partial; v.dvec = W.dvec;
    v.scale = W.scale; v.coef = W.coef; v.misc = W.misc; v.flag = W.flag;
    v.pub_dev = W.pinned_dev + kPubBase;
    v.pub_host = W.pinned + kPubBase;
    v.host = W.pinned;
    v.coef_host = W.pinned + kPubBase + (size_t)kMaxRestart * kPubStride;
    v.step_done = W.step_done;
    return gmres_run(S, pc, b, x, o, s, info, v, S->prof);
  }
  ASM_CATCH_ALL
}

asm_status asm_solve_noalloc(asm_system S, asm_precond pc, const double *b, double *x, const asm_solve_opts *o,
                             hipStream_t s, asm_solve_info *info) {
  try {
    TraceRange range_("asm_solve_noalloc");
    g_err.clear();
    asm_status st = check_solve_args(S, pc, b, x, o, info);
    if (st != ASM_OK) return st;
    int64_t ldu = 0;
    const int64_t n = 3 * (int64_t)S->pat.N;
    if (noalloc_doubles(o->restart, n, &ldu) * (int64_t)sizeof(double) > (int64_t)kNoAllocScratchBytes)
      return fail(ASM_ERR_INVALID, "system too large for the no-allocation solve (ASM_NOALLOC_SCRATCH_BYTES)");
    void *base = nullptr;
    ASM_HIP(noalloc_scratch(&base));
    // carve the fixed array (every part 256-byte aligned)
    double *p = static_cast<double *>(base);
    auto take = [&](int64_t count) {
      double *q = p;
      p += (count + 31) & ~int64_t(31);
      return q;
    };
    KrylovView v;
    v.ldu = ldu;
    v.U = take((int64_t)(o->restart + 1) * ldu);
    v.w = take(n);
    v.z = take(n);
    v.t = take(n);
    v.partial = take(partial_doubles(S->pat.N));
    v.dvec = take(kMaxRestart + 2);
    v.scale = take(kMaxRestart + 2);
    v.coef = take(kMaxRestart + 2);
    v.misc = take(kMaxRestart + 2);
    v.flag = reinterpret_cast<int *>(take(kMaxRestart + 2));
    v.pub_dev = take((int64_t)kMaxRestart * kPubStride);
    // host side: this call's own stack (pageable memory, copied synchronously)
    double pub_host[kMaxRestart * kPubStride];
    double host[kMaxRestart + 2], coef_host[kMaxRestart + 2];
    v.pub_host = pub_host;
    v.host = host;
    v.coef_host = coef_host;
    v.step_done = nullptr;
    Profiler none;
    return gmres_run(S, pc, b, x, o, s, info, v, none);
  }
  ASM_CATCH_ALL
}

// Restarted GMRES with every cycle run as one captured graph (see asm.h).
// The arithmetic is that of asm_solve; the Givens rotations and the small
// triangular solve run on the device, the host reads k, beta and the
// residual estimate once per cycle.
asm_status asm_solve_graph(asm_system S, asm_precond pc, const double *b, double *x, const asm_solve_opts *o,
                           hipStream_t user_stream, asm_solve_info *info) {
  try {
    TraceRange range_("asm_solve_graph");
    g_err.clear();
    if (!S || !pc || !b || !x || !o || !info) return fail(ASM_ERR_INVALID, "NULL argument");
    if (pc->sys != S) return fail(ASM_ERR_INVALID, "preconditioner belongs to another system");
    std::memset(info, 0, sizeof *info);
    const int m = o->restart;
    if (m < 1 || m > kMaxRestart || !(o->rtol >= 0.0) || o->max_iters < 1 || o->fixed_iters < 0)
      return fail(ASM_ERR_INVALID, "bad solver option");
    if (pc->opts.kind != ASM_KIND_NONE &&
        (pc->opts.local != ASM_LOCAL_ILU0 || pc->opts.coarse != ASM_COARSE_NONE))
      return fail(ASM_ERR_INVALID, "graph cycles support ILU(0) local solves without a global coarse grid");
    const int64_t n = 3 * (int64_t)S->pat.N;
    asm_status st = ensure_workspace(S, m, user_stream);
    if (st != ASM_OK) return st;
    Workspace &W = S->ws;
    // the graphs run on a stream of the library's own (a capture needs a
    // stream that is not the legacy default one), after the caller's work
    if (!W.gstream) ASM_HIP(hipStreamCreateWithFlags(&W.gstream, hipStreamNonBlocking));
    if (!W.gready) ASM_HIP(hipEventCreateWithFlags(&W.gready, hipEventDisableTiming));
    hipStream_t s = W.gstream;
    ASM_HIP(hipEventRecord(W.gready, user_stream));
    ASM_HIP(hipStreamWaitEvent(s, W.gready, 0));
    if ((st = ensure_tuned(S, m, s)) != ASM_OK) return st;
    bool bad = false;
    if ((st = any_nonfinite(S, b, n, s, &bad)) != ASM_OK) return st;
    if (!bad && (st = any_nonfinite(S, x, n, s, &bad)) != ASM_OK) return st;
    if (bad) return fail(ASM_ERR_NONFINITE, "non-finite b or x0");
    const int ld = m + 1;
    double *hp = W.pinned;
    int nb = 0;
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
    // initial residual: beta into misc[1], 1/beta into scale[0], r into U_0
    int nbr = 0;
    ASM_HIP(launch_residual(S->sell, x, b, W.U, W.partial, &nbr, s));
    ASM_HIP(launch_norm_finalize(nbr, W.partial, 0, nullptr, nullptr, W.misc + 1, W.scale, nullptr, s));
    ASM_HIP(hipMemcpyAsync(hp, W.misc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    ASM_HIP(hipStreamSynchronize(s));
    double beta = hp[0];
    info->rel_res_true = info->rel_res_est = beta / scl;
    if (o->fixed_iters == 0 && beta <= tol) return ASM_OK;
    const int limit = o->fixed_iters > 0 ? o->fixed_iters : o->max_iters;
    // stopping test of the cycles (host-written, read by the Givens kernel).
    // Pinned scalars: [4, 7) this state, [8, 11) what a cycle publishes,
    // [12] the step limit of the next cycle.
    static_assert(sizeof(CycleState) <= 3 * sizeof(double), "cycle state fits its pinned slot");
    CycleState cs0{};
    cs0.use_tol = o->fixed_iters == 0 ? 1 : 0;
    cs0.tol = tol;
    std::memcpy(hp + 4, &cs0, sizeof cs0);
    ASM_HIP(hipMemcpyAsync(W.cst, hp + 4, sizeof cs0, hipMemcpyHostToDevice, s));
    ASM_HIP(hipStreamSynchronize(s));
    double *pub = W.pinned_dev + 8;
    const void *key[4] = {pc, b, x, reinterpret_cast<const void *>((intptr_t)m)};
    if (!W.gexec || std::memcmp(W.gkey, key, sizeof key) != 0) {
      W.drop_graph();
      // one cycle: m steps whose kernels return at once after the cycle's
      // end, then the correction x += B^-1 V_k y and the true residual
      const int *skip = &W.cst->done;
      ASM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      auto record = [&]() -> asm_status {
        Profiler none;
        ASM_HIP(launch_cycle_start(W.cst, W.gg, W.misc + 1, s));
        for (int j = 0; j < m; ++j) {
          const double *Uj = W.U + (size_t)j * W.ldu;
          asm_status e2 = apply_precond(pc, Uj, W.scale + j, W.z, s, &none, skip);
          if (e2 != ASM_OK) return e2;
          ASM_HIP(launch_spmv(S->sell, W.z, W.w, s, skip, S->tune.spmv_rows));
          int nbd = 0, nbu = 0;
          ASM_HIP(launch_multidot(n, j + 1, W.U, W.ldu, W.w, W.partial, &nbd, s, skip, S->tune.red_blocks));
          ASM_HIP(launch_reduce_cols(nbd, j + 2, W.partial, W.dvec, s, skip));
          ASM_HIP(launch_update(n, j + 1, W.U, W.ldu, W.dvec, W.scale, W.w, W.U + (size_t)(j + 1) * W.ldu, W.partial,
                                &nbu, s, skip, S->tune.red_blocks));
          ASM_HIP(launch_norm_finalize(nbu, W.partial, j + 1, W.dvec, W.scale, W.H + (size_t)j * ld, W.scale + j + 1,
                                       nullptr, s, skip));
          ASM_HIP(launch_givens(j, ld, W.H, W.gcs, W.gsn, W.gg, W.dvec, W.cst, s));
        }
        ASM_HIP(launch_cycle_end(ld, W.H, W.gg, W.scale, W.coef, W.cst, s));
        ASM_HIP(launch_lincomb_dev(n, W.cst, W.U, W.ldu, W.coef, W.t, s));
        asm_status e2 = apply_precond(pc, W.t, nullptr, W.z, s, &none);
        if (e2 != ASM_OK) return e2;
        ASM_HIP(launch_axpy(n, W.z, x, s));
        int nbe = 0;
        ASM_HIP(launch_residual(S->sell, x, b, W.U, W.partial, &nbe, s));
        ASM_HIP(launch_norm_finalize(nbe, W.partial, 0, nullptr, nullptr, W.misc + 1, W.scale, nullptr, s));
        ASM_HIP(launch_cycle_publish(W.cst, W.gg, W.misc + 1, pub, s));
        return ASM_OK;
      };
      const asm_status rec = record();
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(s, &graph);
      if (rec != ASM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rec;
      }
      if (ec != hipSuccess) return fail(ASM_ERR_HIP, hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&W.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        W.gexec = nullptr;
        return fail(ASM_ERR_HIP, hipGetErrorString(ei));
      }
      std::memcpy(W.gkey, key, sizeof key);
    }
    asm_status result = ASM_NOT_CONVERGED;
    int *kmax_host = reinterpret_cast<int *>(hp + 12);
    while (true) {
      if (beta == 0.0) { result = ASM_OK; break; }
      info->cycles++;
      *kmax_host = std::min(m, limit - info->iters);
      ASM_HIP(hipMemcpyAsync(&W.cst->kmax, kmax_host, sizeof(int), hipMemcpyHostToDevice, s));
      ASM_HIP(hipGraphLaunch(W.gexec, s));
      ASM_HIP(hipStreamSynchronize(s));
      const double *pr = hp + 8;
      info->iters += (int)pr[0];
      beta = pr[1];
      info->rel_res_est = pr[2] / scl;
      info->rel_res_true = beta / scl;
      if (o->fixed_iters > 0) {
        if (info->iters >= o->fixed_iters) { result = ASM_OK; break; }
      } else if (beta <= tol) {
        result = ASM_OK;
        break;
      }
      if (info->iters >= limit) { result = ASM_NOT_CONVERGED; break; }
    }
    return result;
  }
  ASM_CATCH_ALL
}

asm_status asm_set_allocator(asm_alloc_fn alloc, asm_free_fn free_fn, void *ctx) {
  try {
    g_err.clear();
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(ASM_ERR_INVALID, "set both hooks or neither");
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    g_allocator.alloc = alloc;
    g_allocator.free = free_fn;
    g_allocator.ctx = alloc ? ctx : nullptr;
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_tuning_get(asm_system S, asm_tuning *out) {
  try {
    g_err.clear();
    if (!S || !out) return fail(ASM_ERR_INVALID, "NULL argument");
    const Tuning &t = S->tune;
    std::memset(out, 0, sizeof *out);
    out->spmv_rows = t.spmv_rows;
    out->red_blocks = t.red_blocks;
    out->source = t.source;
    out->restart = t.restart;
    for (int k = 0; k < 3; ++k) out->spmv_us[k] = t.spmv_us[k];
    for (int k = 0; k < 4; ++k) out->krylov_us[k] = t.krylov_us[k];
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_tuning_set(asm_system S, int32_t spmv_rows, int32_t red_blocks) {
  try {
    g_err.clear();
    if (!S) return fail(ASM_ERR_INVALID, "NULL argument");
    Tuning t;
    if (spmv_rows == 0 && red_blocks == 0) {
      t.retime = true;  // untuned: the next solve times again
    } else {
      if (spmv_rows != 1 && spmv_rows != 2 && spmv_rows != 4) return fail(ASM_ERR_INVALID, "spmv_rows must be 1, 2 or 4");
      if (red_blocks != 512 && red_blocks != 1024 && red_blocks != 2048 && red_blocks != 4096)
        return fail(ASM_ERR_INVALID, "red_blocks must be 512, 1024, 2048 or 4096");
      t.spmv_rows = spmv_rows;
      t.red_blocks = red_blocks;
      t.source = ASM_TUNE_SET;
    }
    S->ws.drop_graph();  // a captured cycle holds the old launch shapes
    S->tune = t;
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_profile_enable(asm_system S, int32_t phase_mask) {
  try {
    g_err.clear();
    if (!S) return fail(ASM_ERR_INVALID, "NULL argument");
    S->prof.on = (phase_mask != 0);
    S->prof.mask = (uint32_t)phase_mask;
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_profile_read(asm_system S, asm_profile *out, int32_t reset) {
  try {
    g_err.clear();
    if (!S || !out) return fail(ASM_ERR_INVALID, "NULL argument");
    for (int k = 0; k < ASM_NPHASE; ++k) {
      out->launches[k] = S->prof.launches[k];
      out->ms[k] = S->prof.ms[k];
    }
    if (reset) S->prof.reset();
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

void asm_destroy_precond(asm_precond pc) {
  // a cycle graph captured for this preconditioner holds its device
  // pointers: it goes with it (a later handle may reuse the address)
  if (pc && pc->sys && pc->sys->ws.gkey[0] == pc) pc->sys->ws.drop_graph();
  delete pc;
}
void asm_destroy_system(asm_system S) { delete S; }

}  // extern "C"
