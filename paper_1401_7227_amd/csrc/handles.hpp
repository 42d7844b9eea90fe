// Internal definitions shared by the C ABI sources: device memory owners,
// the per-system Krylov workspace and the system / preconditioner handles.
#pragma once
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/asm.h"
#include "dense.hpp"
#include "kernels.hpp"
#include "setup.hpp"

namespace asmx {

// Thread-local message of the last failing call (asm_last_error).
extern thread_local std::string g_err;

inline asm_status fail(asm_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

// Every C entry point returns its errors: the body runs in a try block and
// no C++ exception (a host allocation failing inside a container, say)
// crosses the ABI.  Handles under construction are held by unique_ptr until
// they are handed out, so nothing leaks on that path either.
#define ASM_CATCH_ALL                                                                          \
  catch (const std::bad_alloc &) {                                                             \
    return fail(ASM_ERR_OOM, "host allocation failed");                                        \
  }                                                                                            \
  catch (const std::exception &ex_) {                                                          \
    return fail(ASM_ERR_INVALID, std::string("internal error: ") + ex_.what());                \
  }                                                                                            \
  catch (...) {                                                                                \
    return fail(ASM_ERR_INVALID, "internal error");                                            \
  }

#define ASM_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return ::asmx::fail(e_ == hipErrorOutOfMemory ? ASM_ERR_OOM : ASM_ERR_HIP,             \
                          std::string(#call) + ": " + hipGetErrorString(e_));                \
  } while (0)

// Device-memory hooks (asm_set_allocator): NULL functions mean
// hipMalloc / hipFree.
struct Allocator {
  asm_alloc_fn alloc = nullptr;
  asm_free_fn free = nullptr;
  void *ctx = nullptr;
};
Allocator current_allocator();

// Owner of device allocations; frees everything on destruction, through
// the allocator that was current when it was created.
struct DevMem {
  struct Block {
    void *p;
    size_t bytes;
    int dev;
  };
  Allocator a = current_allocator();
  std::vector<Block> ptrs;
  size_t bytes = 0;
  ~DevMem() { release(); }
  void release() {
    if (a.free && !ptrs.empty()) {
      // hooked memory returns to its owner at once: no kernel on its device
      // may still use it
      int cur = 0;
      (void)hipGetDevice(&cur);
      int synced = -1;
      for (const Block &q : ptrs) {
        if (q.dev != synced) {
          if (q.dev != cur) (void)hipSetDevice(q.dev);
          (void)hipDeviceSynchronize();
          synced = q.dev;
        }
        a.free(q.p, q.bytes, q.dev, a.ctx);
      }
      if (synced != cur) (void)hipSetDevice(cur);
    } else {
      for (const Block &q : ptrs) (void)hipFree(q.p);
    }
    ptrs.clear();
    bytes = 0;
  }
  template <typename T>
  hipError_t alloc(T **out, size_t n) {
    *out = nullptr;
    if (n == 0) n = 1;
    void *p = nullptr;
    const size_t nb = n * sizeof(T);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (a.alloc) {
      p = a.alloc(nb, dev, a.ctx);
      if (!p) return hipErrorOutOfMemory;
      if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {  // the kernels' 16-byte loads need less; keep hipMalloc's
        a.free(p, nb, dev, a.ctx);
        return hipErrorInvalidValue;
      }
    } else {
      e = hipMalloc(&p, nb);
      if (e != hipSuccess) return e;
    }
    ptrs.push_back(Block{p, nb, dev});
    bytes += nb;
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
  int32_t n1 = 0;      // destinations of the first segment
  int32_t lanes = 1;   // threads per destination in [0, n1) (about the mean fan-in)
  int32_t lanes2 = 1;  // threads per destination in [n1, n)
  int32_t *ptr = nullptr, *idx = nullptr;
};

// Largest power of two (at most 64) not above the mean fan-in of
// destinations [d0, d1).
inline int32_t gather_lanes(const GatherList &h, int32_t d0, int32_t d1) {
  if (d1 <= d0) return 1;
  const double mean = (double)(h.ptr[d1] - h.ptr[d0]) / (d1 - d0);
  int32_t g = 1;
  while (g < 64 && 2 * g <= mean) g *= 2;
  return g;
}

inline hipError_t upload_gather(DevMem &m, GatherDev &g, const GatherList &h, hipStream_t s) {
  g.n = h.size();
  g.n1 = (h.split >= 0 && h.split <= g.n) ? h.split : g.n;
  g.lanes = gather_lanes(h, 0, g.n1);
  g.lanes2 = gather_lanes(h, g.n1, g.n);
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
  double *misc = nullptr;     // [1] beta, [2] scratch norm
  int *flag = nullptr;
  double *pinned = nullptr;   // host staging: scalars, then one published column per step
  double *pinned_dev = nullptr;  // the same memory as seen by kernels
  hipEvent_t step_done[kMaxRestart] = {};
  // restart cycles run as graphs (asm_solve_graph): device cycle state and
  // Givens arrays, the stream the graphs run on, and the executable graph
  // with what it was captured for (preconditioner, b, x, restart length)
  asmx::CycleState *cst = nullptr;
  double *gcs = nullptr, *gsn = nullptr, *gg = nullptr;
  hipStream_t gstream = nullptr;
  hipEvent_t gready = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void *gkey[4] = {};
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    gkey[0] = gkey[1] = gkey[2] = gkey[3] = nullptr;
  }
  ~Workspace() {
    drop_graph();
    if (gstream) (void)hipStreamDestroy(gstream);
    if (gready) (void)hipEventDestroy(gready);
    if (pinned) (void)hipHostFree(pinned);
    for (hipEvent_t e : step_done)
      if (e) (void)hipEventDestroy(e);
  }
};

// Pinned layout: [0, 16) scalars; column j of a cycle at kPubBase + j*kPubStride
// holds H(0..j+1, j) and then ||w|| (the breakdown reference).
constexpr int kPubBase = 16, kPubStride = kMaxRestart + 4;

// Krylov workspace of a system (allocated on first use), the batched-solve
// helpers and the preconditioner application shared by the solvers.
asm_status ensure_workspace(asm_system S, int m, hipStream_t s);
// Times the launch-shape candidates of an untuned system (or takes the
// process-wide cached choice of its size class); needs the workspace.
asm_status ensure_tuned(asm_system S, int m, hipStream_t s);
// Structure checks of asm_create_system (host copy of the pattern).
asm_status validate_pattern(const HostPattern &P);
// Option checks of asm_setup_precond against a pattern, and its device part:
// uploads a host plan built by build_plan, then assembles and factorises.
asm_status check_precond_opts(const HostPattern &A, const asm_precond_opts *o);
asm_status setup_from_plan(asm_system S, const asm_precond_opts *o, std::shared_ptr<PlanHost> plan,
                           hipStream_t stream, asm_precond *out);
// skip: optional device flag of a graph-mode cycle (the ILU(0) and
// unpreconditioned paths only).
asm_status apply_precond(asm_precond pc, const double *r, const double *scale, double *z, hipStream_t s,
                         Profiler *prof = nullptr, const int *skip = nullptr);

}  // namespace asmx

namespace asmx {
// A named roctx range over one library call (seen by rocprofv3
// --marker-trace; a no-op without a profiler).
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

// The launch-shape choices of a system's Krylov kernels (see asm_tuning).
struct Tuning {
  int spmv_rows = 1;
  int red_blocks = kReduceBlocks;
  int source = ASM_TUNE_DEFAULT;
  int restart = 0;
  bool retime = false;  // asm_tuning_set(0, 0): time again, bypass the cache
  double spmv_us[3] = {};
  double krylov_us[4] = {};
};
}  // namespace asmx

struct asm_system_s {
  int device = 0;
  asmx::Tuning tune;
  asmx::HostPattern pat;
  asmx::DevMem mem;
  int32_t *rp = nullptr, *ci = nullptr;
  double *vals = nullptr;  // CSR values (sources of the assembly)
  asmx::SellDev sell;
  asmx::Workspace ws;
  asmx::Profiler prof;
};

struct asm_precond_s {
  asm_system sys = nullptr;
  asm_precond_opts opts{};
  // Pattern-only state, shared by the preconditioners cloned from one
  // setup: host-side parts kept for export and messages, and the device
  // arrays that never change after setup (maps, schedules, gather lists).
  std::shared_ptr<asmx::PlanHost> plan;
  std::shared_ptr<asmx::DevMem> smem;
  asmx::DevMem mem;       // this handle's own arrays: records, factors, work vectors
  size_t rec_bytes = 0;
  asmx::DevPlan dp{};     // factorisation
  asmx::ApplyPlan ap{};   // sweeps
  asmx::GatherDev l1, l2, asrc, c1, c2, c3;
  double *L1 = nullptr, *L2 = nullptr;  // lumped block values
  double *aval = nullptr;               // assembled A_i (CSR)
  double *PA = nullptr, *PNF = nullptr; // lumped residual sums
  void *recbuf = nullptr;               // sweep records
  int32_t *rl_src = nullptr, *rl_base = nullptr, *rl_stride = nullptr;
  uint8_t *rl_to32 = nullptr;
  int64_t rl_n = 0;
  int32_t *cptr = nullptr, *cidx = nullptr;
  unsigned long long *bad = nullptr;
  // global coarse grid: pattern-only maps (shared), then this handle's A_C
  // values, dense matrix and inverse, and work vectors
  int32_t ncv = 0;
  int32_t *cvar = nullptr;
  asmx::GatherDev cbox, casrc;
  int32_t *acp = nullptr, *acc = nullptr;
  double *acv = nullptr, *cM = nullptr, *cMinv = nullptr, *cfcol = nullptr, *crc = nullptr, *cxc = nullptr;
  double *crtmp = nullptr, *cr2 = nullptr, *cpart = nullptr;
  int *cbad = nullptr;
  // exact local solves: dense inverses of every A_i
  asmx::DenseLocal xd{};
  int32_t xmaxn3 = 0;
  asm_precond_stats stats{};
};

