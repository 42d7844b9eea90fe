// Batched restarted GMRES: many independent systems iterate in lockstep and
// every kernel launch serves all of them.  The engine below runs restart
// cycles over a changing set of solves (solves may join between cycles);
// asm_solve_batch and the request server are built on it.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <deque>
#include <future>
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_set>

#include "handles.hpp"

namespace asmx {

// One solve in flight: the host side of its Arnoldi process.
struct BatchEntry {
  asm_system S = nullptr;
  asm_precond pc = nullptr;
  const double *b = nullptr;
  double *x = nullptr;
  int64_t key = 0;
  double scl = 1.0, tol = 0.0, beta = 0.0;
  asm_solve_info info{};
  int32_t status = ASM_NOT_CONVERGED;
  std::vector<double> H, cs, sn, g, sc;
  int k = 0, kmax = 0;
  bool in_cycle = false;
  bool busy = false;     // slot holds a solve (iterating or finished, not yet released)
  bool iterating = false;
};

// Restart cycles of up to `cap` solves.  Each solve keeps the block counts
// of a single-system launch in every batched kernel, so its arithmetic, and
// therefore its result, is exactly that of asm_solve.
class BatchEngine {
 public:
  ~BatchEngine() { release_all(); }

  asm_status init(int cap, const asm_solve_opts &o, hipStream_t s) {
    if (cap < 1) return fail(ASM_ERR_INVALID, "batch capacity must be positive");
    o_ = o;
    s_ = s;
    cap_ = cap;
    m_ = o.restart;
    ld_ = m_ + 1;
    limit_ = o.fixed_iters > 0 ? o.fixed_iters : o.max_iters;
    region_ = 1 + (size_t)m_ * kPubStride + 1 + m_;
    ent_.assign(cap, BatchEntry{});
    ASM_HIP(hipHostMalloc((void **)&pin_, sizeof(double) * (region_ * cap + 16), hipHostMallocCoherent));
    ASM_HIP(hipHostGetDevicePointer((void **)&pin_dev_, pin_, 0));
    ASM_HIP(hipHostMalloc((void **)&tabh_, sizeof(BatchSys) * cap, hipHostMallocDefault));
    ASM_HIP(hipMalloc((void **)&tabd_, sizeof(BatchSys) * cap));
    slot_ints_ = (size_t)kBkCount * (2 * (size_t)cap + 1);
    ASM_HIP(hipHostMalloc((void **)&segh_, sizeof(int32_t) * slot_ints_ * kRing, hipHostMallocDefault));
    ASM_HIP(hipMalloc((void **)&segd_, sizeof(int32_t) * slot_ints_ * kRing));
    for (hipEvent_t &e : ring_ev_) ASM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (hipEvent_t &e : step_ev_) ASM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return ASM_OK;
  }

  int capacity() const { return cap_; }
  int free_slots() const {
    int n = 0;
    for (const BatchEntry &e : ent_) n += !e.busy;
    return n;
  }
  int iterating() const {
    int n = 0;
    for (const BatchEntry &e : ent_) n += e.iterating;
    return n;
  }
  BatchEntry &entry(int slot) { return ent_[slot]; }
  void release(int slot) { ent_[slot] = BatchEntry{}; }

  struct NewSolve {
    asm_system S;
    asm_precond pc;
    const double *b;
    double *x;
    int64_t key;
  };

  // Places the solves in free slots (slots[i] receives the slot of add[i]),
  // checks b and x0, computes ||b|| and the initial residual.  A solve with
  // non-finite input finishes at once with ASM_ERR_NONFINITE; one that needs
  // no iteration finishes with ASM_OK.  The others iterate from the next
  // cycle.  With all_or_none, one non-finite input stops the others too,
  // before anything is written (they are left not iterating).
  asm_status add(const std::vector<NewSolve> &add, std::vector<int> &slots, bool all_or_none) {
    slots.assign(add.size(), -1);
    std::vector<int> fresh;
    for (size_t a = 0; a < add.size(); ++a) {
      int sl = -1;
      for (int i = 0; i < cap_; ++i)
        if (!ent_[i].busy) { sl = i; break; }
      if (sl < 0) return fail(ASM_ERR_INVALID, "batch is full");
      BatchEntry &E = ent_[sl];
      E = BatchEntry{};
      E.S = add[a].S; E.pc = add[a].pc; E.b = add[a].b; E.x = add[a].x; E.key = add[a].key;
      E.busy = true;
      slots[a] = sl;
      fresh.push_back(sl);
      asm_status st = ensure_workspace(E.S, m_, s_);
      if (st == ASM_OK) st = ensure_tuned(E.S, m_, s_);
      if (st != ASM_OK) return st;
      fill_table(sl);
    }
    if (fresh.empty()) return ASM_OK;
    ASM_HIP(hipMemcpyAsync(tabd_, tabh_, sizeof(BatchSys) * cap_, hipMemcpyHostToDevice, s_));
    for (int i : fresh) {
      BatchEntry &E = ent_[i];
      Workspace &W = E.S->ws;
      const int64_t n = 3 * (int64_t)E.S->pat.N;
      ASM_HIP(hipMemsetAsync(W.flag, 0, sizeof(int), s_));
      ASM_HIP(launch_check_finite(n, E.b, W.flag, s_));
      ASM_HIP(launch_check_finite(n, E.x, W.flag, s_));
      int nb = 0;
      ASM_HIP(launch_norm2(n, E.b, W.partial, &nb, s_));
      ASM_HIP(launch_reduce_cols(nb, 1, W.partial, W.misc + 2, s_));
      ASM_HIP(hipMemcpyAsync(pin_ + region_ * i, W.misc + 2, sizeof(double), hipMemcpyDeviceToHost, s_));
      ASM_HIP(hipMemcpyAsync(pin_ + region_ * i + 1, W.flag, sizeof(int), hipMemcpyDeviceToHost, s_));
    }
    ASM_HIP(hipStreamSynchronize(s_));
    if (all_or_none)
      for (int i : fresh) {
        int flag = 0;
        std::memcpy(&flag, pin_ + region_ * i + 1, sizeof(int));
        if (flag) {
          for (int i2 : fresh) {
            std::memcpy(&flag, pin_ + region_ * i2 + 1, sizeof(int));
            if (flag) ent_[i2].status = ASM_ERR_NONFINITE;
          }
          return ASM_OK;
        }
      }
    std::vector<int> need;
    for (int i : fresh) {
      BatchEntry &E = ent_[i];
      int flag = 0;
      std::memcpy(&flag, pin_ + region_ * i + 1, sizeof(int));
      if (flag) {
        E.status = ASM_ERR_NONFINITE;
        continue;
      }
      const double bn = std::sqrt(pin_[region_ * i]);
      if (bn == 0.0 && o_.fixed_iters == 0) {  // b = 0: x = 0, as asm_solve
        ASM_HIP(hipMemsetAsync(E.x, 0, 3 * (size_t)E.S->pat.N * sizeof(double), s_));
        E.status = ASM_OK;
        continue;
      }
      E.scl = bn > 0.0 ? bn : 1.0;
      E.tol = o_.rtol * bn;
      need.push_back(i);
    }
    if (need.empty()) {
      ASM_HIP(hipStreamSynchronize(s_));
      return ASM_OK;
    }
    asm_status st = residuals(need);
    if (st != ASM_OK) return st;
    for (int i : need) {
      BatchEntry &E = ent_[i];
      E.info.rel_res_true = E.info.rel_res_est = E.beta / E.scl;
      if ((o_.fixed_iters == 0 && E.beta <= E.tol) || E.beta == 0.0) E.status = ASM_OK;
      else E.iterating = true;
    }
    return ASM_OK;
  }

  // Order of the solves in every launch of the next cycles: as placed, or
  // the largest systems first (their workgroups start first, so the launch
  // ends with the small ones).  Results do not depend on it.
  void set_largest_first(bool on) { largest_first_ = on; }
  // Work of the last cycle: block rows summed over the steps each solve ran.
  double last_cycle_work() const { return last_work_; }

  // One restart cycle of every iterating solve; solves that end (converged,
  // iteration limit) stop iterating and keep their slot until released.
  asm_status cycle() {
    std::vector<int> active;
    for (int i = 0; i < cap_; ++i)
      if (ent_[i].iterating) active.push_back(i);
    last_work_ = 0.0;
    if (active.empty()) return ASM_OK;
    if (largest_first_)
      std::stable_sort(active.begin(), active.end(),
                       [&](int a, int b) { return ent_[a].S->pat.N > ent_[b].S->pat.N; });
    asm_status st;
    int K = 0;
    for (int i : active) {
      BatchEntry &E = ent_[i];
      E.H.assign((size_t)ld_ * m_, 0.0);
      E.cs.assign(m_, 0.0);
      E.sn.assign(m_, 0.0);
      E.g.assign(m_ + 1, 0.0);
      E.sc.assign(m_ + 1, 0.0);
      E.g[0] = E.beta;
      E.sc[0] = 1.0 / E.beta;
      E.k = 0;
      E.kmax = std::min(m_, limit_ - E.info.iters);
      E.in_cycle = true;
      E.info.cycles++;
      K = std::max(K, E.kmax);
    }
    std::vector<std::vector<int>> ran(K);  // solves that ran step j
    auto enqueue_step = [&](int j) -> asm_status {
      std::vector<int> act;
      for (int i : active)
        if (ent_[i].in_cycle && ent_[i].kmax > j) {
          act.push_back(i);
          last_work_ += (double)ent_[i].S->pat.N;
        }
      ran[j] = act;
      if (act.empty()) return ASM_OK;
      BatchSeg seg[kBkCount];
      int sl = 0;
      asm_status e2 = segs_for(act, seg, &sl);
      if (e2 != ASM_OK) return e2;
      ASM_HIP(launch_batch_precond(tabd_, seg, j, s_));
      ASM_HIP(launch_batch_spmv(tabd_, seg[kBkSpmv], false, s_));
      ASM_HIP(launch_batch_multidot(tabd_, seg[kBkRed], j + 1, s_));
      ASM_HIP(launch_batch_reduce(tabd_, seg[kBkOne], j + 2, true, 0, s_));
      ASM_HIP(launch_batch_update(tabd_, seg[kBkRed], j + 1, ld_, s_));
      ASM_HIP(launch_batch_norm_finalize(tabd_, seg[kBkOne], j, ld_, kPubStride, 0, s_));
      ASM_HIP(hipEventRecord(step_ev_[j], s_));
      ASM_HIP(hipEventRecord(ring_ev_[sl], s_));
      return ASM_OK;
    };
    if ((st = enqueue_step(0)) != ASM_OK) return st;
    for (int j = 0; j < K; ++j) {
      // keep the next step queued while step j's columns are read back
      if (j + 1 < K && (st = enqueue_step(j + 1)) != ASM_OK) return st;
      if (ran[j].empty()) continue;
      ASM_HIP(hipEventSynchronize(step_ev_[j]));
      for (int i : ran[j]) {
        BatchEntry &E = ent_[i];
        if (!E.in_cycle) continue;  // left the cycle at an earlier step; this step is discarded
        auto Hh = [&](int r, int c) -> double & { return E.H[(size_t)c * ld_ + r]; };
        const double *col = pin_ + region_ * i + 1 + (size_t)j * kPubStride;
        for (int r = 0; r <= j + 1; ++r) Hh(r, j) = col[r];
        const double w0 = col[j + 2];
        const double hn = Hh(j + 1, j);
        E.sc[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
        for (int r = 0; r < j; ++r) {
          const double a = Hh(r, j), c = Hh(r + 1, j);
          Hh(r, j) = E.cs[r] * a + E.sn[r] * c;
          Hh(r + 1, j) = -E.sn[r] * a + E.cs[r] * c;
        }
        const double rho = std::hypot(Hh(j, j), Hh(j + 1, j));
        if (rho == 0.0) {
          E.cs[j] = 1.0;
          E.sn[j] = 0.0;
        } else {
          E.cs[j] = Hh(j, j) / rho;
          E.sn[j] = Hh(j + 1, j) / rho;
        }
        Hh(j, j) = rho;
        Hh(j + 1, j) = 0.0;
        E.g[j + 1] = -E.sn[j] * E.g[j];
        E.g[j] = E.cs[j] * E.g[j];
        E.k = j + 1;
        E.info.rel_res_est = std::fabs(E.g[j + 1]) / E.scl;
        if (hn <= 1e-14 * w0 || (o_.fixed_iters == 0 && std::fabs(E.g[j + 1]) <= E.tol) || E.k >= E.kmax)
          E.in_cycle = false;
      }
    }
    // cycle end: x += B^-1 (V y) for every solve of the cycle
    for (int i : active) {
      BatchEntry &E = ent_[i];
      E.info.iters += E.k;
      auto Hh = [&](int r, int c) -> double & { return E.H[(size_t)c * ld_ + r]; };
      std::vector<double> y(E.k);
      for (int r = E.k - 1; r >= 0; --r) {
        double acc = E.g[r];
        for (int c = r + 1; c < E.k; ++c) acc -= Hh(r, c) * y[c];
        y[r] = acc / Hh(r, r);
      }
      double *coefh = pin_ + region_ * i + 1 + (size_t)m_ * kPubStride;
      coefh[0] = (double)E.k;
      for (int r = 0; r < E.k; ++r) coefh[1 + r] = y[r] * E.sc[r];
    }
    {
      BatchSeg seg[kBkCount];
      int sl = 0;
      if ((st = segs_for(active, seg, &sl)) != ASM_OK) return st;
      ASM_HIP(launch_batch_lincomb(tabd_, seg[kBkVec], s_));
      ASM_HIP(launch_batch_precond(tabd_, seg, -1, s_));
      ASM_HIP(launch_batch_axpy(tabd_, seg[kBkVec], s_));
      ASM_HIP(hipEventRecord(ring_ev_[sl], s_));
    }
    if ((st = residuals(active)) != ASM_OK) return st;
    for (int i : active) {
      BatchEntry &E = ent_[i];
      E.info.rel_res_true = E.beta / E.scl;
      bool end = false;
      if (o_.fixed_iters > 0) {
        if (E.info.iters >= o_.fixed_iters) { E.status = ASM_OK; end = true; }
      } else if (E.beta <= E.tol) {
        E.status = ASM_OK;
        end = true;
      }
      if (!end && (E.info.iters >= limit_ || E.beta == 0.0)) {
        E.status = E.beta == 0.0 ? ASM_OK : ASM_NOT_CONVERGED;
        end = true;
      }
      if (end) E.iterating = false;
    }
    return ASM_OK;
  }

 private:
  static constexpr int kRing = kMaxRestart + 4;

  void fill_table(int i) {
    BatchEntry &E = ent_[i];
    asm_system S = E.S;
    asm_precond pc = E.pc;
    Workspace &W = S->ws;
    BatchSys &T = tabh_[i];
    std::memset(&T, 0, sizeof T);
    T.n = 3 * (int64_t)S->pat.N;
    T.ldu = W.ldu;
    T.U = W.U; T.w = W.w; T.z = W.z; T.t = W.t;
    T.partial = W.partial; T.dvec = W.dvec; T.H = W.H; T.scale = W.scale; T.misc = W.misc;
    T.red_blocks = S->tune.red_blocks;
    T.pub = pin_dev_ + region_ * i + 1;
    T.coefh = pin_dev_ + region_ * i + 1 + (size_t)m_ * kPubStride;
    T.b = E.b;
    T.x = E.x;
    T.N = S->pat.N;
    T.nlog = (S->pat.N + 255) / 256;
    T.sptr = S->sell.sptr; T.cols = S->sell.cols; T.vals = S->sell.vals;
    T.kind = pc->opts.kind;
    T.restricted = pc->opts.combine == ASM_COMBINE_RESTRICTED;
    if (pc->opts.kind != ASM_KIND_NONE) {
      T.npos = (int32_t)pc->plan->total_pos;
      T.nsub = pc->ap.nsub;
      T.ap = pc->ap;
      T.c1n = pc->c1.n; T.c1n1 = pc->c1.n1; T.c1lanes = pc->c1.lanes; T.c1lanes2 = pc->c1.lanes2;
      T.c1ptr = pc->c1.ptr; T.c1idx = pc->c1.idx;
      T.c2n = pc->c2.n; T.c2n1 = pc->c2.n1; T.c2lanes = pc->c2.lanes; T.c2lanes2 = pc->c2.lanes2;
      T.c2ptr = pc->c2.ptr; T.c2idx = pc->c2.idx;
      T.PA = pc->PA; T.PNF = pc->PNF;
      T.cptr = pc->cptr; T.cidx = pc->cidx;
    }
  }

  // Block-to-solve tables of every kernel kind for the solves in `act`,
  // written to the next ring slot.  A slot is rewritten only after the
  // stream passed the event recorded after its last use.
  asm_status segs_for(const std::vector<int> &act, BatchSeg *seg, int *slot) {
    const int sl = ring_next_;
    ASM_HIP(hipEventSynchronize(ring_ev_[sl]));
    ring_next_ = (ring_next_ + 1) % kRing;
    int32_t *h = segh_ + slot_ints_ * sl, *d = segd_ + slot_ints_ * sl;
    const int na = (int)act.size();
    for (int k = 0; k < kBkCount; ++k) {
      int32_t *st0 = h + (size_t)k * (2 * cap_ + 1), *sy = st0 + cap_ + 1;
      int nseg = 0, tot = 0;
      for (int a = 0; a < na; ++a) {
        const BatchSys &T = tabh_[act[a]];
        int nb = batch_blocks((BatchKernel)k, T);
        if (k == kBkCopy && T.kind != ASM_KIND_NONE) nb = 0;
        if ((k == kBkC1 || k == kBkC2 || k == kBkCrs || k == kBkApply || k == kBkCombine) && T.kind == ASM_KIND_NONE)
          nb = 0;
        if (k == kBkCombine && T.restricted) nb = 0;
        if (nb <= 0) continue;
        st0[nseg] = tot;
        sy[nseg] = act[a];
        ++nseg;
        tot += nb;
      }
      st0[nseg] = tot;
      seg[k].start = d + (size_t)k * (2 * cap_ + 1);
      seg[k].sys = seg[k].start + cap_ + 1;
      seg[k].n = nseg;
      seg[k].total = tot;
    }
    ASM_HIP(hipMemcpyAsync(d, h, sizeof(int32_t) * slot_ints_, hipMemcpyHostToDevice, s_));
    *slot = sl;
    return ASM_OK;
  }

  // True residual norms of the solves in `act` (synchronises the stream).
  asm_status residuals(const std::vector<int> &act) {
    BatchSeg seg[kBkCount];
    int sl = 0;
    asm_status st = segs_for(act, seg, &sl);
    if (st != ASM_OK) return st;
    ASM_HIP(launch_batch_spmv(tabd_, seg[kBkSpmv], true, s_));
    ASM_HIP(launch_batch_norm_finalize(tabd_, seg[kBkOne], -1, ld_, kPubStride, 1, s_));
    ASM_HIP(hipEventRecord(ring_ev_[sl], s_));
    ASM_HIP(hipStreamSynchronize(s_));
    for (int i : act) ent_[i].beta = pin_[region_ * i];
    return ASM_OK;
  }

  void release_all() {
    if (s_) (void)hipStreamSynchronize(s_);
    if (pin_) (void)hipHostFree(pin_);
    if (tabh_) (void)hipHostFree(tabh_);
    if (tabd_) (void)hipFree(tabd_);
    if (segh_) (void)hipHostFree(segh_);
    if (segd_) (void)hipFree(segd_);
    for (hipEvent_t e : ring_ev_)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : step_ev_)
      if (e) (void)hipEventDestroy(e);
  }

  asm_solve_opts o_{};
  hipStream_t s_ = nullptr;
  bool largest_first_ = false;
  double last_work_ = 0.0;
  int cap_ = 0, m_ = 0, ld_ = 0, limit_ = 0;
  size_t region_ = 0;  // pinned doubles per slot: [beta][m published columns][1 + m coefficients]
  std::vector<BatchEntry> ent_;
  double *pin_ = nullptr, *pin_dev_ = nullptr;
  BatchSys *tabh_ = nullptr, *tabd_ = nullptr;
  size_t slot_ints_ = 0;
  int32_t *segh_ = nullptr, *segd_ = nullptr;
  int ring_next_ = 0;
  hipEvent_t ring_ev_[kRing] = {};
  hipEvent_t step_ev_[kMaxRestart] = {};
};

asm_status check_solve_opts(const asm_solve_opts *o) {
  if (o->restart < 1 || o->restart > kMaxRestart || !(o->rtol >= 0.0) || o->max_iters < 1 || o->fixed_iters < 0)
    return fail(ASM_ERR_INVALID, "bad solver option");
  return ASM_OK;
}

int64_t system_bytes(asm_system S) { return (int64_t)(S->mem.bytes + S->ws.mem.bytes); }

// Device bytes of a system's Krylov workspace for restart m.
int64_t workspace_bytes(int64_t N, int m) {
  const int64_t n = 3 * N, ldu = (n + 1) & ~(int64_t)1;
  return 8 * ((m + 1) * ldu + 3 * n + partial_doubles(N) + (kMaxRestart + 2) +
              (m + 1) * m + 2 * (m + 1) + 8) + 4;
}

}  // namespace asmx

using namespace asmx;

// ---------------------------------------------------------------------------
// The request server: queued requests are admitted in arrival order within a
// device-memory budget; the solves of all admitted requests iterate together
// in the batch engine, and new solves join between restart cycles.
// ---------------------------------------------------------------------------
namespace {

struct Plan {  // a cached preconditioner whose pattern-only state is cloned
  asm_grid grid{};
  int32_t nb = 0;
  int64_t nnzb = 0;
  asm_precond_opts popts{};
  // host planning, run on a worker thread while the device keeps iterating
  bool building = false;
  std::shared_ptr<PlanHost> host;
  std::future<std::pair<asm_status, std::string>> job;
  asm_status failed = ASM_OK;  // planning error, reported to the requests of this plan
  std::string err;
  asm_system S = nullptr;
  asm_precond pc = nullptr;
  int64_t bytes = 0;      // device bytes held by the cached system and preconditioner
  int64_t req_bytes = 0;  // device bytes of one request on this plan (0 until known)
  int users = 0;   // running requests on this plan
  int served = 0;  // requests that used it so far
  uint64_t last_use = 0;
};

struct Request {
  asm_request d{};
  int next = 0;  // solve in flight, or the next one
  asm_system S = nullptr;
  asm_precond pc = nullptr;
  int plan = -1;
  int64_t bytes = 0;
  int slot = -1;
  int32_t status = ASM_OK;
  int32_t iters = 0;
  double rel_res = 0.0;
  int32_t hit = 0;
};

bool same_opts(const asm_precond_opts &a, const asm_precond_opts &b) { return std::memcmp(&a, &b, sizeof a) == 0; }

}  // namespace

struct asm_server_s {
  asm_server_opts o{};
  hipStream_t s = nullptr;
  BatchEngine eng;
  std::deque<Request *> queue;
  std::vector<Request *> running;
  std::vector<Request *> ready;  // next solve of a running request, to join the batch
  std::deque<asm_completion> done;
  std::unordered_set<int64_t> live_tags;  // tags queued, running or completed but not yet returned
  std::vector<Plan> plans;
  int64_t bytes_in_use = 0;
  int64_t plan_builds = 0, plan_hits = 0;
  double bytes_per_block = 0.0;  // device bytes of a plan plus one request, per stored block
  uint64_t clock = 0;
  ~asm_server_s() {
    if (s) (void)hipStreamSynchronize(s);
    for (Request *r : queue) delete r;
    for (Request *r : running) {
      if (r->pc) asm_destroy_precond(r->pc);
      if (r->S) asm_destroy_system(r->S);
      delete r;
    }
    for (Plan &p : plans) {
      if (p.pc) asm_destroy_precond(p.pc);
      if (p.S) asm_destroy_system(p.S);
    }
  }
};

namespace {

int64_t plan_bytes(asm_system S, asm_precond pc) {
  int64_t b = system_bytes(S);
  if (pc->smem) b += (int64_t)pc->smem->bytes;
  return b + (int64_t)pc->mem.bytes;
}

// Drops cached plans that no request uses (other than `keep`), least
// recently used first, until `need` more bytes fit the budget.
void evict_for(asm_server srv, int64_t need, int keep) {
  if (srv->o.hbm_budget_bytes <= 0) return;
  while (srv->bytes_in_use + need > srv->o.hbm_budget_bytes) {
    int best = -1;
    for (int i = 0; i < (int)srv->plans.size(); ++i)
      if (i != keep && srv->plans[i].users == 0 && srv->plans[i].pc &&
          (best < 0 || srv->plans[i].last_use < srv->plans[best].last_use))
        best = i;
    if (best < 0) return;
    Plan &p = srv->plans[best];
    asm_destroy_precond(p.pc);
    asm_destroy_system(p.S);
    srv->bytes_in_use -= p.bytes;
    srv->plans.erase(srv->plans.begin() + best);
    for (Request *r : srv->running)
      if (r->plan > best) --r->plan;
    if (keep > best) --keep;
  }
}

int find_plan(asm_server srv, const asm_request &d) {
  for (int i = 0; i < (int)srv->plans.size(); ++i) {
    const Plan &p = srv->plans[i];
    if (p.grid.nx == d.grid.nx && p.grid.ny == d.grid.ny && p.grid.nz == d.grid.nz && p.nb == d.nb &&
        p.nnzb == d.nnzb && same_opts(p.popts, d.precond))
      return i;
  }
  return -1;
}

// Device bytes a queued request is expected to add (0 if nothing is known).
int64_t admission_estimate(asm_server srv, const asm_request &d) {
  const int p = find_plan(srv, d);
  if (p >= 0 && srv->plans[p].req_bytes > 0) return srv->plans[p].req_bytes;
  return (int64_t)(srv->bytes_per_block * (double)d.nnzb);
}

void complete(asm_server srv, Request *r) {
  if (r->slot >= 0) srv->eng.release(r->slot);
  if (r->pc) asm_destroy_precond(r->pc);
  if (r->S) asm_destroy_system(r->S);
  srv->bytes_in_use -= r->bytes;
  if (r->plan >= 0) srv->plans[r->plan].users--;
  asm_completion c{};
  c.tag = r->d.tag;
  c.status = r->status;
  c.solves = r->next;
  c.iters = r->iters;
  c.rel_res_true = r->rel_res;
  c.plan_cached = r->hit;
  srv->done.push_back(c);
  srv->running.erase(std::find(srv->running.begin(), srv->running.end(), r));
  delete r;
}

constexpr int kPlanLookahead = 8;  // queued requests whose plans are built ahead
constexpr int kMaxBuilds = 3;      // host plannings in flight at once

// Starts the host planning of the first queued requests whose grid, pattern
// size and options have no plan yet (on worker threads; the pattern is
// copied to the host and checked here).
void start_builds(asm_server srv) {
  int k = 0, inflight = 0;
  for (const Plan &p : srv->plans) inflight += p.building;
  for (Request *r : srv->queue) {
    if (k++ >= kPlanLookahead || inflight >= kMaxBuilds) break;
    const asm_request &d = r->d;
    if (find_plan(srv, d) >= 0) continue;
    ++inflight;
    Plan np{};
    np.grid = d.grid;
    np.nb = d.nb;
    np.nnzb = d.nnzb;
    np.popts = d.precond;
    np.last_use = ++srv->clock;
    auto pat = std::make_shared<HostPattern>();
    pat->nx = d.grid.nx; pat->ny = d.grid.ny; pat->nz = d.grid.nz; pat->N = d.nb; pat->nnzb = d.nnzb;
    if (d.grid.nx < 1 || d.grid.ny < 1 || d.grid.nz < 1 || (int64_t)d.grid.nx * d.grid.ny * d.grid.nz != d.nb ||
        d.nnzb < d.nb || d.nnzb >= ((int64_t)1 << 31) / 9) {
      np.failed = ASM_ERR_INVALID;
      np.err = "grid or nnzb out of range";
    } else {
      pat->rp.resize(d.nb + 1);
      pat->ci.resize(d.nnzb);
      hipError_t e = hipMemcpy(pat->rp.data(), d.row_ptr_dev, (d.nb + 1) * sizeof(int32_t), hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(pat->ci.data(), d.col_idx_dev, d.nnzb * sizeof(int32_t), hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        np.failed = ASM_ERR_HIP;
        np.err = std::string("pattern copy: ") + hipGetErrorString(e);
      } else if ((np.failed = validate_pattern(*pat)) != ASM_OK ||
                 (np.failed = check_precond_opts(*pat, &d.precond)) != ASM_OK) {
        np.err = g_err;
      }
    }
    if (np.failed == ASM_OK) {
      np.building = true;
      np.host = std::make_shared<PlanHost>();
      auto host = np.host;
      const asm_precond_opts o = d.precond;
      np.job = std::async(std::launch::async, [pat, host, o]() {
        std::string err;
        const asm_status st = build_plan(*pat, o, *host, err);
        return std::make_pair(st, err);
      });
    }
    srv->plans.push_back(std::move(np));
  }
}

// Device part of a plan whose host planning finished: the cached system
// (values of the request that first needed it) and the preconditioner.
asm_status finish_plan(asm_server srv, int p, const asm_request &d) {
  Plan &pl = srv->plans[p];
  auto res = pl.job.get();
  pl.building = false;
  if (res.first != ASM_OK) {
    pl.failed = res.first;
    pl.err = res.second;
    pl.host.reset();
    return ASM_OK;
  }
  asm_status st = asm_create_system(&d.grid, d.nb, d.nnzb, d.row_ptr_dev, d.col_idx_dev, d.vals_dev[0], srv->s, &pl.S);
  if (st == ASM_OK) st = setup_from_plan(pl.S, &d.precond, pl.host, srv->s, &pl.pc);
  pl.host.reset();
  if (st != ASM_OK) {
    if (pl.S) asm_destroy_system(pl.S);
    pl.S = nullptr;
    pl.failed = st;
    pl.err = g_err;
    return ASM_OK;
  }
  pl.bytes = plan_bytes(pl.S, pl.pc);
  srv->bytes_in_use += pl.bytes;
  srv->plan_builds++;
  return ASM_OK;
}

// Creates the request's system and its preconditioner: a clone of the cached
// plan for its grid, options and pattern, the plan being built first if
// there is none.
asm_status materialise(asm_server srv, Request *r) {
  const asm_request &d = r->d;
  asm_status st = asm_create_system(&d.grid, d.nb, d.nnzb, d.row_ptr_dev, d.col_idx_dev, d.vals_dev[0], srv->s, &r->S);
  if (st != ASM_OK) return st;
  int p = find_plan(srv, d);
  if (p >= 0) {
    st = asm_precond_clone(srv->plans[p].pc, r->S, srv->s, &r->pc);
    if (st == ASM_OK) {
      r->hit = srv->plans[p].served > 0;  // the plan's first request built it
      srv->plan_hits += r->hit;
    } else if (st == ASM_ERR_INVALID) {
      p = -1;  // same grid and options but another pattern: no plan to share
    } else {
      return st;
    }
  }
  if (p < 0) {
    Plan np{};
    np.grid = d.grid;
    np.nb = d.nb;
    np.nnzb = d.nnzb;
    np.popts = d.precond;
    st = asm_create_system(&d.grid, d.nb, d.nnzb, d.row_ptr_dev, d.col_idx_dev, d.vals_dev[0], srv->s, &np.S);
    if (st != ASM_OK) return st;
    st = asm_setup_precond(np.S, &d.precond, srv->s, &np.pc);
    if (st != ASM_OK) {
      asm_destroy_system(np.S);
      return st;
    }
    np.bytes = plan_bytes(np.S, np.pc);
    np.last_use = ++srv->clock;
    srv->plans.push_back(std::move(np));
    srv->bytes_in_use += srv->plans.back().bytes;
    srv->plan_builds++;
    p = (int)srv->plans.size() - 1;
    st = asm_precond_clone(srv->plans[p].pc, r->S, srv->s, &r->pc);
    if (st != ASM_OK) return st;
  }
  r->plan = p;
  srv->plans[p].users++;
  srv->plans[p].served++;
  srv->plans[p].last_use = ++srv->clock;
  return ASM_OK;
}

// The solve in a finished slot ended: start the request's next solve (new
// values on the same pattern, refactored) or complete the request.
void solve_ended(asm_server srv, Request *r) {
  const BatchEntry &E = srv->eng.entry(r->slot);
  r->iters += E.info.iters;
  r->rel_res = E.info.rel_res_true;
  const int32_t st = E.status;
  srv->eng.release(r->slot);
  r->slot = -1;
  if (st < 0) {
    r->status = st;
    complete(srv, r);
    return;
  }
  if (st == ASM_NOT_CONVERGED) r->status = ASM_NOT_CONVERGED;
  r->next++;
  if (r->next >= r->d.nsolves) {
    complete(srv, r);
    return;
  }
  asm_status e = asm_update_values(r->S, r->d.vals_dev[r->next], srv->s);
  if (e == ASM_OK) e = asm_refactor(r->pc, srv->s);
  if (e != ASM_OK) {
    r->status = e;
    complete(srv, r);
    return;
  }
  srv->ready.push_back(r);
}

}  // namespace

namespace asmx {
namespace {

// The order of the systems in batched launches (see asm_batch_order_set):
// the process-wide setting, the choices made per size class (device, log2
// of the system count, log2 of the total block rows), and this thread's
// record of its last batched solve.
std::mutex g_order_mu;
int g_order_setting = ASM_BATCH_ORDER_TUNE;
std::map<std::tuple<int, int, int>, asm_batch_tuning> g_order_cache;
thread_local asm_batch_tuning t_last_batch{};

int log2_ceil(int64_t v) {
  int c = 0;
  while (((int64_t)1 << c) < v) ++c;
  return c;
}

// Runs the batch's restart cycles to the end.  Tuning: the first two cycles
// run in each order, timed on the host (each cycle ends in a synchronised
// residual) per block row and step; the faster order, if at least 3%
// faster, is kept for the rest of the batch and for later batches of the
// same size class.
asm_status batch_cycles(BatchEngine &eng, int count, int64_t cells, int device) {
  asm_batch_tuning rec{};
  int setting;
  {
    std::lock_guard<std::mutex> lock(g_order_mu);
    setting = g_order_setting;
  }
  const char *env = std::getenv("ASM_TUNE");
  const bool tune_off = env && env[0] == '0' && env[1] == 0;
  const auto key = std::make_tuple(device, log2_ceil(count), log2_ceil(cells));
  bool timing = false;
  if (setting != ASM_BATCH_ORDER_TUNE) {
    rec.order = setting;
    rec.source = ASM_TUNE_SET;
  } else if (tune_off || count < 2) {
    rec.order = ASM_BATCH_ORDER_SUBMITTED;
    rec.source = ASM_TUNE_DEFAULT;
  } else {
    std::lock_guard<std::mutex> lock(g_order_mu);
    auto it = g_order_cache.find(key);
    if (it != g_order_cache.end()) {
      rec = it->second;
      rec.source = ASM_TUNE_CACHED;
    } else {
      timing = true;
      rec.order = ASM_BATCH_ORDER_SUBMITTED;
      rec.source = ASM_TUNE_DEFAULT;
    }
  }
  int timed = 0;
  while (eng.iterating() > 0) {
    const int order = timing ? timed : rec.order;
    eng.set_largest_first(order == ASM_BATCH_ORDER_LARGEST_FIRST);
    const auto t0 = std::chrono::steady_clock::now();
    asm_status st = eng.cycle();
    if (st != ASM_OK) return st;
    if (!timing) continue;
    const double ns = std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t0).count();
    const double work = eng.last_cycle_work();
    rec.ns_per_row_step[timed] = work > 0.0 ? ns / work : 0.0;
    if (++timed == 2) {
      timing = false;
      rec.order = rec.ns_per_row_step[1] < 0.97 * rec.ns_per_row_step[0] ? ASM_BATCH_ORDER_LARGEST_FIRST
                                                                         : ASM_BATCH_ORDER_SUBMITTED;
      rec.source = ASM_TUNE_TIMED;
      std::lock_guard<std::mutex> lock(g_order_mu);
      g_order_cache[key] = rec;
    }
  }
  t_last_batch = rec;
  return ASM_OK;
}

}  // namespace
}  // namespace asmx

extern "C" {

asm_status asm_solve_batch(int32_t count, const asm_system *systems, const asm_precond *preconds,
                           const double *const *b, double *const *x, const asm_solve_opts *o, hipStream_t s,
                           asm_solve_info *infos, int32_t *status) {
  try {
    TraceRange range_("asm_solve_batch");
    g_err.clear();
    if (count < 1 || !systems || !preconds || !b || !x || !o || !infos || !status)
      return fail(ASM_ERR_INVALID, "NULL argument or empty batch");
    asm_status st = check_solve_opts(o);
    if (st != ASM_OK) return st;
    for (int i = 0; i < count; ++i) {
      if (!systems[i] || !preconds[i] || !b[i] || !x[i]) return fail(ASM_ERR_INVALID, "NULL system, preconditioner or vector");
      if (preconds[i]->sys != systems[i]) return fail(ASM_ERR_INVALID, "preconditioner belongs to another system");
      if (preconds[i]->opts.coarse != ASM_COARSE_NONE || preconds[i]->opts.local != ASM_LOCAL_ILU0)
        return fail(ASM_ERR_INVALID, "coarse corrections and exact local solves are not available in batched solves");
      for (int k = 0; k < i; ++k)
        if (systems[k] == systems[i]) return fail(ASM_ERR_INVALID, "a system appears twice in the batch");
    }
    BatchEngine eng;
    if ((st = eng.init(count, *o, s)) != ASM_OK) return st;
    std::vector<BatchEngine::NewSolve> add(count);
    for (int i = 0; i < count; ++i) add[i] = {systems[i], preconds[i], b[i], x[i], i};
    std::vector<int> slots;
    if ((st = eng.add(add, slots, true)) != ASM_OK) return st;
    for (int i = 0; i < count; ++i)
      if (eng.entry(slots[i]).status == ASM_ERR_NONFINITE)
        return fail(ASM_ERR_NONFINITE, "non-finite b or x0 in batch entry " + std::to_string(i));
    int64_t cells = 0;
    for (int i = 0; i < count; ++i) cells += systems[i]->pat.N;
    if ((st = batch_cycles(eng, count, cells, systems[0]->device)) != ASM_OK) return st;
    ASM_HIP(hipStreamSynchronize(s));
    asm_status result = ASM_OK;
    for (int i = 0; i < count; ++i) {
      const BatchEntry &E = eng.entry(slots[i]);
      infos[i] = E.info;
      status[i] = E.status;
      if (E.status != ASM_OK) result = ASM_NOT_CONVERGED;
    }
    return result;
  }
  ASM_CATCH_ALL
}

asm_status asm_batch_order_set(int32_t order) {
  try {
    g_err.clear();
    if (order != ASM_BATCH_ORDER_TUNE && order != ASM_BATCH_ORDER_SUBMITTED && order != ASM_BATCH_ORDER_LARGEST_FIRST)
      return fail(ASM_ERR_INVALID, "unknown batch order");
    std::lock_guard<std::mutex> lock(g_order_mu);
    g_order_setting = order;
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_batch_tuning_last(asm_batch_tuning *out) {
  try {
    g_err.clear();
    if (!out) return fail(ASM_ERR_INVALID, "NULL argument");
    *out = t_last_batch;
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_server_create(const asm_server_opts *o, hipStream_t stream, asm_server *out) {
  try {
    g_err.clear();
    if (!o || !out) return fail(ASM_ERR_INVALID, "NULL argument");
    *out = nullptr;
    asm_status st = check_solve_opts(&o->solve);
    if (st != ASM_OK) return st;
    if (o->max_active < 1 || o->max_active > ASM_SERVER_MAX_ACTIVE || o->hbm_budget_bytes < 0)
      return fail(ASM_ERR_INVALID, "bad server option");
    std::unique_ptr<asm_server_s> srv(new (std::nothrow) asm_server_s());
    if (!srv) return fail(ASM_ERR_OOM, "host allocation failed");
    srv->o = *o;
    srv->s = stream;
    if ((st = srv->eng.init(o->max_active, o->solve, stream)) != ASM_OK) return st;
    *out = srv.release();
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_server_submit(asm_server srv, const asm_request *req) {
  try {
    g_err.clear();
    if (!srv || !req) return fail(ASM_ERR_INVALID, "NULL argument");
    if (req->nsolves < 1 || req->nsolves > ASM_SERVER_MAX_SOLVES) return fail(ASM_ERR_INVALID, "nsolves out of range");
    if (!req->row_ptr_dev || !req->col_idx_dev) return fail(ASM_ERR_INVALID, "NULL pattern");
    for (int k = 0; k < req->nsolves; ++k)
      if (!req->vals_dev[k] || !req->b_dev[k] || !req->x_dev[k]) return fail(ASM_ERR_INVALID, "NULL values or vector");
    if (req->precond.kind == ASM_KIND_NONE) return fail(ASM_ERR_INVALID, "requests need a Schwarz preconditioner");
    if (req->precond.coarse != ASM_COARSE_NONE || req->precond.local != ASM_LOCAL_ILU0)
      return fail(ASM_ERR_INVALID, "coarse corrections and exact local solves are not available in served solves");
    // a completion names its request by tag: two live requests with one tag
    // could not be told apart (and the caller's buffers of the first would
    // be released with the second's completion)
    if (srv->live_tags.count(req->tag)) return fail(ASM_ERR_INVALID, "tag already in use by a live request");
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return fail(ASM_ERR_OOM, "host allocation failed");
    r->d = *req;
    srv->live_tags.insert(req->tag);
    srv->queue.push_back(r.get());
    r.release();  // owned by the queue from here
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_server_poll(asm_server srv, int32_t max, asm_completion *out, int32_t *ndone) {
  try {
    g_err.clear();
    if (!srv || !ndone || max < 0 || (max > 0 && !out)) return fail(ASM_ERR_INVALID, "NULL argument");
    *ndone = 0;
    asm_status st;
    // 1. admission in arrival order; stop at the first request that does not
    //    fit the budget (unless nothing else holds memory) or the batch
    std::vector<Request *> join;
    join.swap(srv->ready);
    int slots = srv->eng.free_slots() - (int)join.size();
    start_builds(srv);
    while (!srv->queue.empty() && slots > 0) {
      Request *r = srv->queue.front();
      const int p = find_plan(srv, r->d);
      if (p >= 0 && srv->plans[p].building) {
        // the head waits for its plan (no overtaking); with nothing else to
        // run, wait here rather than return empty-handed
        const bool idle = srv->eng.iterating() == 0 && join.empty();
        if (!idle && srv->plans[p].job.wait_for(std::chrono::seconds(0)) != std::future_status::ready) break;
        if ((st = finish_plan(srv, p, r->d)) != ASM_OK) return st;
      }
      if (p >= 0 && srv->plans[p].failed != ASM_OK) {
        srv->queue.pop_front();
        srv->running.push_back(r);
        r->status = srv->plans[p].failed;
        g_err = srv->plans[p].err;
        complete(srv, r);
        srv->plans.erase(srv->plans.begin() + p);
        for (Request *q : srv->running)
          if (q->plan > p) --q->plan;
        continue;
      }
      const int64_t need = admission_estimate(srv, r->d);
      if (srv->o.hbm_budget_bytes > 0 && srv->bytes_in_use + need > srv->o.hbm_budget_bytes) {
        evict_for(srv, need, find_plan(srv, r->d));
        if (srv->bytes_in_use + need > srv->o.hbm_budget_bytes && !srv->running.empty()) break;
      }
      srv->queue.pop_front();
      srv->running.push_back(r);
      st = materialise(srv, r);
      if (st != ASM_OK) {
        r->status = st;
        complete(srv, r);
        continue;
      }
      join.push_back(r);
      --slots;
    }
    // 2. the new solves join the batch (checks, ||b||, initial residuals)
    if (!join.empty()) {
      std::vector<BatchEngine::NewSolve> add;
      for (Request *r : join) add.push_back({r->S, r->pc, r->d.b_dev[r->next], r->d.x_dev[r->next], r->d.tag});
      std::vector<int> sl;
      if ((st = srv->eng.add(add, sl, false)) != ASM_OK) return st;
      for (size_t a = 0; a < join.size(); ++a) {
        Request *r = join[a];
        r->slot = sl[a];
        if (r->bytes == 0) {  // first solve: the system's workspace now exists
          r->bytes = system_bytes(r->S) + (int64_t)r->pc->mem.bytes;
          srv->bytes_in_use += r->bytes;
          Plan &p = srv->plans[r->plan];
          if (p.req_bytes == 0) {
            p.req_bytes = r->bytes;
            const double bpb = (double)(p.bytes + r->bytes) / (double)std::max<int64_t>(p.nnzb, 1);
            srv->bytes_per_block = std::max(srv->bytes_per_block, bpb);
          }
        }
      }
      for (Request *r : join)
        if (!srv->eng.entry(r->slot).iterating) solve_ended(srv, r);
    }
    // 3. one restart cycle of every iterating solve
    if (srv->eng.iterating() > 0) {
      if ((st = srv->eng.cycle()) != ASM_OK) return st;
      std::vector<Request *> ended;
      for (Request *r : srv->running)
        if (r->slot >= 0 && !srv->eng.entry(r->slot).iterating) ended.push_back(r);
      for (Request *r : ended) solve_ended(srv, r);
    }
    ASM_HIP(hipStreamSynchronize(srv->s));
    // 4. completions
    while (*ndone < max && !srv->done.empty()) {
      out[(*ndone)++] = srv->done.front();
      srv->live_tags.erase(srv->done.front().tag);
      srv->done.pop_front();
    }
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

asm_status asm_server_get_state(asm_server srv, asm_server_state *st) {
  try {
    g_err.clear();
    if (!srv || !st) return fail(ASM_ERR_INVALID, "NULL argument");
    std::memset(st, 0, sizeof *st);
    st->queued = (int32_t)srv->queue.size();
    st->running = (int32_t)srv->running.size();
    st->iterating = srv->eng.iterating();
    st->completed_unread = (int32_t)srv->done.size();
    st->cached_plans = (int32_t)srv->plans.size();
    st->bytes_in_use = srv->bytes_in_use;
    st->plan_builds = srv->plan_builds;
    st->plan_hits = srv->plan_hits;
    return ASM_OK;
  }
  ASM_CATCH_ALL
}

void asm_server_destroy(asm_server srv) { delete srv; }

}  // extern "C"
