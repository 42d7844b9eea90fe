// Host-only run of the preconditioner planner (test infrastructure).
//
// Builds the block pattern of the 7-point stencil on an nx x ny x nz grid
// (cell c = (ix*ny + iy)*nz + iz, columns sorted, diagonal present), runs
// the library's host planner on it and checks the plan's internal
// consistency: every record and its row inputs fit one LDS record buffer,
// every record section lies inside its record, every factor slot of the
// relayout map lies inside the record buffer, and every index points into
// the array it indexes.  Prints the plan's sizes as one JSON line.  The test
// suite builds this file with AddressSanitizer and UndefinedBehaviorSanitizer,
// so the planner's own memory accesses are checked on the same runs.
//
// Usage: planner_check nx ny nz kind combine sx sy overlap
//                      nearx neary nearz farx fary farz precision field
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <string>

#include "../../paper_1401_7227_amd/csrc/setup.hpp"

using namespace asmx;

static int fails = 0;
#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      if (fails < 20) {                                 \
        std::fprintf(stderr, "check failed: %s: ", #c); \
        std::fprintf(stderr, __VA_ARGS__);              \
        std::fprintf(stderr, "\n");                     \
      }                                                 \
      ++fails;                                          \
    }                                                   \
  } while (0)

static HostPattern stencil(int nx, int ny, int nz) {
  HostPattern A;
  A.nx = nx; A.ny = ny; A.nz = nz; A.N = nx * ny * nz;
  A.rp.push_back(0);
  for (int ix = 0; ix < nx; ++ix)
    for (int iy = 0; iy < ny; ++iy)
      for (int iz = 0; iz < nz; ++iz) {
        const int c = (ix * ny + iy) * nz + iz;
        // sorted: -x, -y, -z, self, +z, +y, +x
        if (ix > 0) A.ci.push_back(c - ny * nz);
        if (iy > 0) A.ci.push_back(c - nz);
        if (iz > 0) A.ci.push_back(c - 1);
        A.ci.push_back(c);
        if (iz + 1 < nz) A.ci.push_back(c + 1);
        if (iy + 1 < ny) A.ci.push_back(c + nz);
        if (ix + 1 < nx) A.ci.push_back(c + ny * nz);
        A.rp.push_back((int32_t)A.ci.size());
      }
  A.nnzb = (int64_t)A.ci.size();
  return A;
}

static void check_steps(const PlanHost &P, const std::vector<RecStep> &steps, const char *which) {
  const int64_t rbytes = (int64_t)P.rec.size();
  for (size_t k = 0; k < steps.size(); ++k) {
    const RecStep &d = steps[k];
    const int64_t b0 = (int64_t)d.rec * 16, len = (int64_t)d.len * 16;
    CHECK(d.rec >= 0 && d.len * 16 >= kRecHead && b0 + len <= rbytes, "%s step %zu: record [%lld, +%lld)", which, k,
          (long long)b0, (long long)len);
    if (!(b0 >= 0 && b0 + len <= rbytes && len >= kRecHead)) continue;
    RecHead h;
    std::memcpy(&h, P.rec.data() + b0, sizeof h);
    CHECK(h.nrows == d.nrows, "%s step %zu: head rows %d, step rows %d", which, k, h.nrows, d.nrows);
    CHECK(d.nrows >= 0 && d.nrows <= kMaxStepRows, "%s step %zu: %d rows", which, k, d.nrows);
    // inputs from the 1 KiB chunk after the record, whole groups of 32 rows
    const int64_t in_off = (len + 1023) / 1024 * 1024;
    const int64_t in = ((d.nrows > 1 ? d.nrows : 1) + 31) / 32 * 32 * 32;

    CHECK(in_off + in <= kRecBytes, "%s step %zu: %lld record bytes + inputs exceed the buffer", which, k,
          (long long)len);
    CHECK(h.in == in_off, "%s step %zu: inputs at %d, record length %lld", which, k, h.in, (long long)len);
    CHECK(h.n32 >= 0 && h.n64 >= 0 && h.n32 + h.n64 <= h.nrows, "%s step %zu: sections", which, k);
    CHECK(d.pos >= 0 && d.pos + d.nrows <= P.total_pos, "%s step %zu: positions", which, k);
    // the streaming loads read whole chunks past the record (the record
    // array's padding), 64 sources and 32 input rows past the step's rows
    // (the padding of the sources and of the work vector)
    CHECK(b0 + len + kRecPadBytes <= rbytes, "%s step %zu: no record padding after it", which, k);
    const int64_t rows = d.nrows > 1 ? d.nrows : 1;
    CHECK(d.pos + (rows + 63) / 64 * 64 <= P.total_pos + kSrcPad, "%s step %zu: source loads", which, k);
    CHECK(d.pos + (rows + 31) / 32 * 32 <= P.total_pos + kPosPad, "%s step %zu: input loads", which, k);
    const int32_t offs[] = {h.slots32, h.slots64, h.vals32, h.vals64, h.lvals, h.ldeps, h.lrptr, h.dinv32, h.dinv64};
    if (h.nrows > 0)
      for (int32_t o : offs) CHECK(o >= kRecHead && o <= len && o % 16 == 0, "%s step %zu: section at %d", which, k, o);
    if (h.nfill > 0) {
      CHECK(h.nrows == 0 && h.fill >= kRecHead && h.fill + 8LL * h.nfill <= len, "%s step %zu: fill list", which, k);
      const int32_t *fl = reinterpret_cast<const int32_t *>(P.rec.data() + b0 + h.fill);
      for (int q = 0; q < h.nfill && q < 4096; ++q) {
        CHECK(fl[2 * q] >= 0 && fl[2 * q] < P.total_pos, "%s step %zu: fill position", which, k);
        CHECK(fl[2 * q + 1] >= kVecSlots - kFillSlots && fl[2 * q + 1] < kVecSlots, "%s step %zu: fill slot", which, k);
      }
    }
    CHECK(h.piece >= kPieceWhole && h.piece <= kPieceLast, "%s step %zu: piece %d", which, k, h.piece);
    if (h.piece != kPieceWhole) CHECK(h.nrows == 1 && h.n32 + h.n64 == 0, "%s step %zu: a piece is one long row", which, k);
    // row headers: slot | flags | count, then backward position (forward
    // sweep) or output cell (backward sweep)
    const bool fwd = which[0] == 'f';
    for (int j = 0; j < h.nrows && kRecHead + (int64_t)kRecRowBytes * (j + 1) <= len; ++j) {
      const int32_t *m = reinterpret_cast<const int32_t *>(P.rec.data() + b0 + kRecHead + (int64_t)kRecRowBytes * j);
      const int slot = m[0] & 0xffff;
      CHECK(slot == kRecNoSlot || slot < kVecSlots - kFillSlots, "%s step %zu row %d: slot %d", which, k, j, slot);
      if (fwd) CHECK(m[1] >= 0 && m[1] < P.total_pos, "%s step %zu row %d: position %d", which, k, j, m[1]);
      else CHECK(m[1] >= -1, "%s step %zu row %d: output cell", which, k, j);
    }
    // short rows' dependency slots: one per entry, inside the record, each
    // a slot of the pool
    if (h.nrows > 0) {
      const int32_t so[2] = {h.slots32, h.slots64}, ns[2] = {h.nslots32, h.nslots64};
      for (int q = 0; q < 2; ++q) {
        CHECK(so[q] + 2LL * ns[q] <= len, "%s step %zu: slot array %d past the record", which, k, q);
        if (so[q] + 2LL * ns[q] > len) continue;
        const uint16_t *sl = reinterpret_cast<const uint16_t *>(P.rec.data() + b0 + so[q]);
        for (int e = 0; e < ns[q]; ++e) CHECK(sl[e] < kVecSlots, "%s step %zu: dependency slot %d", which, k, sl[e]);
      }
    }
  }
}

int main(int argc, char **argv) {
  if (argc != 17) {
    std::fprintf(stderr, "usage: planner_check nx ny nz kind combine sx sy overlap nearx neary nearz farx fary farz "
                         "precision field\n");
    return 2;
  }
  int v[16];
  for (int i = 0; i < 16; ++i) v[i] = std::atoi(argv[i + 1]);
  const HostPattern A = stencil(v[0], v[1], v[2]);
  asm_precond_opts o{};
  o.kind = v[3]; o.combine = v[4]; o.sx = v[5]; o.sy = v[6]; o.overlap = v[7];
  for (int k = 0; k < 3; ++k) { o.near_box[k] = v[8 + k]; o.far_box[k] = v[11 + k]; }
  o.precision = v[14]; o.field = v[15];
  o.coarse = ASM_COARSE_NONE; o.local = ASM_LOCAL_ILU0;
  PlanHost P;
  std::string err;
  const asm_status st = build_plan(A, o, P, err);
  if (st != ASM_OK) {
    std::fprintf(stderr, "build_plan: status %d: %s\n", (int)st, err.c_str());
    return 1;
  }
  CHECK((int)P.sub.size() == P.nsub && P.nsub == o.sx * o.sy, "subdomains %zu", P.sub.size());
  int64_t ext = 0;
  for (int s = 0; s < P.nsub; ++s) {
    const SubDesc &d = P.sub[s];
    CHECK(d.ext_off == ext && d.n >= d.nfine && d.nfine > 0, "sub %d rows", s);
    ext += d.n;
    CHECK(d.rf0 <= d.rf1 && d.rf1 <= (int)P.rf.size() && d.rb0 <= d.rb1 && d.rb1 <= (int)P.rb.size(),
          "sub %d step ranges", s);
    CHECK(d.fstep0 <= d.fstep1 && d.fstep1 <= (int)P.fstep.size(), "sub %d factorisation steps", s);
  }
  CHECK(ext == P.total_ext, "extended rows %lld vs %lld", (long long)ext, (long long)P.total_ext);
  CHECK((int64_t)P.fsrc.size() == P.total_pos + kSrcPad, "forward sources");
  for (int32_t f : P.fsrc) CHECK(f < A.N && -f - 1 < P.total_coarse, "forward source %d", f);
  for (int q = 0; q < kSrcPad; ++q) CHECK(P.fsrc[P.total_pos + q] == 0, "source padding %d", q);
  CHECK((int64_t)P.arp.size() == P.total_ext + 1 && P.arp.back() == P.total_entries, "factor CSR");
  check_steps(P, P.rf, "forward");
  check_steps(P, P.rb, "backward");
  // each head names the step kHeadAhead later in its subdomain's sweep (or the last)
  for (int s = 0; s < P.nsub; ++s)
    for (int sweep = 0; sweep < 2; ++sweep) {
      const std::vector<RecStep> &st = sweep ? P.rb : P.rf;
      const int a = sweep ? P.sub[s].rb0 : P.sub[s].rf0, b = sweep ? P.sub[s].rb1 : P.sub[s].rf1;
      for (int k = a; k < b; ++k) {
        RecHead h;
        std::memcpy(&h, P.rec.data() + (int64_t)st[k].rec * 16, sizeof h);
        const RecStep &ah = st[std::min(k + kHeadAhead, b - 1)];
        CHECK(h.ahead.rec == ah.rec && h.ahead.len == ah.len && h.ahead.pos == ah.pos && h.ahead.nrows == ah.nrows,
              "sub %d sweep %d step %d: step ahead", s, sweep, k - a);
      }
    }
  // factor slots of the record buffer
  const int64_t rbytes = (int64_t)P.rec.size();
  for (size_t t = 0; t < P.rl.src.size(); ++t) {
    const bool f32 = P.rl.to32[t] & 1, gran = P.rl.to32[t] & 2;
    const int64_t sz = f32 ? 4 : 8, b0 = P.rl.base[t];
    int64_t hi;
    if (gran) {
      const int64_t S = P.rl.stride[t] & 0xffff, q = (int64_t)((uint32_t)P.rl.stride[t] >> 16);
      CHECK(q < S, "slot %zu: entry %lld of %lld", t, (long long)q, (long long)S);
      hi = b0 + 8 * S + q;
    } else {
      hi = b0 + 8LL * P.rl.stride[t];
    }
    CHECK(P.rl.src[t] >= 0 && P.rl.src[t] < P.total_entries, "slot %zu: source %d", t, P.rl.src[t]);
    CHECK(b0 >= 0 && (hi + 1) * sz <= rbytes, "slot %zu: [%lld, %lld] of %lld bytes", t, (long long)(b0 * sz),
          (long long)(hi * sz), (long long)rbytes);
  }
  std::printf("{\"nsub\": %d, \"ext_rows\": %lld, \"coarse_rows\": %lld, \"factor_blocks\": %lld, "
              "\"max_levels\": %d, \"sweep_steps\": %lld, \"reloaded_rows\": %lld, \"split_rows\": %lld, "
              "\"record_bytes\": %lld, \"fails\": %d}\n",
              P.nsub, (long long)P.total_ext, (long long)P.total_coarse, (long long)P.total_entries, P.max_levels,
              (long long)(P.rf.size() + P.rb.size()), (long long)P.lds_spilled_rows, (long long)P.split_rows,
              (long long)P.rec.size(), fails);
  return fails ? 1 : 0;
}
