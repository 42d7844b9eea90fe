// Device-side data layout shared by the host setup and the HIP kernels.
//
// A preconditioner is a set of subdomains; subdomain s owns "extended rows"
// ext_off .. ext_off+n-1 (its fine cells, then its coarse rows), stored in a
// global CSR (entries sorted by local column) from which the factors are
// computed, and re-laid out per level step for the triangular solves.
#pragma once
#include <cstddef>
#include <cstdint>

namespace asmx {

// Rows of one factorisation step: one level of the forward schedule (or a
// chunk of it); consecutive steps are separated by a workgroup barrier.
struct Step {
  int32_t pos;    // first position in the step row list
  int32_t nrows;  // rows in the step
};

// Apply-sweep layout: every level step of a sweep is one contiguous record
// in a global buffer, streamed into LDS ahead of its use.
#ifndef ASM_REC_BUFS
#define ASM_REC_BUFS 3
#endif
#ifndef ASM_REC_BYTES
#if ASM_REC_BUFS == 4
#define ASM_REC_BYTES 27584
#else
#define ASM_REC_BYTES 36864
#endif
#endif
constexpr int kRecBufs = ASM_REC_BUFS;    // LDS record buffers of a sweep
constexpr int kRecBytes = ASM_REC_BYTES;  // LDS bytes of one record buffer
static_assert((kRecBufs == 3 || kRecBufs == 4) && kRecBytes % 16 == 0, "three or four buffers of whole 16-byte words");
#ifndef ASM_VEC_SLOTS
// what the record buffers, three source slots and the trash area leave of a
// CU's 160 KiB of LDS
#if ASM_REC_BUFS == 3 && ASM_REC_BYTES == 36864
#define ASM_VEC_SLOTS 2046
#else
#define ASM_VEC_SLOTS 2048
#endif
#endif
constexpr int kVecSlots = ASM_VEC_SLOTS;  // LDS vector slots (3 doubles each)
static_assert(kVecSlots <= 65536, "slots are stored as 16-bit indices");
constexpr int kMaxJdsWidth = 8;    // mode-0 rows have at most this many entries
constexpr int kMaxStepRows = 256;  // rows per step
// The streaming waves copy a record into LDS in chunks of 1 KiB (64 lanes x
// 16 bytes per wave and load); lanes past the record's end still write
// their chunk, so a record's row inputs start at the next chunk boundary.
// A row's input (3 doubles) arrives as two 16-byte loads, doubles (0, 1)
// and (1, 2), so in LDS row j's input takes 32 bytes, component c at
// double 4j + c + (c >> 1); 32 rows per load, the input area is sized in
// whole groups of 32 rows.
constexpr int kRecRowBytes = 8;  // per-row header of a record
constexpr int kRecNoSlot = 0xffff;
constexpr int kRecChunk = 1024;
constexpr int kInRowsPerLoad = 32;
constexpr int kInRowBytes = 32;
constexpr int32_t rec_in_offset(int64_t stored_bytes) {
  return (int32_t)((stored_bytes + kRecChunk - 1) / kRecChunk * kRecChunk);
}
constexpr int32_t rec_in_bytes(int nrows) {
  return (int32_t)(((nrows > 1 ? nrows : 1) + kInRowsPerLoad - 1) / kInRowsPerLoad * kInRowsPerLoad * kInRowBytes);
}
// The streaming loads read whole chunks and whole groups of rows: up to one
// chunk past a record's end, 64 input sources past a step's last position
// and 32 input rows past it.  The arrays they read are padded by that much
// (the sources' padding holds zeros: cell 0, a valid gather).
constexpr int kRecPadBytes = kRecChunk;
constexpr int kSrcPad = 64;
constexpr int kPosPad = kInRowsPerLoad;
// A record's head names the record kHeadAhead steps later in its sweep (the
// last one past the end): the streaming waves read it there and load that
// record's input sources, two steps before they load the record itself
// into the buffer that frees up last.
constexpr int kHeadAhead = kRecBufs + 1;
static_assert(kMaxStepRows * kMaxJdsWidth < 65536, "section entries are packed in 16 bits");

#ifndef ASM_FILL_SLOTS
#define ASM_FILL_SLOTS 256
#endif
constexpr int kFillSlots = ASM_FILL_SLOTS;  // top slots of the pool: values reloaded from global memory

// One step of a sweep.  The record starts with its own descriptor (read
// from LDS once the record has arrived); a compact {rec, len, pos, nrows}
// array per sweep drives the prefetch.  A step holds the rows of one level
// (or part of one), in up to three sections, stored in this order:
//   short FP32 rows [0, n32)      (FP32 factors; fine rows in FP32 mode)
//   short FP64 rows [n32, n32+n64)
//   long rows       [n32+n64, nrows), FP64
// A short row has at most kMaxJdsWidth entries (four lanes per row); a
// long row takes a whole wavefront.  Record sections (byte offsets from the
// record start, each 16-byte aligned):
//   head    RecHead (kRecHead bytes).
//   rows    kRecRowBytes (8) per row: int2 {slot | flags << 16 | count
//           << 18, index}: the LDS slot of the result (0xffff: none);
//           flags bit 0 = store the value to the global vector (always in
//           the forward sweep), bit 1 = the row's input is a cell value of
//           r, to be multiplied by the basis scale (forward fine rows); the
//           row's entry count; index = forward sweep: the row's backward
//           position (where its value goes in the global vector), backward
//           sweep: the output cell or -1 (the row's own position is the
//           step's position plus its index in the step).
//   slots32, slots64  short rows: the LDS slot of each entry's dependency,
//           uint16, in the order of the section's values (entry q = koff[k]
//           + i, below).
//   ldeps   long rows: int per entry, the LDS slot of the dependency.
//   lrptr   long rows: relative entry offsets (nlong+1).
//   vals32, vals64  short rows: jagged diagonals; entry q = koff[k] + i for
//           the k-th entry of the section's row i (rows sorted by entry
//           count, descending).  Granule layout (S = entries of the
//           section, W = values per 16 bytes: 2 doubles or 4 floats):
//           component c < 8 of entry q at [(c/W)*W*S + W*q + c%W], the
//           ninth at [8*S + q], so a block takes five (FP64) or three
//           (FP32) 16-byte-or-smaller reads.
//   lvals   long rows: 9 values per entry.
//   dinv32, dinv64  backward: component e of section row i at
//           [e*rows + i] (dinv64 covers the short FP64 and the long rows).
//   fill    int2 per value {global position, slot}: values of the NEXT step
//           that have no LDS slot of their own, reloaded from the global
//           vector into the fill slots (only in empty "fill" steps).
// The stored record ends there (len 16-byte units); in LDS it is followed,
// from the next 1 KiB boundary (rec_in_offset), by the "in" section, 32
// bytes per row (see kInRowBytes): the rows' inputs, which the streaming waves fetch
// (forward: gathered from r and the coarse rows' lumped inputs through the
// position's source; backward: the forward results at the step's
// positions).  Record, padding and input area (rec_in_bytes) fit one
// buffer of kRecBytes.
// A long row whose record would not fit one LDS buffer is split into
// pieces in consecutive one-row steps that carry the partial sum in LDS.
// A value reloaded by a fill step is produced at least two steps before
// it (the host inserts empty steps where needed).
enum { kPieceWhole = 0, kPieceFirst = 1, kPieceMiddle = 2, kPieceLast = 3 };

struct RecStep {
  int32_t rec;    // record start, in 16-byte units
  int32_t len;    // record length, in 16-byte units
  int32_t pos;    // position of the step's first row (forward / backward order)
  int32_t nrows;
};

struct RecHead {
  int32_t nrows, n32, n64, piece;
  int32_t nslots32, nslots64, pos, in;
  int32_t vals32, vals64, lvals, ldeps;
  int32_t lrptr, dinv32, dinv64, nfill;
  RecStep ahead;                     // the step kHeadAhead later (16-byte aligned)
  int32_t fill, slots32, slots64, pad2;
  int32_t koff32[kMaxJdsWidth + 1];  // first entry of each jagged diagonal
  int32_t koff64[kMaxJdsWidth + 1];
  int32_t pad3[2];
};
constexpr int kRecHead = (int)sizeof(RecHead);
static_assert(kRecHead % 16 == 0, "record head must keep 16-byte alignment");
static_assert(offsetof(RecHead, ahead) % 16 == 0, "the step ahead is read as one 16-byte word");

struct ApplyPlan {
  int32_t nsub;
  const struct SubDesc *sub;
  const RecStep *fstep, *bstep;
  const void *rec;              // all records (16-byte aligned)
  double *rs;                   // 3 doubles per forward position: gathered rhs (dense local solves)
  double *yx;                   // 3 doubles per backward position
  const int32_t *fsrc;          // forward position -> cell (>= 0) or -(1+coarse row)
  const int32_t *cptr3, *cidx3;  // coarse row -> its near/far atom sums (two-level only)
  const double *pnf;             // 3 doubles per near/far atom: lumped residual sums
  double *crs;                   // 3 doubles per coarse row: its lumped input (two-level only)
  int32_t ncoarse;               // coarse rows
};

struct SubDesc {
  int32_t ext_off;         // first extended row (global)
  int32_t n;               // rows of A_i
  int32_t nfine;           // fine rows of A_i
  int32_t fstep0, fstep1;  // factorisation level steps [fstep0, fstep1)
  int32_t rf0, rf1;        // forward sweep records
  int32_t rb0, rb1;        // backward sweep records
  int32_t pad[3];
};

// Pointers handed to the factorisation kernel.
struct DevPlan {
  int32_t nsub;
  const SubDesc *sub;
  const Step *fstep;             // factorisation level steps (pos, nrows)
  const int32_t *frow;           // local row of each step position
  const int32_t *arp;            // per ext row: first CSR entry (global)
  const int32_t *aci;            // per entry: local column
  const int32_t *adiag;          // per ext row: CSR entry of the diagonal
  const int32_t *tptr;           // per entry: first update pair
  const int32_t *tdst, *tsrc;    // update pairs: a[dst] -= L * a[src]
  double *fact;                  // CSR values being factorised
};

}  // namespace asmx
