// Host-side symbolic setup of the Schwarz preconditioner.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/asm.h"
#include "plan.hpp"

namespace asmx {

struct HostPattern {
  int32_t nx = 0, ny = 0, nz = 0, N = 0;
  int64_t nnzb = 0;
  std::vector<int32_t> rp, ci;
};

// Slots copied from the CSR factors into a step layout: to32[t] bit 0 selects
// the FP32 array; bit 1 the granule layout of short-row sections (stride[t]
// = entries of the section | entry << 16); otherwise component q of slot t
// goes to out[base[t] + q*stride[t]].
struct RelayoutMap {
  std::vector<int32_t> src, base, stride;
  std::vector<uint8_t> to32;
};

// Gather-sum description: dst entry d sums sources idx[ptr[d] .. ptr[d+1]).
struct GatherList {
  std::vector<int32_t> ptr{0}, idx;
  // destinations [0, split) and [split, size) have different fan-ins and
  // are gathered with their own lane counts (-1: one segment)
  int32_t split = -1;
  int32_t size() const { return (int32_t)ptr.size() - 1; }
};

struct PlanHost {
  int32_t nsub = 0;
  int64_t total_ext = 0, total_coarse = 0, total_entries = 0, fine_row_entries = 0;
  int32_t max_levels = 0;
  int64_t sweep_steps = 0;       // forward + backward records
  int64_t lds_spilled_rows = 0;  // rows whose values went through global memory
  int64_t split_rows = 0;        // rows computed in pieces over several sweep steps
  std::vector<SubDesc> sub;
  // factorisation level steps
  std::vector<Step> fstep;
  std::vector<int32_t> frow;
  // sweep records
  std::vector<RecStep> rf, rb;
  std::vector<uint8_t> rec;      // all records, 16-byte aligned
  std::vector<int32_t> fsrc;     // forward position -> cell or -(1+coarse row)
  int64_t total_pos = 0;         // rows in forward (= backward) order
  RelayoutMap rl;                // factor blocks -> record value slots
  std::vector<int32_t> rhs_src;  // per ext row: cell or -(1+coarse row)
  std::vector<int32_t> arp, aci, adiag, tptr, tdst, tsrc;
  // Assembly of A_i values: sources index the pool [A blocks | lumped L2].
  GatherList asm_src;
  // Lumped matrices: L1 (fine atoms) from A blocks; L2 (near/far atoms)
  // from L1 blocks.
  GatherList l1, l2;
  // Lumped right-hand side: atom sums of cells, then near/far atom sums of
  // fine atoms, then coarse rows of near/far atoms.
  GatherList c1, c2, c3;
  // Additive combine: per cell the backward positions holding its value.
  std::vector<int32_t> cptr, cidx;
  // Global coarse grid (when a coarse correction is asked for): coarse
  // variable (box) of each cell, the cells of each box, and the block CSR
  // of A_C = R_C A R_C^T with the A blocks summed into each entry.
  int32_t ncv = 0;
  std::vector<int32_t> cvar;
  GatherList cbox_cells;
  std::vector<int32_t> acp, acc;
  GatherList ac_src;
  // Exact local solves: per extended row its position in the subdomain's
  // forward order; per position its subdomain, owned output cell (or -1)
  // and backward position; per subdomain the offset of its dense matrix.
  std::vector<int32_t> xlpos, xpsub, xout, xbpos;
  std::vector<int64_t> xdoff;
  int32_t xmaxn3 = 0;
  bool any_fp32 = false;
};

// Builds everything that depends only on the sparsity pattern and options.
asm_status build_plan(const HostPattern &A, const asm_precond_opts &o, PlanHost &P, std::string &err);

}  // namespace asmx
