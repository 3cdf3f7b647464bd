// symbolic.h -- host-side symbolic object (reordering, tile pattern, task
// DAGs, schedules).  Built by analyze.cpp, consumed by capi.cpp.
#pragma once
#include <stdint.h>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stiles.h"
#include "stiles_internal.h"

// Selected-inversion DAG (task words as in stiles_internal.h, ticket order)
struct SelinvPlan {
  std::vector<int32_t> task, succ, list;
  double flops_alg = 0.0;    // sum_j 2 eta_j (eta_j + 1) over the envelope
  double flops_exec = 0.0;   // tile products executed (padded tiles)
};

// Merged factorization + solve DAG (ticket order; solve pairs follow the
// factorization pairs)
struct MergedPlan {
  std::vector<int32_t> task, succ, pairs;
};

struct stiles_symbolic {
  stiles_opts opts;
  int64_t N = 0, n = 0, a = 0;
  int64_t a_in = 0;            // arrow width of the input (before ND adds separators)
  int64_t w_in = 0;            // largest lower half-width of the band rows before ND
  int32_t T = 64;
  int32_t ordering_used = STILES_ORDER_NONE;
  bool profile_input = false;

  std::vector<int64_t> perm;   // permuted row i <- original row perm[i]
  std::vector<int64_t> iperm;  // original row -> permuted row
  std::vector<int64_t> f;      // element profile of P A P^T (first column per row)

  bool perm_identity = true;
  int32_t nd_parts = 1;        // adaptable ND partitions (1: not used)
  int64_t nd_chain = 0;        // ND: estimated chain of the plan, in tile steps
  std::vector<int32_t> band_part;   // ND: partition of each band tile row/column
  std::vector<int64_t> f_pre;  // profile before adaptable ND (flops_alg), empty if unused

  // input value placement
  std::vector<int64_t> in_rp;  // start of each row of the permuted envelope (N+1);
                               // for profile input with the identity also the value layout
  std::vector<int64_t> fin;    // profile input under a permutation: input first columns (N)
  std::vector<int64_t> in_rp_in;// ... and input row pointers (N+1)
  std::vector<int64_t> map;    // CSC input: value index -> element offset in the tile store

  // tile rows
  int32_t ntb = 0, nta = 0, ntr = 0;
  std::vector<int64_t> row_base;  // ntr
  std::vector<int32_t> row_cnt;   // real rows in each tile row (<= T)

  // tile pattern of L: tiles of tile row m are ids [trow_ptr[m], trow_ptr[m+1]),
  // ascending column; the diagonal tile is the last one of its row.
  std::vector<int32_t> trow_ptr;
  std::vector<int32_t> tcol;
  std::vector<int32_t> trow;
  int64_t ntiles = 0;

  // factorization DAG (topologically sorted by the static schedule)
  std::vector<int32_t> ftask;     // TASK_WORDS per task
  std::vector<int32_t> fsucc;
  std::vector<int32_t> fpairs;
  std::vector<float> fest;        // scheduled start estimate (merging batches)
  std::vector<float> fcost;       // cost model of each factorization task (list schedule of a batch)
  int32_t npart = 0;
  int32_t tree_used = 0;
  int64_t corner_acc = 0;
  int64_t ublocks = 0;      // 2 x 2 update blocks in the factorization DAG

  // solve DAG
  int32_t nspart = 0;             // partial slots of long forward rows
  std::vector<int32_t> stask;
  std::vector<int32_t> ssucc;
  std::vector<int32_t> spairs;

  // selected inversion: built on first use (guarded; the object stays
  // logically immutable)
  mutable std::mutex selinv_mu;
  mutable std::unique_ptr<SelinvPlan> selinv;
  mutable std::mutex merged_mu;
  mutable std::unique_ptr<MergedPlan> merged;

  // statistics
  int64_t nnzL = 0;
  int64_t nnzL_alg = 0;   // envelope entries before adaptable ND (the method's nnz(L))
  double flops_alg = 0.0;
  double flops_exec = 0.0;
};

namespace stiles {
// set by every entry point that rejects an argument (thread-local)
void set_error_arg(int32_t idx);
// the selected-inversion plan of a symbolic object (built once, thread-safe)
const SelinvPlan& selinv_plan(const stiles_symbolic& s);
// the merged factorization + solve plan (built once, thread-safe)
const MergedPlan& merged_plan(const stiles_symbolic& s);
// start order of a list schedule of a DAG (successors in CSR form) on
// `workers` workers, longest remaining path (bl) first
std::vector<int32_t> list_schedule(int32_t nt, const float* cost, const int32_t* succ_ptr, const int32_t* succ,
                                   const int32_t* npred, const float* bl, int workers, float hop);
// workgroups of the list schedule for these options (0 = earliest-start order)
int schedule_workers(const stiles_opts& o);
// per stored tile: 1 if an entry of A falls in it (or it is diagonal), 0 if
// it holds fill only (zero in A)
std::vector<int32_t> tiles_with_entries(const stiles_symbolic& s);
}
