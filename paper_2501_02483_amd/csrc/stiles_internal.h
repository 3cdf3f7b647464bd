// stiles_internal.h -- layouts shared by the host planner (analyze.cpp,
// capi.cpp) and the device kernels (kernels.hip).  Not part of the public ABI.
//
// Tile store (CTSF, Section III-B): the permuted matrix is cut into T x T
// tiles.  Band tile row m covers permuted rows [m*T, m*T+T) of the band part;
// arrow tile row m >= ntb covers rows [n + (m-ntb)*T, ...) of the arrow (the
// arrow keeps tile rows of its own).  Rows beyond the matrix are padding with
// a unit diagonal.  Only tiles of the (tile-level) filled pattern of L are
// stored, row by row, each T x T column-major; tile id t lives at t*T*T.
//
// Work is a DAG of tile tasks executed by a persistent kernel: workgroups take
// tickets in a precomputed topological order and wait on per-task counters of
// unfinished predecessors (the static schedule and progress table of
// Algorithm 2, with counters instead of flags).
#pragma once
#include <stdint.h>

namespace stiles {

enum TaskType : int32_t {
  TK_UPD = 1,    // C_t -= sum over pairs (X_p Y_p^T)            [Alg. 1 SYRK/GEMM]
  TK_PART = 2,   // P_s  = sum over pairs (X_p Y_p^T)            [Alg. 3 partial T[ID]]
  TK_TREE = 3,   // P_o = P_a + P_b, or C_t -= P_a (+ P_b)       [Alg. 3 GEADD tree]
  TK_POTRF = 4,  // [C_kk -= X X^T]; L_kk = chol(C_kk); Linv_k   [Alg. 1 SYRK, POTRF]
  TK_TRSM = 5,   // [C_t -= X Y^T]; L_t = C_t Linv_k^T           [Alg. 1 GEMM, TRSM]
  TK_UPDB = 6,   // 2 x 2 block: C_(r,c) -= sum_j L_(r,j) L_(c,j)^T  [Alg. 1 SYRK/GEMM]
  TK_FUPD = 8,   // solve, forward:  Y_m -= sum L_(m,j) Y_j
  TK_FDIAG = 9,  // solve, forward:  Y_m  = Linv_m (Y_m - [L_(m,j) Y_j])
  TK_BUPD = 10,  // solve, backward: Z_m  = (first ? Y_m : Z_m) - sum L_(i,m)^T Z_i
  TK_BDIAG = 11, // solve, backward: Z_m  = Linv_m^T ((Z_m or Y_m) - [L_(i,m)^T Z_i])
  TK_FPART = 12, // solve, forward:  Q_s  = sum L_(m,j) Y_j  (one chunk of a long row)
  TK_FSUM = 13,  // solve, forward:  Y_m -= Q_a + Q_(a+1) + ... + Q_(b-1)
  // selected inversion (Sigma = A^{-1} on the tile pattern of L), by tile
  // columns k in reverse order; S(k) = tile rows below k in column k,
  // p = min S(k) (the parent of k in the tile elimination tree)
  TK_SWE = 16,   // W_(r,k) [+]= sum_s Sig~_(r,s) L_(s,k), s in S(k) \ {p}  (r != p)
  TK_SW = 17,    // Sig_(r,k) = -(W + products + pushed partials) Linv_k; D, pushes
  TK_SDIAG = 18, // Sig_kk = Linv_k^T (Linv_k - sum_r D_(r,k))
  TK_TSUM = 19,  // a per-tile partial slot = sum of listed slots (off the chain)
};

enum TaskFlag : int32_t {
  TF_DIAG = 1 << 8,   // UPD target is a diagonal tile (lower half only)
  TF_FIRST = 1 << 9,  // BUPD: first chunk reads Y_m; BDIAG: no BUPD, reads Y_m
  TF_ACC = 1 << 10,   // PART: P_s += sum (continues a chain) instead of P_s = sum
  TF_SPLIT = 1 << 11, // POTRF/TRSM/FDIAG/BDIAG: two-stage wait (early predecessors, then the chain one)
  TF_ARROW = 1 << 12, // PART: partial of an arrow-corner tile (FP64 in mixed mode)
};

// One task = 8 int32.
//  w0 type | flags     w1 tile (target tile id / tile row / -1)
//  w2 a                w3 b              w4 c
//  w5 succ_lo          w6 succ_hi        w7 ndeps
// UPD:  a,b = pair range          PART: a,b = pair range, c = out slot
// UPDB: a = first pair of its list, b = column count nj; list (int32 words):
//       the targets (ra,k), (rb,k), (ra,k+1), (rb,k+1) (-1: absent), then per
//       column j the operand tiles (ra,j), (rb,j), (k,j), (k+1,j); TF_DIAG:
//       the diagonal block (ra, rb) = (k, k+1), whose (ra,j) = (k,j)
// TREE: a = slot, b = slot or -1, c = out slot or -1 (then subtract into tile)
// POTRF: a = tile row k, b,c = fused pair range (C_kk -= X X^T first, 0 or 1 pair)
// TRSM:  a = tile row k of the diagonal tile, b,c = fused pair range
// FUPD/BUPD: w1 = tile row m, a,b = solve-pair range
// FDIAG/BDIAG: w1 = m, a,b = fused solve-pair range applied before the diagonal
// FPART: w1 = m, a,b = solve-pair range, c = partial slot
// FSUM:  w1 = m, a,b = partial slot range (summed in index order)
// SWE:   w1 = target tile, a = offset of its pairs in the list array, b = pair
//        count; TF_ACC adds to the target (a later chunk).  A pair is
//        (Sigma tile | SIG_TRANS if used transposed, L tile).
// SW:    w1 = target tile (r,k), a = k, b = list offset, c = nsum | npush << 8
//        | nprod << 16; list: nprod (1 or 2) pairs as in SWE, nsum pushed-
//        partial slots, npush L tiles (at most 64 words); TF_ACC: the target
//        holds an early sum W to add.
// SDIAG: w1 = diagonal tile of k, a = k, b = list offset, c = count of D slots
// TSUM:  w1 = output slot, a = list offset, b = count, c = 0: D slots (dpart),
//        1: pushed-partial slots (qpart); summed in list order
constexpr int TASK_WORDS = 8;
constexpr int32_t SIG_TRANS = 1 << 30;
// Two-stage waits.  A task's counter can hold some predecessors with weight
// MERGED_FDEP ("early" ones) and the others with weight 1; a successor entry
// with SUCC_FDEP set subtracts MERGED_FDEP.  Once the counter falls below
// MERGED_FDEP every early predecessor has finished, and the task can stage
// what those produced while the others are still running.
// Merged factorization + solve DAG: the early predecessors of a solve task
// are its factorization predecessors (its factor tiles are then final).
// Factorization DAG (TF_SPLIT): a TRSM's early predecessors are the update
// chain of its tile and the tasks that finalize its fused operands, its
// late one the POTRF of its column, so it prefetches its tile and does its
// fused product before the POTRF ends; a POTRF with a fused product waits
// late for the TRSM of that operand (the panel of the previous column) and
// prefetches its tile before.
// Solve DAG (TF_SPLIT): a diagonal step with two fused products waits late
// for the step that solves the block of its second product (the previous
// step of the chain) and does the product with the other one before.  In
// the merged DAG its early solve predecessors weigh SPLIT_W (their successor
// entries carry SUCC_MID) below the factorization predecessors' MERGED_FDEP.
constexpr int32_t MERGED_FDEP = 1 << 16;
constexpr int32_t SUCC_FDEP = 1 << 30;
constexpr int32_t SPLIT_W = 1 << 8;
constexpr int32_t SUCC_MID = 1 << 29;
// Tile rows the library's fixed log-determinant array holds (one FP64
// partial per tile row, 512 KiB); the public limit of stiles_logdet_static.
constexpr int32_t STATIC_LOGDET_ROWS = 65536;

// Device-side description of one matrix (or one solve) for the executor.
struct ExecMat {
  double* tiles;            // ntiles * T*T
  double* linv;             // ntr * T*T   inverse diagonal tiles
  float* shadow;            // ntiles * T*T FP32 copies of L tiles (mixed) or null
  double* part;             // npart * T*T  tree partials
  double* vy;               // solve: ntr * T * nrhs (forward result)
  double* vz;               // solve: ntr * T * nrhs (backward result)
  double* vpart;            // solve: partial slots, T * nrhs each
  double* sigma;            // selected inversion: ntiles * T*T (the pattern of L)
  double* dpart;            // selected inversion: D_(r,k) = L_(r,k)^T Sig_(r,k), per tile
  double* qpart;            // selected inversion: pushed partials Sig_(s,p)^T L_(s,k), per tile
  const int32_t* tasks;     // ntasks * TASK_WORDS
  const int32_t* succ;      // successor lists
  int32_t* remaining;       // per-task unfinished-predecessor counters
  const int32_t* pairs;     // 2 ints per pair
  unsigned long long* info; // first failing permuted column + 1, ~0ull if none
  const int64_t* row_base;  // ntr: first permuted row of each tile row
  unsigned long long* trace;// per task {claim, start, end, wg<<32|type<<24|ticket} or null
  int32_t ntasks;
  int32_t ntr;
  int32_t mixed;
  int32_t pad;
};

// Per-matrix tables for the batched scatter and log-determinant launches
// (one launch over every matrix of a batch instead of one per matrix).
struct BatchDesc {
  const int64_t* in_rp;     // row pointers of the row-profile input
  const int64_t* f;         // first column of each row
  const int64_t* perm;      // new row -> input row, or null (natural order: in_rp/f are those of P A P^T)
  const int32_t* trow;      // tile row of each stored tile
  const int32_t* tcol;      // tile column of each stored tile
  const int32_t* trow_ptr;  // first stored tile of each tile row
  const int64_t* row_base;
  const int32_t* row_cnt;
  double* tiles;
  double* orig;             // mixed mode: copy of the scattered values, else null
  double* ldpart;           // per tile row partial sums of log L_ii
  unsigned long long* info;
  int32_t ntiles;
  int32_t ntr;
};

// Launch control block (one per concurrent launch).  `abort` is set by the
// first workgroup whose wait for its predecessors passes the launch's
// deadline; every later wait of the launch then gives up at once, so all
// workgroups skip their remaining tasks and exit.  The last workgroup to
// leave re-arms the block (and, after an abort, every progress counter).
// `abort` sits on a cache line of its own, away from the ticket counter.
struct ExecCtrl {
  int32_t ticket;
  int32_t exited;
  int32_t pad0[30];
  int32_t abort;
  int32_t pad1[31];
};
static_assert(sizeof(ExecCtrl) == 256, "ExecCtrl spans two 128-byte cache lines");

}  // namespace stiles
