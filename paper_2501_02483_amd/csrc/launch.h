// launch.h -- host-callable launchers of the device kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stiles_internal.h"

namespace stiles {

// Persistent DAG executor: `total` tickets of factorization, triangular-solve
// (nrhs >= 1 right-hand sides) or selected-inversion tasks.  order == nullptr
// means one matrix (mats[0]) with tasks in their own order, else order[2t],
// order[2t+1] = (matrix index, task id).
// EXEC_FACTOR_SOLVE runs a merged DAG of factorization and solve tasks.
// wait_ticks bounds every wait for predecessors (ticks of the 100 MHz device
// wall clock); past it the launch is abandoned: the skipped tasks' matrices
// get info = 0 (timeout) and every workgroup exits normally.
enum ExecKind { EXEC_FACTOR = 0, EXEC_SOLVE = 1, EXEC_SELINV = 2, EXEC_FACTOR_SOLVE = 3 };
hipError_t launch_exec(int T, int kind, const ExecMat* d_mats, const int32_t* d_order, int32_t total,
                       ExecCtrl* d_ctrl, int nrhs, int nwg, uint64_t wait_ticks, hipStream_t st);

// diagonal of the selected inverse in the original ordering (NaN on failure)
hipError_t launch_selinv_diag(int T, const double* sigma, const int32_t* trow_ptr, const int64_t* row_base,
                              const int32_t* row_cnt, const int64_t* perm, int32_t ntr,
                              const unsigned long long* info, double* out, hipStream_t st);

// values (row-profile order) -> tile store (gather per tile, zero fill, unit
// padding diagonal); also writes `orig` when not null; resets *info.
hipError_t launch_scatter_profile(int T, const double* vals, const int64_t* in_rp, const int64_t* f,
                                  const int32_t* trow, const int32_t* tcol, const int64_t* row_base,
                                  const int32_t* row_cnt, int64_t ntiles, double* tiles, double* orig,
                                  unsigned long long* info, hipStream_t st);

// CSC values -> tile store through an element map (after a zero/unit fill).
hipError_t launch_scatter_map(int T, const double* vals, const int64_t* map, int64_t nnz, const int32_t* trow,
                              const int32_t* tcol, const int32_t* row_cnt, int64_t ntiles, double* tiles,
                              double* orig, unsigned long long* info, hipStream_t st);

// tile store -> row-profile values of the permuted envelope (lower, with diagonal)
hipError_t launch_extract(int T, const double* tiles, const int64_t* rp, const int64_t* f, const int32_t* trow,
                          const int32_t* tcol, const int64_t* row_base, const int32_t* row_cnt, int64_t ntiles,
                          int64_t nnz, double* out, hipStream_t st);

// out-of-core factorization: S = Lc Lc^T of a factor's dense trailing block
// (row-profile storage), and 2 sum log diag over a range of its rows
hipError_t launch_gram_lower(int32_t c, const double* L, const int64_t* rp, const int64_t* f, int64_t r0, int64_t c0,
                             double* S, hipStream_t st);
hipError_t launch_logdet_rows(const double* L, const int64_t* rp, int64_t r0, int64_t r1, double* acc, hipStream_t st);

hipError_t launch_logdet(int T, const double* tiles, const int32_t* trow_ptr, int32_t ntr, double* part,
                         const unsigned long long* info, double* out, hipStream_t st);

// the same with the per-tile-row partials in the library's fixed device
// array (STATIC_LOGDET_ROWS rows): allocates nothing; hipErrorInvalidValue
// when ntr is out of range
hipError_t launch_logdet_static(int T, const double* tiles, const int32_t* trow_ptr, int32_t ntr,
                                const unsigned long long* info, double* out, hipStream_t st);

// row-profile values of the input ordering -> tile store of P A P^T
// (perm: new row -> input row); same conventions as launch_scatter_profile
hipError_t launch_scatter_perm(int T, const double* vals, const int64_t* in_rp, const int64_t* fin, const int64_t* perm,
                               const int32_t* trow, const int32_t* tcol, const int64_t* row_base,
                               const int32_t* row_cnt, int64_t ntiles, double* tiles, double* orig,
                               unsigned long long* info, hipStream_t st);

// every tile of every matrix of a batch (tmap: matrix, tile pairs)
hipError_t launch_scatter_batch(int T, const BatchDesc* desc, const double* const* vals, const int2* tmap,
                                int64_t total_tiles, hipStream_t st);

// log-determinants of every matrix of a batch into out[0..count)
hipError_t launch_logdet_batch(int T, const BatchDesc* desc, int32_t count, const int2* rmap, int64_t total_rows,
                               double* out, hipStream_t st);

// B (original order, column-major, ldb) -> Y (tile rows, T x nrhs blocks)
hipError_t launch_pack(int T, const double* B, int64_t ldb, int nrhs, const int64_t* perm, const int64_t* row_base,
                       const int32_t* row_cnt, int32_t ntr, double* Y, hipStream_t st);
// Z -> B (original order); NaN when the factorization failed
hipError_t launch_unpack(int T, const double* Z, int nrhs, const int64_t* perm, const int64_t* row_base,
                         const int32_t* row_cnt, int32_t ntr, const unsigned long long* info, double* B, int64_t ldb,
                         hipStream_t st);

// Mixed-mode refinement helpers (FP64, pristine tiles of A).
// Residual items: 4 int32 each (tile row m, kind, lo, hi); kind 0 sums
// A_(m,j) X_j over the tiles rtile[lo..hi) of row m (the diagonal tile used
// symmetrically), kind 1 sums A_(i,m)^T X_i over column entries [lo,hi) of
// ccol_*.  Item q writes partial block q; row m owns items
// [item_ptr[m], item_ptr[m+1]).  absmode != 0 replaces A by |A| and X by
// ones (row sums of |A|).  With apart (items x T doubles) and D (ntr x T),
// a residual pass (absmode 0) also writes the row sums of |A| to D, from
// the same reads of A.
hipError_t launch_residual(int T, const double* orig, const int32_t* rtile, const int32_t* tcol,
                           const int32_t* ccol_tile, const int32_t* ccol_row, const int32_t* items, int32_t nitems,
                           const int32_t* item_ptr, int32_t ntr, const double* X, const double* B, double* part,
                           double* R, int nrhs, int absmode, hipStream_t st, double* apart = nullptr,
                           double* D = nullptr);
// stats[2c] = max_i |R_ic|, stats[2c+1] = max_i |X_ic| (bit patterns, atomically maxed)
hipError_t launch_norms(int T, int32_t ntr, int nrhs, const double* R, const double* X, unsigned long long* stats,
                        hipStream_t st);
// X(:, c) += D(:, c) for the right-hand sides c set in mask
hipError_t launch_axpy(int T, int32_t ntr, int nrhs, double* X, const double* D, uint32_t mask, hipStream_t st);
// X(:, c) = P(:, c) for the right-hand sides c set in mask
hipError_t launch_copy_cols(int T, int32_t ntr, int nrhs, double* X, const double* P, uint32_t mask, hipStream_t st);

}  // namespace stiles
