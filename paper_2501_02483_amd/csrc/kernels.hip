// kernels.hip -- gfx950 (CDNA4) device code of the sparse tile Cholesky.
//
// One persistent kernel executes every tile task of the factorization
// (Algorithm 1: SYRK/GEMM updates, POTRF, TRSM; Algorithm 3: partial
// accumulations and the GEADD tree) and of the triangular solves.  Workgroups
// of 256 threads (4 wave64) take tickets in the static order computed on the
// host and wait on a per-task counter of unfinished predecessors, the
// counterpart of the paper's progress table (Algorithm 2).
//
// Tile products use the FP64 matrix cores (v_mfma_f64_16x16x4f64) or, in the
// mixed mode, the FP32 ones (v_mfma_f32_16x16x4f32) on FP32 copies of the
// factor tiles.  Each wave owns a (T/2) x (T/2) quarter of the output tile.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "launch.h"
#include "stiles_internal.h"

namespace stiles {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int NT = 256;

// Global-memory accesses go through address-space-1 pointers, so that they
// are global (not flat) instructions: they then count only in vmcnt, and a
// wait for LDS data (lgkmcnt) never waits for a tile prefetch in flight.
#define GLOBAL __attribute__((address_space(1)))
template <typename E>
__device__ __forceinline__ GLOBAL E* gp(E* p) { return (GLOBAL E*)p; }
template <typename E>
__device__ __forceinline__ const GLOBAL E* gp(const E* p) { return (const GLOBAL E*)p; }

// The pair (or slot) words of a task, read once: lane l of every wave holds
// word l (at most 64 words); word i is then taken with readlane into a scalar
// register, so the loop over the pairs issues no dependent metadata loads.
__device__ __forceinline__ int load_words(const int32_t* w, int n) {
  const int l = threadIdx.x & 63;
  return l < n ? gp(w)[l] : 0;
}
__device__ __forceinline__ int word(int v, int i) { return __builtin_amdgcn_readlane(v, i); }

// Stores of task results are device-scope (sc1) stores: they are written
// through to the point of coherence of all XCDs, so once they have completed
// (s_waitcnt) they are visible to a task on any XCD that acquires after it.
// A task's release then needs no L2 write-back (buffer_wbl2), which costs
// about as much as several tile products.  Every global store of the task
// bodies must go through these.
__device__ __forceinline__ void st_dev(GLOBAL double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(GLOBAL float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) { st_dev(gp(p), v); }

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int ld_relaxed(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// 1/sqrt(d): hardware estimate, then one third-order correction
// y = y0 (1 + e/2 + 3 e^2 / 8), e = 1 - d y0^2 (four dependent FP64 steps
// instead of six for two Newton steps; the estimate's error is cubed)
__device__ __forceinline__ double rsqrt_c(double d) {
  const double y0 = __builtin_amdgcn_rsq(d);
  const double e = fma(-d * y0, y0, 1.0);
  const double p = fma(0.375, e, 0.5);
  return fma(y0 * e, p, y0);
}

// ------------------------------------------------------- tile products (MFMA)
// acc[i][j] covers C rows r0 + 16 j + (lane & 15) and C columns
// c0 + 16 i + (lane >> 4) + 4 r (FP64 MFMA output layout on gfx950: lane l,
// register r holds D[(l >> 4) + 4 r][l & 15]).  The A operand is taken from
// Y (C columns), the B operand from X (C rows), so that the 16 lanes of one
// row group touch 16 consecutive rows of a column-major tile.  Operands are
// read from LDS, where a whole tile pair has been staged.

template <int T>
__device__ __forceinline__ void mma_f64(v4d (&acc)[T / 32][T / 32], const double* X, const double* Y, int r0, int c0,
                                        int lane) {
  constexpr int NB = T / 32;
  const double* xp = X + r0 + (lane & 15) + (lane >> 4) * T;
  const double* yp = Y + c0 + (lane & 15) + (lane >> 4) * T;
  // the operands of step k + 4 are read from LDS while step k's MFMAs run
  double a[NB], b[NB];
#pragma unroll
  for (int q = 0; q < NB; q++) {
    a[q] = yp[q * 16];
    b[q] = xp[q * 16];
  }
#pragma unroll
  for (int k = 0; k < T; k += 4) {
    double an[NB], bn[NB];
    if (k + 4 < T) {
#pragma unroll
      for (int q = 0; q < NB; q++) {
        an[q] = yp[q * 16 + (k + 4) * T];
        bn[q] = xp[q * 16 + (k + 4) * T];
      }
    }
    // keep the next step's LDS reads ahead of this step's MFMAs
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    if (k + 4 < T) {
#pragma unroll
      for (int q = 0; q < NB; q++) {
        a[q] = an[q];
        b[q] = bn[q];
      }
    }
  }
}

// FP32 variant (mixed mode); FP32 MFMA output layout: lane l, register r holds
// D[4 (l >> 4) + r][l & 15], so acc[i][j][r] covers column c0 + 16 i + 4 (lane >> 4) + r.
template <int T>
__device__ __forceinline__ void mma_f32(v4f (&acc)[T / 32][T / 32], const float* X, const float* Y, int r0, int c0,
                                        int lane) {
  constexpr int NB = T / 32;
  const float* xp = X + r0 + (lane & 15) + (lane >> 4) * T;
  const float* yp = Y + c0 + (lane & 15) + (lane >> 4) * T;
  // the operands of step k + 4 are read from LDS while step k's MFMAs run
  float a[NB], b[NB];
#pragma unroll
  for (int q = 0; q < NB; q++) {
    a[q] = yp[q * 16];
    b[q] = xp[q * 16];
  }
#pragma unroll
  for (int k = 0; k < T; k += 4) {
    float an[NB], bn[NB];
    if (k + 4 < T) {
#pragma unroll
      for (int q = 0; q < NB; q++) {
        an[q] = yp[q * 16 + (k + 4) * T];
        bn[q] = xp[q * 16 + (k + 4) * T];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    if (k + 4 < T) {
#pragma unroll
      for (int q = 0; q < NB; q++) {
        a[q] = an[q];
        b[q] = bn[q];
      }
    }
  }
}

// Whole-tile staging through registers: every thread moves its share of a
// T x T tile with 16-byte loads, so a tile arrives after one memory latency
// and the next pair can be in flight while the current one is multiplied.
template <int T, typename E>
struct TileStage {
  typedef E vec __attribute__((ext_vector_type(16 / sizeof(E))));
  static constexpr int EPV = 16 / sizeof(E);
  static constexpr int NV = T * T / NT / EPV;
  vec r[NV];
  __device__ __forceinline__ void load(const E* __restrict__ g) {
    const GLOBAL vec* v = (const GLOBAL vec*)g;
#pragma unroll
    for (int q = 0; q < NV; q++) r[q] = v[threadIdx.x + q * NT];
  }
  __device__ __forceinline__ void store(E* l) const {
    vec* v = reinterpret_cast<vec*>(l);
#pragma unroll
    for (int q = 0; q < NV; q++) v[threadIdx.x + q * NT] = r[q];
  }
};

// ------------------------------------------------------------ task bodies

// The calling workgroup waits until *cnt < bound (all predecessors, or all
// predecessors of one kind, have finished), then acquires.  Wave 0 polls.
// The wait is bounded: it gives up when another workgroup of the launch has
// given up (ctrl->abort) or when `limit` ticks of the 100 MHz wall clock pass
// without the counter falling; the first to give up sets ctrl->abort.  The
// result is the same for every thread (false: gave up).  The outcome goes
// through LDS; the second barrier keeps a later wait from overwriting it
// before every wave has read it.
__device__ __forceinline__ bool wait_below(int32_t* cnt, int32_t bound, ExecCtrl* ctrl, uint64_t limit) {
  __shared__ int32_t s_ok;
  if (threadIdx.x < 64) {
    int32_t ok = 1;
    if (__builtin_amdgcn_readfirstlane(ld_relaxed(cnt)) >= bound) {
      const uint64_t t0 = wall_clock64();
      for (;;) {
        __builtin_amdgcn_s_sleep(1);
        if (__builtin_amdgcn_readfirstlane(ld_relaxed(cnt)) < bound) break;
        if (__builtin_amdgcn_readfirstlane(ld_relaxed(&ctrl->abort)) != 0) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > limit) {
          st_relaxed(&ctrl->abort, 1);
          ok = 0;
          break;
        }
      }
    }
    fence_acquire();
    if (threadIdx.x == 0) s_ok = ok;
  }
  __syncthreads();
  const bool ok = __builtin_amdgcn_readfirstlane(s_ok) != 0;
  __syncthreads();
  return ok;
}


// UPD / PART: acc = sum_p X_p Y_p^T over a list of tile pairs (at most 32).
// mode 0: C_t -= acc (UPD), mode 1: P = acc (PART).  LX, LY: LDS tiles.
template <int T, int K>
__device__ __attribute__((noinline)) void task_update(const ExecMat& M, const int32_t* w, int mode, double* LX, double* LY) {
  constexpr int TT = T * T, W = T / 2, NB = T / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int r0 = wr * W, c0 = wc * W;
  const bool diag = (w[0] & TF_DIAG) != 0;
  const bool active = !(diag && wc > wr);   // strictly upper quarter of a diagonal tile
  const int p0 = __builtin_amdgcn_readfirstlane(w[2]), np = __builtin_amdgcn_readfirstlane(w[3]) - p0;
  // FP32 products in mixed mode: the updates, and the partials of corner
  // tiles other than the arrow corner (separator rows under adaptable ND);
  // the arrow corner's partials too in the all-FP32 variant (mixed == 2)
  const bool mixed = M.mixed && (mode == 0 || M.mixed == 2 || (w[0] & TF_ARROW) == 0);
  const bool accum = mode == 1 && (w[0] & TF_ACC) != 0;   // partial chain: P += sum
  GLOBAL double* out = gp(mode == 0 ? M.tiles + (int64_t)w[1] * TT : M.part + (int64_t)w[4] * TT);
  const int pv = load_words(M.pairs + 2 * p0, 2 * np);
  // the target's current value is needed only at the end: fetch it now
  double cin[NB][NB][4];
  if ((mode == 0 || accum) && active) {
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = r0 + 16 * j + (lane & 15);
          const int col = c0 + 16 * i + (mixed ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r);
          cin[i][j][r] = out[row + col * T];
        }
  }
  if (!mixed) {
    const double* tiles = M.tiles;
    v4d acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    TileStage<T, double> sx, sy;
    sx.load(tiles + (int64_t)word(pv, 0) * TT);
    sy.load(tiles + (int64_t)word(pv, 1) * TT);
    for (int p = 0; p < np; p++) {
      __syncthreads();
      sx.store(LX);
      sy.store(LY);
      __syncthreads();
      if (p + 1 < np) {
        sx.load(tiles + (int64_t)word(pv, 2 * p + 2) * TT);
        sy.load(tiles + (int64_t)word(pv, 2 * p + 3) * TT);
      }
      if (active) mma_f64<T>(acc, LX, LY, r0, c0, lane);
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
            if (mode == 0) {
              if (!diag || row >= col) st_dev(out + row + col * T, cin[i][j][r] - acc[i][j][r]);
            } else {
              st_dev(out + row + col * T, accum ? cin[i][j][r] + acc[i][j][r] : acc[i][j][r]);
            }
          }
    } else if (mode == 1) {   // keep the partial fully defined
#pragma unroll
      for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
            st_dev(out + row + col * T, 0.0);
          }
    }
  } else {
    const float* shadow = M.shadow;
    float* FX = reinterpret_cast<float*>(LX);
    float* FY = reinterpret_cast<float*>(LY);
    v4f acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    TileStage<T, float> sx, sy;
    sx.load(shadow + (int64_t)word(pv, 0) * TT);
    sy.load(shadow + (int64_t)word(pv, 1) * TT);
    for (int p = 0; p < np; p++) {
      __syncthreads();
      sx.store(FX);
      sy.store(FY);
      __syncthreads();
      if (p + 1 < np) {
        sx.load(shadow + (int64_t)word(pv, 2 * p + 2) * TT);
        sy.load(shadow + (int64_t)word(pv, 2 * p + 3) * TT);
      }
      if (active) mma_f32<T>(acc, FX, FY, r0, c0, lane);
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + 4 * (lane >> 4) + r;
            if (mode == 0) {
              if (!diag || row >= col) st_dev(out + row + col * T, cin[i][j][r] - (double)acc[i][j][r]);
            } else {
              st_dev(out + row + col * T, accum ? cin[i][j][r] + (double)acc[i][j][r] : (double)acc[i][j][r]);
            }
          }
    }
  }
}

// UPDB: a 2 x 2 block of update targets C_(r,c) -= sum_j L_(r,j) L_(c,j)^T,
// r in {ra, rb}, c in {k, k+1}, over a list of columns j.  Wave q owns
// target q: rows from operand X_(q & 1) = L_(ra|rb, j), columns from
// Y_(q >> 1) = L_(k|k+1, j), a whole T x T tile in its registers, so each
// operand tile is read once from memory for two products.  Per column j
// the four operand tiles go through LDS in two halves of T/2 k-columns
// (X halves in LX, Y halves in LY; a half of a column-major tile is
// contiguous); the next half is in flight in registers while the current
// one is multiplied.  The diagonal block (TF_DIAG: ra = k, rb = k+1) reads
// X_a = Y_k and X_b = Y_(k+1), stages only the Y halves, and its two
// diagonal targets compute their lower 16 x 16 blocks only.  E = double on
// the FP64 factor tiles, float on the FP32 copies in mixed mode (the
// product is then subtracted from the FP64 tile).
template <int T, typename E>
struct BlockOps;
template <int T>
struct BlockOps<T, double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ __forceinline__ const double* src(const ExecMat& M) { return M.tiles; }
};
template <int T>
struct BlockOps<T, float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ const float* src(const ExecMat& M) { return M.shadow; }
};

template <int T, typename E>
__device__ __forceinline__ void update_block(const ExecMat& M, const int32_t* w, double* LXd, double* LYd) {
  typedef BlockOps<T, E> O;
  typedef typename O::acc_t acc_t;
  typedef E vec __attribute__((ext_vector_type(16 / sizeof(E))));
  constexpr int TT = T * T, H = T / 2, HE = T * H, NB = T / 16;
  constexpr int EPV = 16 / sizeof(E), NV = HE / NT / EPV;   // vectors per thread per half tile
  E* LX = reinterpret_cast<E*>(LXd);
  E* LY = reinterpret_cast<E*>(LYd);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool dg = (__builtin_amdgcn_readfirstlane(w[0]) & TF_DIAG) != 0;
  const int p0 = __builtin_amdgcn_readfirstlane(w[2]), nj = __builtin_amdgcn_readfirstlane(w[3]);
  const int pv = load_words(M.pairs + 2 * p0, 4 + 4 * nj);
  const int tgt = word(pv, wave);
  const bool active = tgt >= 0;
  const bool tdiag = dg && wave != 1;
  const int xs = wave & 1, ys = wave >> 1;
  const E* tiles = O::src(M);
  // staged halves: the Y tiles (k, j), (k+1, j), then (non-diagonal block)
  // the X tiles (ra, j), (rb, j)
  const int nst = dg ? 2 : 4;
  vec st[4][NV];
  // an operand tile id of -1 (absent) is neither loaded nor used: the waves
  // whose X or Y it is skip that column
  auto stage_load = [&](int step) {
    const int j = step >> 1, h = step & 1;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      // slot order in the list: xa, xb, yk, yk1
      const int id = q < nst ? word(pv, 4 + 4 * j + (q < 2 ? 2 + q : q - 2)) : -1;
      if (id >= 0) {
        const GLOBAL vec* g = (const GLOBAL vec*)(tiles + (int64_t)id * TT + h * HE);
#pragma unroll
        for (int v = 0; v < NV; v++) st[q][v] = g[threadIdx.x + v * NT];
      }
    }
  };
  auto stage_store = [&](int step) {
    const int j = step >> 1;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int id = q < nst ? word(pv, 4 + 4 * j + (q < 2 ? 2 + q : q - 2)) : -1;
      if (id >= 0) {
        vec* l = reinterpret_cast<vec*>((q < 2 ? LY : LX) + (q & 1) * HE);
#pragma unroll
        for (int v = 0; v < NV; v++) l[threadIdx.x + v * NT] = st[q][v];
      }
    }
  };
  acc_t acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; i++)
#pragma unroll
    for (int jj = 0; jj < NB; jj++) acc[i][jj] = acc_t{0, 0, 0, 0};
  const E* xl = (dg ? LY : LX) + xs * HE + (lane & 15) + (lane >> 4) * T;
  const E* yl = LY + ys * HE + (lane & 15) + (lane >> 4) * T;
  const int nsteps = 2 * nj;
  bool any = false;   // this wave's target received a product
  stage_load(0);
  for (int step = 0; step < nsteps; step++) {
    __syncthreads();
    stage_store(step);
    __syncthreads();
    if (step + 1 < nsteps) stage_load(step + 1);
    const int j = step >> 1;
    const bool use = active && word(pv, 4 + 4 * j + xs) >= 0 && word(pv, 4 + 4 * j + 2 + ys) >= 0;
    any |= use;
    if (use) {
#pragma unroll 2
      for (int k = 0; k < H; k += 4) {
        E a[NB], b[NB];
#pragma unroll
        for (int q = 0; q < NB; q++) {
          a[q] = yl[q * 16 + k * T];
          b[q] = xl[q * 16 + k * T];
        }
#pragma unroll
        for (int i = 0; i < NB; i++)
#pragma unroll
          for (int jj = 0; jj < NB; jj++)
            if (!tdiag || jj >= i) acc[i][jj] = O::mfma(a[i], b[jj], acc[i][jj]);
      }
    }
  }
  if (!any) return;
  GLOBAL double* out = gp(M.tiles + (int64_t)tgt * TT);
#pragma unroll
  for (int i = 0; i < NB; i++) {
    double cin[NB][4];
#pragma unroll
    for (int jj = 0; jj < NB; jj++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = 16 * jj + (lane & 15), col = 16 * i + O::col(lane, r);
        cin[jj][r] = (!tdiag || jj >= i) ? out[row + col * T] : 0.0;
      }
#pragma unroll
    for (int jj = 0; jj < NB; jj++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = 16 * jj + (lane & 15), col = 16 * i + O::col(lane, r);
        if (!tdiag || row >= col) st_dev(out + row + col * T, cin[jj][r] - (double)acc[i][jj][r]);
      }
  }
}

template <int T, int K>
__device__ __attribute__((noinline)) void task_update_block(const ExecMat& M, const int32_t* w, double* LX, double* LY) {
  if (M.mixed) update_block<T, float>(M, w, LX, LY);
  else update_block<T, double>(M, w, LX, LY);
}

// TREE: P_c = P_a + P_b, or C_t -= P_a (+ P_b) at the root (Alg. 3 GEADD).
template <int T, int K>
__device__ __attribute__((noinline)) void task_tree(const ExecMat& M, const int32_t* w) {
  constexpr int TT = T * T;
  typedef double d2 __attribute__((ext_vector_type(2)));
  const GLOBAL d2* pa = (const GLOBAL d2*)(M.part + (int64_t)w[2] * TT);
  const GLOBAL d2* pb = w[3] >= 0 ? (const GLOBAL d2*)(M.part + (int64_t)w[3] * TT) : nullptr;
  GLOBAL d2* dst = w[4] >= 0 ? (GLOBAL d2*)(M.part + (int64_t)w[4] * TT) : (GLOBAL d2*)(M.tiles + (int64_t)w[1] * TT);
  const bool apply = w[4] < 0;
#pragma unroll 4
  for (int e = threadIdx.x; e < TT / 2; e += NT) {
    const d2 s = pb ? pa[e] + pb[e] : pa[e];
    const d2 v = apply ? dst[e] - s : s;
    GLOBAL double* o = (GLOBAL double*)(dst + e);
    st_dev(o, v.x);
    st_dev(o + 1, v.y);
  }
}

// TRSM: L_t = (C_t - [sum X Y^T]) Linv_k^T as staged tile products; FP32
// copy in mixed mode.  The optional fused products (at most two) are the
// updates with the most recent columns.  The task waits for its
// predecessors itself: with TF_SPLIT, first for the early ones (its tile's
// update chain and the fused operands), then it stages its tile and does
// the fused products, and only then waits for the POTRF of its column, so
// that the pivot chain sees one tile product.  Returns the time its last
// wait ended (per-task trace); `ok` as for the solve tasks.
template <int T, int K>
__device__ __attribute__((noinline)) uint64_t task_trsm(const ExecMat& M, const int32_t* w, double* LX, double* LY,
                                                        int32_t* cnt, ExecCtrl* ctrl, uint64_t limit, bool& ok) {
  constexpr int TT = T * T, W = T / 2, NB = T / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (wave >> 1) * W, c0 = (wave & 1) * W;
  const bool split = (__builtin_amdgcn_readfirstlane(w[0]) & TF_SPLIT) != 0;
  if (ok) ok = wait_below(cnt, split ? MERGED_FDEP : 1, ctrl, limit);
  if (!ok) return 0;
  uint64_t t_start = M.trace ? wall_clock64() : 0;
  double* C = M.tiles + (int64_t)w[1] * TT;
  const double* Li = M.linv + (int64_t)w[2] * TT;
  GLOBAL double* Cg = gp(C);
  const int f0 = __builtin_amdgcn_readfirstlane(w[3]), nf = __builtin_amdgcn_readfirstlane(w[4]) - f0;
  TileStage<T, double> sx, sy;
  v4d acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; i++)
#pragma unroll
    for (int j = 0; j < NB; j++) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  if (nf > 0) {
    sx.load(M.tiles + (int64_t)M.pairs[2 * f0] * TT);
    sy.load(M.tiles + (int64_t)M.pairs[2 * f0 + 1] * TT);
    for (int q = 0; q < nf; q++) {
      __syncthreads();
      sx.store(LX);
      sy.store(LY);
      if (q + 1 < nf) {
        sx.load(M.tiles + (int64_t)M.pairs[2 * (f0 + q + 1)] * TT);
        sy.load(M.tiles + (int64_t)M.pairs[2 * (f0 + q + 1) + 1] * TT);
      } else {
        sx.load(C);
        if (!split) sy.load(Li);
      }
      __syncthreads();
      mma_f64<T>(acc, LX, LY, r0, c0, lane);   // X Y^T
    }
    __syncthreads();
    sx.store(LX);
    __syncthreads();
    // C -= X Y^T in LDS, each wave on its own quarter
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
          LX[row + col * T] -= acc[i][j][r];
          acc[i][j][r] = 0.0;
        }
  } else {
    sx.load(C);
    if (!split) sy.load(Li);
    sx.store(LX);
  }
  if (split) {
    // the POTRF of the column: its inverse is the last operand
    ok = wait_below(cnt, 1, ctrl, limit);
    if (!ok) return 0;
    if (M.trace) t_start = wall_clock64();
    sy.load(Li);
  }
  sy.store(LY);
  __syncthreads();
  mma_f64<T>(acc, LX, LY, r0, c0, lane);
  GLOBAL float* S = M.mixed ? gp(M.shadow + (int64_t)w[1] * TT) : nullptr;
#pragma unroll
  for (int i = 0; i < NB; i++)
#pragma unroll
    for (int j = 0; j < NB; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
        st_dev(Cg + row + col * T, acc[i][j][r]);
        if (S) st_dev(S + row + col * T, (float)acc[i][j][r]);
      }
  return t_start;
}

// ------------------------------------------------- diagonal tile: POTRF + TRTRI
// Blocked right-looking Cholesky of one T x T tile held in LDS, with 16-wide
// panels.  For each panel the 16 x 16 diagonal block is factored in the
// registers of wave 0 (diag_block16) and inverted by all four waves
// (inv_block16), the panel below is solved against the inverse block and
// the trailing matrix is updated, both as 16 x 16 x 16 MFMA products.  The inverse of the whole factor is built one
// block row at a time, as soon as its diagonal block is inverted, on the
// waves the panel leaves idle:
//   X_ii = D_i^{-1},  X_ib = -D_i^{-1} sum_{b <= q < i} L_iq X_qb.

__device__ __forceinline__ double bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// broadcast of lane r of every 16-lane row to the whole row (DPP row_newbcast)
__device__ __forceinline__ int row_bcast32(int v, int r) {
  switch (r) {
    case 0: return __builtin_amdgcn_update_dpp(0, v, 0x150, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0x151, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0x152, 0xF, 0xF, false);
    case 3: return __builtin_amdgcn_update_dpp(0, v, 0x153, 0xF, 0xF, false);
    case 4: return __builtin_amdgcn_update_dpp(0, v, 0x154, 0xF, 0xF, false);
    case 5: return __builtin_amdgcn_update_dpp(0, v, 0x155, 0xF, 0xF, false);
    case 6: return __builtin_amdgcn_update_dpp(0, v, 0x156, 0xF, 0xF, false);
    case 7: return __builtin_amdgcn_update_dpp(0, v, 0x157, 0xF, 0xF, false);
    case 8: return __builtin_amdgcn_update_dpp(0, v, 0x158, 0xF, 0xF, false);
    case 9: return __builtin_amdgcn_update_dpp(0, v, 0x159, 0xF, 0xF, false);
    case 10: return __builtin_amdgcn_update_dpp(0, v, 0x15A, 0xF, 0xF, false);
    case 11: return __builtin_amdgcn_update_dpp(0, v, 0x15B, 0xF, 0xF, false);
    case 12: return __builtin_amdgcn_update_dpp(0, v, 0x15C, 0xF, 0xF, false);
    case 13: return __builtin_amdgcn_update_dpp(0, v, 0x15D, 0xF, 0xF, false);
    case 14: return __builtin_amdgcn_update_dpp(0, v, 0x15E, 0xF, 0xF, false);
    default: return __builtin_amdgcn_update_dpp(0, v, 0x15F, 0xF, 0xF, false);
  }
}

__device__ __forceinline__ double row_bcast(double v, int r) {
  return __hiloint2double(row_bcast32(__double2hiint(v), r), row_bcast32(__double2loint(v), r));
}

// Cholesky factor of one 16 x 16 diagonal block on one wave.  Lane l holds
// row i = l & 15 of the columns g + 4 s (g = l >> 4, s = 0..3).  Column j:
// the pivot is read from its lane, the owner lanes scale the column and
// publish it through LDS (the operations of one wave reach LDS in order),
// and every lane applies its part of the rank-1 update.  The published
// columns (zero above the diagonal) go to pcol (16 columns with leading
// dimension T), the reciprocal pivots to rinv: the caller passes the upper
// block (0, T/16 - 1) of the tile buffer, which no other step uses while a
// diagonal block is factored and inverted.  The wave's issue rate, not the
// latency of the pivot chain, sets its time, so the inverse is left to all
// four waves (inv_block16).
template <int T>
__device__ __forceinline__ void diag_block16(double* S, double* rinv, double* pcol, int c0, int lane, int& fail) {
  const int i = lane & 15, g = lane >> 4;
  double a[4];
#pragma unroll
  for (int s = 0; s < 4; s++) a[s] = S[(c0 + i) + (c0 + g + 4 * s) * T];
  double piv[16];
  // the pivot of column j + 1 is formed from broadcast values as soon as
  // L(j + 1, j) exists, ahead of the lane updates that go through LDS
  double d = bcast(a[0], 0);
#pragma unroll
  for (int j = 0; j < 16; j++) {
    const int gj = j & 3, sj = j >> 2;
    const double rs = rsqrt_c(d);
    if (!(d > 0.0) && fail < 0) fail = c0 + j;
    piv[j] = rs;
    const double v = i == j ? d * rs : (i > j ? a[sj] * rs : 0.0);
    if (j < 15) {
      const int gn = (j + 1) & 3, sn = (j + 1) >> 2;
      const double pold = bcast(a[sn], (j + 1) + 16 * gn);   // A(j+1, j+1) before column j
      const double l1 = bcast(v, (j + 1) + 16 * gj);         // L(j+1, j)
      d = fma(-l1, l1, pold);
    }
    if (g == gj) {
      a[sj] = v;
      pcol[i + j * T] = v;
    }
    __builtin_amdgcn_wave_barrier();
    const double lij = pcol[i + j * T];
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const int q = g + 4 * s;
      if (q > j) a[s] = fma(-lij, pcol[q + j * T], a[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < 4; s++) {
    const int c = g + 4 * s;
    if (i >= c) S[(c0 + i) + (c0 + c) * T] = a[s];
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 16; j++) rinv[c0 + j] = piv[j];
  }
}

// Inverse of a factored 16 x 16 diagonal block (its columns in pcol, the
// reciprocal pivots in rinv), by all four waves after a barrier: the
// 16-lane row g of wave w computes column 4 w + g of D^{-1} by forward
// substitution, each final entry broadcast inside its 16-lane row by DPP.
template <int T>
__device__ __forceinline__ void inv_block16(double* Xi, const double* rinv, const double* pcol, int c0, int wave,
                                            int lane) {
  const int i = lane & 15, c = 4 * wave + (lane >> 4);
  double x = i == c ? 1.0 : 0.0;
#pragma unroll
  for (int rr = 0; rr < 16; rr++) {
    const double lir = pcol[i + rr * T];   // L(i, rr)
    if (i == rr) x *= rinv[c0 + rr];
    const double xb = row_bcast(x, rr);
    if (i > rr) x = fma(-lir, xb, x);
  }
  if (i >= c) Xi[(c0 + i) + (c0 + c) * T] = x;
}

template <int T>
__device__ __forceinline__ void inv_row_block(double* S, double* Xi, int b, int q, int lane) {
  v4d u = v4d{0.0, 0.0, 0.0, 0.0};
  for (int p = q; p < b; p++) {
#pragma unroll
    for (int kq = 0; kq < 16; kq += 4) {
      const double av = S[(16 * b + (lane & 15)) + (16 * p + kq + (lane >> 4)) * T];    // L(b, p)
      const double bv = Xi[(16 * p + kq + (lane >> 4)) + (16 * q + (lane & 15)) * T];   // X(p, q)
      u = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, u, 0, 0, 0);
    }
  }
#pragma unroll
  for (int rr = 0; rr < 4; rr++) S[(16 * q + (lane >> 4) + 4 * rr) + (16 * b + (lane & 15)) * T] = u[rr];
  __builtin_amdgcn_wave_barrier();
  v4d xv = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kq = 0; kq < 16; kq += 4) {
    const double av = Xi[(16 * b + (lane & 15)) + (16 * b + kq + (lane >> 4)) * T];   // D_b^{-1}
    const double bv = S[(16 * q + kq + (lane >> 4)) + (16 * b + (lane & 15)) * T];    // U
    xv = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, xv, 0, 0, 0);
  }
#pragma unroll
  for (int rr = 0; rr < 4; rr++) Xi[(16 * b + (lane >> 4) + 4 * rr) + (16 * q + (lane & 15)) * T] = -xv[rr];
}

// POTRF waits for its predecessors itself: with TF_SPLIT it prefetches its
// tile once the early ones (its update chain) have finished and waits last
// for the TRSM of its fused operand X = L_(k,k-1) (the panel of the previous
// column, on the pivot chain).  Returns the time its last wait ended.
template <int T, int K>
__device__ __attribute__((noinline)) uint64_t task_potrf(const ExecMat& M, const int32_t* w, double* S, double* Xi,
                                                         double* rinv, int32_t* cnt, ExecCtrl* ctrl, uint64_t limit,
                                                         bool& ok) {
  constexpr int TT = T * T, NBK = T / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool split = (__builtin_amdgcn_readfirstlane(w[0]) & TF_SPLIT) != 0;
  if (ok) ok = wait_below(cnt, split ? MERGED_FDEP : 1, ctrl, limit);
  if (!ok) return 0;
  uint64_t t_start = M.trace ? wall_clock64() : 0;
  double* C = M.tiles + (int64_t)w[1] * TT;
  const int k = w[2];
  {
    // C is prefetched; the fused operand X = L_(k,k-1) follows the last wait
    const bool fused = w[4] > w[3];
    const int64_t xt = fused ? __builtin_amdgcn_readfirstlane(M.pairs[2 * w[3]]) : 0;
    TileStage<T, double> st, sx;
    st.load(C);
    if (split) {
      ok = wait_below(cnt, 1, ctrl, limit);
      if (!ok) return 0;
      if (M.trace) t_start = wall_clock64();
    }
    if (fused) sx.load(M.tiles + xt * TT);
    st.store(S);
    if (fused) {
      // fused update with column k-1: C_kk -= X X^T
      constexpr int W = T / 2, NB = T / 32;
      const int r0 = (wave >> 1) * W, c0 = (wave & 1) * W;
      sx.store(Xi);
      __syncthreads();
      v4d acc[NB][NB];
#pragma unroll
      for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      mma_f64<T>(acc, Xi, Xi, r0, c0, lane);
#pragma unroll
      for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
            S[row + col * T] -= acc[i][j][r];
          }
      __syncthreads();
    }
  }
  for (int e = tid; e < TT; e += NT) Xi[e] = 0.0;
  __syncthreads();
  int fail = -1;
  double* pcol = S + (T - 16) * T;   // upper block (0, T/16 - 1), unused by the factorization
  if (tid < 64) diag_block16<T>(S, rinv, pcol, 0, lane, fail);
#pragma unroll 1
  for (int b = 0; b < NBK; b++) {
    const int c0 = 16 * b;
    __syncthreads();   // diagonal block b factored, trailing updates of step b-1 done
    inv_block16<T>(Xi, rinv, pcol, c0, wave, lane);
    __syncthreads();   // D_b^{-1} complete
    // ---- row block b of the inverse, X(b, q) for q < b, on the waves that
    //      the panel below leaves idle (every input is final by now)
    {
      const int q = wave - (NBK - 1 - b);
      if (q >= 0 && q < b) inv_row_block<T>(S, Xi, b, q, lane);
    }
    if (b + 1 == NBK) __syncthreads();
    if (b + 1 < NBK) {
      // ---- panel: L(R, c0:c0+16) = A(R, c0:c0+16) D^{-T}, R = rows below (MFMA)
      //      one 16-row block per wave
      const int nrb = NBK - 1 - b;
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      const int rb = c0 + 16 + 16 * wave;
      if (wave < nrb) {
        // D^{-T}(l, j) = Dinv(j, l): B(l, j) at Xi[(c0 + j) + (c0 + l) * T] -> ldb swap
        const double* A = S + rb + c0 * T;
#pragma unroll
        for (int kq = 0; kq < 16; kq += 4) {
          const double av = A[(lane & 15) + (kq + (lane >> 4)) * T];
          const double bv = Xi[(c0 + (lane & 15)) + (c0 + kq + (lane >> 4)) * T];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
      }
      __syncthreads();
      if (wave < nrb) {
#pragma unroll
        for (int q = 0; q < 4; q++) S[(rb + (lane >> 4) + 4 * q) + (c0 + (lane & 15)) * T] = acc[q];
      }
      __syncthreads();
      // ---- trailing update A22 -= P P^T over lower 16 x 16 blocks (MFMA).
      //      Lookahead: wave 0 updates the next diagonal block (block 0 of
      //      the trailing matrix) and factors it at once; waves 1..3 update
      //      the other blocks meanwhile (disjoint LDS regions)
      const int nb2 = nrb * (nrb + 1) / 2;
      const int q0 = wave, qstep = wave == 0 ? nb2 : NT / 64 - 1;
      for (int q = q0; q < nb2; q += qstep) {
        int bi = 0, rem = q;
        while (rem > bi) { rem -= bi + 1; bi++; }
        const int bj = rem;   // bj <= bi
        const int gi = c0 + 16 + 16 * bi, gj = c0 + 16 + 16 * bj;
        v4d u = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kq = 0; kq < 16; kq += 4) {
          const double av = S[(gi + (lane & 15)) + (c0 + kq + (lane >> 4)) * T];   // P(gi + i, l)
          const double bv = S[(gj + (lane & 15)) + (c0 + kq + (lane >> 4)) * T];   // P(gj + j, l)
          u = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, u, 0, 0, 0);
        }
#pragma unroll
        for (int rr = 0; rr < 4; rr++) S[(gi + (lane >> 4) + 4 * rr) + (gj + (lane & 15)) * T] -= u[rr];
      }
      if (tid < 64) {
        __builtin_amdgcn_wave_barrier();
        diag_block16<T>(S, rinv, pcol, c0 + 16, lane, fail);
      }
    }
  }
  if (tid == 0 && fail >= 0) atomicMin(M.info, (unsigned long long)(M.row_base[k] + fail + 1));
  double* Li = M.linv + (int64_t)k * TT;
  for (int e = tid; e < TT; e += NT) {
    const int row = e % T, col = e / T;
    st_dev(C + e, row >= col ? S[e] : 0.0);
    st_dev(Li + e, Xi[e]);
  }
  return t_start;
}

// ---------------------------------------------------------- solve tasks
// Vector blocks are T x nrhs column-major (nrhs <= 16).  Each task computes
// out = sum_p A_p V_p with A_p a factor tile (or its transpose) and V_p a
// vector block, as 16 x 16 x 4 FP64 MFMA products with the right-hand sides
// padded to 16 columns.
// MFMA operands are read from global memory straight into registers.  At
// MFMA step s the four k-groups of the 16 x 16 x 4 instruction (lane >> 4 =
// g) take k = (T/4) g + s, so that one lane's operands are contiguous: the
// B operand (vector block, column lane & 15) is one run of T/4 doubles, and
// so is the A operand of a transposed tile (backward sweep: A(r, k) =
// L(k, r), a piece of column r); a direct tile (forward sweep) is read as
// T/4 loads whose 16 lanes cover 16 consecutive rows.  Wave w owns rows
// 16 w .. 16 w + 15 of the T x 16 result (waves past T/16 idle).
template <int T>
struct SolveOps {
  static constexpr int NS = T / 4;   // MFMA steps per tile
  typedef double d2 __attribute__((ext_vector_type(2)));
  // A operand of tile Lt for rows 16 w + (lane & 15)
  static __device__ __forceinline__ void load_a(double (&a)[NS], const double* Lt, bool trans, int wave, int lane) {
    const int r = 16 * wave + (lane & 15), g = lane >> 4;
    if (trans) {
      const GLOBAL d2* p = (const GLOBAL d2*)(Lt + NS * g + (int64_t)r * T);
#pragma unroll
      for (int q = 0; q < NS / 2; q++) {
        const d2 v = p[q];
        a[2 * q] = v.x;
        a[2 * q + 1] = v.y;
      }
    } else {
      const GLOBAL double* p = gp(Lt) + r + (int64_t)NS * g * T;
#pragma unroll
      for (int q = 0; q < NS; q++) a[q] = p[(int64_t)q * T];
    }
  }
  // B operand of a vector block (T x nrhs, leading dimension T) in global memory
  static __device__ __forceinline__ void load_b(double (&b)[NS], const double* V, int nrhs, int lane) {
    const int j = lane & 15, g = lane >> 4;
    const GLOBAL d2* p = (const GLOBAL d2*)(V + NS * g + (int64_t)j * T);
    const bool ok = j < nrhs;
#pragma unroll
    for (int q = 0; q < NS / 2; q++) {
      const d2 v = ok ? p[q] : d2{0.0, 0.0};
      b[2 * q] = v.x;
      b[2 * q + 1] = v.y;
    }
  }
  // the same from a T x 16 block in LDS
  static __device__ __forceinline__ void load_b_lds(double (&b)[NS], const double* V, int lane) {
    const int j = lane & 15, g = lane >> 4;
    const d2* p = (const d2*)(V + NS * g + j * T);
#pragma unroll
    for (int q = 0; q < NS / 2; q++) {
      const d2 v = p[q];
      b[2 * q] = v.x;
      b[2 * q + 1] = v.y;
    }
  }
  // acc += A B over the T/4 steps, two accumulation chains
  static __device__ __forceinline__ v4d mma(v4d acc, const double (&a)[NS], const double (&b)[NS]) {
    v4d acc1 = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NS; q += 2) {
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q + 1], b[q + 1], acc1, 0, 0, 0);
    }
    return acc + acc1;
  }
};

// A solve task (FUPD, FDIAG, BUPD, BDIAG, FPART).  It waits for its
// predecessors itself (*cnt): the factor tiles of a diagonal step (at most
// two fused products and the inverse diagonal tile) are read into registers
// first, so that only the small vector blocks are loaded once the
// predecessors are done.  A diagonal step with TF_SPLIT waits in two
// stages: once its early predecessors are done (the counter below
// MERGED_FDEP in a solve launch, below SPLIT_W in the merged launch, whose
// executor has already waited for the factorization predecessors) it loads
// its right-hand side block and does the first fused product, then waits
// for the previous step of the chain, whose block the second product reads.
// The factor tiles must be final when it is called.
// `ok` enters false when the launch was already abandoned and leaves false
// when this task's own wait gave up; the task then writes nothing.
template <int T, int K>
__device__ __forceinline__ uint64_t task_solve_r(const ExecMat& M, const int32_t* w, int nrhs, int32_t* cnt,
                                                 double* LV, ExecCtrl* ctrl, uint64_t limit, bool& ok) {
  typedef SolveOps<T> O;
  constexpr int TT = T * T, NS = O::NS;
  const int type = __builtin_amdgcn_readfirstlane(w[0]) & 0xff;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool act = 16 * wave < T;
  const int m = __builtin_amdgcn_readfirstlane(w[1]);
  const int64_t vb = (int64_t)T * nrhs;
  const bool fwd = type == TK_FUPD || type == TK_FDIAG || type == TK_FPART;
  const bool diag = type == TK_FDIAG || type == TK_BDIAG;
  const double* vsrc = fwd ? M.vy : M.vz;
  const int p0 = __builtin_amdgcn_readfirstlane(w[2]), np = __builtin_amdgcn_readfirstlane(w[3]) - p0;
  const int pv = load_words(M.pairs + 2 * p0, 2 * np);
  // output element of this lane, register r: row 16 wave + (lane >> 4) + 4 r, column lane & 15
  const int col = lane & 15;
  const double* base = fwd ? M.vy + m * vb : ((w[0] & TF_FIRST) ? M.vy + m * vb : M.vz + m * vb);
  GLOBAL double* dst = gp(fwd ? M.vy + m * vb : M.vz + m * vb);
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  if (diag) {
    // static operands first (at most two fused products), then the wait
    const bool split = (__builtin_amdgcn_readfirstlane(w[0]) & TF_SPLIT) != 0;
    double a0[NS], a1[NS], ai[NS], b0[NS], b1[NS];
    if (act) {
      if (np > 0) O::load_a(a0, M.tiles + (int64_t)word(pv, 0) * TT, !fwd, wave, lane);
      if (np > 1) O::load_a(a1, M.tiles + (int64_t)word(pv, 2) * TT, !fwd, wave, lane);
      O::load_a(ai, M.linv + (int64_t)m * TT, !fwd, wave, lane);
    }
    if (ok) ok = wait_below(cnt, split ? (K == EXEC_FACTOR_SOLVE ? SPLIT_W : MERGED_FDEP) : 1, ctrl, limit);
    if (!ok) return 0;
    uint64_t t_start = M.trace ? wall_clock64() : 0;
    double bs[4];
    if (act) {
      if (np > 0) O::load_b(b0, vsrc + word(pv, 1) * vb, nrhs, lane);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = 16 * wave + (lane >> 4) + 4 * r;
        bs[r] = col < nrhs ? gp(base)[row + col * T] : 0.0;
      }
      if (np > 0) acc = O::mma(acc, a0, b0);
    }
    if (split) {
      // the previous step of the chain: its block is the second operand
      ok = wait_below(cnt, 1, ctrl, limit);
      if (!ok) return 0;
      if (M.trace) t_start = wall_clock64();
    }
    if (act) {
      if (np > 1) {
        O::load_b(b1, vsrc + word(pv, 3) * vb, nrhs, lane);
        acc = O::mma(acc, a1, b1);
      }
      // base - acc into LDS (T x 16, leading dimension T) for the product
      // with the inverse diagonal tile
#pragma unroll
      for (int r = 0; r < 4; r++) LV[(16 * wave + (lane >> 4) + 4 * r) + col * T] = bs[r] - acc[r];
    }
    __syncthreads();
    if (act) {
      O::load_b_lds(b0, LV, lane);
      const v4d out = O::mma(v4d{0.0, 0.0, 0.0, 0.0}, ai, b0);
      if (col < nrhs) {
#pragma unroll
        for (int r = 0; r < 4; r++) st_dev(dst + (16 * wave + (lane >> 4) + 4 * r) + col * T, out[r]);
      }
    }
    return t_start;
  }
  // a chunk of products: the factor tiles of the first two pairs are read
  // before the wait; then two pairs stay in flight (the operands of pair
  // p + 2 are loaded while pair p + 1 is multiplied)
  double a[2][NS], b[2][NS], bs[4];
  if (act && np > 0) {
    O::load_a(a[0], M.tiles + (int64_t)word(pv, 0) * TT, !fwd, wave, lane);
    if (np > 1) O::load_a(a[1], M.tiles + (int64_t)word(pv, 2) * TT, !fwd, wave, lane);
  }
  if (ok) ok = wait_below(cnt, 1, ctrl, limit);
  if (!ok) return 0;
  const uint64_t t_start = M.trace ? wall_clock64() : 0;
  if (act) {
    if (np > 0) O::load_b(b[0], vsrc + word(pv, 1) * vb, nrhs, lane);
    if (np > 1) O::load_b(b[1], vsrc + word(pv, 3) * vb, nrhs, lane);
    if (type != TK_FPART) {
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = 16 * wave + (lane >> 4) + 4 * r;
        bs[r] = col < nrhs ? gp(base)[row + col * T] : 0.0;
      }
    }
    for (int p = 0; p < np; p += 2) {
      acc = O::mma(acc, a[0], b[0]);
      if (p + 2 < np) {
        O::load_a(a[0], M.tiles + (int64_t)word(pv, 2 * p + 4) * TT, !fwd, wave, lane);
        O::load_b(b[0], vsrc + word(pv, 2 * p + 5) * vb, nrhs, lane);
      }
      if (p + 1 < np) {
        acc = O::mma(acc, a[1], b[1]);
        if (p + 3 < np) {
          O::load_a(a[1], M.tiles + (int64_t)word(pv, 2 * p + 6) * TT, !fwd, wave, lane);
          O::load_b(b[1], vsrc + word(pv, 2 * p + 7) * vb, nrhs, lane);
        }
      }
    }
  }
  if (!act) return t_start;
  if (type == TK_FPART) {
    // one chunk of a long row: the partial product into its slot
    GLOBAL double* q = gp(M.vpart + (int64_t)w[4] * vb);
    if (col < nrhs) {
#pragma unroll
      for (int r = 0; r < 4; r++) st_dev(q + (16 * wave + (lane >> 4) + 4 * r) + col * T, acc[r]);
    }
    return t_start;
  }
  if (col < nrhs) {
#pragma unroll
    for (int r = 0; r < 4; r++) st_dev(dst + (16 * wave + (lane >> 4) + 4 * r) + col * T, bs[r] - acc[r]);
  }
  return t_start;
}

// Y_m -= Q_a + ... + Q_(b-1): the partial products of a long row, summed in
// a fixed order (so the result does not depend on the schedule)
template <int T, int K>
__device__ __attribute__((noinline)) void task_fsum(const ExecMat& M, const int32_t* w, int nrhs) {
  const int64_t vb = (int64_t)T * nrhs;
  double* y = M.vy + (int64_t)w[1] * vb;
  const int a = w[2], b = w[3];
  for (int e = threadIdx.x; e < T * nrhs; e += NT) {
    // four running sums (slot q goes to sum q mod 4) keep four loads in
    // flight; the order is fixed, so the result does not depend on timing
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = a;
    for (; q + 4 <= b; q += 4) {
      s0 += M.vpart[(int64_t)q * vb + e];
      s1 += M.vpart[(int64_t)(q + 1) * vb + e];
      s2 += M.vpart[(int64_t)(q + 2) * vb + e];
      s3 += M.vpart[(int64_t)(q + 3) * vb + e];
    }
    for (; q < b; q++) s0 += M.vpart[(int64_t)q * vb + e];
    st_dev(y + e, y[e] - ((s0 + s1) + (s2 + s3)));
  }
}

// ------------------------------------------------------- selected inversion
// Tile products of the form C = op(X) op(Y)^T, op = identity or transpose,
// on tiles staged in LDS with leading dimension LP = T + 2: reading a
// column-major tile directly or transposed is then free of bank conflicts
// within each group of 16 lanes, and the 16-byte staging stores stay aligned.
// Output layout as in mma_f64 (each wave owns one (T/2) x (T/2) quarter).

template <int T>
struct PadStage {
  typedef double d2 __attribute__((ext_vector_type(2)));
  static constexpr int LP = T + 2;
  static constexpr int NV = T * T / NT / 2;
  d2 r[NV];
  __device__ __forceinline__ void load(const double* __restrict__ g) {
    const GLOBAL d2* v = (const GLOBAL d2*)g;
#pragma unroll
    for (int q = 0; q < NV; q++) r[q] = v[threadIdx.x + q * NT];
  }
  __device__ __forceinline__ void store(double* l) const {
#pragma unroll
    for (int q = 0; q < NV; q++) {
      const int e = 2 * ((int)threadIdx.x + q * NT);
      *reinterpret_cast<d2*>(l + (e % T) + (e / T) * LP) = r[q];
    }
  }
};

// acc += op(X) op(Y)^T: Xe(row, kk) = TX ? X[kk + row LP] : X[row + kk LP],
// the same for Y (rows of C from X, columns from Y)
template <int T, bool TX, bool TY>
__device__ __forceinline__ void mma_lp(v4d (&acc)[T / 32][T / 32], const double* X, const double* Y, int r0, int c0,
                                       int lane) {
  constexpr int NB = T / 32, LP = T + 2;
  const int li = lane & 15, lk = lane >> 4;
  auto ya = [&](int q, int kk) { const int yi = c0 + 16 * q + li; return TY ? Y[kk + yi * LP] : Y[yi + kk * LP]; };
  auto xb = [&](int q, int kk) { const int xi = r0 + 16 * q + li; return TX ? X[kk + xi * LP] : X[xi + kk * LP]; };
  double a[NB], b[NB];
#pragma unroll
  for (int q = 0; q < NB; q++) {
    a[q] = ya(q, lk);
    b[q] = xb(q, lk);
  }
#pragma unroll
  for (int k = 0; k < T; k += 4) {
    double an[NB], bn[NB];
    if (k + 4 < T) {
#pragma unroll
      for (int q = 0; q < NB; q++) {
        an[q] = ya(q, k + 4 + lk);
        bn[q] = xb(q, k + 4 + lk);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    if (k + 4 < T) {
#pragma unroll
      for (int q = 0; q < NB; q++) {
        a[q] = an[q];
        b[q] = bn[q];
      }
    }
  }
}

template <int T>
__device__ __forceinline__ void zero_acc(v4d (&acc)[T / 32][T / 32]) {
#pragma unroll
  for (int i = 0; i < T / 32; i++)
#pragma unroll
    for (int j = 0; j < T / 32; j++) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
}

// acc += sum over pairs of Sig~ L: the pair words (Sigma tile code, L tile)
// are in pv (at most 32 pairs); LX, LY: padded LDS tiles.  Two register
// stages alternate, so the global loads of a pair are issued two products
// before it is used.
template <int T>
__device__ __forceinline__ void sig_pair_load(PadStage<T>& sx, PadStage<T>& sy, const ExecMat& M, int pv, int p) {
  constexpr int TT = T * T;
  sx.load(M.sigma + (int64_t)(word(pv, 2 * p) & ~SIG_TRANS) * TT);
  sy.load(M.tiles + (int64_t)word(pv, 2 * p + 1) * TT);
}

template <int T>
__device__ __forceinline__ void sig_pair_mma(v4d (&acc)[T / 32][T / 32], int code, const double* LX, const double* LY,
                                             int r0, int c0, int lane) {
  // C = Sig~ L: op(X) = Sig or Sig^T, op(Y)^T = L
  if (code & SIG_TRANS) mma_lp<T, true, true>(acc, LX, LY, r0, c0, lane);
  else mma_lp<T, false, true>(acc, LX, LY, r0, c0, lane);
}

template <int T>
__device__ __forceinline__ void sig_products(v4d (&acc)[T / 32][T / 32], const ExecMat& M, int pv, int np,
                                             double* LX, double* LY, int r0, int c0, int lane) {
  if (np <= 0) return;
  PadStage<T> ax, ay, bx, by;
  sig_pair_load<T>(ax, ay, M, pv, 0);
  if (np > 1) sig_pair_load<T>(bx, by, M, pv, 1);
  for (int p = 0; p < np; p += 2) {
    __syncthreads();
    ax.store(LX);
    ay.store(LY);
    __syncthreads();
    if (p + 2 < np) sig_pair_load<T>(ax, ay, M, pv, p + 2);
    sig_pair_mma<T>(acc, word(pv, 2 * p), LX, LY, r0, c0, lane);
    if (p + 1 < np) {
      __syncthreads();
      bx.store(LX);
      by.store(LY);
      __syncthreads();
      if (p + 3 < np) sig_pair_load<T>(bx, by, M, pv, p + 3);
      sig_pair_mma<T>(acc, word(pv, 2 * p + 2), LX, LY, r0, c0, lane);
    }
  }
}

// out (global, column-major T x T) <- s * acc, element by element
template <int T>
__device__ __forceinline__ void put_acc_g(const v4d (&acc)[T / 32][T / 32], double* out, double sc, int r0, int c0,
                                          int lane) {
  GLOBAL double* o = gp(out);
#pragma unroll
  for (int i = 0; i < T / 32; i++)
#pragma unroll
    for (int j = 0; j < T / 32; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
        st_dev(o + row + col * T, sc * acc[i][j][r]);
      }
}

// out (LDS, leading dimension T + 2) <- s * acc
template <int T>
__device__ __forceinline__ void put_acc_l(const v4d (&acc)[T / 32][T / 32], double* out, double sc, int r0, int c0,
                                          int lane) {
#pragma unroll
  for (int i = 0; i < T / 32; i++)
#pragma unroll
    for (int j = 0; j < T / 32; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
        out[row + col * (T + 2)] = sc * acc[i][j][r];
      }
}

// acc += tile g (column-major T x T, global), element by element
template <int T>
__device__ __forceinline__ void add_tile(v4d (&acc)[T / 32][T / 32], const double* __restrict__ g, int r0, int c0,
                                         int lane) {
  const GLOBAL double* s = gp(g);
#pragma unroll
  for (int i = 0; i < T / 32; i++)
#pragma unroll
    for (int j = 0; j < T / 32; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
        acc[i][j][r] += s[row + col * T];
      }
}

// SWE: W_t (+)= sum over pairs of Sig~ L, kept in the Sigma tile of t until
// its SW task finishes it
template <int T>
__device__ __attribute__((noinline)) void task_swe(const ExecMat& M, const int32_t* w, double* LX, double* LY) {
  constexpr int TT = T * T, W = T / 2, NB = T / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (wave >> 1) * W, c0 = (wave & 1) * W;
  double* out = M.sigma + (int64_t)__builtin_amdgcn_readfirstlane(w[1]) * TT;
  const int np = __builtin_amdgcn_readfirstlane(w[3]);
  const int pv = load_words(M.pairs + __builtin_amdgcn_readfirstlane(w[2]), 2 * np);
  v4d acc[NB][NB];
  zero_acc<T>(acc);
  if (w[0] & TF_ACC) add_tile<T>(acc, out, r0, c0, lane);
  sig_products<T>(acc, M, pv, np, LX, LY, r0, c0, lane);
  put_acc_g<T>(acc, out, 1.0, r0, c0, lane);
}

// Static operands of a selected-inversion task (the factor is final), staged
// before the task waits for its predecessors: the L tile of SW's first
// product into LY, the inverse diagonal tile of SDIAG into LX.
template <int T>
__device__ __forceinline__ void selinv_prefetch(const ExecMat& M, const int32_t* w, double* LX, double* LY) {
  constexpr int TT = T * T;
  const int type = __builtin_amdgcn_readfirstlane(w[0]) & 0xff;
  PadStage<T> st;
  if (type == TK_SW) {
    const int32_t* lst = M.pairs + __builtin_amdgcn_readfirstlane(w[3]);
    st.load(M.tiles + (int64_t)__builtin_amdgcn_readfirstlane(lst[1]) * TT);
    st.store(LY);
  } else if (type == TK_SDIAG) {
    st.load(M.linv + (int64_t)__builtin_amdgcn_readfirstlane(w[2]) * TT);
    st.store(LX);
  }
}

// SW: Sig_t = -(W + pushed partials + sum of its one or two products Sig~ L_y)
// Linv_k, then D_t = L_t^T Sig_t and, for every listed tile u = (r,c),
// Q_u = Sig_t^T L_u.  The first product's L_y was staged in LY by
// selinv_prefetch.  w4 = nsum | npush << 8 | nprod << 16; the list holds the
// product pairs, then the slots, then the push tiles (at most 64 words).
template <int T>
__device__ __attribute__((noinline)) void task_sw(const ExecMat& M, const int32_t* w, double* LX, double* LY) {
  constexpr int TT = T * T, W = T / 2, NB = T / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (wave >> 1) * W, c0 = (wave & 1) * W;
  const int cnt = __builtin_amdgcn_readfirstlane(w[4]);
  const int nsum = cnt & 0xff, npush = (cnt >> 8) & 0xff, nprod = cnt >> 16;
  const int pv = load_words(M.pairs + __builtin_amdgcn_readfirstlane(w[3]), 2 * nprod + nsum + npush);
  const int sw0 = 2 * nprod, pw0 = 2 * nprod + nsum;   // first slot word, first push word
  const int64_t t = __builtin_amdgcn_readfirstlane(w[1]);
  const int64_t k = __builtin_amdgcn_readfirstlane(w[2]);
  double* sig = M.sigma + t * TT;
  PadStage<T> sx, sy, st;
  sx.load(M.sigma + (int64_t)(word(pv, 0) & ~SIG_TRANS) * TT);
  if (nprod > 1) {
    sy.load(M.tiles + (int64_t)word(pv, 3) * TT);
    st.load(M.sigma + (int64_t)(word(pv, 2) & ~SIG_TRANS) * TT);
  } else {
    st.load(M.linv + k * TT);
  }
  v4d acc[NB][NB];
  zero_acc<T>(acc);
  if (w[0] & TF_ACC) add_tile<T>(acc, sig, r0, c0, lane);
  for (int q = 0; q < nsum; q++) add_tile<T>(acc, M.qpart + (int64_t)word(pv, sw0 + q) * TT, r0, c0, lane);
  sx.store(LX);
  __syncthreads();
  // W += Sig~ L_y  (op(X) = Sig or Sig^T, op(Y)^T = L_y)
  sig_pair_mma<T>(acc, word(pv, 0), LX, LY, r0, c0, lane);
  if (nprod > 1) {
    __syncthreads();
    st.store(LX);
    sy.store(LY);
    __syncthreads();
    st.load(M.linv + k * TT);
    sig_pair_mma<T>(acc, word(pv, 2), LX, LY, r0, c0, lane);
  }
  // Sig_t = -W Linv_k  (op(X) = W, op(Y)^T = Linv_k)
  __syncthreads();
  put_acc_l<T>(acc, LX, 1.0, r0, c0, lane);
  st.store(LY);
  __syncthreads();
  st.load(M.tiles + t * TT);
  zero_acc<T>(acc);
  mma_lp<T, false, true>(acc, LX, LY, r0, c0, lane);
  put_acc_g<T>(acc, sig, -1.0, r0, c0, lane);
  __syncthreads();
  put_acc_l<T>(acc, LX, -1.0, r0, c0, lane);   // LX = Sig_t
  st.store(LY);                                // LY = L_t
  __syncthreads();
  if (npush > 0) st.load(M.tiles + (int64_t)word(pv, pw0) * TT);
  // D_t = L_t^T Sig_t  (op(X) = L_t^T, op(Y)^T = Sig_t)
  zero_acc<T>(acc);
  mma_lp<T, true, true>(acc, LY, LX, r0, c0, lane);
  put_acc_g<T>(acc, M.dpart + t * TT, 1.0, r0, c0, lane);
  for (int q = 0; q < npush; q++) {
    const int64_t u = word(pv, pw0 + q);
    __syncthreads();
    st.store(LY);                              // LY = L_u
    __syncthreads();
    if (q + 1 < npush) st.load(M.tiles + (int64_t)word(pv, pw0 + q + 1) * TT);
    // Q_u = Sig_t^T L_u  (op(X) = Sig_t^T, op(Y)^T = L_u)
    zero_acc<T>(acc);
    mma_lp<T, true, true>(acc, LX, LY, r0, c0, lane);
    put_acc_g<T>(acc, M.qpart + u * TT, 1.0, r0, c0, lane);
  }
}

// SDIAG: Sig_kk = Linv_k^T (Linv_k - sum_r D_(r,k)), the D in list order
// (w4 = count, at most 64); the lower triangle is kept and mirrored, so the
// stored tile is symmetric.  Linv_k was staged in LX by selinv_prefetch.
template <int T>
__device__ __attribute__((noinline)) void task_sdiag(const ExecMat& M, const int32_t* w, double* LX, double* LY) {
  constexpr int TT = T * T, W = T / 2, NB = T / 32, LP = T + 2;
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (wave >> 1) * W, c0 = (wave & 1) * W;
  const int nd = __builtin_amdgcn_readfirstlane(w[4]);
  const int pv = load_words(M.pairs + __builtin_amdgcn_readfirstlane(w[3]), nd);
  PadStage<T> z;
#pragma unroll
  for (int v = 0; v < PadStage<T>::NV; v++) {
    const int e = 2 * ((int)threadIdx.x + v * NT);
    z.r[v] = *reinterpret_cast<const d2*>(LX + (e % T) + (e / T) * LP);
  }
  for (int q = 0; q < nd; q++) {
    const GLOBAL d2* dp = (const GLOBAL d2*)(M.dpart + (int64_t)word(pv, q) * TT);
#pragma unroll
    for (int v = 0; v < PadStage<T>::NV; v++) z.r[v] -= dp[threadIdx.x + v * NT];
  }
  z.store(LY);
  __syncthreads();
  v4d acc[NB][NB];
  zero_acc<T>(acc);
  // op(X) = Linv_k^T, op(Y)^T = Z
  mma_lp<T, true, true>(acc, LX, LY, r0, c0, lane);
  GLOBAL double* out = gp(M.sigma + (int64_t)__builtin_amdgcn_readfirstlane(w[1]) * TT);
#pragma unroll
  for (int i = 0; i < NB; i++)
#pragma unroll
    for (int j = 0; j < NB; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
        if (row >= col) {
          st_dev(out + row + col * T, acc[i][j][r]);
          st_dev(out + col + row * T, acc[i][j][r]);
        }
      }
}

// TSUM: slot w1 = sum of the listed slots of dpart (c = 0) or qpart (c = 1),
// in list order; four running sums keep four loads in flight
template <int T>
__device__ __attribute__((noinline)) void task_tsum(const ExecMat& M, const int32_t* w) {
  constexpr int TT = T * T;
  typedef double d2 __attribute__((ext_vector_type(2)));
  const double* base = __builtin_amdgcn_readfirstlane(w[4]) == 1 ? M.qpart : M.dpart;
  const int32_t* lst = M.pairs + __builtin_amdgcn_readfirstlane(w[2]);
  const int n = __builtin_amdgcn_readfirstlane(w[3]);
  GLOBAL d2* out = (GLOBAL d2*)(base + (int64_t)__builtin_amdgcn_readfirstlane(w[1]) * TT);
  constexpr int NV = TT / 2 / NT;
  d2 s0[NV], s1[NV], s2[NV], s3[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) s0[v] = s1[v] = s2[v] = s3[v] = d2{0.0, 0.0};
  auto slot = [&](int id) { return (const GLOBAL d2*)(base + (int64_t)id * TT); };
  for (int blk = 0; blk < n; blk += 64) {   // 64 slot words per load
    const int nb = n - blk < 64 ? n - blk : 64;
    const int pv = load_words(lst + blk, nb);
    int q = 0;
    for (; q + 4 <= nb; q += 4) {
      const GLOBAL d2* a = slot(word(pv, q));
      const GLOBAL d2* b = slot(word(pv, q + 1));
      const GLOBAL d2* c = slot(word(pv, q + 2));
      const GLOBAL d2* d = slot(word(pv, q + 3));
#pragma unroll
      for (int v = 0; v < NV; v++) {
        const int e = threadIdx.x + v * NT;
        s0[v] += a[e];
        s1[v] += b[e];
        s2[v] += c[e];
        s3[v] += d[e];
      }
    }
    for (; q < nb; q++) {
      const GLOBAL d2* a = slot(word(pv, q));
#pragma unroll
      for (int v = 0; v < NV; v++) s0[v] += a[threadIdx.x + v * NT];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; v++) {
    const d2 t = (s0[v] + s1[v]) + (s2[v] + s3[v]);
    GLOBAL double* o = (GLOBAL double*)(out + threadIdx.x + v * NT);
    st_dev(o, t.x);
    st_dev(o + 1, t.y);
  }
}

// ---------------------------------------------------------------- executor

// The task bodies take the kernel kind as a template argument so that every
// executor kernel gets its own copies: a noinline function shared by two
// kernels is compiled for both call sites at once, which cost the
// factorization kernel register spills.
// KIND selects the task set: factorization tasks (UPD, PART, TREE, POTRF,
// TRSM), triangular-solve tasks, or selected-inversion tasks; they are
// separate kernels so that each carries only its own code.
template <int T, int KIND>
__global__ __launch_bounds__(NT, 2) void exec_kernel(const ExecMat* __restrict__ mats, const int32_t* __restrict__ order,
                                                  int32_t total, ExecCtrl* ctrl, int nrhs, uint64_t limit) {
  constexpr bool SOLVE = KIND == EXEC_SOLVE, SELINV = KIND == EXEC_SELINV, BOTH = KIND == EXEC_FACTOR_SOLVE;
  // LDS: factorization tasks use S (tile, ld T+1 room), Xi (T x T) and rinv;
  // solve tasks only a T x 16 block (Xi in the solve kernel, LI in the
  // combined factorization + solve kernel); selected-inversion tasks two
  // padded tiles.
  __shared__ __attribute__((aligned(16))) double S[SOLVE ? 2 : SELINV ? T * (T + 2) : T * (T + 1)];
  __shared__ __attribute__((aligned(16))) double Xi[SOLVE ? T * 16 : SELINV ? T * (T + 2) : T * T];
  __shared__ double rinv[(KIND == EXEC_FACTOR || BOTH) ? T : 1];
  __shared__ __attribute__((aligned(16))) double LI[BOTH ? T * 16 : 2];
  __shared__ int32_t s_ticket;
  // Control flow outside the task bodies is kept uniform across the
  // workgroup (values broadcast with readfirstlane, loops with uniform bounds
  // and predicated bodies): the compiler must never see a lane-divergent
  // region that straddles a barrier or the loop back-edge.
  for (;;) {
    if (threadIdx.x == 0) s_ticket = atomicAdd(&ctrl->ticket, 1);
    __syncthreads();
    const int32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    __syncthreads();
    if (t >= total) break;
    int32_t mi = 0, lid = t;
    if (order) {
      mi = __builtin_amdgcn_readfirstlane(order[2 * t]);
      lid = __builtin_amdgcn_readfirstlane(order[2 * t + 1]);
    }
    const ExecMat& M = mats[mi];
    const int32_t* w = M.tasks + (int64_t)lid * TASK_WORDS;
    int32_t* cnt = M.remaining + lid;
    uint64_t t_claim = 0, t_start = 0;
    if (M.trace) t_claim = wall_clock64();
    const int type = __builtin_amdgcn_readfirstlane(w[0]) & 0xff;
    if constexpr (SELINV) selinv_prefetch<T>(M, w, S, Xi);
    // merged factorization + solve DAG: a solve task first waits for its
    // factorization predecessors only (the counter falls below MERGED_FDEP);
    // its factor tiles are final then
    bool ok = true;
    if constexpr (BOTH) {
      if (type >= TK_FUPD) ok = wait_below(cnt, MERGED_FDEP, ctrl, limit);
    }
    // solve tasks other than FSUM wait for their predecessors themselves,
    // after reading their factor tiles; so do POTRF and TRSM (two-stage)
    const bool self_wait = ((SOLVE || BOTH) && type >= TK_FUPD && type != TK_FSUM) ||
                           (!SOLVE && !SELINV && (type == TK_POTRF || type == TK_TRSM));
    // wait until every predecessor has finished (Alg. 2 progress check);
    // wave 0 polls, then acquires for the workgroup (all its waves share
    // the CU's caches that the acquire invalidates)
    if (!self_wait && ok) ok = wait_below(cnt, 1, ctrl, limit);
    if (M.trace) t_start = wall_clock64();
    // tasks on the pivot chain (diagonal factorization, panel solve, diagonal
    // solve steps) raise their waves' issue priority over the co-resident
    // update work of other workgroups on the same SIMDs
    const bool chain = SOLVE    ? (type == TK_FDIAG || type == TK_BDIAG)
                       : SELINV ? (type == TK_SW || type == TK_SDIAG)
                                : (type == TK_POTRF || type == TK_TRSM || type == TK_FDIAG || type == TK_BDIAG);
    if (chain) __builtin_amdgcn_s_setprio(3);
    if constexpr (SELINV) {
      if (!ok) {
      } else if (type == TK_SWE) task_swe<T>(M, w, S, Xi);
      else if (type == TK_SW) task_sw<T>(M, w, S, Xi);
      else if (type == TK_SDIAG) task_sdiag<T>(M, w, S, Xi);
      else task_tsum<T>(M, w);
    } else if constexpr (SOLVE) {
      if (type == TK_FSUM) {
        if (ok) task_fsum<T, KIND>(M, w, nrhs);
      } else {
        t_start = task_solve_r<T, KIND>(M, w, nrhs, cnt, Xi, ctrl, limit, ok);
      }
    } else if (BOTH && type >= TK_FUPD) {
      if (type == TK_FSUM) {
        if (ok) task_fsum<T, KIND>(M, w, nrhs);
      } else {
        t_start = task_solve_r<T, KIND>(M, w, nrhs, cnt, LI, ctrl, limit, ok);
      }
    } else if (ok) {
      switch (type) {
        case TK_UPD: task_update<T, KIND>(M, w, 0, S, Xi); break;
        case TK_UPDB: task_update_block<T, KIND>(M, w, S, Xi); break;
        case TK_PART: task_update<T, KIND>(M, w, 1, S, Xi); break;
        case TK_TREE: task_tree<T, KIND>(M, w); break;
        case TK_POTRF: t_start = task_potrf<T, KIND>(M, w, S, Xi, rinv, cnt, ctrl, limit, ok); break;
        default: t_start = task_trsm<T, KIND>(M, w, S, Xi, cnt, ctrl, limit, ok); break;
      }
    }
    if (chain) __builtin_amdgcn_s_setprio(0);
    if (!ok) {
      // abandoned launch: the task is skipped and its matrix marked as timed
      // out (info 0, below every failing column); no successor is notified
      // and the counters are re-armed by the last workgroup to leave
      if (threadIdx.x == 0) atomicMin(M.info, 0ull);
      __syncthreads();
      continue;
    }
    // every wave waits for its own stores (device-scope stores, coherent
    // once complete), then wave 0 notifies the successors (Alg. 2 progress
    // update); the workgroup-scope release only orders the notification
    // after the stores in the compiler
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (threadIdx.x == 0) st_relaxed(cnt, w[7]);   // re-arm for the next launch
    const int32_t s0 = __builtin_amdgcn_readfirstlane(w[5]), s1 = __builtin_amdgcn_readfirstlane(w[6]);
    for (int32_t q0 = s0; q0 < s1; q0 += 64) {
      const int32_t q = q0 + (int32_t)threadIdx.x;
      if (threadIdx.x < 64 && q < s1) {
        int32_t sq = M.succ[q], dec = 1;
        if (sq & SUCC_FDEP) {   // an early predecessor of a two-stage wait
          dec = MERGED_FDEP;
          sq &= ~SUCC_FDEP;
        } else if (sq & SUCC_MID) {   // merged DAG: early solve predecessor of a diagonal step
          dec = SPLIT_W;
          sq &= ~SUCC_MID;
        }
        __hip_atomic_fetch_add(M.remaining + sq, -dec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (M.trace && threadIdx.x == 0) {
      unsigned long long* tr = M.trace + 4 * (int64_t)lid;
      tr[0] = t_claim;
      tr[1] = t_start;
      tr[2] = wall_clock64();
      tr[3] = ((unsigned long long)blockIdx.x << 32) | ((unsigned)type << 24) | ((unsigned)t & 0xffffffu);
    }
  }
  // the last workgroup to leave re-arms the control block; after an abort it
  // also re-arms every progress counter of the launch (skipped tasks did not
  // re-arm theirs, and some were notified after being skipped).  Every
  // workgroup's notifications are complete before it counts itself out.
  __shared__ int32_t s_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    fence_release();
    const int e = atomicAdd(&ctrl->exited, 1);
    s_last = e == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (__builtin_amdgcn_readfirstlane(s_last)) {
    fence_acquire();
    if (__builtin_amdgcn_readfirstlane(ld_relaxed(&ctrl->abort)) != 0) {
      for (int32_t t = threadIdx.x; t < total; t += NT) {
        int32_t mi = 0, lid = t;
        if (order) {
          mi = order[2 * t];
          lid = order[2 * t + 1];
        }
        st_relaxed(mats[mi].remaining + lid, mats[mi].tasks[(int64_t)lid * TASK_WORDS + 7]);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      st_relaxed(&ctrl->abort, 0);
      ctrl->ticket = 0;
      ctrl->exited = 0;
    }
  }
}

hipError_t launch_exec(int T, int kind, const ExecMat* d_mats, const int32_t* d_order, int32_t total,
                       ExecCtrl* d_ctrl, int nrhs, int nwg, uint64_t wait_ticks, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  if (nwg > total) nwg = total;
#define STILES_EXEC(TT, KK) \
  hipLaunchKernelGGL((exec_kernel<TT, KK>), dim3(nwg), dim3(NT), 0, st, d_mats, d_order, total, d_ctrl, nrhs, wait_ticks)
  if (T == 64) {
    if (kind == EXEC_SOLVE) STILES_EXEC(64, EXEC_SOLVE);
    else if (kind == EXEC_SELINV) STILES_EXEC(64, EXEC_SELINV);
    else if (kind == EXEC_FACTOR_SOLVE) STILES_EXEC(64, EXEC_FACTOR_SOLVE);
    else STILES_EXEC(64, EXEC_FACTOR);
  } else {
    if (kind == EXEC_SOLVE) STILES_EXEC(32, EXEC_SOLVE);
    else if (kind == EXEC_SELINV) STILES_EXEC(32, EXEC_SELINV);
    else if (kind == EXEC_FACTOR_SOLVE) STILES_EXEC(32, EXEC_FACTOR_SOLVE);
    else STILES_EXEC(32, EXEC_FACTOR);
  }
#undef STILES_EXEC
  return hipGetLastError();
}

// diagonal of Sigma (selected inversion) in the original ordering; NaN when
// the factorization failed.  One workgroup per tile row, one thread per row.
template <int T>
__global__ void selinv_diag_kernel(const double* __restrict__ sigma, const int32_t* __restrict__ trow_ptr,
                                   const int64_t* __restrict__ row_base, const int32_t* __restrict__ row_cnt,
                                   const int64_t* __restrict__ perm, int32_t ntr, const unsigned long long* info,
                                   double* __restrict__ out) {
  const int m = blockIdx.x, i = threadIdx.x;
  if (m >= ntr || i >= row_cnt[m]) return;
  const double v = sigma[(int64_t)(trow_ptr[m + 1] - 1) * T * T + i + i * T];
  out[perm[row_base[m] + i]] = *info != ~0ull ? __builtin_nan("") : v;
}

hipError_t launch_selinv_diag(int T, const double* sigma, const int32_t* trow_ptr, const int64_t* row_base,
                              const int32_t* row_cnt, const int64_t* perm, int32_t ntr,
                              const unsigned long long* info, double* out, hipStream_t st) {
  if (ntr <= 0) return hipSuccess;
  if (T == 64)
    hipLaunchKernelGGL((selinv_diag_kernel<64>), dim3(ntr), dim3(64), 0, st, sigma, trow_ptr, row_base, row_cnt, perm,
                       ntr, info, out);
  else
    hipLaunchKernelGGL((selinv_diag_kernel<32>), dim3(ntr), dim3(32), 0, st, sigma, trow_ptr, row_base, row_cnt, perm,
                       ntr, info, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ value scatter

// column-major T x T tile out (and o2) from the row-major LDS buffer
// (leading dimension T + 1): two rows per 16-byte streaming store
template <int T>
__device__ __forceinline__ void store_tile_cm(const double* buf, double* out, double* o2) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  constexpr int TT = T * T;
  GLOBAL d2* go = (GLOBAL d2*)out;
  GLOBAL d2* g2 = o2 ? (GLOBAL d2*)o2 : nullptr;
  for (int e2 = threadIdx.x; e2 < TT / 2; e2 += NT) {
    const int e = 2 * e2, c = e / T, r = e % T;
    const d2 v = d2{buf[r * (T + 1) + c], buf[(r + 1) * (T + 1) + c]};
    __builtin_nontemporal_store(v, go + e2);
    if (g2) __builtin_nontemporal_store(v, g2 + e2);
  }
}

// One T x T tile of the store from row-profile values: staged through LDS so
// that the reads follow the input rows and the stores the column-major tile.
// The first column and start offset of each of the tile's rows are read once
// into LDS, so every element costs one global load.
template <int T>
__device__ __forceinline__ void scatter_tile(const double* __restrict__ vals, const int64_t* __restrict__ in_rp,
                                             const int64_t* __restrict__ f, int m, int j,
                                             const int64_t* __restrict__ row_base,
                                             const int32_t* __restrict__ row_cnt, double* out, double* o2,
                                             double* buf) {
  constexpr int TT = T * T;
  __shared__ int64_t sf[T], sp[T];
  const int64_t rb = row_base[m], cb = row_base[j];
  const int rc = row_cnt[m], cc = row_cnt[j];
  if ((int)threadIdx.x < rc) {
    sf[threadIdx.x] = f[rb + threadIdx.x];
    sp[threadIdx.x] = in_rp[rb + threadIdx.x];
  }
  __syncthreads();
  // row-wise: consecutive threads read consecutive values; all of a
  // thread's loads are issued before any LDS store
  constexpr int NQ = TT / NT;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const int e = (int)threadIdx.x + q * NT;
    const int r = e / T, c = e % T;
    v[q] = (r >= rc && m == j && r == c) ? 1.0 : 0.0;   // padding row: unit diagonal
    if (r < rc) {
      const int64_t i = rb + r, g = cb + c;
      const int64_t fi = sf[r];
      if (c < cc && g <= i && g >= fi) v[q] = gp(vals)[sp[r] + (g - fi)];
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const int e = (int)threadIdx.x + q * NT;
    buf[(e / T) * (T + 1) + e % T] = v[q];
  }
  __syncthreads();
  store_tile_cm<T>(buf, out, o2);
}

template <int T>
__global__ __launch_bounds__(NT) void scatter_profile_kernel(const double* __restrict__ vals,
                                                             const int64_t* __restrict__ in_rp,
                                                             const int64_t* __restrict__ f,
                                                             const int32_t* __restrict__ trow,
                                                             const int32_t* __restrict__ tcol,
                                                             const int64_t* __restrict__ row_base,
                                                             const int32_t* __restrict__ row_cnt, double* tiles,
                                                             double* orig, unsigned long long* info) {
  constexpr int TT = T * T;
  __shared__ double buf[T * (T + 1)];
  const int64_t t = blockIdx.x;
  scatter_tile<T>(vals, in_rp, f, trow[t], tcol[t], row_base, row_cnt, tiles + t * TT, orig ? orig + t * TT : nullptr,
                  buf);
  if (t == 0 && threadIdx.x == 0) *info = ~0ull;
}

// Tile of P A P^T from row-profile values of the input ordering: element
// (r, c) of tile (m, j) is the input entry (perm[row], perm[col]), taken from
// the lower triangle (larger index as the row).  The gathers follow the tile
// rows; entries of reversed blocks are read transposed.
template <int T>
__device__ __forceinline__ void scatter_tile_perm(const double* __restrict__ vals, const int64_t* __restrict__ in_rp,
                                                  const int64_t* __restrict__ fin, const int64_t* __restrict__ perm,
                                                  int m, int j, const int64_t* __restrict__ row_base,
                                                  const int32_t* __restrict__ row_cnt, double* out, double* o2,
                                                  double* buf) {
  constexpr int TT = T * T;
  // per row and per column of the tile: input index, its first column and
  // its value offset (the larger input index of an entry names its row)
  __shared__ int64_t pr[T], pc[T], fr[T], fc[T], sr[T], sc[T];
  const int64_t rb = row_base[m], cb = row_base[j];
  const int rc = row_cnt[m], cc = row_cnt[j];
  if (threadIdx.x < T) {
    const int r = threadIdx.x;
    if (r < rc) {
      const int64_t o = perm[rb + r];
      pr[r] = o;
      fr[r] = fin[o];
      sr[r] = in_rp[o];
    }
  } else if (threadIdx.x < 2 * T) {
    const int c = threadIdx.x - T;
    if (c < cc) {
      const int64_t o = perm[cb + c];
      pc[c] = o;
      fc[c] = fin[o];
      sc[c] = in_rp[o];
    }
  }
  __syncthreads();
  // all of a thread's loads are issued before any LDS store (TT / NT of them
  // in flight per thread)
  constexpr int NQ = TT / NT;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const int e = (int)threadIdx.x + q * NT;
    const int r = e / T, c = e % T;
    v[q] = (r >= rc && m == j && r == c) ? 1.0 : 0.0;   // padding row: unit diagonal
    if (r < rc && c < cc && cb + c <= rb + r) {
      const int64_t oi = pr[r], oj = pc[c];
      const bool rowi = oi > oj;
      const int64_t lo = rowi ? oj : oi;
      const int64_t fh = rowi ? fr[r] : fc[c];
      const int64_t base = rowi ? sr[r] : sc[c];
      if (lo >= fh) v[q] = gp(vals)[base + (lo - fh)];
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const int e = (int)threadIdx.x + q * NT;
    buf[(e / T) * (T + 1) + e % T] = v[q];
  }
  __syncthreads();
  store_tile_cm<T>(buf, out, o2);
}

template <int T>
__global__ __launch_bounds__(NT) void scatter_perm_kernel(const double* __restrict__ vals,
                                                          const int64_t* __restrict__ in_rp,
                                                          const int64_t* __restrict__ fin,
                                                          const int64_t* __restrict__ perm,
                                                          const int32_t* __restrict__ trow,
                                                          const int32_t* __restrict__ tcol,
                                                          const int64_t* __restrict__ row_base,
                                                          const int32_t* __restrict__ row_cnt, double* tiles,
                                                          double* orig, unsigned long long* info) {
  constexpr int TT = T * T;
  __shared__ double buf[T * (T + 1)];
  const int64_t t = blockIdx.x;
  scatter_tile_perm<T>(vals, in_rp, fin, perm, trow[t], tcol[t], row_base, row_cnt, tiles + t * TT,
                       orig ? orig + t * TT : nullptr, buf);
  if (t == 0 && threadIdx.x == 0) *info = ~0ull;
}

hipError_t launch_scatter_perm(int T, const double* vals, const int64_t* in_rp, const int64_t* fin, const int64_t* perm,
                               const int32_t* trow, const int32_t* tcol, const int64_t* row_base,
                               const int32_t* row_cnt, int64_t ntiles, double* tiles, double* orig,
                               unsigned long long* info, hipStream_t st) {
  if (T == 64)
    hipLaunchKernelGGL(scatter_perm_kernel<64>, dim3((unsigned)ntiles), dim3(NT), 0, st, vals, in_rp, fin, perm, trow,
                       tcol, row_base, row_cnt, tiles, orig, info);
  else
    hipLaunchKernelGGL(scatter_perm_kernel<32>, dim3((unsigned)ntiles), dim3(NT), 0, st, vals, in_rp, fin, perm, trow,
                       tcol, row_base, row_cnt, tiles, orig, info);
  return hipGetLastError();
}

// every tile of every matrix of a batch: block b handles tile tmap[b].y of
// matrix tmap[b].x
template <int T>
__global__ __launch_bounds__(NT) void scatter_batch_kernel(const BatchDesc* __restrict__ desc,
                                                           const double* const* __restrict__ vals,
                                                           const int2* __restrict__ tmap) {
  constexpr int TT = T * T;
  __shared__ double buf[T * (T + 1)];
  const int2 mt = tmap[blockIdx.x];
  const BatchDesc& d = desc[mt.x];
  const int64_t t = mt.y;
  if (d.perm)
    scatter_tile_perm<T>(vals[mt.x], d.in_rp, d.f, d.perm, d.trow[t], d.tcol[t], d.row_base, d.row_cnt,
                         d.tiles + t * TT, d.orig ? d.orig + t * TT : nullptr, buf);
  else
    scatter_tile<T>(vals[mt.x], d.in_rp, d.f, d.trow[t], d.tcol[t], d.row_base, d.row_cnt, d.tiles + t * TT,
                    d.orig ? d.orig + t * TT : nullptr, buf);
  if (t == 0 && threadIdx.x == 0) *d.info = ~0ull;
}

hipError_t launch_scatter_batch(int T, const BatchDesc* desc, const double* const* vals, const int2* tmap,
                                int64_t total_tiles, hipStream_t st) {
  if (total_tiles <= 0) return hipSuccess;
  if (T == 64)
    hipLaunchKernelGGL(scatter_batch_kernel<64>, dim3((unsigned)total_tiles), dim3(NT), 0, st, desc, vals, tmap);
  else
    hipLaunchKernelGGL(scatter_batch_kernel<32>, dim3((unsigned)total_tiles), dim3(NT), 0, st, desc, vals, tmap);
  return hipGetLastError();
}

hipError_t launch_scatter_profile(int T, const double* vals, const int64_t* in_rp, const int64_t* f,
                                  const int32_t* trow, const int32_t* tcol, const int64_t* row_base,
                                  const int32_t* row_cnt, int64_t ntiles, double* tiles, double* orig,
                                  unsigned long long* info, hipStream_t st) {
  if (T == 64)
    hipLaunchKernelGGL(scatter_profile_kernel<64>, dim3((unsigned)ntiles), dim3(NT), 0, st, vals, in_rp, f, trow, tcol,
                       row_base, row_cnt, tiles, orig, info);
  else
    hipLaunchKernelGGL(scatter_profile_kernel<32>, dim3((unsigned)ntiles), dim3(NT), 0, st, vals, in_rp, f, trow, tcol,
                       row_base, row_cnt, tiles, orig, info);
  return hipGetLastError();
}

template <int T>
__global__ __launch_bounds__(NT) void fill_tiles_kernel(const int32_t* __restrict__ trow,
                                                        const int32_t* __restrict__ tcol,
                                                        const int32_t* __restrict__ row_cnt, double* tiles,
                                                        unsigned long long* info) {
  constexpr int TT = T * T;
  const int64_t t = blockIdx.x;
  const int m = trow[t], j = tcol[t], rc = row_cnt[m];
  double* out = tiles + t * TT;
  for (int e = threadIdx.x; e < TT; e += NT) {
    const int r = e % T, c = e / T;
    out[e] = (m == j && r == c && r >= rc) ? 1.0 : 0.0;
  }
  if (t == 0 && threadIdx.x == 0) *info = ~0ull;
}

__global__ void map_scatter_kernel(const double* __restrict__ vals, const int64_t* __restrict__ map, int64_t nnz,
                                   double* tiles, double* orig) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) {
    const int64_t o = map[e];
    tiles[o] = vals[e];
    if (orig) orig[o] = vals[e];
  }
}

hipError_t launch_scatter_map(int T, const double* vals, const int64_t* map, int64_t nnz, const int32_t* trow,
                              const int32_t* tcol, const int32_t* row_cnt, int64_t ntiles, double* tiles,
                              double* orig, unsigned long long* info, hipStream_t st) {
  if (T == 64) {
    hipLaunchKernelGGL(fill_tiles_kernel<64>, dim3((unsigned)ntiles), dim3(NT), 0, st, trow, tcol, row_cnt, tiles, info);
    if (orig)
      hipLaunchKernelGGL(fill_tiles_kernel<64>, dim3((unsigned)ntiles), dim3(NT), 0, st, trow, tcol, row_cnt, orig, info);
  } else {
    hipLaunchKernelGGL(fill_tiles_kernel<32>, dim3((unsigned)ntiles), dim3(NT), 0, st, trow, tcol, row_cnt, tiles, info);
    if (orig)
      hipLaunchKernelGGL(fill_tiles_kernel<32>, dim3((unsigned)ntiles), dim3(NT), 0, st, trow, tcol, row_cnt, orig, info);
  }
  if (nnz > 0)
    hipLaunchKernelGGL(map_scatter_kernel, dim3((unsigned)((nnz + NT - 1) / NT)), dim3(NT), 0, st, vals, map, nnz,
                       tiles, orig);
  return hipGetLastError();
}

template <int T>
__global__ __launch_bounds__(NT) void extract_kernel(const double* __restrict__ tiles, const int64_t* __restrict__ rp,
                                                     const int64_t* __restrict__ f, const int32_t* __restrict__ trow,
                                                     const int32_t* __restrict__ tcol,
                                                     const int64_t* __restrict__ row_base,
                                                     const int32_t* __restrict__ row_cnt, double* out) {
  constexpr int TT = T * T;
  const int64_t t = blockIdx.x;
  const int m = trow[t], j = tcol[t];
  const int64_t rb = row_base[m], cb = row_base[j];
  const int rc = row_cnt[m], cc = row_cnt[j];
  const double* src = tiles + t * TT;
  for (int e = threadIdx.x; e < TT; e += NT) {
    const int c = e / T, r = e % T;
    if (r >= rc || c >= cc) continue;
    const int64_t i = rb + r, g = cb + c;
    if (g <= i && g >= f[i]) out[rp[i] + (g - f[i])] = src[e];
  }
}

__global__ void zero_kernel(double* out, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = 0.0;
}

hipError_t launch_extract(int T, const double* tiles, const int64_t* rp, const int64_t* f, const int32_t* trow,
                          const int32_t* tcol, const int64_t* row_base, const int32_t* row_cnt, int64_t ntiles,
                          int64_t nnz, double* out, hipStream_t st) {
  // envelope entries outside the stored tiles (structural zeros of L) are zero
  if (nnz > 0)
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)std::min<int64_t>((nnz + NT - 1) / NT, 65536)), dim3(NT), 0, st, out,
                       nnz);
  if (T == 64)
    hipLaunchKernelGGL(extract_kernel<64>, dim3((unsigned)ntiles), dim3(NT), 0, st, tiles, rp, f, trow, tcol, row_base,
                       row_cnt, out);
  else
    hipLaunchKernelGGL(extract_kernel<32>, dim3((unsigned)ntiles), dim3(NT), 0, st, tiles, rp, f, trow, tcol, row_base,
                       row_cnt, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ logdet

// log-determinant: per tile row a fixed-shape wave reduction of log L_ii,
// then one block sums the tile-row partials (strided, then a binary tree).
// The single-matrix and batched launches share these two steps, so their
// results agree bit for bit.
template <int T>
__device__ __forceinline__ void logdet_row(const double* __restrict__ D, double* part_m, double* ws) {
  double v = threadIdx.x < T ? log(D[threadIdx.x * (T + 1)]) : 0.0;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < NT / 64; q++) s += ws[q];
    *part_m = s;
  }
}

__device__ __forceinline__ void logdet_sum(const double* __restrict__ part, int32_t n,
                                           const unsigned long long* info, double* out, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (*info == ~0ull) ? 2.0 * sh[0] : __builtin_nan("");
}

template <int T>
__global__ __launch_bounds__(NT) void logdet_partial_kernel(const double* __restrict__ tiles,
                                                            const int32_t* __restrict__ trow_ptr, double* part) {
  constexpr int TT = T * T;
  __shared__ double ws[NT / 64];
  const int m = blockIdx.x;
  logdet_row<T>(tiles + (int64_t)(trow_ptr[m + 1] - 1) * TT, part + m, ws);
}

__global__ __launch_bounds__(NT) void logdet_final_kernel(const double* __restrict__ part, int32_t n,
                                                          const unsigned long long* info, double* out) {
  __shared__ double sh[NT];
  logdet_sum(part, n, info, out, sh);
}

template <int T>
__global__ __launch_bounds__(NT) void logdet_partial_batch_kernel(const BatchDesc* __restrict__ desc,
                                                                  const int2* __restrict__ rmap) {
  constexpr int TT = T * T;
  __shared__ double ws[NT / 64];
  const int2 mr = rmap[blockIdx.x];
  const BatchDesc& d = desc[mr.x];
  logdet_row<T>(d.tiles + (int64_t)(d.trow_ptr[mr.y + 1] - 1) * TT, d.ldpart + mr.y, ws);
}

__global__ __launch_bounds__(NT) void logdet_final_batch_kernel(const BatchDesc* __restrict__ desc, double* out) {
  __shared__ double sh[NT];
  const BatchDesc& d = desc[blockIdx.x];
  logdet_sum(d.ldpart, d.ntr, d.info, out + blockIdx.x, sh);
}

hipError_t launch_logdet(int T, const double* tiles, const int32_t* trow_ptr, int32_t ntr, double* part,
                         const unsigned long long* info, double* out, hipStream_t st) {
  if (T == 64)
    hipLaunchKernelGGL(logdet_partial_kernel<64>, dim3(ntr), dim3(NT), 0, st, tiles, trow_ptr, part);
  else
    hipLaunchKernelGGL(logdet_partial_kernel<32>, dim3(ntr), dim3(NT), 0, st, tiles, trow_ptr, part);
  hipLaunchKernelGGL(logdet_final_kernel, dim3(1), dim3(NT), 0, st, part, ntr, info, out);
  return hipGetLastError();
}

// Per-tile-row partial sums of the log-determinant for callers that cannot
// allocate device memory (launch_logdet_static): a fixed array of the
// library, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol): it uses the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.  Every call
// on one GPU shares the array; each launch overwrites the partials of its
// own rows before the final sum reads them, so nothing needs clearing, and
// calls that overlap on one GPU race.
static __device__ __align__(256) double scratch[STATIC_LOGDET_ROWS];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};
}  // namespace

hipError_t static_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_logdet_static(int T, const double* tiles, const int32_t* trow_ptr, int32_t ntr,
                                const unsigned long long* info, double* out, hipStream_t st) {
  if (ntr < 1 || ntr > STATIC_LOGDET_ROWS) return hipErrorInvalidValue;
  double* part = nullptr;
  hipError_t e = static_scratch(&part);
  if (e != hipSuccess) return e;
  return launch_logdet(T, tiles, trow_ptr, ntr, part, info, out, st);
}

hipError_t launch_logdet_batch(int T, const BatchDesc* desc, int32_t count, const int2* rmap, int64_t total_rows,
                               double* out, hipStream_t st) {
  if (count <= 0 || total_rows <= 0) return hipSuccess;
  if (T == 64)
    hipLaunchKernelGGL(logdet_partial_batch_kernel<64>, dim3((unsigned)total_rows), dim3(NT), 0, st, desc, rmap);
  else
    hipLaunchKernelGGL(logdet_partial_batch_kernel<32>, dim3((unsigned)total_rows), dim3(NT), 0, st, desc, rmap);
  hipLaunchKernelGGL(logdet_final_batch_kernel, dim3((unsigned)count), dim3(NT), 0, st, desc, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ pack / unpack

__global__ void pack_kernel(int T, const double* __restrict__ B, int64_t ldb, int nrhs, const int64_t* __restrict__ perm,
                            const int64_t* __restrict__ row_base, const int32_t* __restrict__ row_cnt, int32_t ntr,
                            double* Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vb = (int64_t)T * nrhs;
  if (e >= vb * ntr) return;
  const int64_t m = e / vb, rem = e % vb;
  const int c = (int)(rem / T), r = (int)(rem % T);
  Y[e] = r < row_cnt[m] ? B[perm[row_base[m] + r] + c * ldb] : 0.0;
}

__global__ void unpack_kernel(int T, const double* __restrict__ Z, int nrhs, const int64_t* __restrict__ perm,
                              const int64_t* __restrict__ row_base, const int32_t* __restrict__ row_cnt, int32_t ntr,
                              const unsigned long long* info, double* B, int64_t ldb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vb = (int64_t)T * nrhs;
  if (e >= vb * ntr) return;
  const int64_t m = e / vb, rem = e % vb;
  const int c = (int)(rem / T), r = (int)(rem % T);
  if (r < row_cnt[m]) B[perm[row_base[m] + r] + c * ldb] = (*info == ~0ull) ? Z[e] : __builtin_nan("");
}

hipError_t launch_pack(int T, const double* B, int64_t ldb, int nrhs, const int64_t* perm, const int64_t* row_base,
                       const int32_t* row_cnt, int32_t ntr, double* Y, hipStream_t st) {
  const int64_t n = (int64_t)T * nrhs * ntr;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, T, B, ldb, nrhs, perm, row_base,
                     row_cnt, ntr, Y);
  return hipGetLastError();
}

hipError_t launch_unpack(int T, const double* Z, int nrhs, const int64_t* perm, const int64_t* row_base,
                         const int32_t* row_cnt, int32_t ntr, const unsigned long long* info, double* B, int64_t ldb,
                         hipStream_t st) {
  const int64_t n = (int64_t)T * nrhs * ntr;
  hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, T, Z, nrhs, perm, row_base,
                     row_cnt, ntr, info, B, ldb);
  return hipGetLastError();
}

}  // namespace stiles

// ------------------------------------------------- refinement (mixed mode)

namespace stiles {

// Residual items on MFMA: each tile of the item is staged in LDS
// (with |.| in absmode), multiplied with the vector block (A x for row items,
// A^T x for column items; a diagonal tile adds its strict lower part
// transposed), and the item's partial written once.
template <int T>
__global__ __launch_bounds__(NT) void residual_mma_kernel(const double* __restrict__ orig,
                                                          const int32_t* __restrict__ rtile,
                                                          const int32_t* __restrict__ tcol,
                                                          const int32_t* __restrict__ ccol_tile,
                                                          const int32_t* __restrict__ ccol_row,
                                                          const int32_t* __restrict__ items,
                                                          const double* __restrict__ X, double* part, double* apart,
                                                          int nrhs, int absmode) {
  // operands straight from global memory into registers (SolveOps layout),
  // two tiles in flight; wave w owns rows 16 w .. 16 w + 15 of the T x 16 result.
  // With apart (residual pass), the row sums of |A| over the same operands
  // are accumulated too (one pass over A gives both).
  typedef SolveOps<T> O;
  constexpr int TT = T * T, NS = O::NS;
  const int q = blockIdx.x;
  const int m = items[4 * q], kind = items[4 * q + 1], lo = items[4 * q + 2], hi = items[4 * q + 3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool act = 16 * wave < T;
  const int col = lane & 15, g = lane >> 4, r = 16 * wave + (lane & 15);
  const int64_t vb = (int64_t)T * nrhs;
  const int ncol = absmode ? 1 : nrhs;
  const bool trans = kind == 1;
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  double rs = 0.0;   // this lane's share of the row sum of |A| (apart)
  if (!act) return;
  double a[2][NS], b[2][NS];
  // operands of item entry e into slot u
  auto load = [&](int u, int e) {
    const int tile = kind == 0 ? rtile[e] : ccol_tile[e];
    const int src = kind == 0 ? tcol[tile] : ccol_row[e];
    O::load_a(a[u], orig + (int64_t)tile * TT, trans, wave, lane);
    if (absmode) {
#pragma unroll
      for (int s = 0; s < NS; s++) b[u][s] = col == 0 ? 1.0 : 0.0;
    } else {
      O::load_b(b[u], X + src * vb, nrhs, lane);
    }
  };
  auto use = [&](int u, int e) {
    if (absmode) {
#pragma unroll
      for (int s = 0; s < NS; s++) a[u][s] = fabs(a[u][s]);
    } else if (apart) {
#pragma unroll
      for (int s = 0; s < NS; s++) rs += fabs(a[u][s]);
    }
    acc = O::mma(acc, a[u], b[u]);
    const int tile = kind == 0 ? rtile[e] : -1;
    if (kind == 0 && tcol[tile] == m) {
      // diagonal tile: only its lower triangle is stored; add the strict
      // lower part transposed (A(r, k) = L(k, r), zero on the diagonal)
      double at[NS];
      O::load_a(at, orig + (int64_t)tile * TT, true, wave, lane);
#pragma unroll
      for (int s = 0; s < NS; s++) {
        const double v = NS * g + s == r ? 0.0 : at[s];
        at[s] = absmode ? fabs(v) : v;
        if (apart && !absmode) rs += fabs(v);
      }
      acc = O::mma(acc, at, b[u]);
    }
  };
  if (lo < hi) load(0, lo);
  for (int e = lo; e < hi; e += 2) {
    if (e + 1 < hi) load(1, e + 1);
    use(0, e);
    if (e + 1 < hi) {
      if (e + 2 < hi) load(0, e + 2);
      use(1, e + 1);
    }
  }
  double* out = part + (int64_t)q * vb;
  if (col < ncol) {
#pragma unroll
    for (int rr = 0; rr < 4; rr++) out[(16 * wave + (lane >> 4) + 4 * rr) + col * T] = acc[rr];
  }
  if (apart) {
    // the four lanes of a row (k groups g = 0..3) hold its whole sum
    rs += __shfl_xor(rs, 16, 64);
    rs += __shfl_xor(rs, 32, 64);
    if (g == 0) apart[(int64_t)q * T + r] = rs;
  }
}

__global__ void residual_combine_kernel(int T, const int32_t* __restrict__ item_ptr, const double* __restrict__ part,
                                        const double* __restrict__ B, double* R, int nrhs, int absmode,
                                        const double* __restrict__ apart, double* D) {
  const int m = blockIdx.x;
  const int64_t vb = (int64_t)T * nrhs;
  const int ncol = absmode ? 1 : nrhs;
  for (int e = threadIdx.x; e < T * ncol; e += blockDim.x) {
    double s = 0.0;
    for (int q = item_ptr[m]; q < item_ptr[m + 1]; q++) s += part[(int64_t)q * vb + e];
    R[m * vb + e] = absmode ? s : B[m * vb + e] - s;
  }
  if (apart) {
    for (int e = threadIdx.x; e < T; e += blockDim.x) {
      double s = 0.0;
      for (int q = item_ptr[m]; q < item_ptr[m + 1]; q++) s += apart[(int64_t)q * T + e];
      D[(int64_t)m * T + e] = s;
    }
  }
}

hipError_t launch_residual(int T, const double* orig, const int32_t* rtile, const int32_t* tcol,
                           const int32_t* ccol_tile, const int32_t* ccol_row, const int32_t* items, int32_t nitems,
                           const int32_t* item_ptr, int32_t ntr, const double* X, const double* B, double* part,
                           double* R, int nrhs, int absmode, hipStream_t st, double* apart, double* D) {
  if (absmode) apart = nullptr;
  if (nitems > 0) {
    if (T == 64)
      hipLaunchKernelGGL(residual_mma_kernel<64>, dim3(nitems), dim3(NT), 0, st, orig, rtile, tcol, ccol_tile, ccol_row,
                         items, X, part, apart, nrhs, absmode);
    else
      hipLaunchKernelGGL(residual_mma_kernel<32>, dim3(nitems), dim3(NT), 0, st, orig, rtile, tcol, ccol_tile, ccol_row,
                         items, X, part, apart, nrhs, absmode);
  }
  hipLaunchKernelGGL(residual_combine_kernel, dim3(ntr), dim3(NT), 0, st, T, item_ptr, part, B, R, nrhs, absmode,
                     apart, D);
  return hipGetLastError();
}

// ------------------------------------------------ out-of-core factorization
// S = Lc Lc^T (lower part, c x c, row-major) for the dense lower-triangular
// trailing block Lc of a factor stored in row-profile order: Lc(i, t) =
// L[rp[r0 + i] + (c0 + t - f[r0 + i])], t <= i.  16 x 16 tiles of S per
// workgroup, 64 columns of both row panels staged in LDS per step.
__global__ __launch_bounds__(256) void gram_lower_kernel(int32_t c, const double* __restrict__ L,
                                                         const int64_t* __restrict__ rp, const int64_t* __restrict__ f,
                                                         int64_t r0, int64_t c0, double* __restrict__ S) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  __shared__ double A[16][65], B[16][65];
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int ri = 16 * bi + ty, rj = 16 * bj + ty;   // rows staged by this thread
  const int64_t oi = ri < c ? rp[r0 + ri] + c0 - f[r0 + ri] : 0;
  const int64_t oj = rj < c ? rp[r0 + rj] + c0 - f[r0 + rj] : 0;
  const int tmax = min(c, 16 * bj + 16);            // Lc(j, t) = 0 for t > j
  double acc = 0.0;
  for (int t0 = 0; t0 < tmax; t0 += 64) {
#pragma unroll
    for (int q = tx; q < 64; q += 16) {
      const int t = t0 + q;
      A[ty][q] = (ri < c && t <= ri) ? L[oi + t] : 0.0;
      B[ty][q] = (rj < c && t <= rj) ? L[oj + t] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int q = 0; q < 64; q++) acc = fma(A[ty][q], B[tx][q], acc);
    __syncthreads();
  }
  const int i = 16 * bi + ty, j = 16 * bj + tx;
  if (i < c && j <= i) S[(int64_t)i * c + j] = acc;
}

hipError_t launch_gram_lower(int32_t c, const double* L, const int64_t* rp, const int64_t* f, int64_t r0, int64_t c0,
                             double* S, hipStream_t st) {
  if (c <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((c + 15) / 16);
  hipLaunchKernelGGL(gram_lower_kernel, dim3(nb, nb), dim3(256), 0, st, c, L, rp, f, r0, c0, S);
  return hipGetLastError();
}

// acc += 2 sum_r log L(r, r) over rows [r0, r1) of a factor in row-profile
// order (diagonal = last entry of a row); one workgroup, fixed summation
// order (per-thread strided sums, then a tree), so the result is
// reproducible.  NaN when a pivot is not positive.
__global__ __launch_bounds__(256) void logdet_rows_kernel(const double* __restrict__ L, const int64_t* __restrict__ rp,
                                                          int64_t r0, int64_t r1, double* acc) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    const double d = L[rp[r + 1] - 1];
    s += d > 0.0 ? 2.0 * log(d) : NAN;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *acc += red[0];
}

hipError_t launch_logdet_rows(const double* L, const int64_t* rp, int64_t r0, int64_t r1, double* acc, hipStream_t st) {
  hipLaunchKernelGGL(logdet_rows_kernel, dim3(1), dim3(256), 0, st, L, rp, r0, r1, acc);
  return hipGetLastError();
}

// Per-column max |R| and max |X| over the tile-row blocks (T x nrhs each).
// Block (x, c) covers 16 tile rows of column c and reduces in LDS before one
// atomic per value.  Maxima are taken on the bit patterns of |v|
// (non-negative doubles order like their bits), so a NaN propagates.
__global__ __launch_bounds__(NT) void norms_kernel(int32_t ntr, int T, int nrhs, const double* __restrict__ R,
                                                   const double* __restrict__ X, unsigned long long* stats) {
  __shared__ unsigned long long sr[NT], sx[NT];
  const int c = blockIdx.y;
  const int64_t vb = (int64_t)T * nrhs;
  const int m0 = blockIdx.x * 16;
  unsigned long long rm = 0, xm = 0;
  for (int idx = threadIdx.x; idx < 16 * T; idx += NT) {
    const int m = m0 + idx / T, r = idx % T;
    if (m < ntr) {
      const int64_t e = (int64_t)m * vb + (int64_t)c * T + r;
      const unsigned long long ur = (unsigned long long)__double_as_longlong(fabs(R[e]));
      const unsigned long long ux = (unsigned long long)__double_as_longlong(fabs(X[e]));
      rm = ur > rm ? ur : rm;
      xm = ux > xm ? ux : xm;
    }
  }
  sr[threadIdx.x] = rm;
  sx[threadIdx.x] = xm;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sr[threadIdx.x] = sr[threadIdx.x + o] > sr[threadIdx.x] ? sr[threadIdx.x + o] : sr[threadIdx.x];
      sx[threadIdx.x] = sx[threadIdx.x + o] > sx[threadIdx.x] ? sx[threadIdx.x + o] : sx[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(stats + 2 * c, sr[0]);
    atomicMax(stats + 2 * c + 1, sx[0]);
  }
}

hipError_t launch_norms(int T, int32_t ntr, int nrhs, const double* R, const double* X, unsigned long long* stats,
                        hipStream_t st) {
  if (ntr <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(norms_kernel, dim3((unsigned)((ntr + 15) / 16), (unsigned)nrhs), dim3(NT), 0, st, ntr, T, nrhs, R,
                     X, stats);
  return hipGetLastError();
}

// X(:, c) += D(:, c) (assign = 0) or X(:, c) = D(:, c) (assign = 1) for the
// right-hand sides c whose bit is set in `mask`; blocks of T x nrhs, so
// element e belongs to column (e / T) mod nrhs
__global__ void colmask_kernel(int64_t n, int T, int nrhs, double* X, const double* __restrict__ D, uint32_t mask,
                               int assign) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)((e / T) % nrhs);
  if (!((mask >> c) & 1u)) return;
  X[e] = assign ? D[e] : X[e] + D[e];
}

hipError_t launch_axpy(int T, int32_t ntr, int nrhs, double* X, const double* D, uint32_t mask, hipStream_t st) {
  const int64_t n = (int64_t)T * nrhs * ntr;
  hipLaunchKernelGGL(colmask_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, T, nrhs, X, D, mask, 0);
  return hipGetLastError();
}

hipError_t launch_copy_cols(int T, int32_t ntr, int nrhs, double* X, const double* P, uint32_t mask, hipStream_t st) {
  const int64_t n = (int64_t)T * nrhs * ntr;
  hipLaunchKernelGGL(colmask_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, T, nrhs, X, P, mask, 1);
  return hipGetLastError();
}

}  // namespace stiles
