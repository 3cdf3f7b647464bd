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

#include "launch.h"
#include "stiles_internal.h"

namespace stiles {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int NT = 256;

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int ld_relaxed(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// 1/sqrt(d): hardware estimate (about 24 bits) refined by two Newton steps
// y <- y + y (1 - d y^2) / 2, which reach full double precision (to ~1 ulp).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  double e = fma(-d * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-d * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  return y;
}

// ------------------------------------------------------- tile products (MFMA)
// acc[i][j] covers C rows r0 + 16 j + (lane & 15) and C columns
// c0 + 16 i + (lane >> 4) + 4 r (FP64 MFMA output layout on gfx950: lane l,
// register r holds D[(l >> 4) + 4 r][l & 15]).  The A operand is taken from
// Y (C columns), the B operand from X (C rows), so that the 16 lanes of one
// row group touch 16 consecutive rows of a column-major tile.

template <int T>
__device__ __forceinline__ void mma_f64(v4d (&acc)[T / 32][T / 32], const double* __restrict__ X,
                                        const double* __restrict__ Y, int r0, int c0, int lane) {
  constexpr int NB = T / 32;
  const double* xp = X + r0 + (lane & 15) + (lane >> 4) * T;
  const double* yp = Y + c0 + (lane & 15) + (lane >> 4) * T;
#pragma unroll 4
  for (int k = 0; k < T; k += 4) {
    double a[NB], b[NB];
#pragma unroll
    for (int q = 0; q < NB; q++) {
      a[q] = yp[q * 16 + k * T];
      b[q] = xp[q * 16 + k * T];
    }
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// FP32 variant (mixed mode); FP32 MFMA output layout: lane l, register r holds
// D[4 (l >> 4) + r][l & 15], so acc[i][j][r] covers column c0 + 16 i + 4 (lane >> 4) + r.
template <int T>
__device__ __forceinline__ void mma_f32(v4f (&acc)[T / 32][T / 32], const float* __restrict__ X,
                                        const float* __restrict__ Y, int r0, int c0, int lane) {
  constexpr int NB = T / 32;
  const float* xp = X + r0 + (lane & 15) + (lane >> 4) * T;
  const float* yp = Y + c0 + (lane & 15) + (lane >> 4) * T;
#pragma unroll 4
  for (int k = 0; k < T; k += 4) {
    float a[NB], b[NB];
#pragma unroll
    for (int q = 0; q < NB; q++) {
      a[q] = yp[q * 16 + k * T];
      b[q] = xp[q * 16 + k * T];
    }
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// ------------------------------------------------------------ task bodies

// UPD / PART: acc = sum_p X_p Y_p^T over a list of tile pairs.
// mode 0: C_t -= acc (UPD), mode 1: P = acc (PART).
template <int T>
__device__ void task_update(const ExecMat& M, const int32_t* w, int mode) {
  constexpr int TT = T * T, W = T / 2, NB = T / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int r0 = wr * W, c0 = wc * W;
  const bool diag = (w[0] & TF_DIAG) != 0;
  const bool active = !(diag && wc > wr);   // strictly upper quarter of a diagonal tile
  const int p0 = w[2], p1 = w[3];
  const bool mixed = M.mixed && mode == 0;
  double* out = mode == 0 ? M.tiles + (int64_t)w[1] * TT : M.part + (int64_t)w[4] * TT;
  if (!active) {
    if (mode == 1) {   // keep the partial fully defined
#pragma unroll
      for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
            out[row + col * T] = 0.0;
          }
    }
    return;
  }
  if (!mixed) {
    v4d acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int p = p0; p < p1; p++) {
      const double* X = M.tiles + (int64_t)M.pairs[2 * p] * TT;
      const double* Y = M.tiles + (int64_t)M.pairs[2 * p + 1] * TT;
      mma_f64<T>(acc, X, Y, r0, c0, lane);
    }
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
          if (mode == 0) {
            if (!diag || row >= col) out[row + col * T] -= acc[i][j][r];
          } else {
            out[row + col * T] = acc[i][j][r];
          }
        }
  } else {
    v4f acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int p = p0; p < p1; p++) {
      const float* X = M.shadow + (int64_t)M.pairs[2 * p] * TT;
      const float* Y = M.shadow + (int64_t)M.pairs[2 * p + 1] * TT;
      mma_f32<T>(acc, X, Y, r0, c0, lane);
    }
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < NB; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + 4 * (lane >> 4) + r;
          if (!diag || row >= col) out[row + col * T] -= (double)acc[i][j][r];
        }
  }
}

// TREE: P_c = P_a + P_b, or C_t -= P_a (+ P_b) at the root (Alg. 3 GEADD).
template <int T>
__device__ void task_tree(const ExecMat& M, const int32_t* w) {
  constexpr int TT = T * T;
  const double* pa = M.part + (int64_t)w[2] * TT;
  const double* pb = w[3] >= 0 ? M.part + (int64_t)w[3] * TT : nullptr;
  if (w[4] >= 0) {
    double* po = M.part + (int64_t)w[4] * TT;
    for (int e = threadIdx.x; e < TT; e += NT) po[e] = pa[e] + (pb ? pb[e] : 0.0);
  } else {
    double* c = M.tiles + (int64_t)w[1] * TT;
    for (int e = threadIdx.x; e < TT; e += NT) c[e] -= (pb ? pa[e] + pb[e] : pa[e]);
  }
}

// TRSM: L_t = C_t Linv_k^T as a tile product; FP32 copy in mixed mode.
template <int T>
__device__ void task_trsm(const ExecMat& M, const int32_t* w) {
  constexpr int TT = T * T, W = T / 2, NB = T / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (wave >> 1) * W, c0 = (wave & 1) * W;
  double* C = M.tiles + (int64_t)w[1] * TT;
  const double* Li = M.linv + (int64_t)w[2] * TT;
  v4d acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; i++)
#pragma unroll
    for (int j = 0; j < NB; j++) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  mma_f64<T>(acc, C, Li, r0, c0, lane);
  __syncthreads();   // every wave has read C before it is overwritten
  float* S = M.mixed ? M.shadow + (int64_t)w[1] * TT : nullptr;
#pragma unroll
  for (int i = 0; i < NB; i++)
#pragma unroll
    for (int j = 0; j < NB; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        int row = r0 + 16 * j + (lane & 15), col = c0 + 16 * i + (lane >> 4) + 4 * r;
        C[row + col * T] = acc[i][j][r];
        if (S) S[row + col * T] = (float)acc[i][j][r];
      }
}

// POTRF + TRTRI of one diagonal tile in LDS.
// Column-by-column right-looking Cholesky; then the inverse of the lower
// factor by forward substitution, one column per group of NT/T threads.
template <int T>
__device__ void task_potrf(const ExecMat& M, const int32_t* w, double* S, double* Xi, double* rinv) {
  constexpr int TT = T * T, G = NT / T;
  const int tid = threadIdx.x;
  double* C = M.tiles + (int64_t)w[1] * TT;
  const int k = w[2];
  for (int e = tid; e < TT; e += NT) {
    S[e] = C[e];
    Xi[e] = 0.0;
  }
  __syncthreads();
  int fail = -1;
  for (int j = 0; j < T; j++) {
    const double d = S[j + j * T];
    const double r = rsqrt_nr(d);
    if (!(d > 0.0) && fail < 0) fail = j;
    if (tid == 0) rinv[j] = r;
    if (tid > j && tid < T) S[tid + j * T] *= r;
    __syncthreads();
    if (tid == 0) S[j + j * T] = d * r;
    const int m = T - j - 1;
    for (int e = tid; e < m * m; e += NT) {
      const int i = j + 1 + e % m, c = j + 1 + e / m;
      if (c <= i) S[i + c * T] -= S[i + j * T] * S[c + j * T];
    }
    __syncthreads();
  }
  if (tid == 0 && fail >= 0) atomicMin(M.info, (unsigned long long)(M.row_base[k] + fail + 1));
  // inverse: column c by the G threads of one group, rows in sequence
  {
    const int c = tid / G, q = tid % G;
    if (c < T) {
      if (q == 0) Xi[c + c * T] = rinv[c];
      for (int i = c + 1; i < T; i++) {
        double s = 0.0;
        for (int kk = c + q; kk < i; kk += G) s += S[i + kk * T] * Xi[kk + c * T];
#pragma unroll
        for (int o = 1; o < G; o <<= 1) s += __shfl_xor(s, o, G);
        const double x = -s * rinv[i];
        if (q == 0) Xi[i + c * T] = x;
        // the group's lanes live in one wave; LDS accesses of a wave complete
        // in order, so only the compiler must not move the next reads up
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
  __syncthreads();
  double* Li = M.linv + (int64_t)k * TT;
  for (int e = tid; e < TT; e += NT) {
    const int row = e % T, col = e / T;
    C[e] = row >= col ? S[e] : 0.0;
    Li[e] = Xi[e];
  }
}

// ---------------------------------------------------------------- solves
// Vector blocks are T x nrhs column-major; thread (row = tid % T, group =
// tid / T) owns right-hand sides group, group + G, ...

template <int T>
__device__ void task_solve(const ExecMat& M, const int32_t* w, int nrhs) {
  constexpr int TT = T * T, G = NT / T, MAXC = 16 / G;
  const int type = __builtin_amdgcn_readfirstlane(w[0]) & 0xff;
  const int row = threadIdx.x % T, grp = threadIdx.x / T;
  const int m = w[1];
  const int64_t vb = (int64_t)T * nrhs;
  double acc[MAXC];
#pragma unroll
  for (int c = 0; c < MAXC; c++) acc[c] = 0.0;
  if (type == TK_FUPD) {
    for (int p = w[2]; p < w[3]; p++) {
      const double* L = M.tiles + (int64_t)M.pairs[2 * p] * TT;
      const double* y = M.vy + M.pairs[2 * p + 1] * vb;
      for (int l = 0; l < T; l++) {
        const double lv = L[row + l * T];
#pragma unroll
        for (int c = 0; c < MAXC; c++) {
          const int cc = grp + c * G;
          if (cc < nrhs) acc[c] += lv * y[l + cc * T];
        }
      }
    }
    double* ym = M.vy + m * vb;
#pragma unroll
    for (int c = 0; c < MAXC; c++) {
      const int cc = grp + c * G;
      if (cc < nrhs) ym[row + cc * T] -= acc[c];
    }
  } else if (type == TK_BUPD) {
    for (int p = w[2]; p < w[3]; p++) {
      const double* L = M.tiles + (int64_t)M.pairs[2 * p] * TT;
      const double* z = M.vz + M.pairs[2 * p + 1] * vb;
      for (int l = 0; l < T; l++) {
        const double lv = L[l + row * T];
#pragma unroll
        for (int c = 0; c < MAXC; c++) {
          const int cc = grp + c * G;
          if (cc < nrhs) acc[c] += lv * z[l + cc * T];
        }
      }
    }
    const double* src = (w[0] & TF_FIRST) ? M.vy + m * vb : M.vz + m * vb;
    double* zm = M.vz + m * vb;
#pragma unroll
    for (int c = 0; c < MAXC; c++) {
      const int cc = grp + c * G;
      if (cc < nrhs) zm[row + cc * T] = src[row + cc * T] - acc[c];
    }
  } else {
    // FDIAG: Y_m = Linv_m Y_m ; BDIAG: Z_m = Linv_m^T (Z_m or Y_m)
    const double* Li = M.linv + (int64_t)m * TT;
    const bool fwd = type == TK_FDIAG;
    const double* src = fwd ? M.vy + m * vb : ((w[0] & TF_FIRST) ? M.vy + m * vb : M.vz + m * vb);
    double* dst = fwd ? M.vy + m * vb : M.vz + m * vb;
    for (int l = 0; l < T; l++) {
      const double lv = fwd ? Li[row + l * T] : Li[l + row * T];
#pragma unroll
      for (int c = 0; c < MAXC; c++) {
        const int cc = grp + c * G;
        if (cc < nrhs) acc[c] += lv * src[l + cc * T];
      }
    }
    __syncthreads();   // all reads of src done before dst (== src for FDIAG) changes
#pragma unroll
    for (int c = 0; c < MAXC; c++) {
      const int cc = grp + c * G;
      if (cc < nrhs) dst[row + cc * T] = acc[c];
    }
  }
}

// ---------------------------------------------------------------- executor

template <int T>
__global__ __launch_bounds__(NT) void exec_kernel(const ExecMat* __restrict__ mats, const int32_t* __restrict__ order,
                                                  int32_t total, ExecCtrl* ctrl, int nrhs) {
  __shared__ double S[T * T];
  __shared__ double Xi[T * T];
  __shared__ double rinv[T];
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
    // wait until every predecessor has finished (Alg. 2 progress check)
    while (__builtin_amdgcn_readfirstlane(ld_relaxed(cnt)) > 0) __builtin_amdgcn_s_sleep(2);
    __syncthreads();
    if (threadIdx.x == 0) st_relaxed(cnt, w[7]);   // re-arm for the next launch
    fence_acquire();
    const int type = __builtin_amdgcn_readfirstlane(w[0]) & 0xff;
    switch (type) {
      case TK_UPD: task_update<T>(M, w, 0); break;
      case TK_PART: task_update<T>(M, w, 1); break;
      case TK_TREE: task_tree<T>(M, w); break;
      case TK_POTRF: task_potrf<T>(M, w, S, Xi, rinv); break;
      case TK_TRSM: task_trsm<T>(M, w); break;
      default: task_solve<T>(M, w, nrhs); break;
    }
    fence_release();
    __syncthreads();
    // notify successors (Alg. 2 progress update)
    const int32_t s0 = __builtin_amdgcn_readfirstlane(w[5]), s1 = __builtin_amdgcn_readfirstlane(w[6]);
    for (int32_t q0 = s0; q0 < s1; q0 += NT) {
      const int32_t q = q0 + (int32_t)threadIdx.x;
      if (q < s1) __hip_atomic_fetch_add(M.remaining + M.succ[q], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (threadIdx.x == 0) {
    const int e = atomicAdd(&ctrl->exited, 1);
    if (e == (int)gridDim.x - 1) {   // every other workgroup has left: re-arm
      ctrl->ticket = 0;
      ctrl->exited = 0;
    }
  }
}

hipError_t launch_exec(int T, const ExecMat* d_mats, const int32_t* d_order, int32_t total, ExecCtrl* d_ctrl, int nrhs,
                       int nwg, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  if (nwg > total) nwg = total;
  if (T == 64)
    hipLaunchKernelGGL(exec_kernel<64>, dim3(nwg), dim3(NT), 0, st, d_mats, d_order, total, d_ctrl, nrhs);
  else
    hipLaunchKernelGGL(exec_kernel<32>, dim3(nwg), dim3(NT), 0, st, d_mats, d_order, total, d_ctrl, nrhs);
  return hipGetLastError();
}

// ------------------------------------------------------------ value scatter

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
  const int m = trow[t], j = tcol[t];
  const int64_t rb = row_base[m], cb = row_base[j];
  const int rc = row_cnt[m], cc = row_cnt[j];
  for (int e = threadIdx.x; e < TT; e += NT) {
    const int r = e / T, c = e % T;   // row-wise: consecutive threads read consecutive values
    double v = 0.0;
    if (r < rc) {
      const int64_t i = rb + r, g = cb + c;
      const int64_t fi = f[i];
      if (c < cc && g <= i && g >= fi) v = vals[in_rp[i] + (g - fi)];
    } else if (m == j && r == c) {
      v = 1.0;   // padding row: unit diagonal
    }
    buf[r * (T + 1) + c] = v;
  }
  __syncthreads();
  double* out = tiles + t * TT;
  double* o2 = orig ? orig + t * TT : nullptr;
  for (int e = threadIdx.x; e < TT; e += NT) {
    const int c = e / T, r = e % T;   // column-major store
    const double v = buf[r * (T + 1) + c];
    out[e] = v;
    if (o2) o2[e] = v;
  }
  if (t == 0 && threadIdx.x == 0) *info = ~0ull;
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

hipError_t launch_extract(int T, const double* tiles, const int64_t* rp, const int64_t* f, const int32_t* trow,
                          const int32_t* tcol, const int64_t* row_base, const int32_t* row_cnt, int64_t ntiles,
                          double* out, hipStream_t st) {
  if (T == 64)
    hipLaunchKernelGGL(extract_kernel<64>, dim3((unsigned)ntiles), dim3(NT), 0, st, tiles, rp, f, trow, tcol, row_base,
                       row_cnt, out);
  else
    hipLaunchKernelGGL(extract_kernel<32>, dim3((unsigned)ntiles), dim3(NT), 0, st, tiles, rp, f, trow, tcol, row_base,
                       row_cnt, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ logdet

template <int T>
__global__ __launch_bounds__(NT) void logdet_partial_kernel(const double* __restrict__ tiles,
                                                            const int32_t* __restrict__ trow_ptr, double* part) {
  constexpr int TT = T * T;
  __shared__ double ws[NT / 64];
  const int m = blockIdx.x;
  const double* D = tiles + (int64_t)(trow_ptr[m + 1] - 1) * TT;
  double v = threadIdx.x < T ? log(D[threadIdx.x * (T + 1)]) : 0.0;
  // fixed-shape wave reduction, then waves in index order
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < NT / 64; q++) s += ws[q];
    part[m] = s;
  }
}

__global__ __launch_bounds__(NT) void logdet_final_kernel(const double* __restrict__ part, int32_t n,
                                                          const unsigned long long* info, double* out) {
  __shared__ double sh[NT];
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

hipError_t launch_logdet(int T, const double* tiles, const int32_t* trow_ptr, int32_t ntr, double* part,
                         const unsigned long long* info, double* out, hipStream_t st) {
  if (T == 64)
    hipLaunchKernelGGL(logdet_partial_kernel<64>, dim3(ntr), dim3(NT), 0, st, tiles, trow_ptr, part);
  else
    hipLaunchKernelGGL(logdet_partial_kernel<32>, dim3(ntr), dim3(NT), 0, st, tiles, trow_ptr, part);
  hipLaunchKernelGGL(logdet_final_kernel, dim3(1), dim3(NT), 0, st, part, ntr, info, out);
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

template <int T>
__global__ __launch_bounds__(NT) void residual_item_kernel(const double* __restrict__ orig,
                                                           const int32_t* __restrict__ trow,
                                                           const int32_t* __restrict__ tcol,
                                                           const int32_t* __restrict__ ccol_tile,
                                                           const int32_t* __restrict__ ccol_row,
                                                           const int32_t* __restrict__ items,
                                                           const double* __restrict__ X, double* part, int nrhs,
                                                           int absmode) {
  constexpr int TT = T * T, G = NT / T, MAXC = 16 / G;
  const int q = blockIdx.x;
  const int m = items[4 * q], kind = items[4 * q + 1], lo = items[4 * q + 2], hi = items[4 * q + 3];
  const int row = threadIdx.x % T, grp = threadIdx.x / T;
  const int64_t vb = (int64_t)T * nrhs;
  const int ncol = absmode ? 1 : nrhs;
  double acc[MAXC];
#pragma unroll
  for (int c = 0; c < MAXC; c++) acc[c] = 0.0;
  for (int e = lo; e < hi; e++) {
    int tile, src;
    if (kind == 0) { tile = e; src = tcol[e]; } else { tile = ccol_tile[e]; src = ccol_row[e]; }
    const double* A = orig + (int64_t)tile * TT;
    const double* x = X + src * vb;
    const bool dg = kind == 0 && src == m;
    for (int l = 0; l < T; l++) {
      double av;
      if (kind == 1) av = A[l + row * T];
      else if (dg) av = l <= row ? A[row + l * T] : A[l + row * T];
      else av = A[row + l * T];
      if (absmode) av = fabs(av);
#pragma unroll
      for (int c = 0; c < MAXC; c++) {
        const int cc = grp + c * G;
        if (cc < ncol) acc[c] += av * (absmode ? 1.0 : x[l + cc * T]);
      }
    }
  }
  double* out = part + (int64_t)q * vb;
#pragma unroll
  for (int c = 0; c < MAXC; c++) {
    const int cc = grp + c * G;
    if (cc < ncol) out[row + cc * T] = acc[c];
  }
}

__global__ void residual_combine_kernel(int T, const int32_t* __restrict__ item_ptr, const double* __restrict__ part,
                                        const double* __restrict__ B, double* R, int nrhs, int absmode) {
  const int m = blockIdx.x;
  const int64_t vb = (int64_t)T * nrhs;
  const int ncol = absmode ? 1 : nrhs;
  for (int e = threadIdx.x; e < T * ncol; e += blockDim.x) {
    double s = 0.0;
    for (int q = item_ptr[m]; q < item_ptr[m + 1]; q++) s += part[(int64_t)q * vb + e];
    R[m * vb + e] = absmode ? s : B[m * vb + e] - s;
  }
}

hipError_t launch_residual(int T, const double* orig, const int32_t* trow, const int32_t* tcol,
                           const int32_t* ccol_tile, const int32_t* ccol_row, const int32_t* items, int32_t nitems,
                           const int32_t* item_ptr, int32_t ntr, const double* X, const double* B, double* part,
                           double* R, int nrhs, int absmode, hipStream_t st) {
  if (T == 64)
    hipLaunchKernelGGL(residual_item_kernel<64>, dim3(nitems), dim3(NT), 0, st, orig, trow, tcol, ccol_tile, ccol_row,
                       items, X, part, nrhs, absmode);
  else
    hipLaunchKernelGGL(residual_item_kernel<32>, dim3(nitems), dim3(NT), 0, st, orig, trow, tcol, ccol_tile, ccol_row,
                       items, X, part, nrhs, absmode);
  hipLaunchKernelGGL(residual_combine_kernel, dim3(ntr), dim3(NT), 0, st, T, item_ptr, part, B, R, nrhs, absmode);
  return hipGetLastError();
}

__global__ void norms_kernel(int64_t n, int T, int nrhs, const double* __restrict__ R, const double* __restrict__ X,
                             unsigned long long* stats) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t vb = (int64_t)T * nrhs;
  const int c = (int)((e % vb) / T);
  const double r = fabs(R[e]), x = fabs(X[e]);
  // non-negative doubles order like their bit patterns
  atomicMax(stats + 2 * c, (unsigned long long)__double_as_longlong(r));
  atomicMax(stats + 2 * c + 1, (unsigned long long)__double_as_longlong(x));
}

hipError_t launch_norms(int T, int32_t ntr, int nrhs, const double* R, const double* X, unsigned long long* stats,
                        hipStream_t st) {
  const int64_t n = (int64_t)T * nrhs * ntr;
  hipLaunchKernelGGL(norms_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, T, nrhs, R, X, stats);
  return hipGetLastError();
}

__global__ void axpy_kernel(int64_t n, double* X, const double* __restrict__ D) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) X[e] += D[e];
}

hipError_t launch_axpy(int T, int32_t ntr, int nrhs, double* X, const double* D, hipStream_t st) {
  const int64_t n = (int64_t)T * nrhs * ntr;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, X, D);
  return hipGetLastError();
}

}  // namespace stiles
