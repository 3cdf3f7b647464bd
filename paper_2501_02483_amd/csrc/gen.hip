// gen.hip -- device-side synthetic inputs (separate library libstiles_gen.so).
//
// Holds none of the factorization's arithmetic: it only fills the value array
// of a band-plus-arrow envelope (row-profile order, see include/stiles.h) with
// seeded off-diagonal values and a dominant diagonal, so that serving
// workloads can draw fresh matrices per request without host generation and
// transfers.  Off-diagonal entry number q (0-based, in row-profile order,
// diagonals skipped) gets the q-th standard normal of the stream
//   (u1, u2) = Philox4x32-10(key = seed, counter = q / 2)  (Salmon et al., SC'11)
//   z = sqrt(-2 ln u1) * (cos, sin)(2 pi u2)                 (Box-Muller)
// and the diagonal is the absolute sum of the full symmetric row plus one
// (or plus eps for the Laplacian law with -|z| off-diagonals).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox_round(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
  U4 r;
  r.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
  r.y = (uint32_t)p1;
  r.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
  r.w = (uint32_t)p0;
  return r;
}

__device__ __forceinline__ U4 philox10(uint64_t ctr, uint64_t key) {
  U4 c{(uint32_t)ctr, (uint32_t)(ctr >> 32), 0u, 0u};
  uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
  for (int i = 0; i < 10; i++) {
    c = philox_round(c, k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ double normal_at(uint64_t q, uint64_t seed) {
  const U4 r = philox10(q >> 1, seed);
  // 53-bit uniforms in (0, 1]
  const double u1 = ((double)(((uint64_t)r.x << 21) ^ (r.y >> 11)) + 1.0) * (1.0 / 9007199254740992.0);
  const double u2 = ((double)(((uint64_t)r.z << 21) ^ (r.w >> 11))) * (1.0 / 9007199254740992.0);
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;
  return (q & 1) ? rad * sin(ang) : rad * cos(ang);
}

// one block per row: off-diagonal values and |row part| sum
__global__ void gen_rows(const int64_t* __restrict__ rp, const int64_t* __restrict__ f, int64_t N, uint64_t seed,
                         int laplacian, double* v, double* rowsum) {
  const int64_t i = blockIdx.x;
  const int64_t b = rp[i], len = i - f[i];   // off-diagonal count of row i
  const int64_t q0 = b - i;                  // off-diagonals before row i
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < len; e += blockDim.x) {
    double z = normal_at((uint64_t)(q0 + e), seed);
    if (laplacian) z = -fabs(z);
    v[b + e] = z;
    s += fabs(z);
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) rowsum[i] = sh[0];
}

// one thread per column j: |column part| sum over rows i > j with f_i <= j;
// rows are scanned in [j+1, min(N, j+1+wmax)) plus the dense rows from full0
__global__ void gen_cols(const int64_t* __restrict__ rp, const int64_t* __restrict__ f, int64_t N, int64_t wmax,
                         int64_t full0, const double* __restrict__ v, double* colsum) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double s = 0.0;
  const int64_t hi = j + 1 + wmax < full0 ? j + 1 + wmax : full0;
  for (int64_t i = j + 1; i < hi; i++)
    if (f[i] <= j) s += fabs(v[rp[i] + (j - f[i])]);
  for (int64_t i = (full0 > j + 1 ? full0 : j + 1); i < N; i++)
    if (f[i] <= j) s += fabs(v[rp[i] + (j - f[i])]);
  colsum[j] = s;
}

__global__ void gen_diag(const int64_t* __restrict__ rp, int64_t N, const double* __restrict__ rowsum,
                         const double* __restrict__ colsum, double shift, double* v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) v[rp[i + 1] - 1] = rowsum[i] + colsum[i] + shift;
}

}  // namespace

extern "C" {

// Fill d_v (row-profile values of the envelope d_rp/d_f, N rows) with seeded
// off-diagonals (law 0: N(0,1); law 1: -|N(0,1)|) and write the absolute row
// and column-part sums to d_tmp[0..N) and d_tmp[N..2N).  wmax: max over rows
// with f > 0 of i - f_i; full0: first row index from which all rows are dense
// (the arrow).  Returns a hipError_t code.
int stiles_gen_offdiag(const int64_t* d_rp, const int64_t* d_f, int64_t N, int64_t wmax, int64_t full0, uint64_t seed,
                       int32_t law, double* d_v, double* d_tmp, hipStream_t st) {
  if (N <= 0) return 0;
  hipLaunchKernelGGL(gen_rows, dim3((unsigned)N), dim3(256), 0, st, d_rp, d_f, N, seed, law, d_v, d_tmp);
  hipLaunchKernelGGL(gen_cols, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, d_rp, d_f, N, wmax, full0, d_v,
                     d_tmp + N);
  return (int)hipGetLastError();
}

// diagonal_i = row sum + column sum + shift (after stiles_gen_offdiag)
int stiles_gen_diag(const int64_t* d_rp, int64_t N, const double* d_tmp, double shift, double* d_v, hipStream_t st) {
  if (N <= 0) return 0;
  hipLaunchKernelGGL(gen_diag, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, d_rp, N, d_tmp, d_tmp + N, shift,
                     d_v);
  return (int)hipGetLastError();
}

}  // extern "C"
