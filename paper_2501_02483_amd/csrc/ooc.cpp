// ooc.cpp -- out-of-core (streamed) factorization of a band-plus-arrow
// envelope whose factor does not fit in device memory at once (the paper
// names handling matrices beyond device memory as future work for its GPU
// path, Sections IV-B and VI).
//
// The band rows are cut into consecutive segments.  Segment k is factored
// in core as an arrowhead matrix of its own, M_k: its band part is the
// segment's rows followed by the rows of the next segment that couple back
// into segment k (the interface, each row with its own profile), its arrow
// the true arrow.  The segment's rows of M_k's factor and the interface and
// arrow rows' entries in the segment's columns are final entries of L
// (block Cholesky: eliminating the segment's columns does not depend on
// anything after them).  Its trailing block (interface and arrow rows and
// columns) factors the Schur complement S_k of the segment, so S_k = Lc Lc^T
// with Lc that block of M_k's factor (a device kernel); S_k replaces the
// interface block, the arrow rows' interface columns and the arrow corner
// in M_(k+1).  The last segment has no interface; its trailing block is the
// final factor of the arrow corner.  Only one segment's matrix, factor and
// Schur complement are resident at a time; factors stream back to host
// memory.  The log-determinant is accumulated on the device, segment by
// segment, over the rows whose factor is final.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "launch.h"
#include "symbolic.h"

using namespace stiles;

namespace {

// device buffer that grows on demand (freed with the call)
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  bool reserve(size_t bytes) {
    if (bytes <= n) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) { p = nullptr; return false; }
    n = std::max<size_t>(bytes, 256);
    return true;
  }
  ~DevBuf() { if (p) (void)hipFree(p); }
  template <typename E>
  E* as() const { return static_cast<E*>(p); }
};

// f(lo, hi) over [0, n) in contiguous chunks on up to 16 host threads (the
// caller's thread takes the first chunk, and any chunk no thread could be
// started for); every chunk writes its own rows
template <typename F>
void parallel_rows(int64_t n, F&& f) {
  const unsigned hc = std::thread::hardware_concurrency();
  const int64_t T = std::min<int64_t>({(int64_t)std::clamp(hc, 1u, 16u), n / 16, (int64_t)16});
  if (T <= 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t started = 1;
  try {
    th.reserve((size_t)T - 1);
    for (int64_t t = 1; t < T; t++) {
      th.emplace_back([&f, n, t, T] { f(n * t / T, n * (t + 1) / T); });
      started = t + 1;
    }
  } catch (...) {
  }
  f((int64_t)0, n / T);
  for (int64_t t = started; t < T; t++) f(n * t / T, n * (t + 1) / T);
  for (auto& x : th) x.join();
}

}  // namespace

extern "C" stiles_status stiles_factorize_ooc(int64_t n, int64_t a, const int64_t* first_col, const double* h_values,
                                              int64_t seg_rows, int32_t tile, double* h_L, double* logdet,
                                              int64_t* info, size_t* peak_device_bytes, hipStream_t st) {
  set_error_arg(0);
  if (n < 1) { set_error_arg(1); return STILES_EINVAL; }
  if (a < 0) { set_error_arg(2); return STILES_EINVAL; }
  if (!first_col) { set_error_arg(3); return STILES_EINVAL; }
  for (int64_t i = 0; i < n; i++)
    if (first_col[i] < 0 || first_col[i] > i) { set_error_arg(3); return STILES_EINVAL; }
  if (!h_values) { set_error_arg(4); return STILES_EINVAL; }
  if (seg_rows < 1) { set_error_arg(5); return STILES_EINVAL; }
  if (tile != 0 && tile != 32 && tile != 64) { set_error_arg(6); return STILES_ENOTSUP; }
  if (!h_L) { set_error_arg(7); return STILES_EINVAL; }
  if (!logdet) { set_error_arg(8); return STILES_EINVAL; }
  if (!info) { set_error_arg(9); return STILES_EINVAL; }
  const int64_t N = n + a;
  std::vector<int64_t> rpA(N + 1, 0);
  for (int64_t i = 0; i < N; i++) rpA[i + 1] = rpA[i] + (i - (i < n ? first_col[i] : 0) + 1);
  auto fA = [&](int64_t i) { return i < n ? first_col[i] : (int64_t)0; };
  auto A = [&](int64_t i, int64_t j) { return j >= fA(i) ? h_values[rpA[i] + j - fA(i)] : 0.0; };
  // segment boundaries and interfaces: rows >= s_(k+1) that couple to a
  // column before it, a range [s_(k+1), e_(k+1)) inside the next segment
  std::vector<int64_t> sb{0}, eb{0};
  while (sb.back() < n) sb.push_back(std::min(n, sb.back() + seg_rows));
  const int m = (int)sb.size() - 1;
  eb.assign(sb.size(), 0);
  for (int k = 1; k < m; k++) {
    int64_t e = sb[k];
    for (int64_t i = sb[k]; i < n; i++)
      if (first_col[i] < sb[k]) e = i + 1;
    if (e > sb[k + 1]) { set_error_arg(5); return STILES_EINVAL; }   // segments narrower than the band
    eb[k] = e;
  }
  *info = 0;
  *logdet = 0.0;
  size_t peak = 0;
  DevBuf ws, vals, lbuf, rpb, fb, sbuf, acc;
  const double zero = 0.0;
  if (!acc.reserve(8) || hipMemcpyAsync(acc.p, &zero, 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return STILES_EDEVICE;
  std::vector<double> S_prev, hM, vM;
  int64_t c_prev = 0, ni_prev = 0;
  stiles_opts o;
  stiles_default_opts(&o);
  o.tile = tile;
  o.ordering = STILES_ORDER_NONE;
  // M_k's profile and its symbolic analysis (host only, independent of the
  // values): band rows from the segment and the interface rows (each from
  // its first column in A, which is not before s0), the arrow rows dense.
  // An interface row starts at the segment's last column at the latest (a
  // row of the range that does not couple back then holds one explicit zero
  // there), so that every row of the trailing block covers all of its
  // columns, as the Gram kernel reads them.  The analysis of segment k + 1
  // runs on a helper thread while segment k is assembled and factored.
  struct Seg {
    std::vector<int64_t> fM, rpM;
    stiles_symbolic* sym = nullptr;
    stiles_status status = STILES_OK;
    ~Seg() { if (sym) stiles_symbolic_destroy(sym); }
  };
  auto prepare = [&](int k, Seg& g) {
    const int64_t s0 = sb[k], s1 = sb[k + 1];
    const int64_t nb = s1 - s0, ni = k + 1 < m ? eb[k + 1] - s1 : 0, Nk = nb + ni + a;
    g.fM.assign(Nk, 0);
    g.rpM.assign(Nk + 1, 0);
    for (int64_t r = 0; r < nb; r++) g.fM[r] = std::max(first_col[s0 + r], s0) - s0;
    for (int64_t ii = 0; ii < ni; ii++) g.fM[nb + ii] = std::min(first_col[s1 + ii] - s0, nb - 1);
    for (int64_t r = 0; r < Nk; r++) g.rpM[r + 1] = g.rpM[r] + (r - g.fM[r] + 1);
    g.status = stiles_analyze_profile(nb + ni, a, g.fM.data(), &o, &g.sym);
  };
  std::unique_ptr<Seg> cur(new Seg), nxt;
  prepare(0, *cur);
  for (int k = 0; k < m; k++) {
    const int64_t s0 = sb[k], s1 = sb[k + 1];
    const int64_t nb = s1 - s0, ni = k + 1 < m ? eb[k + 1] - s1 : 0, Nk = nb + ni + a;
    const bool last = k + 1 == m;
    nxt.reset(last ? nullptr : new Seg);
    std::thread helper;
    if (nxt) {
      try {
        helper = std::thread(prepare, k + 1, std::ref(*nxt));
      } catch (...) {
        prepare(k + 1, *nxt);
      }
    }
    struct Join {
      std::thread& t;
      ~Join() { if (t.joinable()) t.join(); }
    } join{helper};
    const std::vector<int64_t>& fM = cur->fM;
    const std::vector<int64_t>& rpM = cur->rpM;
    vM.assign(rpM[Nk], 0.0);
    // values: the original entries, except the previous segment's Schur
    // complement on its interface block, the arrow rows' interface columns
    // and the arrow corner
    auto Sp = [&](int64_t i, int64_t j) { return S_prev[(size_t)i * c_prev + j]; };
    parallel_rows(nb, [&](int64_t lo, int64_t hi) {
      for (int64_t r = lo; r < hi; r++) {
        const int64_t i = s0 + r;
        for (int64_t cM = fM[r]; cM <= r; cM++) {
          const int64_t gc = s0 + cM;
          vM[rpM[r] + cM - fM[r]] = (k > 0 && i < eb[k] && gc < eb[k]) ? Sp(i - s0, gc - s0) : A(i, gc);
        }
      }
    });
    parallel_rows(ni, [&](int64_t lo, int64_t hi) {
      for (int64_t ii = lo; ii < hi; ii++) {
        const int64_t i = s1 + ii, r = nb + ii;
        for (int64_t cM = fM[r]; cM <= r; cM++) vM[rpM[r] + cM - fM[r]] = A(i, cM < nb ? s0 + cM : s1 + (cM - nb));
      }
    });
    parallel_rows(a, [&](int64_t lo, int64_t hi) {
      for (int64_t t = lo; t < hi; t++) {
        const int64_t r = nb + ni + t;
        for (int64_t cM = 0; cM <= r; cM++) {
          double v;
          if (cM < nb) {
            const int64_t gc = s0 + cM;
            v = (k > 0 && gc < eb[k]) ? Sp(ni_prev + t, gc - s0) : A(n + t, gc);
          } else if (cM < nb + ni) {
            v = A(n + t, s1 + (cM - nb));
          } else {
            const int64_t u = cM - nb - ni;
            v = k > 0 ? Sp(ni_prev + t, ni_prev + u) : A(n + t, n + u);
          }
          vM[rpM[r] + cM] = v;
        }
      }
    });
    // in-core factorization of M_k
    stiles_symbolic* sym = cur->sym;
    stiles_status r = cur->status;
    if (r != STILES_OK) return r;
    size_t wsb = 0;
    r = stiles_workspace_size(sym, STILES_FP64, 1, &wsb);
    const size_t nnz = (size_t)rpM[Nk], c = (size_t)(ni + a);
    const size_t need = wsb + nnz * 16 + (size_t)(Nk + 1) * 8 + (size_t)Nk * 8 + (last ? 0 : c * c * 8) + 8;
    if (r != STILES_OK || !ws.reserve(wsb) || !vals.reserve(nnz * 8) || !lbuf.reserve(nnz * 8) ||
        !rpb.reserve((Nk + 1) * 8) || !fb.reserve(Nk * 8) || (!last && !sbuf.reserve(c * c * 8)))
      return r != STILES_OK ? r : STILES_EDEVICE;
    peak = std::max(peak, need);
    stiles_factor* fac = nullptr;
    r = stiles_workspace_init(sym, STILES_FP64, 1, ws.p, ws.n, st, &fac);
    hipError_t e = hipSuccess;
    int64_t inf = 0;
    if (r == STILES_OK) {
      e = hipMemcpyAsync(vals.p, vM.data(), nnz * 8, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) r = stiles_factorize(fac, vals.as<double>(), st);
      if (r == STILES_OK && e == hipSuccess) r = stiles_factor_info(fac, st, &inf);
      if (r == STILES_OK && inf == 0) r = stiles_factor_extract(fac, lbuf.as<double>(), st);
    }
    // the symbolic object's tables were uploaded asynchronously
    if (hipStreamSynchronize(st) != hipSuccess) e = hipErrorUnknown;
    if (fac) stiles_factor_release(fac);
    if (e != hipSuccess) return STILES_EDEVICE;
    if (r != STILES_OK) return r;
    if (inf > 0) {
      // first failing pivot, in the numbering of A
      const int64_t q = inf - 1;
      *info = 1 + (q < nb ? s0 + q : q < nb + ni ? s1 + (q - nb) : n + (q - nb - ni));
      *logdet = NAN;
      if (peak_device_bytes) *peak_device_bytes = peak;
      return STILES_OK;
    }
    // Schur complement of the segment and the final rows' log-determinant,
    // on the device; the factor streams back to host memory
    hM.resize(nnz);
    e = hipMemcpyAsync(rpb.p, rpM.data(), (Nk + 1) * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(fb.p, fM.data(), Nk * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !last)
      e = launch_gram_lower((int32_t)c, lbuf.as<double>(), rpb.as<int64_t>(), fb.as<int64_t>(), nb, nb,
                            sbuf.as<double>(), st);
    if (e == hipSuccess)
      e = launch_logdet_rows(lbuf.as<double>(), rpb.as<int64_t>(), 0, last ? Nk : nb, acc.as<double>(), st);
    if (e == hipSuccess) e = hipMemcpyAsync(hM.data(), lbuf.p, nnz * 8, hipMemcpyDeviceToHost, st);
    std::vector<double> S;
    if (e == hipSuccess && !last) {
      S.assign(c * c, 0.0);
      e = hipMemcpyAsync(S.data(), sbuf.p, c * c * 8, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return STILES_EDEVICE;
    // final entries of L in the numbering and row-profile order of A
    parallel_rows(nb, [&](int64_t lo, int64_t hi) {
      for (int64_t rr = lo; rr < hi; rr++) {
        const int64_t i = s0 + rr;
        for (int64_t cM = fM[rr]; cM <= rr; cM++) h_L[rpA[i] + (s0 + cM) - fA(i)] = hM[rpM[rr] + cM - fM[rr]];
      }
    });
    parallel_rows(ni, [&](int64_t lo, int64_t hi) {
      for (int64_t ii = lo; ii < hi; ii++) {
        const int64_t i = s1 + ii, rr = nb + ii;
        for (int64_t cM = std::max(fM[rr], first_col[i] - s0); cM < nb; cM++)
          h_L[rpA[i] + (s0 + cM) - first_col[i]] = hM[rpM[rr] + cM - fM[rr]];
      }
    });
    parallel_rows(a, [&](int64_t lo, int64_t hi) {
      for (int64_t t = lo; t < hi; t++) {
        const int64_t rr = nb + ni + t;
        for (int64_t cM = 0; cM < nb; cM++) h_L[rpA[n + t] + s0 + cM] = hM[rpM[rr] + cM];
        if (last)
          for (int64_t u = 0; u <= t; u++) h_L[rpA[n + t] + n + u] = hM[rpM[rr] + nb + u];
      }
    });
    S_prev.swap(S);
    c_prev = (int64_t)c;
    ni_prev = ni;
    if (helper.joinable()) helper.join();
    cur = std::move(nxt);
  }
  if (hipMemcpyAsync(logdet, acc.p, 8, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return STILES_EDEVICE;
  if (peak_device_bytes) *peak_device_bytes = peak;
  return STILES_OK;
}
