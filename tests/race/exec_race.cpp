// Threaded host emulation of the persistent executor's protocol, for
// ThreadSanitizer.  Worker threads take tickets in the plan's static order,
// wait on per-task counters (two-stage for TF_SPLIT tasks: the early
// predecessors, which weigh 2^16, then the late one), run the task on host
// tiles and notify the successors (an entry with bit 30 set subtracts 2^16)
// -- the counter protocol of the device executor with C++ acquire/release
// atomics in place of the device's coherent stores and fences.  A missing
// dependency in the plan, or a task that reads before its wait, is a data
// race between the tile accesses of two tasks, which ThreadSanitizer
// reports; random delays vary the interleavings.  Task semantics are those
// of the device task bodies (factorization DAG: UPD, PART, TREE, POTRF,
// TRSM, UPDB; merged factorization + solve DAG: also FUPD, FPART, FSUM,
// FDIAG, BUPD, BDIAG), written here as plain loops.  In the merged DAG a
// solve task first waits for its factorization predecessors (weight 2^16)
// and reads its factor tiles, then for its solve predecessors; a two-stage
// diagonal step waits for its early solve predecessors (weight 2^8, entries
// with bit 29), reads its right-hand side block and the first fused
// product's block, then waits for the last one.
//
// Input (binary, little-endian int32 header then arrays):
//   T, ntiles, ntr, ntasks, nsucc, npairw (int32 words of the pair array),
//   npart; tasks (8 int32 per task), succ, pair words, tiles (ntiles T x T
//   column-major doubles); for a merged DAG then nrhs (int32) and the
//   right-hand side blocks (ntr blocks of T x nrhs column-major doubles).
//   Output: the tiles, then (merged DAG) the solution blocks.
// Usage: exec_race <in> <out> <threads> <seed> [drop_edge]
//   out receives the factored tiles; drop_edge removes one successor entry
//   (and its weight from the successor's counter) to plant a missing
//   dependency; the task that lost the edge then starts 20 ms late, so that
//   its former successor runs first in every interleaving.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

namespace {

constexpr int TK_UPD = 1, TK_PART = 2, TK_TREE = 3, TK_POTRF = 4, TK_TRSM = 5, TK_UPDB = 6;
constexpr int TK_FUPD = 8, TK_FDIAG = 9, TK_BUPD = 10, TK_BDIAG = 11, TK_FPART = 12, TK_FSUM = 13;
constexpr int TF_DIAG = 1 << 8, TF_FIRST = 1 << 9, TF_ACC = 1 << 10, TF_SPLIT = 1 << 11;
constexpr int32_t W = 1 << 16, FDEP = 1 << 30, WMID = 1 << 8, MID = 1 << 29;

struct Plan {
  int32_t T = 0, ntiles = 0, ntr = 0, ntasks = 0, nsucc = 0, npairw = 0, npart = 0, nrhs = 0;
  std::vector<int32_t> tasks, succ, pairs;
  std::vector<double> tiles, y;
};

bool read_plan(const char* path, Plan& p) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  int32_t h[7];
  bool ok = std::fread(h, 4, 7, f) == 7;
  if (ok) {
    p.T = h[0]; p.ntiles = h[1]; p.ntr = h[2]; p.ntasks = h[3]; p.nsucc = h[4]; p.npairw = h[5]; p.npart = h[6];
    p.tasks.resize((size_t)p.ntasks * 8);
    p.succ.resize(p.nsucc);
    p.pairs.resize(p.npairw);
    p.tiles.resize((size_t)p.ntiles * p.T * p.T);
    ok = std::fread(p.tasks.data(), 4, p.tasks.size(), f) == p.tasks.size() &&
         std::fread(p.succ.data(), 4, p.succ.size(), f) == p.succ.size() &&
         std::fread(p.pairs.data(), 4, p.pairs.size(), f) == p.pairs.size() &&
         std::fread(p.tiles.data(), 8, p.tiles.size(), f) == p.tiles.size();
  }
  int32_t nrhs = 0;
  if (ok && std::fread(&nrhs, 4, 1, f) == 1 && nrhs > 0) {
    p.nrhs = nrhs;
    p.y.resize((size_t)p.ntr * p.T * nrhs);
    ok = std::fread(p.y.data(), 8, p.y.size(), f) == p.y.size();
  }
  std::fclose(f);
  return ok;
}

struct Exec {
  Plan& p;
  std::vector<double> linv, part, z, q;
  std::vector<std::atomic<int32_t>> cnt;
  std::atomic<int32_t> ticket{0};
  std::atomic<bool> failed{false};
  explicit Exec(Plan& pl)
      : p(pl), linv((size_t)pl.ntr * pl.T * pl.T), part((size_t)std::max(pl.npart, 1) * pl.T * pl.T), cnt(pl.ntasks) {
    for (int32_t t = 0; t < pl.ntasks; t++) cnt[t].store(pl.tasks[(size_t)t * 8 + 7], std::memory_order_relaxed);
    if (pl.nrhs > 0) {
      int32_t nq = 1;
      for (int32_t t = 0; t < pl.ntasks; t++)
        if ((pl.tasks[(size_t)t * 8] & 0xff) == TK_FPART) nq = std::max(nq, pl.tasks[(size_t)t * 8 + 4] + 1);
      z.assign(pl.y.size(), 0.0);
      q.assign((size_t)nq * pl.T * pl.nrhs, 0.0);
    }
  }
  double* tile(int32_t id) { return p.tiles.data() + (size_t)id * p.T * p.T; }
  double* slot(int32_t id) { return part.data() + (size_t)id * p.T * p.T; }
  size_t vb() const { return (size_t)p.T * p.nrhs; }
  double* yb(int32_t m) { return p.y.data() + (size_t)m * vb(); }
  double* zb(int32_t m) { return z.data() + (size_t)m * vb(); }
  double* qb(int32_t s) { return q.data() + (size_t)s * vb(); }
  // v -= op(L) x (op = transpose when `trans`), x and v T x nrhs blocks
  void sub_mv(double* v, const double* L, const double* x, bool trans) {
    const int T = p.T;
    for (int c = 0; c < p.nrhs; c++)
      for (int r = 0; r < T; r++) {
        double s = 0.0;
        for (int k = 0; k < T; k++) s += (trans ? L[k + r * T] : L[r + k * T]) * x[k + c * T];
        v[r + c * T] -= s;
      }
  }
  // C -= X Y^T (lower only when `lower`)
  void sub_prod(double* C, const double* X, const double* Y, bool lower) {
    const int T = p.T;
    for (int c = 0; c < T; c++)
      for (int r = lower ? c : 0; r < T; r++) {
        double s = 0.0;
        for (int k = 0; k < T; k++) s += X[r + k * T] * Y[c + k * T];
        C[r + c * T] -= s;
      }
  }
  void wait_below(int32_t t, int32_t bound, std::mt19937& rng) {
    int spins = 0;
    while (cnt[t].load(std::memory_order_acquire) >= bound) {
      if (++spins > 64) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 20));
      else std::this_thread::yield();
      if (failed.load(std::memory_order_relaxed)) return;
    }
  }
  int32_t slow_task = -1;   // the source of a planted missing edge
  void run_task(int32_t t, std::mt19937& rng) {
    if (t == slow_task) std::this_thread::sleep_for(std::chrono::milliseconds(20));
    const int32_t* w = &p.tasks[(size_t)t * 8];
    const int type = w[0] & 0xff, T = p.T;
    const bool split = (w[0] & TF_SPLIT) != 0;
    std::vector<double> C((size_t)T * T);
    if (type == TK_POTRF || type == TK_TRSM) {
      wait_below(t, split ? W : 1, rng);
      std::memcpy(C.data(), tile(w[1]), C.size() * 8);   // its own tile: an early input
      if (type == TK_TRSM)                                  // fused products: early inputs
        for (int32_t q = w[3]; q < w[4]; q++) sub_prod(C.data(), tile(p.pairs[2 * q]), tile(p.pairs[2 * q + 1]), false);
      if (split) wait_below(t, 1, rng);
      if (type == TK_POTRF) {
        for (int32_t q = w[3]; q < w[4]; q++) sub_prod(C.data(), tile(p.pairs[2 * q]), tile(p.pairs[2 * q + 1]), true);
        // Cholesky of the lower triangle, then the inverse of the factor
        for (int j = 0; j < T; j++) {
          double d = C[j + j * T];
          for (int k = 0; k < j; k++) d -= C[j + k * T] * C[j + k * T];
          if (!(d > 0.0)) { failed.store(true); return; }
          const double l = std::sqrt(d);
          C[j + j * T] = l;
          for (int i = j + 1; i < T; i++) {
            double s = C[i + j * T];
            for (int k = 0; k < j; k++) s -= C[i + k * T] * C[j + k * T];
            C[i + j * T] = s / l;
          }
        }
        for (int c = 0; c < T; c++)
          for (int r = 0; r < c; r++) C[r + c * T] = 0.0;
        double* Li = linv.data() + (size_t)w[2] * T * T;
        for (int c = 0; c < T; c++)
          for (int r = 0; r < T; r++) {
            if (r < c) { Li[r + c * T] = 0.0; continue; }
            double s = r == c ? 1.0 : 0.0;
            for (int k = c; k < r; k++) s -= C[r + k * T] * Li[k + c * T];
            Li[r + c * T] = s / C[r + r * T];
          }
      } else {
        const double* Li = linv.data() + (size_t)w[2] * T * T;
        std::vector<double> out((size_t)T * T, 0.0);
        for (int c = 0; c < T; c++)
          for (int r = 0; r < T; r++) {
            double s = 0.0;
            for (int k = 0; k < T; k++) s += C[r + k * T] * Li[c + k * T];
            out[r + c * T] = s;
          }
        C.swap(out);
      }
      std::memcpy(tile(w[1]), C.data(), C.size() * 8);
      return;
    }
    if (type >= TK_FUPD) {
      run_solve(t, w, type, rng);
      return;
    }
    wait_below(t, 1, rng);
    if (type == TK_UPD) {
      for (int32_t q = w[2]; q < w[3]; q++)
        sub_prod(tile(w[1]), tile(p.pairs[2 * q]), tile(p.pairs[2 * q + 1]), (w[0] & TF_DIAG) != 0);
    } else if (type == TK_PART) {
      std::fill(C.begin(), C.end(), 0.0);
      for (int32_t q = w[2]; q < w[3]; q++) sub_prod(C.data(), tile(p.pairs[2 * q]), tile(p.pairs[2 * q + 1]), false);
      double* P = slot(w[4]);
      for (size_t e = 0; e < C.size(); e++) P[e] = (w[0] & TF_ACC) ? P[e] - C[e] : -C[e];
    } else if (type == TK_TREE) {
      const double* a = slot(w[2]);
      const double* b = w[3] >= 0 ? slot(w[3]) : nullptr;
      double* dst = w[4] >= 0 ? slot(w[4]) : tile(w[1]);
      for (size_t e = 0; e < C.size(); e++) {
        const double s = a[e] + (b ? b[e] : 0.0);
        dst[e] = w[4] >= 0 ? s : dst[e] - s;
      }
    } else if (type == TK_UPDB) {
      const int32_t* words = &p.pairs[2 * (size_t)w[2]];
      const int32_t nj = w[3];
      for (int q = 0; q < 4; q++) {
        if (words[q] < 0) continue;
        const bool lower = (w[0] & TF_DIAG) && q != 1;
        for (int32_t j = 0; j < nj; j++) {
          const int32_t* o = words + 4 + 4 * j;
          if (o[q & 1] < 0 || o[2 + (q >> 1)] < 0) continue;
          sub_prod(tile(words[q]), tile(o[q & 1]), tile(o[2 + (q >> 1)]), lower);
        }
      }
    } else {
      std::fprintf(stderr, "exec_race: unknown task type %d\n", type);
      failed.store(true);
    }
  }
  // merged DAG solve task: factor tiles after the factorization predecessors
  // (counter below 2^16), vector blocks after the solve predecessors
  void run_solve(int32_t t, const int32_t* w, int type, std::mt19937& rng) {
    const int T = p.T, m = w[1];
    const size_t TT = (size_t)T * T, nb = vb();
    wait_below(t, W, rng);
    std::vector<double> Ls;   // the factor tiles this task reads, copied now
    const int np = type == TK_FSUM ? 0 : w[3] - w[2];
    for (int k = 0; k < np; k++) Ls.insert(Ls.end(), tile(p.pairs[2 * (w[2] + k)]), tile(p.pairs[2 * (w[2] + k)]) + TT);
    const bool diag = type == TK_FDIAG || type == TK_BDIAG, fwd = type == TK_FUPD || type == TK_FDIAG || type == TK_FPART;
    std::vector<double> Li;
    if (diag) Li.assign(linv.data() + (size_t)m * TT, linv.data() + (size_t)(m + 1) * TT);
    auto blk = [&](int k) { const int32_t b = p.pairs[2 * (w[2] + k) + 1]; return fwd ? yb(b) : zb(b); };
    std::vector<double> v(nb, 0.0);
    int k0 = 0;
    if (diag && (w[0] & TF_SPLIT)) {
      wait_below(t, WMID, rng);   // early solve predecessors
      const double* base = fwd ? yb(m) : ((w[0] & TF_FIRST) ? yb(m) : zb(m));
      std::memcpy(v.data(), base, nb * 8);
      sub_mv(v.data(), Ls.data(), blk(0), !fwd);
      k0 = 1;
      wait_below(t, 1, rng);      // the previous step of the chain
    } else {
      wait_below(t, 1, rng);
      if (type != TK_FPART && type != TK_FSUM) {
        const double* base = fwd ? yb(m) : ((w[0] & TF_FIRST) ? yb(m) : zb(m));
        std::memcpy(v.data(), base, nb * 8);
      } else if (type == TK_FSUM) {
        std::memcpy(v.data(), yb(m), nb * 8);
      }
    }
    if (type == TK_FSUM) {
      for (int32_t s = w[2]; s < w[3]; s++)
        for (size_t e = 0; e < nb; e++) v[e] -= qb(s)[e];
      std::memcpy(yb(m), v.data(), nb * 8);
      return;
    }
    for (int k = k0; k < np; k++) sub_mv(v.data(), Ls.data() + (size_t)k * TT, blk(k), !fwd);
    if (type == TK_FPART) {
      for (size_t e = 0; e < nb; e++) qb(w[4])[e] = -v[e];
      return;
    }
    if (diag) {
      std::vector<double> out(nb, 0.0);
      sub_mv(out.data(), Li.data(), v.data(), !fwd);   // out = -op(Linv) v
      for (size_t e = 0; e < nb; e++) out[e] = -out[e];
      std::memcpy(fwd ? yb(m) : zb(m), out.data(), nb * 8);
      return;
    }
    std::memcpy(fwd ? yb(m) : zb(m), v.data(), nb * 8);
  }
  void worker(unsigned seed) {
    std::mt19937 rng(seed);
    for (;;) {
      const int32_t t = ticket.fetch_add(1, std::memory_order_relaxed);
      if (t >= p.ntasks || failed.load(std::memory_order_relaxed)) break;
      run_task(t, rng);
      if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
      const int32_t* w = &p.tasks[(size_t)t * 8];
      for (int32_t q = w[5]; q < w[6]; q++) {
        const int32_t v = p.succ[q];
        if (v == -1) continue;   // a planted missing edge
        cnt[v & ~(FDEP | MID)].fetch_sub((v & FDEP) ? W : (v & MID) ? WMID : 1, std::memory_order_release);
      }
    }
  }
};

}  // namespace

int main(int argc, char** argv) {
  if (argc < 5) {
    std::fprintf(stderr, "usage: exec_race in out threads seed [drop_edge]\n");
    return 2;
  }
  Plan p;
  if (!read_plan(argv[1], p)) {
    std::fprintf(stderr, "exec_race: cannot read %s\n", argv[1]);
    return 2;
  }
  if (argc > 5) {
    // plant a missing dependency: the successor no longer waits for it
    const int32_t e = std::atoi(argv[5]);
    const int32_t v = p.succ[e];
    p.tasks[(size_t)(v & ~(FDEP | MID)) * 8 + 7] -= (v & FDEP) ? W : (v & MID) ? WMID : 1;
    p.succ[e] = -1;
  }
  Exec ex(p);
  if (argc > 5) {
    const int32_t e = std::atoi(argv[5]);
    for (int32_t t = 0; t < p.ntasks; t++)
      if (p.tasks[(size_t)t * 8 + 5] <= e && e < p.tasks[(size_t)t * 8 + 6]) ex.slow_task = t;
  }
  const int nth = std::atoi(argv[3]);
  const unsigned seed = (unsigned)std::atoi(argv[4]);
  std::vector<std::thread> th;
  for (int i = 0; i < nth; i++) th.emplace_back([&ex, seed, i] { ex.worker(seed * 7919u + (unsigned)i); });
  for (auto& x : th) x.join();
  if (ex.failed.load()) {
    std::fprintf(stderr, "exec_race: a task failed\n");
    return 3;
  }
  FILE* f = std::fopen(argv[2], "wb");
  if (!f) return 2;
  bool ok = std::fwrite(p.tiles.data(), 8, p.tiles.size(), f) == p.tiles.size();
  if (ok && p.nrhs > 0) ok = std::fwrite(ex.z.data(), 8, ex.z.size(), f) == ex.z.size();
  std::fclose(f);
  return ok ? 0 : 2;
}
