// capi.cpp -- the C ABI entry points: workspace layout, upload of the static
// task tables, and the stream-ordered launches of the device kernels.
// The library never allocates device memory; every buffer is carved out of
// caller-owned workspaces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "launch.h"
#include "symbolic.h"

using namespace stiles;

namespace {

constexpr size_t ALIGN = 256;
inline size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t ctrl_f, ctrl_s, info, mat_f, mat_s;
  size_t ctrl_m, mat_m, mtask, msucc, mrem, mpairs;   // merged factorization + solve DAG (FP64)
  size_t ftask, fsucc, frem, fpairs;
  size_t stask, ssucc, srem, spairs;
  size_t row_base, row_cnt, trow_ptr, trow, tcol, perm;
  size_t in_rp, fprof, map, fin, in_rp_in;
  size_t tiles, linv, part, shadow, orig;
  size_t vy, vz, vpart, vx, vr, vb, vd, vxp;
  size_t ldpart, stats;
  size_t rtile, ccol_tile, ccol_row, items, item_ptr, rpart, rapart;
  size_t total;
};

struct Plan {   // host-side refinement tables (mixed mode)
  std::vector<int32_t> rtile, ccol_tile, ccol_row, items, item_ptr;
};



// Residual items over the tiles that hold entries of A (tiles of fill only
// are zero in the original tiles and are skipped): kind 0 sums over a row's
// tiles (rtile), kind 1 over a column's tiles below the diagonal (ccol_*).
void make_plan(const stiles_symbolic& s, Plan& p) {
  const std::vector<int32_t> has = tiles_with_entries(s);
  std::vector<std::vector<std::pair<int32_t, int32_t>>> below(s.ntr);
  std::vector<int32_t> rptr(s.ntr + 1, 0);
  p.rtile.clear();
  for (int32_t m = 0; m < s.ntr; m++) {
    for (int32_t t = s.trow_ptr[m]; t < s.trow_ptr[m + 1]; t++) {
      if (!has[t]) continue;
      p.rtile.push_back(t);
      if (s.tcol[t] != m) below[s.tcol[t]].push_back({t, m});
    }
    rptr[m + 1] = (int32_t)p.rtile.size();
  }
  std::vector<int32_t> cptr(s.ntr + 1, 0);
  for (int32_t m = 0; m < s.ntr; m++) cptr[m + 1] = cptr[m] + (int32_t)below[m].size();
  p.ccol_tile.clear();
  p.ccol_row.clear();
  for (int32_t m = 0; m < s.ntr; m++)
    for (auto& e : below[m]) { p.ccol_tile.push_back(e.first); p.ccol_row.push_back(e.second); }
  // long items: the rows of the arrow meet every column, and each item's
  // partial block is summed per row afterwards (refined 16-RHS solve of the
  // n = 500,000 workload: 27.4 ms at 16 tiles per item, 23.6 ms at 64)
  const int32_t CH = 64;
  p.items.clear();
  p.item_ptr.assign(s.ntr + 1, 0);
  for (int32_t m = 0; m < s.ntr; m++) {
    for (int32_t lo = rptr[m]; lo < rptr[m + 1]; lo += CH) {
      int32_t hi = std::min(rptr[m + 1], lo + CH);
      int32_t it[4] = {m, 0, lo, hi};
      p.items.insert(p.items.end(), it, it + 4);
    }
    for (int32_t lo = cptr[m]; lo < cptr[m + 1]; lo += CH) {
      int32_t hi = std::min(cptr[m + 1], lo + CH);
      int32_t it[4] = {m, 1, lo, hi};
      p.items.insert(p.items.end(), it, it + 4);
    }
    p.item_ptr[m + 1] = (int32_t)(p.items.size() / 4);
  }
}

Layout make_layout(const stiles_symbolic& s, int32_t precision, int64_t nrhs_max, const Plan* plan) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = up(o + std::max<size_t>(bytes, 1)); return r; };
  const size_t TT = (size_t)s.T * s.T;
  const size_t nft = s.ftask.size() / TASK_WORDS, nst = s.stask.size() / TASK_WORDS;
  L.ctrl_f = take(sizeof(ExecCtrl));
  L.ctrl_s = take(sizeof(ExecCtrl));
  {
    // merged factorization + solve DAG (every precision: in mixed mode its
    // solve gives the first iterate of the refinement)
    const size_t nm = nft + nst;
    L.ctrl_m = take(sizeof(ExecCtrl));
    L.mat_m = take(sizeof(ExecMat));
    L.mtask = take(nm * TASK_WORDS * 4);
    // successors: the two DAGs' own edges plus at most one cross edge per
    // solve pair and one per diagonal solve step
    L.msucc = take((s.fsucc.size() + s.ssucc.size() + s.spairs.size() / 2 + nst) * 4);
    L.mrem = take(nm * 4);
    L.mpairs = take((s.fpairs.size() + s.spairs.size()) * 4);
  }
  L.info = take(8);
  L.mat_f = take(sizeof(ExecMat));
  L.mat_s = take(sizeof(ExecMat));
  L.ftask = take(s.ftask.size() * 4);
  L.fsucc = take(s.fsucc.size() * 4);
  L.frem = take(nft * 4);
  L.fpairs = take(s.fpairs.size() * 4);
  L.stask = take(s.stask.size() * 4);
  L.ssucc = take(s.ssucc.size() * 4);
  L.srem = take(nst * 4);
  L.spairs = take(s.spairs.size() * 4);
  L.row_base = take(s.row_base.size() * 8);
  L.row_cnt = take(s.row_cnt.size() * 4);
  L.trow_ptr = take(s.trow_ptr.size() * 4);
  L.trow = take(s.trow.size() * 4);
  L.tcol = take(s.tcol.size() * 4);
  L.perm = take(s.perm.size() * 8);
  L.in_rp = take(s.in_rp.size() * 8);   // row pointers of the permuted envelope
  L.fprof = take(s.f.size() * 8);
  L.map = s.profile_input ? 0 : take(s.map.size() * 8);
  L.fin = s.fin.empty() ? 0 : take(s.fin.size() * 8);
  L.in_rp_in = s.in_rp_in.empty() ? 0 : take(s.in_rp_in.size() * 8);
  L.tiles = take(s.ntiles * TT * 8);
  L.linv = take((size_t)s.ntr * TT * 8);
  L.part = take((size_t)s.npart * TT * 8);
  const bool mixed = precision != STILES_FP64;
  L.shadow = mixed ? take(s.ntiles * TT * 4) : 0;
  L.orig = mixed ? take(s.ntiles * TT * 8) : 0;
  const size_t vbytes = (size_t)s.ntr * s.T * nrhs_max * 8;
  L.vy = take(vbytes);
  L.vz = take(vbytes);
  L.vpart = take((size_t)s.nspart * s.T * nrhs_max * 8);
  L.vx = mixed ? take(vbytes) : 0;
  L.vr = mixed ? take(vbytes) : 0;
  L.vb = mixed ? take(vbytes) : 0;
  L.vd = mixed ? take((size_t)s.ntr * s.T * 8) : 0;   // row sums of |A|
  L.vxp = mixed ? take(vbytes) : 0;                      // previous refinement iterate
  L.ldpart = take((size_t)s.ntr * 8);
  L.stats = take(2 * 16 * 8 + 16);
  if (mixed && plan) {
    L.rtile = take(plan->rtile.size() * 4);
    L.ccol_tile = take(plan->ccol_tile.size() * 4);
    L.ccol_row = take(plan->ccol_row.size() * 4);
    L.items = take(plan->items.size() * 4);
    L.item_ptr = take(plan->item_ptr.size() * 4);
    L.rpart = take((plan->items.size() / 4) * (size_t)s.T * nrhs_max * 8);
    L.rapart = take((plan->items.size() / 4) * (size_t)s.T * 8);   // row sums of |A| per item
  }
  L.total = o;
  return L;
}

// default bound of an executor wait for its predecessors: 10 s of the
// 100 MHz device wall clock (far beyond any legitimate wait here)
constexpr uint64_t kDefaultWaitTicks = 1000000000ull;

int device_wg_capacity(int T) {
  static std::mutex mu;
  static int cache[2][64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> g(mu);
  int& c = cache[T == 64 ? 1 : 0][dev];
  if (c == 0) {
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    // LDS of the executor: 2 T^2 doubles + T doubles (+ ticket)
    const size_t lds = (2 * (size_t)T * T + T) * 8 + 64;
    int per_cu = (int)std::min<size_t>(8, (160 * 1024) / lds);
    if (per_cu < 1) per_cu = 1;
    c = cus * per_cu;
  }
  return c;
}

}  // namespace

struct stiles_factor {
  const stiles_symbolic* sym = nullptr;
  int32_t precision = STILES_FP64;
  int64_t nrhs_max = 1;
  char* ws = nullptr;
  size_t bytes = 0;
  Layout L{};
  Plan plan;
  ExecMat mf{}, ms{}, mm{};   // executor descriptors: factorization, solve, merged
  int32_t nmerged = 0;   // tasks of the merged factorization + solve DAG (FP64)
  int32_t max_wg = 0;
  uint64_t wait_ticks = kDefaultWaitTicks;   // bound of every executor wait (100 MHz ticks)
  int32_t state = 0;   // 0 unknown, 1 factored ok, 2 failed (or timed out), -1 not factored
  double anorm = -1.0; // inf-norm of A (mixed mode), computed lazily
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // timing: factor pair, solve pair
  bool timing = false;
  ~stiles_factor() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

template <class T>
T* at(stiles_factor* f, size_t off) { return reinterpret_cast<T*>(f->ws + off); }

hipError_t upload(stiles_factor* f, size_t off, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(f->ws + off, src, bytes, hipMemcpyHostToDevice, st);
}


int nwg_for(const stiles_factor* f, int32_t ntasks) {
  int cap = device_wg_capacity(f->sym->T);
  if (f->max_wg > 0) cap = std::min(cap, (int)f->max_wg);
  return std::max(1, std::min(cap, (int)ntasks));
}

}  // namespace

extern "C" stiles_status stiles_workspace_size(const stiles_symbolic* s, int32_t precision, int64_t nrhs_max,
                                               size_t* bytes) {
  set_error_arg(0);
  if (!s) { set_error_arg(1); return STILES_EINVAL; }
  if (precision != STILES_FP64 && precision != STILES_MIXED32 && precision != STILES_MIXED32_FULL) {
    set_error_arg(2);
    return STILES_EINVAL;
  }
  if (nrhs_max < 1) { set_error_arg(3); return STILES_EINVAL; }
  if (!bytes) { set_error_arg(4); return STILES_EINVAL; }
  Plan p;
  if (precision != STILES_FP64) make_plan(*s, p);
  *bytes = make_layout(*s, precision, nrhs_max, precision != STILES_FP64 ? &p : nullptr).total;
  return STILES_OK;
}

extern "C" stiles_status stiles_workspace_init(const stiles_symbolic* s, int32_t precision, int64_t nrhs_max,
                                               void* d_ws, size_t ws_bytes, hipStream_t st, stiles_factor** out) {
  set_error_arg(0);
  if (!s) { set_error_arg(1); return STILES_EINVAL; }
  if (precision != STILES_FP64 && precision != STILES_MIXED32 && precision != STILES_MIXED32_FULL) {
    set_error_arg(2);
    return STILES_EINVAL;
  }
  if (nrhs_max < 1) { set_error_arg(3); return STILES_EINVAL; }
  if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % ALIGN) != 0) { set_error_arg(4); return STILES_EINVAL; }
  if (!out) { set_error_arg(7); return STILES_EINVAL; }
  stiles_factor* f = new stiles_factor();
  f->sym = s;
  f->precision = precision;
  f->nrhs_max = nrhs_max;
  f->ws = static_cast<char*>(d_ws);
  f->bytes = ws_bytes;
  const bool mixed = precision != STILES_FP64;
  if (mixed) make_plan(*s, f->plan);
  f->L = make_layout(*s, precision, nrhs_max, mixed ? &f->plan : nullptr);
  if (ws_bytes < f->L.total) { delete f; set_error_arg(5); return STILES_ENOMEM; }
  const Layout& L = f->L;
  const size_t nft = s->ftask.size() / TASK_WORDS, nst = s->stask.size() / TASK_WORDS;
  // progress counters start at each task's predecessor count and re-arm
  // themselves after every launch
  std::vector<int32_t> frem(nft), srem(nst);
  for (size_t t = 0; t < nft; t++) frem[t] = s->ftask[t * TASK_WORDS + 7];
  for (size_t t = 0; t < nst; t++) srem[t] = s->stask[t * TASK_WORDS + 7];
  ExecCtrl ctrl{};
  ExecMat& mf = f->mf;
  mf.tiles = at<double>(f, L.tiles);
  mf.linv = at<double>(f, L.linv);
  mf.shadow = mixed ? at<float>(f, L.shadow) : nullptr;
  mf.part = at<double>(f, L.part);
  mf.vy = at<double>(f, L.vy);
  mf.vz = at<double>(f, L.vz);
  mf.vpart = at<double>(f, L.vpart);
  mf.tasks = at<int32_t>(f, L.ftask);
  mf.succ = at<int32_t>(f, L.fsucc);
  mf.remaining = at<int32_t>(f, L.frem);
  mf.pairs = at<int32_t>(f, L.fpairs);
  mf.info = at<unsigned long long>(f, L.info);
  mf.row_base = at<int64_t>(f, L.row_base);
  mf.ntasks = (int32_t)nft;
  mf.ntr = s->ntr;
  mf.mixed = !mixed ? 0 : precision == STILES_MIXED32_FULL ? 2 : 1;
  ExecMat& ms = f->ms;
  ms = mf;
  ms.tasks = at<int32_t>(f, L.stask);
  ms.succ = at<int32_t>(f, L.ssucc);
  ms.remaining = at<int32_t>(f, L.srem);
  ms.pairs = at<int32_t>(f, L.spairs);
  ms.ntasks = (int32_t)nst;
  ms.mixed = 0;
  unsigned long long info0 = ~0ull;
  hipError_t e = hipSuccess;
  auto U = [&](size_t off, const void* src, size_t b) { if (e == hipSuccess) e = upload(f, off, src, b, st); };
  U(L.ctrl_f, &ctrl, sizeof(ctrl));
  U(L.ctrl_s, &ctrl, sizeof(ctrl));
  U(L.info, &info0, 8);
  U(L.mat_f, &mf, sizeof(mf));
  U(L.mat_s, &ms, sizeof(ms));
  U(L.ftask, s->ftask.data(), s->ftask.size() * 4);
  U(L.fsucc, s->fsucc.data(), s->fsucc.size() * 4);
  U(L.frem, frem.data(), frem.size() * 4);
  U(L.fpairs, s->fpairs.data(), s->fpairs.size() * 4);
  U(L.stask, s->stask.data(), s->stask.size() * 4);
  U(L.ssucc, s->ssucc.data(), s->ssucc.size() * 4);
  U(L.srem, srem.data(), srem.size() * 4);
  U(L.spairs, s->spairs.data(), s->spairs.size() * 4);
  U(L.row_base, s->row_base.data(), s->row_base.size() * 8);
  U(L.row_cnt, s->row_cnt.data(), s->row_cnt.size() * 4);
  U(L.trow_ptr, s->trow_ptr.data(), s->trow_ptr.size() * 4);
  U(L.trow, s->trow.data(), s->trow.size() * 4);
  U(L.tcol, s->tcol.data(), s->tcol.size() * 4);
  U(L.perm, s->perm.data(), s->perm.size() * 8);
  U(L.in_rp, s->in_rp.data(), s->in_rp.size() * 8);
  U(L.fprof, s->f.data(), s->f.size() * 8);
  if (!s->profile_input) U(L.map, s->map.data(), s->map.size() * 8);
  if (!s->fin.empty()) U(L.fin, s->fin.data(), s->fin.size() * 8);
  if (!s->in_rp_in.empty()) U(L.in_rp_in, s->in_rp_in.data(), s->in_rp_in.size() * 8);
  std::vector<int32_t> mrem;
  ExecMat& mm = f->mm;
  {
    const MergedPlan& md = merged_plan(*s);
    f->nmerged = (int32_t)(md.task.size() / TASK_WORDS);
    mrem.resize(f->nmerged);
    for (int32_t t = 0; t < f->nmerged; t++) mrem[t] = md.task[(size_t)t * TASK_WORDS + 7];
    mm = mf;
    mm.tasks = at<int32_t>(f, L.mtask);
    mm.succ = at<int32_t>(f, L.msucc);
    mm.remaining = at<int32_t>(f, L.mrem);
    mm.pairs = at<int32_t>(f, L.mpairs);
    mm.ntasks = f->nmerged;
    U(L.ctrl_m, &ctrl, sizeof(ctrl));
    U(L.mat_m, &mm, sizeof(mm));
    U(L.mtask, md.task.data(), md.task.size() * 4);
    U(L.msucc, md.succ.data(), md.succ.size() * 4);
    U(L.mrem, mrem.data(), mrem.size() * 4);
    U(L.mpairs, md.pairs.data(), md.pairs.size() * 4);
  }
  if (mixed) {
    U(L.rtile, f->plan.rtile.data(), f->plan.rtile.size() * 4);
    U(L.ccol_tile, f->plan.ccol_tile.data(), f->plan.ccol_tile.size() * 4);
    U(L.ccol_row, f->plan.ccol_row.data(), f->plan.ccol_row.size() * 4);
    U(L.items, f->plan.items.data(), f->plan.items.size() * 4);
    U(L.item_ptr, f->plan.item_ptr.data(), f->plan.item_ptr.size() * 4);
  }
  // the host vectors above must stay alive until the copies are done
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { delete f; return STILES_EDEVICE; }
  f->state = -1;
  *out = f;
  return STILES_OK;
}

extern "C" stiles_status stiles_factor_set_wait_limit(stiles_factor* f, double seconds) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (!(seconds >= 0.0) || seconds > 3600.0) { set_error_arg(2); return STILES_EINVAL; }
  // 100 MHz device wall clock; at least one tick
  f->wait_ticks = seconds == 0.0 ? kDefaultWaitTicks : std::max<uint64_t>(1, (uint64_t)(seconds * 1e8));
  return STILES_OK;
}

extern "C" stiles_status stiles_factor_set_max_workgroups(stiles_factor* f, int32_t max_wg) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (max_wg < 0) { set_error_arg(2); return STILES_EINVAL; }
  f->max_wg = max_wg;
  return STILES_OK;
}

static stiles_status scatter_values(stiles_factor* f, const double* d_values, hipStream_t st) {
  const stiles_symbolic& s = *f->sym;
  const Layout& L = f->L;
  double* orig = f->precision != STILES_FP64 ? at<double>(f, L.orig) : nullptr;
  hipError_t e;
  if (s.profile_input && !s.perm_identity)
    e = launch_scatter_perm(s.T, d_values, at<int64_t>(f, L.in_rp_in), at<int64_t>(f, L.fin), at<int64_t>(f, L.perm),
                            at<int32_t>(f, L.trow), at<int32_t>(f, L.tcol), at<int64_t>(f, L.row_base),
                            at<int32_t>(f, L.row_cnt), s.ntiles, at<double>(f, L.tiles), orig,
                            at<unsigned long long>(f, L.info), st);
  else if (s.profile_input)
    e = launch_scatter_profile(s.T, d_values, at<int64_t>(f, L.in_rp), at<int64_t>(f, L.fprof), at<int32_t>(f, L.trow),
                               at<int32_t>(f, L.tcol), at<int64_t>(f, L.row_base), at<int32_t>(f, L.row_cnt),
                               s.ntiles, at<double>(f, L.tiles), orig, at<unsigned long long>(f, L.info), st);
  else
    e = launch_scatter_map(s.T, d_values, at<int64_t>(f, L.map), (int64_t)s.map.size(), at<int32_t>(f, L.trow),
                           at<int32_t>(f, L.tcol), at<int32_t>(f, L.row_cnt), s.ntiles, at<double>(f, L.tiles), orig,
                           at<unsigned long long>(f, L.info), st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" stiles_status stiles_factorize(stiles_factor* f, const double* d_values, hipStream_t st) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  const stiles_symbolic& sy = *f->sym;
  const int64_t nvals = !sy.profile_input ? (int64_t)sy.map.size() : sy.perm_identity ? sy.in_rp.back() : sy.in_rp_in.back();
  if (!d_values && nvals > 0) {
    set_error_arg(2);
    return STILES_EINVAL;
  }
  stiles_status r = scatter_values(f, d_values, st);
  if (r != STILES_OK) return r;
  const int32_t nt = f->mf.ntasks;
  if (f->timing) (void)hipEventRecord(f->ev[0], st);
  hipError_t e = launch_exec(f->sym->T, EXEC_FACTOR, at<ExecMat>(f, f->L.mat_f), nullptr, nt, at<ExecCtrl>(f, f->L.ctrl_f), 0,
                             nwg_for(f, nt), f->wait_ticks, st);
  if (f->timing) (void)hipEventRecord(f->ev[1], st);
  if (e != hipSuccess) return STILES_EDEVICE;
  f->state = 0;
  f->anorm = -1.0;
  return STILES_OK;
}

extern "C" stiles_status stiles_factor_info(stiles_factor* f, hipStream_t st, int64_t* info) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (!info) { set_error_arg(3); return STILES_EINVAL; }
  if (f->state == -1) return STILES_ESTATE;
  unsigned long long v = 0;
  if (hipMemcpyAsync(&v, at<unsigned long long>(f, f->L.info), 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return STILES_EDEVICE;
  f->state = v == ~0ull ? 1 : 2;
  if (v == 0) {   // a launch of this factor was abandoned at its wait deadline
    *info = -1;
    return STILES_ETIMEOUT;
  }
  *info = v == ~0ull ? 0 : (int64_t)v;
  return STILES_OK;
}

static stiles_status solve_sweep(stiles_factor* f, const double* d_src, int64_t ldsrc, int nrhs, hipStream_t st) {
  // src (original order) -> Y; run the solve DAG; result in Z
  const stiles_symbolic& s = *f->sym;
  const Layout& L = f->L;
  hipError_t e = launch_pack(s.T, d_src, ldsrc, nrhs, at<int64_t>(f, L.perm), at<int64_t>(f, L.row_base),
                             at<int32_t>(f, L.row_cnt), s.ntr, at<double>(f, L.vy), st);
  if (e == hipSuccess && f->timing) (void)hipEventRecord(f->ev[2], st);
  if (e == hipSuccess)
    e = launch_exec(s.T, EXEC_SOLVE, at<ExecMat>(f, L.mat_s), nullptr, f->ms.ntasks, at<ExecCtrl>(f, L.ctrl_s), nrhs,
                    nwg_for(f, f->ms.ntasks), f->wait_ticks, st);
  if (e == hipSuccess && f->timing) (void)hipEventRecord(f->ev[3], st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

static stiles_status solve_tiles_from_tiles(stiles_factor* f, const double* d_tile_src, int nrhs, hipStream_t st) {
  // tile-layout source -> Y (copy), run the solve DAG; result in Z
  const stiles_symbolic& s = *f->sym;
  const size_t bytes = (size_t)s.ntr * s.T * nrhs * 8;
  if (hipMemcpyAsync(at<double>(f, f->L.vy), d_tile_src, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return STILES_EDEVICE;
  hipError_t e = launch_exec(s.T, EXEC_SOLVE, at<ExecMat>(f, f->L.mat_s), nullptr, f->ms.ntasks, at<ExecCtrl>(f, f->L.ctrl_s),
                             nrhs, nwg_for(f, f->ms.ntasks), f->wait_ticks, st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

// Mixed mode: iterative refinement in FP64 of the nb right-hand sides at B
// (column offset c0 of the caller's report).  x0 = solve(b) (already in vz
// when x0_ready: the merged factorization + solve launch computed it); then
// per right-hand side r = b - A x with the resident FP64 tiles of A,
// d = solve(r), x += d until its own stopping test holds.
stiles_status refine_mixed(stiles_factor* f, double* B, int64_t ldb, int nb, int64_t c0, hipStream_t st,
                           stiles_solve_report* report, bool x0_ready) {
  const stiles_symbolic& s = *f->sym;
  const Layout& L = f->L;
  // ---- mixed mode: x0 = solve(b); repeat r = b - A x, d = solve(r), x += d,
  //      each right-hand side until its own stopping test holds
  const size_t vbytes = (size_t)s.ntr * s.T * nb * 8;
  double* vx = at<double>(f, L.vx);
  double* vxp = at<double>(f, L.vxp);
  double* vr = at<double>(f, L.vr);
  double* vbb = at<double>(f, L.vb);
  double* vz = at<double>(f, L.vz);
  unsigned long long* stats = at<unsigned long long>(f, L.stats);
  // r = b - A x; the first residual after a factorization also gives the
  // row sums of |A| (||A||_inf, kept until the next factorization) from
  // the same pass over A
  auto resid = [&](const double* X, double* R, bool rowsums) {
    return launch_residual(s.T, at<double>(f, L.orig), at<int32_t>(f, L.rtile), at<int32_t>(f, L.tcol),
                           at<int32_t>(f, L.ccol_tile), at<int32_t>(f, L.ccol_row), at<int32_t>(f, L.items),
                           (int32_t)(f->plan.items.size() / 4), at<int32_t>(f, L.item_ptr), s.ntr, X, vbb,
                           at<double>(f, L.rpart), R, nb, 0, st, rowsums ? at<double>(f, L.rapart) : nullptr,
                           rowsums ? at<double>(f, L.vd) : nullptr);
  };
  if (!x0_ready) {
    stiles_status r = solve_sweep(f, B, ldb, nb, st);      // packs b into Y
    if (r != STILES_OK) return r;
  }
  // keep b (tile layout) and x
  if (launch_pack(s.T, B, ldb, nb, at<int64_t>(f, L.perm), at<int64_t>(f, L.row_base), at<int32_t>(f, L.row_cnt),
                  s.ntr, vbb, st) != hipSuccess)
    return STILES_EDEVICE;
  if (hipMemcpyAsync(vx, vz, vbytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return STILES_EDEVICE;
  std::vector<double> bnorm(nb, 0.0);
  {
    // ||b||_inf per column, from the packed copy (host reduction of a small
    // device-side max: reuse the norms kernel with R = b)
    std::vector<unsigned long long> z(2 * 16, 0ull);
    if (hipMemcpyAsync(stats, z.data(), z.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess) return STILES_EDEVICE;
    if (launch_norms(s.T, s.ntr, nb, vbb, vbb, stats, st) != hipSuccess) return STILES_EDEVICE;
    std::vector<unsigned long long> h(2 * 16);
    if (hipMemcpyAsync(h.data(), stats, h.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return STILES_EDEVICE;
    for (int c = 0; c < nb; c++) { double v; std::memcpy(&v, &h[2 * c], 8); bnorm[c] = v; }
  }
  // default stopping test: a backward error of the size the FP64 factor's
  // own solve reaches, u (w + a), w the largest band half-width
  const double tol = f->sym->opts.refine_tol > 0
                         ? f->sym->opts.refine_tol
                         : std::ldexp(1.0, -52) * (double)std::max<int64_t>(1, s.w_in + s.a_in);
  const int maxit = f->sym->opts.refine_max_iter > 0 ? f->sym->opts.refine_max_iter : 30;
  // per right-hand side: backward error of the current x, steps taken,
  // converged, still refining
  std::vector<double> berr(nb, INFINITY);
  std::vector<int> its(nb, 0);
  std::vector<char> conv(nb, 0);
  uint32_t active = (1u << nb) - 1u;   // nb <= 16
  int step = 0;
  for (;;) {
    const bool rowsums = f->anorm < 0;
    if (resid(vx, vr, rowsums) != hipSuccess) return STILES_EDEVICE;
    // per right-hand side max |r| and max |x|; after the first residual
    // also ||A||_inf = the largest row sum of |A| (slot 32, on the device)
    std::vector<unsigned long long> z(2 * 16 + 2, 0ull), h(2 * 16 + 2);
    if (hipMemcpyAsync(stats, z.data(), z.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess) return STILES_EDEVICE;
    if (launch_norms(s.T, s.ntr, nb, vr, vx, stats, st) != hipSuccess) return STILES_EDEVICE;
    if (rowsums) {
      const double* vd = at<double>(f, L.vd);
      if (launch_norms(s.T, s.ntr, 1, vd, vd, stats + 2 * 16, st) != hipSuccess) return STILES_EDEVICE;
    }
    if (hipMemcpyAsync(h.data(), stats, h.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return STILES_EDEVICE;
    if (rowsums) std::memcpy(&f->anorm, &h[2 * 16], 8);
    uint32_t revert = 0;
    for (int c = 0; c < nb; c++) {
      if (!((active >> c) & 1u)) continue;
      double rn, xn;
      std::memcpy(&rn, &h[2 * c], 8);
      std::memcpy(&xn, &h[2 * c + 1], 8);
      const double den = f->anorm * xn + bnorm[c];
      const double be = den > 0 ? rn / den : rn;
      const uint32_t bit = 1u << c;
      if (!(be == be)) {                       // NaN: failed factorization
        berr[c] = be;
        active &= ~bit;
      } else if (be <= tol) {                  // converged
        berr[c] = be;
        conv[c] = 1;
        active &= ~bit;
      } else if (step > 0 && be > 0.5 * berr[c]) {
        // no longer halving (stagnation): keep the better of the last two
        // iterates, with its backward error
        if (be > berr[c]) {
          revert |= bit;   // the last correction is undone
          its[c]--;
        } else {
          berr[c] = be;
        }
        active &= ~bit;
      } else {
        berr[c] = be;
        if (its[c] >= maxit) active &= ~bit;   // step limit
      }
    }
    if (revert && launch_copy_cols(s.T, s.ntr, nb, vx, vxp, revert, st) != hipSuccess) return STILES_EDEVICE;
    if (!active) break;
    // x_prev = x; d = solve(r) (every column: the sweep's cost does not
    // depend on the count); x += d on the columns still refining
    if (hipMemcpyAsync(vxp, vx, vbytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return STILES_EDEVICE;
    stiles_status r2 = solve_tiles_from_tiles(f, vr, nb, st);
    if (r2 != STILES_OK) return r2;
    if (launch_axpy(s.T, s.ntr, nb, vx, vz, active, st) != hipSuccess) return STILES_EDEVICE;
    for (int c = 0; c < nb; c++)
      if ((active >> c) & 1u) its[c]++;
    step++;
  }
  if (launch_unpack(s.T, vx, nb, at<int64_t>(f, L.perm), at<int64_t>(f, L.row_base), at<int32_t>(f, L.row_cnt),
                    s.ntr, at<unsigned long long>(f, L.info), B, ldb, st) != hipSuccess)
    return STILES_EDEVICE;
  if (report) {
    for (int c = 0; c < nb; c++) {
      report->iterations = std::max(report->iterations, its[c]);
      report->converged = report->converged && conv[c];
      report->backward_error = std::max(report->backward_error, berr[c]);
      if (!(berr[c] == berr[c])) report->backward_error = berr[c];
      if (report->backward_errors) report->backward_errors[c0 + c] = berr[c];
      if (report->rhs_iterations) report->rhs_iterations[c0 + c] = its[c];
    }
  }
  return STILES_OK;
}

extern "C" stiles_status stiles_solve(stiles_factor* f, int64_t nrhs, double* d_B, int64_t ldb, hipStream_t st,
                                      stiles_solve_report* report) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (nrhs < 1 || nrhs > f->nrhs_max) { set_error_arg(2); return STILES_EINVAL; }
  if (!d_B) { set_error_arg(3); return STILES_EINVAL; }
  if (ldb < f->sym->N) { set_error_arg(4); return STILES_EINVAL; }
  if (f->state == -1) return STILES_ESTATE;
  if (f->state == 2) return STILES_ESTATE;
  const stiles_symbolic& s = *f->sym;
  const Layout& L = f->L;
  if (report) {
    report->iterations = 0;
    report->converged = 1;
    report->backward_error = -1.0;
    for (int64_t c = 0; c < nrhs; c++) {
      if (report->backward_errors) report->backward_errors[c] = -1.0;
      if (report->rhs_iterations) report->rhs_iterations[c] = 0;
    }
  }
  for (int64_t c0 = 0; c0 < nrhs; c0 += 16) {
    const int nb = (int)std::min<int64_t>(16, nrhs - c0);
    double* B = d_B + c0 * ldb;
    if (f->precision == STILES_FP64) {
      stiles_status r = solve_sweep(f, B, ldb, nb, st);
      if (r != STILES_OK) return r;
      if (launch_unpack(s.T, at<double>(f, L.vz), nb, at<int64_t>(f, L.perm), at<int64_t>(f, L.row_base),
                        at<int32_t>(f, L.row_cnt), s.ntr, at<unsigned long long>(f, L.info), B, ldb, st) != hipSuccess)
        return STILES_EDEVICE;
      continue;
    }
    stiles_status r = refine_mixed(f, B, ldb, nb, c0, st, report, false);
    if (r != STILES_OK) return r;
  }
  return STILES_OK;
}

extern "C" stiles_status stiles_factorize_solve(stiles_factor* f, const double* d_values, int64_t nrhs, double* d_B,
                                                int64_t ldb, hipStream_t st) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  const stiles_symbolic& sy = *f->sym;
  const int64_t nvals = !sy.profile_input ? (int64_t)sy.map.size() : sy.perm_identity ? sy.in_rp.back() : sy.in_rp_in.back();
  if (!d_values && nvals > 0) { set_error_arg(2); return STILES_EINVAL; }
  if (nrhs < 1 || nrhs > f->nrhs_max) { set_error_arg(3); return STILES_EINVAL; }
  if (!d_B) { set_error_arg(4); return STILES_EINVAL; }
  if (ldb < sy.N) { set_error_arg(5); return STILES_EINVAL; }
  stiles_status r = scatter_values(f, d_values, st);
  if (r != STILES_OK) return r;
  const Layout& L = f->L;
  const int nb = (int)std::min<int64_t>(16, nrhs);
  hipError_t e = launch_pack(sy.T, d_B, ldb, nb, at<int64_t>(f, L.perm), at<int64_t>(f, L.row_base),
                             at<int32_t>(f, L.row_cnt), sy.ntr, at<double>(f, L.vy), st);
  if (e != hipSuccess) return STILES_EDEVICE;
  if (f->timing) (void)hipEventRecord(f->ev[0], st);
  e = launch_exec(sy.T, EXEC_FACTOR_SOLVE, at<ExecMat>(f, L.mat_m), nullptr, f->nmerged, at<ExecCtrl>(f, L.ctrl_m), nb,
                  nwg_for(f, f->nmerged), f->wait_ticks, st);
  if (f->timing) (void)hipEventRecord(f->ev[1], st);
  if (e != hipSuccess) return STILES_EDEVICE;
  f->state = 0;
  f->anorm = -1.0;
  if (f->precision != STILES_FP64) {
    // mixed mode: the launch's solve is the first iterate of the refinement
    r = refine_mixed(f, d_B, ldb, nb, 0, st, nullptr, true);
    if (r != STILES_OK) return r;
  } else if (launch_unpack(sy.T, at<double>(f, L.vz), nb, at<int64_t>(f, L.perm), at<int64_t>(f, L.row_base),
                           at<int32_t>(f, L.row_cnt), sy.ntr, at<unsigned long long>(f, L.info), d_B, ldb, st) !=
             hipSuccess) {
    return STILES_EDEVICE;
  }
  // right-hand sides beyond the first 16: ordinary solve sweeps
  for (int64_t c0 = nb; c0 < nrhs; c0 += 16) {
    const int nb2 = (int)std::min<int64_t>(16, nrhs - c0);
    double* B = d_B + c0 * ldb;
    if (f->precision != STILES_FP64) {
      r = refine_mixed(f, B, ldb, nb2, c0, st, nullptr, false);
      if (r != STILES_OK) return r;
      continue;
    }
    r = solve_sweep(f, B, ldb, nb2, st);
    if (r != STILES_OK) return r;
    if (launch_unpack(sy.T, at<double>(f, L.vz), nb2, at<int64_t>(f, L.perm), at<int64_t>(f, L.row_base),
                      at<int32_t>(f, L.row_cnt), sy.ntr, at<unsigned long long>(f, L.info), B, ldb, st) != hipSuccess)
      return STILES_EDEVICE;
  }
  return STILES_OK;
}

extern "C" stiles_status stiles_logdet(stiles_factor* f, double* d_out, hipStream_t st) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (!d_out) { set_error_arg(2); return STILES_EINVAL; }
  if (f->state == -1 || f->state == 2) return STILES_ESTATE;
  const Layout& L = f->L;
  hipError_t e = launch_logdet(f->sym->T, at<double>(f, L.tiles), at<int32_t>(f, L.trow_ptr), f->sym->ntr,
                               at<double>(f, L.ldpart), at<unsigned long long>(f, L.info), d_out, st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" stiles_status stiles_logdet_static(stiles_factor* f, double* d_out, hipStream_t st) {
  static_assert(STILES_STATIC_LOGDET_MAX_ROWS == STATIC_LOGDET_ROWS, "public and internal limits differ");
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (!d_out) { set_error_arg(2); return STILES_EINVAL; }
  if (f->sym->ntr > STATIC_LOGDET_ROWS) { set_error_arg(1); return STILES_ENOTSUP; }
  if (f->state == -1 || f->state == 2) return STILES_ESTATE;
  const Layout& L = f->L;
  hipError_t e = launch_logdet_static(f->sym->T, at<double>(f, L.tiles), at<int32_t>(f, L.trow_ptr), f->sym->ntr,
                                      at<unsigned long long>(f, L.info), d_out, st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

// ------------------------------------------------------------------ batches

namespace {

inline char* b_ws_at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

struct BatchSizes {
  size_t tasks = 0, tiles = 0, rows = 0, succ = 0;
};

BatchSizes batch_sizes(int32_t count, stiles_factor* const* factors) {
  BatchSizes z;
  for (int32_t i = 0; i < count; i++) {
    z.tasks += factors[i]->mf.ntasks;
    z.tiles += factors[i]->sym->ntiles;
    z.rows += factors[i]->sym->ntr;
    z.succ += factors[i]->sym->fsucc.size();
  }
  return z;
}

// batch workspace: control block, executor descriptors, merged ticket order,
// the matrices' task tables without two-stage waits (tasks, successor lists,
// counters), scatter/logdet descriptors, (matrix, tile) and (matrix, tile
// row) maps, and the array of value pointers
struct BatchLayout {
  size_t ctrl, mats, order, tasks, succ, rem, desc, tmap, rmap, vptr, total;
};

BatchLayout batch_layout(int32_t count, const BatchSizes& z) {
  BatchLayout B{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = up(o + std::max<size_t>(bytes, 1)); return r; };
  B.ctrl = take(sizeof(ExecCtrl));
  B.mats = take(sizeof(ExecMat) * count);
  B.order = take(z.tasks * 8);
  B.tasks = take(z.tasks * TASK_WORDS * 4);
  B.succ = take(z.succ * 4);
  B.rem = take(z.tasks * 4);
  B.desc = take(sizeof(BatchDesc) * count);
  B.tmap = take(z.tiles * 8);
  B.rmap = take(z.rows * 8);
  B.vptr = take(sizeof(double*) * count);
  B.total = o;
  return B;
}

}  // namespace

extern "C" stiles_status stiles_batch_workspace_size(int32_t count, stiles_factor* const* factors, size_t* bytes) {
  set_error_arg(0);
  if (count < 1) { set_error_arg(1); return STILES_EINVAL; }
  if (!factors) { set_error_arg(2); return STILES_EINVAL; }
  if (!bytes) { set_error_arg(3); return STILES_EINVAL; }
  for (int32_t i = 0; i < count; i++)
    if (!factors[i]) { set_error_arg(2); return STILES_EINVAL; }
  *bytes = batch_layout(count, batch_sizes(count, factors)).total;
  return STILES_OK;
}

struct stiles_batch {
  std::vector<stiles_factor*> factors;
  char* ws = nullptr;
  int32_t total = 0;
  int T = 64;
  bool all_profile = true;    // every matrix has row-profile input: one scatter launch
  BatchSizes z;
  BatchLayout B;
  std::vector<const double*> vptr;   // value pointers last uploaded
};

extern "C" stiles_status stiles_batch_create(int32_t count, stiles_factor* const* factors, void* d_batch_ws,
                                             size_t batch_ws_bytes, hipStream_t st, stiles_batch** out) {
  set_error_arg(0);
  size_t need = 0;
  stiles_status r = stiles_batch_workspace_size(count, factors, &need);
  if (r != STILES_OK) return r;
  if (!d_batch_ws || (reinterpret_cast<uintptr_t>(d_batch_ws) % ALIGN) != 0) { set_error_arg(3); return STILES_EINVAL; }
  if (batch_ws_bytes < need) { set_error_arg(4); return STILES_ENOMEM; }
  if (!out) { set_error_arg(6); return STILES_EINVAL; }
  const int T = factors[0]->sym->T;
  for (int32_t i = 0; i < count; i++) {
    if (factors[i]->sym->T != T) { set_error_arg(2); return STILES_ENOTSUP; }
    for (int32_t j = 0; j < i; j++)
      if (factors[j]->ws == factors[i]->ws) { set_error_arg(2); return STILES_EINVAL; }
  }
  // one ticket order for the union of the matrices' DAGs: a list schedule on
  // the workgroups of the launch (longest remaining path first), or, when
  // the options ask for the earliest-start order, the per-matrix schedules
  // merged by their start estimates
  const int workers = schedule_workers(factors[0]->sym->opts);
  std::vector<int32_t> order;
  if (workers > 0) {
    const float hop = 0.8f;
    std::vector<int32_t> off(count + 1, 0);
    for (int32_t i = 0; i < count; i++) off[i + 1] = off[i] + factors[i]->mf.ntasks;
    const int32_t n = off[count];
    std::vector<float> cost(n), bl(n);
    std::vector<int32_t> sptr(n + 1, 0), sflat, npred(n), owner(n);
    for (int32_t i = 0; i < count; i++) {
      const stiles_symbolic& sy = *factors[i]->sym;
      for (int32_t t = 0; t < factors[i]->mf.ntasks; t++) {
        const int32_t g = off[i] + t;
        const int32_t* w = &sy.ftask[(size_t)t * TASK_WORDS];
        cost[g] = sy.fcost[t];
        owner[g] = i;
        for (int32_t q = w[5]; q < w[6]; q++) sflat.push_back(off[i] + (sy.fsucc[q] & ~SUCC_FDEP));
        sptr[g + 1] = (int32_t)sflat.size();
      }
    }
    // predecessor counts (the task counters weight early predecessors)
    for (int32_t q = 0; q < (int32_t)sflat.size(); q++) npred[sflat[q]]++;
    // remaining path lengths: each matrix's tasks are in topological order
    for (int32_t g = n - 1; g >= 0; g--) {
      float b2 = 0.f;
      for (int32_t q = sptr[g]; q < sptr[g + 1]; q++) b2 = std::max(b2, bl[sflat[q]] + hop);
      bl[g] = b2 + cost[g];
    }
    const std::vector<int32_t> ord = list_schedule(n, cost.data(), sptr.data(), sflat.data(), npred.data(), bl.data(),
                                                   workers, hop);
    // the executor needs a topological ticket order: verify it
    std::vector<int32_t> pos(n, -1);
    for (int32_t q = 0; q < (int32_t)ord.size(); q++) pos[ord[q]] = q;
    for (int32_t g = 0; g < n; g++) {
      bool ok = pos[g] >= 0;
      for (int32_t q = sptr[g]; ok && q < sptr[g + 1]; q++) ok = pos[sflat[q]] > pos[g];
      if (!ok) { fprintf(stderr, "stiles: batch schedule is not topological\n"); abort(); }
    }
    order.resize((size_t)n * 2);
    for (int32_t q = 0; q < n; q++) { order[2 * q] = owner[ord[q]]; order[2 * q + 1] = ord[q] - off[owner[ord[q]]]; }
  } else {
    struct E { float est; int32_t m, t; };
    std::vector<E> ev;
    for (int32_t i = 0; i < count; i++) {
      const auto& est = factors[i]->sym->fest;
      for (int32_t t = 0; t < factors[i]->mf.ntasks; t++) ev.push_back({est[t], i, t});
    }
    std::stable_sort(ev.begin(), ev.end(), [](const E& a, const E& b) { return a.est < b.est; });
    order.resize(ev.size() * 2);
    for (size_t q = 0; q < ev.size(); q++) { order[2 * q] = ev[q].m; order[2 * q + 1] = ev[q].t; }
  }
  std::vector<ExecMat> mats(count);
  std::vector<BatchDesc> desc(count);
  std::vector<int32_t> tmap, rmap;
  stiles_batch* b = new stiles_batch();
  b->z = batch_sizes(count, factors);
  b->B = batch_layout(count, b->z);
  // The batch runs the matrices' factorization DAGs without their two-stage
  // waits: in a launch over many matrices no single pivot chain bounds the
  // run, and the second counter round trip of a split task only costs
  // throughput (512-matrix batch: executor 14.1 -> 13.7 ms).  Same tasks,
  // same products in the same order: the results do not change.
  std::vector<int32_t> btasks, bsucc, brem;
  btasks.reserve(b->z.tasks * TASK_WORDS);
  bsucc.reserve(b->z.succ);
  std::vector<size_t> task_off(count), succ_off(count);
  for (int32_t i = 0; i < count; i++) {
    const stiles_symbolic& s = *factors[i]->sym;
    const int32_t nt = factors[i]->mf.ntasks;
    task_off[i] = btasks.size() / TASK_WORDS;
    succ_off[i] = bsucc.size();
    std::vector<int32_t> npred(nt, 0);
    for (int32_t v : s.fsucc) npred[v & ~SUCC_FDEP]++;
    for (int32_t t = 0; t < nt; t++) {
      const int32_t* w = &s.ftask[(size_t)t * TASK_WORDS];
      btasks.insert(btasks.end(), w, w + TASK_WORDS);
      int32_t* bw = &btasks[btasks.size() - TASK_WORDS];
      bw[0] &= ~TF_SPLIT;
      bw[7] = npred[t];
      brem.push_back(npred[t]);
    }
    for (int32_t v : s.fsucc) bsucc.push_back(v & ~SUCC_FDEP);
  }
  for (int32_t i = 0; i < count; i++) {
    stiles_factor* f = factors[i];
    const stiles_symbolic& s = *f->sym;
    const Layout& L = f->L;
    mats[i] = f->mf;
    mats[i].tasks = reinterpret_cast<const int32_t*>(b_ws_at(d_batch_ws, b->B.tasks)) + task_off[i] * TASK_WORDS;
    mats[i].succ = reinterpret_cast<const int32_t*>(b_ws_at(d_batch_ws, b->B.succ)) + succ_off[i];
    mats[i].remaining = reinterpret_cast<int32_t*>(b_ws_at(d_batch_ws, b->B.rem)) + task_off[i];
    BatchDesc& d = desc[i];
    if (s.profile_input && !s.perm_identity) {
      d.in_rp = at<int64_t>(f, L.in_rp_in);
      d.f = at<int64_t>(f, L.fin);
      d.perm = at<int64_t>(f, L.perm);
    } else {
      d.in_rp = at<int64_t>(f, L.in_rp);
      d.f = at<int64_t>(f, L.fprof);
      d.perm = nullptr;
    }
    d.trow = at<int32_t>(f, L.trow);
    d.tcol = at<int32_t>(f, L.tcol);
    d.trow_ptr = at<int32_t>(f, L.trow_ptr);
    d.row_base = at<int64_t>(f, L.row_base);
    d.row_cnt = at<int32_t>(f, L.row_cnt);
    d.tiles = at<double>(f, L.tiles);
    d.orig = f->precision != STILES_FP64 ? at<double>(f, L.orig) : nullptr;
    d.ldpart = at<double>(f, L.ldpart);
    d.info = at<unsigned long long>(f, L.info);
    d.ntiles = (int32_t)s.ntiles;
    d.ntr = s.ntr;
    if (!s.profile_input) b->all_profile = false;
    for (int32_t t = 0; t < (int32_t)s.ntiles; t++) { tmap.push_back(i); tmap.push_back(t); }
    for (int32_t m = 0; m < s.ntr; m++) { rmap.push_back(i); rmap.push_back(m); }
  }
  b->factors.assign(factors, factors + count);
  b->ws = static_cast<char*>(d_batch_ws);
  b->total = (int32_t)(order.size() / 2);
  b->T = T;
  ExecCtrl ctrl{};
  char* w = b->ws;
  hipError_t e = hipMemcpyAsync(w + b->B.ctrl, &ctrl, sizeof(ctrl), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + b->B.mats, mats.data(), sizeof(ExecMat) * count, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + b->B.tasks, btasks.data(), btasks.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !bsucc.empty())
    e = hipMemcpyAsync(w + b->B.succ, bsucc.data(), bsucc.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + b->B.rem, brem.data(), brem.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + b->B.order, order.data(), order.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + b->B.desc, desc.data(), sizeof(BatchDesc) * count, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !tmap.empty())
    e = hipMemcpyAsync(w + b->B.tmap, tmap.data(), tmap.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !rmap.empty())
    e = hipMemcpyAsync(w + b->B.rmap, rmap.data(), rmap.size() * 4, hipMemcpyHostToDevice, st);
  // host vectors must outlive the asynchronous copies
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { delete b; return STILES_EDEVICE; }
  *out = b;
  return STILES_OK;
}

extern "C" stiles_status stiles_batch_factorize(stiles_batch* b, const double* const* d_values, hipStream_t st) {
  set_error_arg(0);
  if (!b) { set_error_arg(1); return STILES_EINVAL; }
  if (!d_values) { set_error_arg(2); return STILES_EINVAL; }
  const size_t count = b->factors.size();
  for (size_t i = 0; i < count; i++)
    if (!d_values[i]) { set_error_arg(2); return STILES_EINVAL; }
  if (b->all_profile) {
    // one scatter launch over every tile of every matrix; the value pointers
    // are uploaded when they differ from the last call's (the upload waits
    // for the stream, so earlier launches reading the old array are done)
    if (b->vptr.size() != count || !std::equal(b->vptr.begin(), b->vptr.end(), d_values)) {
      hipError_t e = hipStreamSynchronize(st);
      b->vptr.assign(d_values, d_values + count);
      if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + b->B.vptr, b->vptr.data(), sizeof(double*) * count, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) { b->vptr.clear(); return STILES_EDEVICE; }
    }
    hipError_t e = launch_scatter_batch(b->T, reinterpret_cast<const BatchDesc*>(b->ws + b->B.desc),
                                        reinterpret_cast<const double* const*>(b->ws + b->B.vptr),
                                        reinterpret_cast<const int2*>(b->ws + b->B.tmap), (int64_t)b->z.tiles, st);
    if (e != hipSuccess) return STILES_EDEVICE;
  } else {
    for (size_t i = 0; i < count; i++) {
      stiles_status r = scatter_values(b->factors[i], d_values[i], st);
      if (r != STILES_OK) return r;
    }
  }
  stiles_factor* f0 = b->factors[0];
  // the first factor's workgroup cap bounds the batch launch (batches on
  // different streams can then share the GPU)
  int cap = device_wg_capacity(b->T);
  if (f0->max_wg > 0) cap = std::min(cap, (int)f0->max_wg);
  if (f0->timing) (void)hipEventRecord(f0->ev[0], st);
  hipError_t e = launch_exec(b->T, EXEC_FACTOR, reinterpret_cast<const ExecMat*>(b->ws + b->B.mats),
                             reinterpret_cast<const int32_t*>(b->ws + b->B.order), b->total,
                             reinterpret_cast<ExecCtrl*>(b->ws + b->B.ctrl), 0, std::min<int>(cap, b->total),
                             f0->wait_ticks, st);
  if (f0->timing) (void)hipEventRecord(f0->ev[1], st);
  if (e != hipSuccess) return STILES_EDEVICE;
  for (auto* f : b->factors) { f->state = 0; f->anorm = -1.0; }
  return STILES_OK;
}

extern "C" stiles_status stiles_batch_logdet(stiles_batch* b, double* d_out, hipStream_t st) {
  set_error_arg(0);
  if (!b) { set_error_arg(1); return STILES_EINVAL; }
  if (!d_out) { set_error_arg(2); return STILES_EINVAL; }
  for (auto* f : b->factors)
    if (f->state == -1 || f->state == 2) return STILES_ESTATE;
  hipError_t e = launch_logdet_batch(b->T, reinterpret_cast<const BatchDesc*>(b->ws + b->B.desc),
                                     (int32_t)b->factors.size(), reinterpret_cast<const int2*>(b->ws + b->B.rmap),
                                     (int64_t)b->z.rows, d_out, st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" void stiles_batch_destroy(stiles_batch* b) { delete b; }

extern "C" stiles_status stiles_factorize_batch(int32_t count, stiles_factor* const* factors,
                                                const double* const* d_values, void* d_batch_ws,
                                                size_t batch_ws_bytes, hipStream_t st) {
  set_error_arg(0);
  if (!d_values) { set_error_arg(3); return STILES_EINVAL; }
  stiles_batch* b = nullptr;
  stiles_status r = stiles_batch_create(count, factors, d_batch_ws, batch_ws_bytes, st, &b);
  if (r != STILES_OK) {
    // keep this entry point's argument numbering
    const int32_t a = stiles_last_error_arg();
    set_error_arg(a >= 3 ? a + 1 : a);
    return r;
  }
  r = stiles_batch_factorize(b, d_values, st);
  stiles_batch_destroy(b);
  if (r == STILES_EINVAL) set_error_arg(3);
  return r;
}

extern "C" stiles_status stiles_factor_set_trace(stiles_factor* f, void* d_factor_trace, void* d_solve_trace,
                                                 hipStream_t st) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  f->mf.trace = static_cast<unsigned long long*>(d_factor_trace);
  f->ms.trace = static_cast<unsigned long long*>(d_solve_trace);
  hipError_t e = hipMemcpyAsync(f->ws + f->L.mat_f, &f->mf, sizeof(ExecMat), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(f->ws + f->L.mat_s, &f->ms, sizeof(ExecMat), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" stiles_status stiles_factor_set_merged_trace(stiles_factor* f, void* d_trace, hipStream_t st) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  f->mm.trace = static_cast<unsigned long long*>(d_trace);
  hipError_t e = hipMemcpyAsync(f->ws + f->L.mat_m, &f->mm, sizeof(ExecMat), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" stiles_status stiles_factor_set_timing(stiles_factor* f, int32_t enable) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (enable)
    for (auto& e : f->ev)
      if (!e && hipEventCreate(&e) != hipSuccess) return STILES_EDEVICE;
  f->timing = enable != 0;
  return STILES_OK;
}

extern "C" stiles_status stiles_factor_kernel_ms(stiles_factor* f, int32_t which, float* ms) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (which != 0 && which != 1) { set_error_arg(2); return STILES_EINVAL; }
  if (!ms) { set_error_arg(3); return STILES_EINVAL; }
  if (!f->timing) return STILES_ESTATE;
  hipEvent_t a = f->ev[2 * which], b = f->ev[2 * which + 1];
  if (hipEventSynchronize(b) != hipSuccess) return STILES_EDEVICE;
  if (hipEventElapsedTime(ms, a, b) != hipSuccess) return STILES_ESTATE;
  return STILES_OK;
}

extern "C" stiles_status stiles_factor_extract(stiles_factor* f, double* d_L, hipStream_t st) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (!d_L) { set_error_arg(2); return STILES_EINVAL; }
  if (f->state == -1) return STILES_ESTATE;
  const stiles_symbolic& s = *f->sym;
  const Layout& L = f->L;
  hipError_t e = launch_extract(s.T, at<double>(f, L.tiles), at<int64_t>(f, L.in_rp), at<int64_t>(f, L.fprof),
                                at<int32_t>(f, L.trow), at<int32_t>(f, L.tcol), at<int64_t>(f, L.row_base),
                                at<int32_t>(f, L.row_cnt), s.ntiles, s.nnzL, d_L, st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" void stiles_factor_release(stiles_factor* f) { delete f; }

// ------------------------------------------------------- selected inversion

namespace {

// selected-inversion workspace: control block, executor descriptor, task
// tables and progress counters, then Sigma and the two per-tile partial stores
struct SelinvLayout {
  size_t ctrl, mat, task, succ, rem, list, sigma, dpart, qpart, total;
};

SelinvLayout selinv_layout(const stiles_symbolic& s, const SelinvPlan& P) {
  SelinvLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = up(o + std::max<size_t>(bytes, 1)); return r; };
  const size_t tile_bytes = (size_t)s.ntiles * s.T * s.T * 8;
  L.ctrl = take(sizeof(ExecCtrl));
  L.mat = take(sizeof(ExecMat));
  L.task = take(P.task.size() * 4);
  L.succ = take(P.succ.size() * 4);
  L.rem = take(P.task.size() / TASK_WORDS * 4);
  L.list = take(P.list.size() * 4);
  L.sigma = take(tile_bytes);
  L.dpart = take(tile_bytes);
  L.qpart = take(tile_bytes);
  L.total = o;
  return L;
}

}  // namespace

struct stiles_selinv {
  stiles_factor* f = nullptr;
  char* ws = nullptr;
  SelinvLayout L{};
  int32_t ntasks = 0;
  bool done = false;
  bool timing = false;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~stiles_selinv() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

extern "C" stiles_status stiles_selinv_query(const stiles_symbolic* s, int64_t* tasks, double* flops_alg,
                                             double* flops_exec) {
  set_error_arg(0);
  if (!s) { set_error_arg(1); return STILES_EINVAL; }
  const SelinvPlan& P = selinv_plan(*s);
  if (tasks) *tasks = (int64_t)(P.task.size() / TASK_WORDS);
  if (flops_alg) *flops_alg = P.flops_alg;
  if (flops_exec) *flops_exec = P.flops_exec;
  return STILES_OK;
}

extern "C" stiles_status stiles_selinv_workspace_size(const stiles_symbolic* s, size_t* bytes) {
  set_error_arg(0);
  if (!s) { set_error_arg(1); return STILES_EINVAL; }
  if (!bytes) { set_error_arg(2); return STILES_EINVAL; }
  *bytes = selinv_layout(*s, selinv_plan(*s)).total;
  return STILES_OK;
}

extern "C" stiles_status stiles_selinv_create(stiles_factor* f, void* d_ws, size_t ws_bytes, hipStream_t st,
                                              stiles_selinv** out) {
  set_error_arg(0);
  if (!f) { set_error_arg(1); return STILES_EINVAL; }
  if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % ALIGN) != 0) { set_error_arg(2); return STILES_EINVAL; }
  if (!out) { set_error_arg(5); return STILES_EINVAL; }
  const stiles_symbolic& s = *f->sym;
  const SelinvPlan& P = selinv_plan(s);
  const SelinvLayout L = selinv_layout(s, P);
  if (ws_bytes < L.total) { set_error_arg(3); return STILES_ENOMEM; }
  stiles_selinv* si = new stiles_selinv();
  si->f = f;
  si->ws = static_cast<char*>(d_ws);
  si->L = L;
  si->ntasks = (int32_t)(P.task.size() / TASK_WORDS);
  ExecMat m = f->mf;
  m.tasks = reinterpret_cast<const int32_t*>(si->ws + L.task);
  m.succ = reinterpret_cast<const int32_t*>(si->ws + L.succ);
  m.remaining = reinterpret_cast<int32_t*>(si->ws + L.rem);
  m.pairs = reinterpret_cast<const int32_t*>(si->ws + L.list);
  m.sigma = reinterpret_cast<double*>(si->ws + L.sigma);
  m.dpart = reinterpret_cast<double*>(si->ws + L.dpart);
  m.qpart = reinterpret_cast<double*>(si->ws + L.qpart);
  m.shadow = nullptr;
  m.trace = nullptr;
  m.ntasks = si->ntasks;
  m.mixed = 0;
  std::vector<int32_t> rem(si->ntasks);
  for (int32_t t = 0; t < si->ntasks; t++) rem[t] = P.task[(size_t)t * TASK_WORDS + 7];
  ExecCtrl ctrl{};
  hipError_t e = hipSuccess;
  auto U = [&](size_t off, const void* src, size_t b) {
    if (e == hipSuccess && b) e = hipMemcpyAsync(si->ws + off, src, b, hipMemcpyHostToDevice, st);
  };
  U(L.ctrl, &ctrl, sizeof(ctrl));
  U(L.mat, &m, sizeof(m));
  U(L.task, P.task.data(), P.task.size() * 4);
  U(L.succ, P.succ.data(), P.succ.size() * 4);
  U(L.rem, rem.data(), rem.size() * 4);
  U(L.list, P.list.data(), P.list.size() * 4);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host vectors above die here
  if (e != hipSuccess) { delete si; return STILES_EDEVICE; }
  *out = si;
  return STILES_OK;
}

extern "C" stiles_status stiles_selinv_compute(stiles_selinv* si, hipStream_t st) {
  set_error_arg(0);
  if (!si) { set_error_arg(1); return STILES_EINVAL; }
  stiles_factor* f = si->f;
  if (f->state == -1 || f->state == 2) return STILES_ESTATE;
  if (si->timing) (void)hipEventRecord(si->ev[0], st);
  hipError_t e = launch_exec(f->sym->T, EXEC_SELINV, reinterpret_cast<const ExecMat*>(si->ws + si->L.mat), nullptr,
                             si->ntasks, reinterpret_cast<ExecCtrl*>(si->ws + si->L.ctrl), 0,
                             nwg_for(f, si->ntasks), f->wait_ticks, st);
  if (si->timing) (void)hipEventRecord(si->ev[1], st);
  if (e != hipSuccess) return STILES_EDEVICE;
  si->done = true;
  return STILES_OK;
}

extern "C" stiles_status stiles_selinv_diag(stiles_selinv* si, double* d_diag, hipStream_t st) {
  set_error_arg(0);
  if (!si) { set_error_arg(1); return STILES_EINVAL; }
  if (!d_diag) { set_error_arg(2); return STILES_EINVAL; }
  if (!si->done) return STILES_ESTATE;
  stiles_factor* f = si->f;
  const stiles_symbolic& s = *f->sym;
  const Layout& L = f->L;
  hipError_t e = launch_selinv_diag(s.T, reinterpret_cast<const double*>(si->ws + si->L.sigma),
                                    at<int32_t>(f, L.trow_ptr), at<int64_t>(f, L.row_base), at<int32_t>(f, L.row_cnt),
                                    at<int64_t>(f, L.perm), s.ntr, at<unsigned long long>(f, L.info), d_diag, st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" stiles_status stiles_selinv_extract(stiles_selinv* si, double* d_out, hipStream_t st) {
  set_error_arg(0);
  if (!si) { set_error_arg(1); return STILES_EINVAL; }
  if (!d_out) { set_error_arg(2); return STILES_EINVAL; }
  if (!si->done) return STILES_ESTATE;
  stiles_factor* f = si->f;
  const stiles_symbolic& s = *f->sym;
  const Layout& L = f->L;
  hipError_t e = launch_extract(s.T, reinterpret_cast<const double*>(si->ws + si->L.sigma), at<int64_t>(f, L.in_rp),
                                at<int64_t>(f, L.fprof), at<int32_t>(f, L.trow), at<int32_t>(f, L.tcol),
                                at<int64_t>(f, L.row_base), at<int32_t>(f, L.row_cnt), s.ntiles, s.nnzL, d_out, st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" stiles_status stiles_selinv_set_timing(stiles_selinv* si, int32_t enable) {
  set_error_arg(0);
  if (!si) { set_error_arg(1); return STILES_EINVAL; }
  if (enable)
    for (auto& e : si->ev)
      if (!e && hipEventCreate(&e) != hipSuccess) return STILES_EDEVICE;
  si->timing = enable != 0;
  return STILES_OK;
}

extern "C" stiles_status stiles_selinv_kernel_ms(stiles_selinv* si, float* ms) {
  set_error_arg(0);
  if (!si) { set_error_arg(1); return STILES_EINVAL; }
  if (!ms) { set_error_arg(2); return STILES_EINVAL; }
  if (!si->timing || !si->done) return STILES_ESTATE;
  if (hipEventSynchronize(si->ev[1]) != hipSuccess) return STILES_EDEVICE;
  if (hipEventElapsedTime(ms, si->ev[0], si->ev[1]) != hipSuccess) return STILES_ESTATE;
  return STILES_OK;
}

extern "C" stiles_status stiles_selinv_set_trace(stiles_selinv* si, void* d_trace, hipStream_t st) {
  set_error_arg(0);
  if (!si) { set_error_arg(1); return STILES_EINVAL; }
  ExecMat m;
  hipError_t e = hipMemcpyAsync(&m, si->ws + si->L.mat, sizeof(ExecMat), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  m.trace = static_cast<unsigned long long*>(d_trace);
  if (e == hipSuccess) e = hipMemcpyAsync(si->ws + si->L.mat, &m, sizeof(ExecMat), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? STILES_OK : STILES_EDEVICE;
}

extern "C" void stiles_selinv_destroy(stiles_selinv* si) { delete si; }
