// Round executor, device-memory layout of an instance, and the HALLaR solver
// written as one C++20 coroutine per instance.
//
// A solve suspends at every device operation it needs (a FISTA trial, a
// Lanczos block, a Frank-Wolfe update, ...).  A round collects the pending
// operations of all resident instances, groups equal operations, launches
// each group's kernels once over the concatenated tiles of its instances,
// exchanges the per-instance scalars with the host in one copy each way and
// resumes every coroutine.  A single solve is a pool with one instance.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <random>

#include <rocfft/rocfft.h>

#include "ops.h"

namespace hl {

ResumeWorkers::~ResumeWorkers() {
  {
    std::lock_guard<std::mutex> lk(m_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto &t : th_) t.join();
}

void ResumeWorkers::work(Job &j) {
  for (int i; (i = j.next.fetch_add(1)) < j.n;) {
    (*j.fn)(i);
    j.done.fetch_add(1);
  }
}

void ResumeWorkers::loop() {
  uint64_t seen = 0;
  for (;;) {
    std::shared_ptr<Job> j;
    {
      std::unique_lock<std::mutex> lk(m_);
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      j = job_;
    }
    if (j) work(*j);
  }
}

void ResumeWorkers::run(int n, const std::function<void(int)> &fn) {
  if (th_.empty()) {
    const unsigned hc = std::thread::hardware_concurrency();
    const int nt = (int)std::max(1u, std::min(8u, hc > 1 ? hc - 1 : 1u));
    for (int t = 0; t < nt; ++t) th_.emplace_back([this] { loop(); });
  }
  auto j = std::make_shared<Job>();
  j->fn = &fn;
  j->n = n;
  {
    std::lock_guard<std::mutex> lk(m_);
    job_ = j;
    ++gen_;
  }
  cv_.notify_all();
  work(*j);
  while (j->done.load() < n) std::this_thread::yield();
  // fn outlives no worker call: every index ran to completion, and a late
  // worker finds j->next >= n and leaves without calling fn
  std::lock_guard<std::mutex> lk(m_);
  if (job_ == j) job_.reset();
}


static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

#define HL_TRY(expr, msg)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      err = std::string(msg) + ": " + hipGetErrorString(e_);                           \
      return HALLAR_E_HIP;                                                             \
    }                                                                                  \
  } while (0)

// ------------------------------------------------------------------ arena
bool Arena::init(size_t bytes, std::string &err) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (hipMalloc((void **)&base_, bytes) != hipSuccess) {
    err = "hipMalloc of the pool slab failed";
    base_ = nullptr;
    return false;
  }
  cap_ = bytes;
  used_ = 0;
  free_.clear();
  free_[0] = bytes;
  return true;
}
void Arena::release() {
  if (base_) (void)hipFree(base_);
  base_ = nullptr;
  cap_ = used_ = 0;
  free_.clear();
}
size_t Arena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used_ += bytes;
      return off;
    }
  }
  return SIZE_MAX;
}
void Arena::free(size_t off, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  used_ -= bytes;
  auto it = free_.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

// ------------------------------------------------------------------ layout
int rcap_for(const hallar_options &o, int prec) {
  const int cap = o.rank_cap > 0 ? std::min(o.rank_cap + 1, R_MAX) : R_MAX;
  return r_bucket(cap, prec);
}
int kmax_for(const hallar_options &o, int n) {
  int k = o.eig_kmax > 0 ? std::min(o.eig_kmax, KMAX) : KMAX;
  return std::max(2, std::min(k, n));
}

struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

struct Layout {
  size_t rowptr_u, col_u, pcon, c_u, pa, c64, pa64, rowptr_l, col_l, pid_l, low_pb, upb, b, K0, K064, D0, c_diag;
  size_t eptr, econ, ea64, ew64, cptr, cent, epair, Bpair;
  size_t buf[NBUF], m_xt, m_yp, p, yp, TY, Ty, m64, m64_low, V, V2, w, lzv, hcoef, Z0, part, red_stage, red_count, gram, tiles,
      ilist;
  size_t Kc, Kc64, Dc, lc_con, lc_off, lc_doff, lc_of_con, lc_term, lc_part, lc_Y, lc_Z, lc_T, lc_v, lc_zv, lc_Tv, lc_W[2], lc_wv;
  size_t cdp_d, cdp_S, cdp_S2, cdp_T, cdp_Tv, cdp_wv, cdp_W[2];
  size_t total;
};

static size_t prows_for(const HostProblem &hp) {
  return hp.tiles.size() + ((size_t)hp.m + BLOCK - 1) / BLOCK + 1;
}

static Layout make_layout(const HostProblem &hp, int prec, int Rcap, int kmax) {
  Layout L{};
  Carve c;
  const size_t sz = prec == 0 ? 8 : 4;
  const size_t n = hp.n, m = hp.m, P = hp.npairs, nl = hp.nlower, E = hp.nentries;
  L.rowptr_u = c.take((n + 1) * 4);
  L.col_u = c.take(P * 4);
  L.pcon = c.take(P * 4);
  L.c_u = c.take(P * sz);
  L.pa = c.take(P * sz);
  L.c64 = c.take(P * 8);
  L.pa64 = c.take(P * 8);
  L.rowptr_l = c.take((n + 1) * 4);
  L.col_l = c.take(nl * 4);
  L.pid_l = c.take(nl * 4);
  L.low_pb = c.take(hp.low_recompute ? nl * 16 : 0);
  L.upb = c.take(hp.direct ? P * 16 : 0);
  L.b = c.take(m * 8);
  L.c_diag = c.take(hp.c_diag_only ? n * 8 : 0);
  L.K0 = c.take(n * hp.r0 * sz);
  L.K064 = c.take(n * hp.r0 * 8);
  L.D0 = c.take(hp.r0 * hp.r0 * 8);
  if (!hp.direct) {
    L.eptr = c.take((P + 1) * 4);
    L.econ = c.take(E * 4);
    L.ea64 = c.take(E * 8);
    L.ew64 = c.take(E * 8);
    L.cptr = c.take((m + 1) * 4);
    L.cent = c.take(E * 4);
    L.epair = c.take(E * 4);
    L.Bpair = c.take(P * 8);
  }
  for (int q = 0; q < NBUF; ++q) L.buf[q] = c.take(n * Rcap * sz);
  L.m_xt = c.take(P * sz);
  L.m_yp = c.take(P * sz);
  L.p = c.take(m * 8);
  L.yp = c.take(m * 8);
  L.TY = c.take(m * 8);
  L.Ty = c.take(m * 8);
  L.m64 = c.take(P * 8);
  L.m64_low = c.take(nl * 8);
  L.V = c.take((size_t)(kmax + 1) * n * 8);
  L.V2 = c.take((size_t)(kmax + 1) * n * 8);
  L.w = c.take(n * 8);
  L.lzv = c.take(n * 8);
  L.hcoef = c.take((KMAX + 1) * 8);
  L.Z0 = c.take(2 * LR_MAX * R_MAX * 8);
  const size_t nt = hp.tiles.size();
  L.part = c.take(prows_for(hp) * PSTRIDE * 8);
  L.red_stage = c.take(RED_SPLIT * 8 * 8);
  L.red_count = c.take(4);
  L.gram = c.take(nt * (size_t)Rcap * Rcap * 8);
  L.tiles = c.take(nt * sizeof(Tile));
  L.ilist = c.take(sizeof(int32_t));
  if (hp.rk > 0) {
    const size_t rk = hp.rk, nlc = hp.nlc;
    L.Kc = c.take(n * rk * sz);
    L.Kc64 = prec == 0 ? L.Kc : c.take(n * rk * 8);
    L.Dc = c.take(hp.Dc.size() * 8);
    L.lc_con = c.take(nlc * 4);
    L.lc_off = c.take((nlc + 1) * 4);
    L.lc_doff = c.take(nlc * 4);
    L.lc_of_con = c.take(m * 4);
    L.lc_term = c.take(rk * 4);
    L.lc_part = c.take(nt * rk * R_MAX * 8);
    L.lc_Y = c.take(rk * R_MAX * 8);
    L.lc_Z = c.take(2 * rk * R_MAX * 8);
    L.lc_T = c.take(nlc * 8);
    L.lc_v = c.take(rk * 8);
    L.lc_zv = c.take(rk * 8);
    L.lc_Tv = c.take(nlc * 8);
    for (int z = 0; z < 2; ++z) L.lc_W[z] = c.take(n * Rcap * 8);
    L.lc_wv = c.take(n * 8);
  }
  if (hp.cdp_L > 0) {
    // masks, spectra for up to Rcap columns (and their scaled copy), the
    // constraint values, the adjoint blocks of the two Z-slots
    const size_t nc = hp.cdp_nc, Lp = hp.cdp_L;
    L.cdp_d = c.take(Lp * nc * 16);
    L.cdp_S = c.take(Lp * Rcap * nc * 16);
    L.cdp_S2 = c.take(Lp * Rcap * nc * 16);
    L.cdp_T = c.take(m * 8);
    L.cdp_Tv = c.take(m * 8);
    L.cdp_wv = c.take(n * 8);
    for (int z = 0; z < 2; ++z) L.cdp_W[z] = c.take(n * Rcap * 8);
  }
  L.total = c.off;
  return L;
}

size_t instance_bytes(const HostProblem &hp, int prec, int Rcap, int kmax) {
  return make_layout(hp, prec, Rcap, kmax).total;
}

// ------------------------------------------------------------------ pool
hallar_status pool_init(Pool &P, int max_slots, int prec, const hallar_options &opts, hipStream_t stream,
                        size_t arena_bytes, int64_t tiles_cap, std::string &err) {
  P.prec = prec;
  P.opts = opts;
  P.stream = stream;
  P.max_slots = max_slots;
  P.slots.resize(max_slots);
  P.h_insts.assign(max_slots, InstDev{});
  HL_TRY(hipMalloc((void **)&P.d_insts, sizeof(InstDev) * max_slots), "hipMalloc insts");
  HL_TRY(hipMalloc((void **)&P.d_prm, sizeof(InstParams) * max_slots), "hipMalloc params");
  HL_TRY(hipMalloc((void **)&P.d_res, sizeof(InstRes) * max_slots), "hipMalloc results");
  HL_TRY(hipHostMalloc((void **)&P.h_prm, sizeof(InstParams) * max_slots, hipHostMallocDefault), "hipHostMalloc params");
  HL_TRY(hipHostMalloc((void **)&P.h_res, sizeof(InstRes) * max_slots, hipHostMallocDefault), "hipHostMalloc results");
  std::memset(P.h_prm, 0, sizeof(InstParams) * max_slots);
  std::memset(P.h_res, 0, sizeof(InstRes) * max_slots);
  HL_TRY(hipMemset(P.d_res, 0, sizeof(InstRes) * max_slots), "hipMemset results");
  P.tiles_cap = std::max<int64_t>(tiles_cap, 4096);
  HL_TRY(hipMalloc((void **)&P.d_tiles, sizeof(Tile) * P.tiles_cap), "hipMalloc tiles");
  HL_TRY(hipHostMalloc((void **)&P.h_tiles, sizeof(Tile) * P.tiles_cap, hipHostMallocDefault), "hipHostMalloc tiles");
  P.ilist_cap = 3 * (int64_t)max_slots + 16;
  HL_TRY(hipMalloc((void **)&P.d_ilist, sizeof(int32_t) * P.ilist_cap), "hipMalloc ilist");
  HL_TRY(hipHostMalloc((void **)&P.h_ilist, sizeof(int32_t) * P.ilist_cap, hipHostMallocDefault), "hipHostMalloc ilist");
  P.up_cap = std::max<int64_t>(1 << 16, (int64_t)std::min(max_slots, 256) * KMAX * KMAX);
  P.dl_cap = P.up_cap;
  HL_TRY(hipMalloc((void **)&P.d_up, sizeof(double) * P.up_cap), "hipMalloc upload");
  HL_TRY(hipHostMalloc((void **)&P.h_up, sizeof(double) * P.up_cap, hipHostMallocDefault), "hipHostMalloc upload");
  HL_TRY(hipMalloc((void **)&P.d_dl, sizeof(double) * P.dl_cap), "hipMalloc download");
  HL_TRY(hipHostMalloc((void **)&P.h_dl, sizeof(double) * P.dl_cap, hipHostMallocDefault), "hipHostMalloc download");
  for (int q = 0; q < Pool::NSIDE; ++q) {
    HL_TRY(hipStreamCreateWithFlags(&P.side[q], hipStreamNonBlocking), "hipStreamCreate");
    HL_TRY(hipEventCreateWithFlags(&P.ev_join[q], hipEventDisableTiming), "hipEventCreate");
  }
  HL_TRY(hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming), "hipEventCreate");
  if (opts.graphs) {
    HL_TRY(hipStreamCreateWithFlags(&P.gst, hipStreamNonBlocking), "hipStreamCreate");
    HL_TRY(hipEventCreateWithFlags(&P.ev_gfork, hipEventDisableTiming), "hipEventCreate");
    HL_TRY(hipEventCreateWithFlags(&P.ev_gjoin, hipEventDisableTiming), "hipEventCreate");
  }
  P.profile = opts.profile != 0;
  P.prof_level = opts.profile;
  if (P.profile) {
    P.events.resize(8192);
    for (auto &ev : P.events) HL_TRY(hipEventCreate(&ev), "hipEventCreate");
  }
  if (arena_bytes > 0) {
    if (!P.arena.init(arena_bytes, err)) return HALLAR_E_OOM;
    P.use_arena = true;
    P.budget = arena_bytes;
  }
  return HALLAR_OK;
}

void pool_release(Pool &P) {
  if (P.opts.verbose && P.rounds > 0)
    fprintf(stderr,
            "[hallar] pool: %lld rounds (%lld replayed as graphs, %lld captured), host seconds prep %.3f launch %.3f "
            "wait %.3f resume %.3f\n",
            (long long)P.rounds, (long long)P.graph_replays, (long long)P.graph_captures, P.t_prep, P.t_launch,
            P.t_wait, P.t_resume);
  P.workers.reset();
  for (auto &kv : P.graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  P.graphs.clear();
  for (int s = 0; s < (int)P.slots.size(); ++s)
    if (P.slots[s]) slot_unload(P, s);
  auto fr = [](void *p) {
    if (p) (void)hipFree(p);
  };
  auto frh = [](void *p) {
    if (p) (void)hipHostFree(p);
  };
  fr(P.d_insts); fr(P.d_prm); fr(P.d_res); fr(P.d_tiles); fr(P.d_ilist); fr(P.d_up); fr(P.d_dl);
  frh(P.h_prm); frh(P.h_res); frh(P.h_tiles); frh(P.h_ilist); frh(P.h_up); frh(P.h_dl);
  for (auto &ev : P.events) (void)hipEventDestroy(ev);
  P.events.clear();
  for (int q = 0; q < Pool::NSIDE; ++q) {
    if (P.side[q]) (void)hipStreamDestroy(P.side[q]);
    if (P.ev_join[q]) (void)hipEventDestroy(P.ev_join[q]);
    P.side[q] = nullptr;
    P.ev_join[q] = nullptr;
  }
  if (P.ev_fork) (void)hipEventDestroy(P.ev_fork);
  P.ev_fork = nullptr;
  if (P.gst) (void)hipStreamDestroy(P.gst);
  if (P.ev_gfork) (void)hipEventDestroy(P.ev_gfork);
  if (P.ev_gjoin) (void)hipEventDestroy(P.ev_gjoin);
  P.gst = nullptr;
  P.ev_gfork = P.ev_gjoin = nullptr;
  P.d_insts = nullptr;
  P.arena.release();
}

int pool_active(const Pool &P) {
  int c = 0;
  for (auto &s : P.slots)
    if (s && s->used && !s->done && s->task) ++c;
  return c;
}

template <typename T>
static void put(char *base, size_t off, const std::vector<T> &v, hipStream_t st) {
  if (!v.empty()) (void)hipMemcpyAsync(base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// ------------------------------------------------------------------ FFTs
// rocFFT plans of a coded-diffraction instance: complex double, length n_c,
// in place, forward and inverse (both unnormalised), one pair per batch of
// L r transforms (r the live columns of an operand, 1 for the Lanczos and
// Frank-Wolfe vectors), made when first needed; one work buffer serves them
// all (an instance's transforms run one after another on its stream).
struct CdpFft {
  struct Pair {
    rocfft_plan fwd = nullptr, inv = nullptr;
  };
  size_t len = 0;
  std::map<int, Pair> plans;
  rocfft_execution_info info = nullptr;
  void *work = nullptr;
  size_t work_bytes = 0;
};

static void cdp_release(CdpFft *F) {
  if (!F) return;
  for (auto &kv : F->plans) {
    if (kv.second.fwd) rocfft_plan_destroy(kv.second.fwd);
    if (kv.second.inv) rocfft_plan_destroy(kv.second.inv);
  }
  if (F->info) rocfft_execution_info_destroy(F->info);
  if (F->work) (void)hipFree(F->work);
  delete F;
}

// The plan pair for `batch` transforms, made on first use.  A work buffer
// larger than the one held is allocated after the device has drained (the
// old one may still be in use by transforms already enqueued).
static const CdpFft::Pair *cdp_plan(CdpFft &F, int batch, std::string &err) {
  auto it = F.plans.find(batch);
  if (it != F.plans.end()) return &it->second;
  CdpFft::Pair pr;
  if (rocfft_plan_create(&pr.fwd, rocfft_placement_inplace, rocfft_transform_type_complex_forward,
                         rocfft_precision_double, 1, &F.len, (size_t)batch, nullptr) != rocfft_status_success ||
      rocfft_plan_create(&pr.inv, rocfft_placement_inplace, rocfft_transform_type_complex_inverse,
                         rocfft_precision_double, 1, &F.len, (size_t)batch, nullptr) != rocfft_status_success) {
    if (pr.fwd) rocfft_plan_destroy(pr.fwd);
    err = "rocfft_plan_create failed (length " + std::to_string(F.len) + ", batch " + std::to_string(batch) + ")";
    return nullptr;
  }
  size_t need = 0;
  for (rocfft_plan pl : {pr.fwd, pr.inv}) {
    size_t wb = 0;
    if (rocfft_plan_get_work_buffer_size(pl, &wb) == rocfft_status_success) need = std::max(need, wb);
  }
  if (need > F.work_bytes) {
    (void)hipDeviceSynchronize();
    if (F.work) (void)hipFree(F.work);
    F.work = nullptr;
    F.work_bytes = 0;
    if (hipMalloc(&F.work, need) != hipSuccess ||
        rocfft_execution_info_set_work_buffer(F.info, F.work, need) != rocfft_status_success) {
      rocfft_plan_destroy(pr.fwd);
      rocfft_plan_destroy(pr.inv);
      err = "FFT work buffer allocation failed";
      return nullptr;
    }
    F.work_bytes = need;
  }
  return &(F.plans[batch] = pr);
}

static hallar_status cdp_plans(const HostProblem &h, int prec, int Rcap, CdpFft *&out, std::string &err) {
  static std::once_flag once;
  static rocfft_status setup = rocfft_status_success;
  std::call_once(once, [] { setup = rocfft_setup(); });
  if (setup != rocfft_status_success) {
    err = "rocfft_setup failed";
    return HALLAR_E_HIP;
  }
  CdpFft *F = new CdpFft;
  F->len = (size_t)h.cdp_nc;
  if (rocfft_execution_info_create(&F->info) != rocfft_status_success) {
    cdp_release(F);
    err = "rocfft_execution_info_create failed";
    return HALLAR_E_HIP;
  }
  // the widest batch first (its work buffer is the largest), then the vectors'
  (void)prec;
  if (!cdp_plan(*F, h.cdp_L * Rcap, err) || !cdp_plan(*F, h.cdp_L, err)) {
    cdp_release(F);
    return HALLAR_E_HIP;
  }
  out = F;
  return HALLAR_OK;
}

// one batch of in-place transforms on the instance's stream
// (a failure is recorded in P.launch_err and ends the round with an error)
static void cdp_exec(Pool &P, CdpFft &F, int batch, bool forward, void *buf, hipStream_t st) {
  if (P.launch_err != HALLAR_OK) return;
  const CdpFft::Pair *pr = cdp_plan(F, batch, P.err);
  if (!pr) {
    P.launch_err = HALLAR_E_HIP;
    return;
  }
  void *io[1] = {buf};
  if (rocfft_execution_info_set_stream(F.info, st) != rocfft_status_success ||
      rocfft_execute(forward ? pr->fwd : pr->inv, io, nullptr, F.info) != rocfft_status_success) {
    P.err = "rocfft_execute failed (batch " + std::to_string(batch) + ")";
    P.launch_err = HALLAR_E_HIP;
  }
}

// Spectra F (d_l * u_c) of the first Rc columns of role xrole (vsrc 0, rows
// of stride R) or of a vector (vsrc 1: the Lanczos vector, 2: the Ritz
// vector; R = Rc = 1), and when out >= 0 their |.|^2 sums into cdp_T (out 0)
// or cdp_Tv (out 1).
static void cdp_forward(Pool &P, int s, hipStream_t st, int xrole, int vsrc, int R, int Rc, int out) {
  Slot &S = *P.slots[s];
  const size_t L = S.hp.cdp_L, nc = S.hp.cdp_nc;
  op_cdp_pack(P.prec, st, P.d_insts, s, xrole, vsrc, R, Rc, L * Rc * nc, (int)nc);
  cdp_exec(P, *S.fft, (int)(L * Rc), true, S.dev.cdp_S, st);
  if (out >= 0) op_cdp_abs2(st, P.d_insts, s, Rc, out, L * nc);
}

// The adjoint block sum_l conj(d_l) F^H (y_l * spectra) of the last
// cdp_forward (Rc columns), with multipliers mult (null: the instance's y'),
// into cdp_W[zsel] (vec 0, R columns, those from Rc on zero) or cdp_wv
// (vec 1, R = Rc = 1).
static void cdp_adjoint(Pool &P, int s, hipStream_t st, int R, int Rc, int zsel, int vec, const double *mult) {
  Slot &S = *P.slots[s];
  const size_t L = S.hp.cdp_L, nc = S.hp.cdp_nc;
  op_cdp_scale(st, P.d_insts, s, Rc, mult, L * Rc * nc);
  cdp_exec(P, *S.fft, (int)(L * Rc), false, S.dev.cdp_S2, st);
  op_cdp_gather(st, P.d_insts, s, R, Rc, zsel, vec, (size_t)R * nc, (int)nc);
}

hallar_status slot_load(Pool &P, int s, HostProblem &&hp, std::string &err) {
  P.tile_epoch++;
  auto sl = std::make_unique<Slot>();
  Slot &S = *sl;
  S.hp = std::move(hp);
  HostProblem &h = S.hp;
  if (P.opts.lower_gather) h.low_recompute = false;
  S.Rcap = rcap_for(P.opts, P.prec);
  S.kmax = kmax_for(P.opts, h.n);
  const Layout L = make_layout(h, P.prec, S.Rcap, S.kmax);
  if (h.cdp_L > 0) {
    const hallar_status fs = cdp_plans(h, P.prec, S.Rcap, S.fft, err);
    if (fs != HALLAR_OK) return fs;
  }
  char *base = nullptr;
  if (P.use_arena) {
    const size_t off = P.arena.alloc(L.total);
    if (off == SIZE_MAX) {
      cdp_release(S.fft);
      S.fft = nullptr;
      err = "pool budget exhausted";
      return HALLAR_E_OOM;
    }
    S.slab_off = off;
    base = P.arena.base() + off;
  } else {
    if (hipMalloc((void **)&base, L.total) != hipSuccess) {
      cdp_release(S.fft);
      S.fft = nullptr;
      err = "hipMalloc of the instance slab failed";
      return HALLAR_E_OOM;
    }
  }
  S.slab = base;
  S.slab_bytes = L.total;
  hipStream_t st = P.stream;
  for (auto &t : h.tiles) t.inst = s;
  // operator-type copies
  const bool f32 = P.prec != 0;
  auto conv = [&](const std::vector<double> &v, size_t off) {
    if (v.empty()) return;
    if (f32) {
      std::vector<float> f(v.begin(), v.end());
      (void)hipMemcpy(base + off, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    } else {
      (void)hipMemcpy(base + off, v.data(), v.size() * 8, hipMemcpyHostToDevice);
    }
  };
  put(base, L.rowptr_u, h.rowptr_u, st);
  put(base, L.col_u, h.col_u, st);
  put(base, L.pcon, h.pcon, st);
  conv(h.c_u, L.c_u);
  conv(h.pa, L.pa);
  put(base, L.c64, h.c_u, st);
  put(base, L.pa64, h.pa, st);
  put(base, L.rowptr_l, h.rowptr_l, st);
  put(base, L.col_l, h.col_l, st);
  put(base, L.c_diag, h.c_diag, st);
  put(base, L.pid_l, h.pid_l, st);
  put(base, L.b, h.b, st);
  conv(h.K0, L.K0);
  put(base, L.K064, h.K0, st);
  put(base, L.D0, h.D0, st);
  if (!h.direct) {
    put(base, L.eptr, h.eptr, st);
    put(base, L.econ, h.econ, st);
    put(base, L.ea64, h.ea, st);
    put(base, L.ew64, h.ew, st);
    put(base, L.cptr, h.cptr, st);
    put(base, L.cent, h.cent, st);
    put(base, L.epair, h.epair, st);
  }
  if (h.rk > 0) {
    conv(h.Kc, L.Kc);
    if (f32) put(base, L.Kc64, h.Kc, st);
    put(base, L.Dc, h.Dc, st);
    put(base, L.lc_con, h.lc_con, st);
    put(base, L.lc_off, h.lc_off, st);
    put(base, L.lc_doff, h.lc_doff, st);
    put(base, L.lc_of_con, h.lc_of_con, st);
    put(base, L.lc_term, h.lc_term, st);
    (void)hipMemsetAsync(base + L.lc_Z, 0, 2 * (size_t)h.rk * R_MAX * 8, st);
    (void)hipMemsetAsync(base + L.lc_zv, 0, (size_t)h.rk * 8, st);
    for (int z = 0; z < 2; ++z) (void)hipMemsetAsync(base + L.lc_W[z], 0, (size_t)h.n * S.Rcap * 8, st);
    (void)hipMemsetAsync(base + L.lc_wv, 0, (size_t)h.n * 8, st);
  }
  if (h.cdp_L > 0) {
    put(base, L.cdp_d, h.cdp_d, st);
    for (int z = 0; z < 2; ++z) (void)hipMemsetAsync(base + L.cdp_W[z], 0, (size_t)h.n * S.Rcap * 8, st);
    (void)hipMemsetAsync(base + L.cdp_wv, 0, (size_t)h.n * 8, st);
  }
  put(base, L.tiles, h.tiles, st);
  std::vector<int32_t> il{s};
  put(base, L.ilist, il, st);
  if (h.m > 0) (void)hipMemsetAsync(base + L.p, 0, (size_t)h.m * 8, st);
  // {p_l, b_l} copies start defined (the standalone SDDMM's epilogue reads them)
  if (h.direct && h.npairs > 0) (void)hipMemsetAsync(base + L.upb, 0, (size_t)h.npairs * 16, st);
  if (h.low_recompute && h.nlower > 0) (void)hipMemsetAsync(base + L.low_pb, 0, (size_t)h.nlower * 16, st);
  (void)hipMemsetAsync(base + L.Z0, 0, 2 * LR_MAX * R_MAX * 8, st);
  (void)hipMemsetAsync(base + L.red_count, 0, 4, st);
  for (int q = 0; q < NBUF; ++q) (void)hipMemsetAsync(base + L.buf[q], 0, (size_t)h.n * S.Rcap * (f32 ? 4 : 8), st);
  if (hipStreamSynchronize(st) != hipSuccess) {
    err = "upload of the instance failed";
    return HALLAR_E_HIP;
  }
  InstDev &D = P.h_insts[s];
  D = InstDev{};
  D.n = h.n;
  D.m = h.m;
  D.npairs = (int32_t)h.npairs;
  D.nlower = (int32_t)h.nlower;
  D.r0 = h.r0;
  D.direct = h.direct ? 1 : 0;
  D.ntiles = (int32_t)h.tiles.size();
  D.prows = (int32_t)prows_for(h);
  auto at = [&](size_t off) { return (void *)(base + off); };
  D.rowptr_u = (const int32_t *)at(L.rowptr_u);
  D.col_u = (const int32_t *)at(L.col_u);
  D.pcon = (const int32_t *)at(L.pcon);
  D.c_u = h.has_c ? at(L.c_u) : nullptr;
  D.pa = at(L.pa);
  D.c64 = h.has_c ? (const double *)at(L.c64) : nullptr;
  D.pa64 = (const double *)at(L.pa64);
  D.pa_uniform = h.pa_uniform ? 1 : 0;
  D.con_rule = h.direct ? h.con_rule : 0;
  D.pa_const = h.pa_const;
  D.c_diag_only = h.c_diag_only ? 1 : 0;
  D.c_diag = h.c_diag_only ? (const double *)at(L.c_diag) : nullptr;
  D.b = (const double *)at(L.b);
  D.rowptr_l = (const int32_t *)at(L.rowptr_l);
  D.col_l = (const int32_t *)at(L.col_l);
  D.pid_l = (const int32_t *)at(L.pid_l);
  D.low_mode = h.low_recompute ? 1 : 0;
  D.low_pb = h.low_recompute ? (double *)at(L.low_pb) : nullptr;
  D.upb = h.direct ? (double *)at(L.upb) : nullptr;
  D.K0 = at(L.K0);
  D.K064 = (const double *)at(L.K064);
  D.D0 = (const double *)at(L.D0);
  if (!h.direct) {
    D.eptr = (const int32_t *)at(L.eptr);
    D.econ = (const int32_t *)at(L.econ);
    D.ea64 = (const double *)at(L.ea64);
    D.ew64 = (const double *)at(L.ew64);
    D.cptr = (const int32_t *)at(L.cptr);
    D.cent = (const int32_t *)at(L.cent);
    D.epair = (const int32_t *)at(L.epair);
    D.Bpair = (double *)at(L.Bpair);
  }
  for (int q = 0; q < NBUF; ++q) D.buf[q] = at(L.buf[q]);
  D.m_xt = at(L.m_xt);
  D.m_yp = at(L.m_yp);
  D.p = (double *)at(L.p);
  D.yp = (double *)at(L.yp);
  D.TY = (double *)at(L.TY);
  D.Ty = (double *)at(L.Ty);
  D.m64 = (double *)at(L.m64);
  D.m64_low = (double *)at(L.m64_low);
  D.V = (double *)at(L.V);
  D.V2 = (double *)at(L.V2);
  D.w = (double *)at(L.w);
  D.lzv = (double *)at(L.lzv);
  D.hcoef = (double *)at(L.hcoef);
  D.Z0 = (double *)at(L.Z0);
  D.up_base = P.d_up;
  D.dl_base = P.d_dl;
  D.part = (double *)at(L.part);
  D.red_stage = (double *)at(L.red_stage);
  D.red_count = (uint32_t *)at(L.red_count);
  D.gram = (double *)at(L.gram);
  D.prm = P.d_prm + s;
  D.res = P.d_res + s;
  D.rk = h.rk;
  D.nlc = h.nlc;
  if (h.rk > 0) {
    D.Kc = at(L.Kc);
    D.Kc64 = (const double *)at(L.Kc64);
    D.Dc = (const double *)at(L.Dc);
    D.lc_con = (const int32_t *)at(L.lc_con);
    D.lc_off = (const int32_t *)at(L.lc_off);
    D.lc_doff = (const int32_t *)at(L.lc_doff);
    D.lc_of_con = (const int32_t *)at(L.lc_of_con);
    D.lc_term = (const int32_t *)at(L.lc_term);
    D.lc_part = (double *)at(L.lc_part);
    D.lc_Y = (double *)at(L.lc_Y);
    D.lc_Z = (double *)at(L.lc_Z);
    D.lc_T = (double *)at(L.lc_T);
    D.lc_v = (double *)at(L.lc_v);
    D.lc_zv = (double *)at(L.lc_zv);
    D.lc_Tv = (double *)at(L.lc_Tv);
    for (int z = 0; z < 2; ++z) D.lc_W[z] = (double *)at(L.lc_W[z]);
    D.lc_wv = (double *)at(L.lc_wv);
  }
  D.cdp_L = h.cdp_L;
  D.cdp_nc = h.cdp_nc;
  if (h.cdp_L > 0) {
    D.cdp_d = (const double2 *)at(L.cdp_d);
    D.cdp_S = (double2 *)at(L.cdp_S);
    D.cdp_S2 = (double2 *)at(L.cdp_S2);
    D.cdp_T = (double *)at(L.cdp_T);
    D.cdp_Tv = (double *)at(L.cdp_Tv);
    D.cdp_wv = (double *)at(L.cdp_wv);
    for (int z = 0; z < 2; ++z) D.cdp_W[z] = (double *)at(L.cdp_W[z]);
  }
  S.dev = D;
  S.used = true;
  S.free_bufs.clear();
  for (int q = NBUF - 1; q >= 0; --q) S.free_bufs.push_back(q);
  S.prm = InstParams{};
  S.prm.tau2 = h.tau2;
  S.prm.tau = std::sqrt(h.tau2);
  S.cur_R = r_bucket(1, P.prec);
  S.cur_r = 1;
  P.slots[s] = std::move(sl);
  P.insts_dirty = true;
  // tiles / ilist of the slot live in its slab
  return HALLAR_OK;
}

void slot_unload(Pool &P, int s) {
  P.tile_epoch++;
  if (!P.slots[s]) return;
  Slot &S = *P.slots[s];
  if (S.task) {
    delete S.task;
    S.task = nullptr;
  }
  if (S.slab) {
    if (P.use_arena) P.arena.free(S.slab_off, S.slab_bytes);
    else (void)hipFree(S.slab);
  }
  cdp_release(S.fft);
  S.fft = nullptr;
  P.slots[s].reset();
  P.h_insts[s] = InstDev{};
  P.insts_dirty = true;
}

// ------------------------------------------------------------------ rounds
int PendingOp::key() const {
  return (int)code * 1000003 + R * 131 + R2 * 17 + xrole * 7 + (msel + 1) * 3 + wT * 5 + wyp * 11 + zsel * 13 +
         src * 19 + dst * 23;
}

struct Group {
  OpCode code;
  int R, R2;
  int64_t t0, nt;
  int64_t i0, ni;
  int64_t gi0, gni;  // general-mode instances
  int64_t di0, dni;  // direct-mode instances
  int maxm, maxp;
  const PendingOp *op;
  int first_slot;
  int steps;               // Lanczos steps: the largest request of the group
  std::vector<int> slots;
};

// ------------------------------------------------------------------ profiling
// Whether an instance's FISTA trials run as the fused kernel: a property of
// the instance (and the pool's options) alone, and part of the grouping key,
// so that an instance takes the same kernels -- and produces the same bits --
// alone, in a batch or in the served mix.
static bool trial_fuses(const Pool &P, int s) {
  const HostProblem &h = P.slots[s]->hp;
  return !P.opts.unfused_trial && h.direct && h.low_recompute && h.r0 == 0;
}

// grouping key of a slot's pending operation: packs are never merged (each
// has its own source), trials of fused and unfused instances never are
static int64_t group_key(const Pool &P, int s) {
  const PendingOp &o = P.slots[s]->op;
  int64_t k = o.key();
  if (o.code == OP_PACK) k += (int64_t)s * 7919;
  if (o.code == OP_TRIAL && trial_fuses(P, s)) k += 104729;
  return k;
}

struct ProfScope {
  Pool &P;
  int cls, e0 = -1;
  double bytes;
  hipStream_t st;
  ProfScope(Pool &p, int c, double b, hipStream_t s) : P(p), cls(c), bytes(b), st(s) {
    const bool timed =
        P.prof_level == 1 || c == KC_SDDMM || c == KC_SPMM || c == KC_FUSED || c == KC_LZ_SPMV || c == KC_CDP;
    if (P.profile && timed && P.ev_used + 2 <= (int)P.events.size()) {
      e0 = P.ev_used;
      P.ev_used += 2;
      (void)hipEventRecord(P.events[e0], st);
    }
  }
  ~ProfScope() {
    if (e0 >= 0) {
      (void)hipEventRecord(P.events[e0 + 1], st);
      P.recs.push_back(ProfRec{cls, e0, e0 + 1, bytes});
    }
  }
};

void prof_flush(Pool &P) {
  for (const ProfRec &r : P.recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P.events[r.e0], P.events[r.e1]) == hipSuccess) {
      P.prof_ms[r.cls] += ms;
      P.prof_n[r.cls] += 1;
      P.prof_bytes[r.cls] += r.bytes;
    }
  }
  P.recs.clear();
  P.ev_used = 0;
}

// algorithmic bytes of one launch over the instances of a group
struct GroupBytes {
  double sddmm = 0, spmm_core = 0, fused = 0, urow = 0, lz_spmv = 0, vec_n8 = 0;
};

static void launch_group(Pool &P, const Group &g, hipStream_t st);

// Algorithmic bytes of the coded-diffraction operator's steps for Rc live
// columns of element size xsz in a bucket of R (spectra S = L Rc nc complex
// doubles, each transform one read and one write of S): part 0 packs
// d_l * u_c (reads the columns and the masks, writes S) and transforms;
// part 1 sums |S|^2 into the m constraint values; part 2 scales by the
// multipliers into S2, transforms back and gathers the n x R block.
static double cdp_bytes(const HostProblem &h, double xsz, int R, int Rc, int part) {
  const double S = (double)h.cdp_L * Rc * h.cdp_nc * 16.0, masks = (double)h.cdp_L * h.cdp_nc * 16.0;
  if (part == 0) return h.n * Rc * xsz + masks + 3.0 * S;
  if (part == 1) return S + h.m * 8.0;
  return 2.0 * S + h.m * 8.0 + 2.0 * S + S + masks + h.n * R * 8.0;
}

// live columns of slot s's pending operation in a group of bucket R
static int live_cols(const Pool &P, int s, int R) {
  const int r = P.slots[s]->op.rlive;
  return r > 0 ? std::min(r, R) : R;
}

static GroupBytes group_bytes(const Pool &P, const std::vector<int> &slots, int R) {
  GroupBytes b;
  const double sz = P.prec == 0 ? 8.0 : 4.0;
  for (int s : slots) {
    const HostProblem &h = P.slots[s]->hp;
    const double n = h.n, Pp = (double)h.npairs, nl = (double)h.nlower, m = h.m;
    b.urow += n * R * sz;
    // factor rows once, row pointers, per pair: column, then (direct) constraint
    // id, {p_l, b_l} and the coefficient unless shared, the objective entry
    // unless diagonal-only; general mode reads b and p per constraint
    const double sd = n * R * sz + (n + 1) * 4 +
                      Pp * (4 + (h.direct ? (h.con_rule ? 0 : 4) + 16 + (h.pa_uniform ? 0 : sz) : 0) +
                            (h.has_c && !h.c_diag_only ? sz : 0)) +
                      (h.c_diag_only ? 8 * n : 0) + (h.direct ? 0 : 16 * m);
    b.sddmm += sd;
    // lower half: column and pair id, or column and (p_l, b_l) when recomputed
    b.spmm_core += n * R * sz + 2 * (n + 1) * 4 + Pp * (4 + sz) + nl * (h.low_recompute ? 20 : 8);
    // fused trial: the SDDMM's reads (no pair values written), the lower
    // row pointers, columns and {p_l, b_l}; the SpMM epilogue is added by
    // the caller
    b.fused += sd + (n + 1) * 4 + nl * 20;
    b.lz_spmv += n * 8 * 2 + Pp * (8 + 4) + nl * 12 + 2 * (n + 1) * 4;  // lower: column + lower-order value
    b.vec_n8 += n * 8;
  }
  return b;
}

static void launch_group(Pool &P, const Group &g, hipStream_t st) {
  const Tile *T = P.d_tiles + g.t0;
  const int nt = (int)g.nt;
  const int32_t *IL = P.d_ilist + g.i0;
  const int ni = (int)g.ni;
  const int32_t *GL = P.d_ilist + g.gi0;
  const int gni = (int)g.gni;
  const int32_t *DL = P.d_ilist + g.di0;
  const int dni = (int)g.dni;
  const InstDev *D = P.d_insts;
  const int prec = P.prec;
  const int R = g.R;
  const PendingOp &o = *g.op;
  const GroupBytes B = P.profile ? group_bytes(P, g.slots, R) : GroupBytes{};
  const double sz = prec == 0 ? 8.0 : 4.0;
  double msum = 0, psum = 0;
  bool any_lr = false;
  int64_t max_pb = 0;  // entries of the {p_l, b_l} copies refreshed when p changes
  int64_t max_nl = 0, nrows = 0;
  int max_rk = 0;  // columns of the constraints' low-rank parts
  std::vector<int> cdps;  // instances with coded-diffraction constraints
  // the trial's SDDMM and gradient SpMM run as one kernel when every instance
  // recomputes its lower half, has no low-rank objective term (its product
  // is reduced between the two) and the rows are narrow
  bool fuse = gni == 0 && trial_fusable(prec, R);
  for (int s : g.slots) {
    const HostProblem &h = P.slots[s]->hp;
    fuse = fuse && trial_fuses(P, s);
    msum += h.m;
    psum += (double)h.npairs;
    any_lr = any_lr || h.r0 > 0;
    if (h.direct) max_pb = std::max<int64_t>(max_pb, h.npairs);
    if (h.low_recompute) max_pb = std::max<int64_t>(max_pb, h.nlower);
    max_nl = std::max<int64_t>(max_nl, h.nlower);
    nrows += h.n;
    max_rk = std::max(max_rk, h.rk);
    if (h.cdp_L > 0) cdps.push_back(s);
  }
  // the trial's reduces are split over several workgroups for instances with
  // thousands of tiles (one workgroup then waits on its own loads); each
  // instance decides by its own tile count, so the launch is split when any
  // instance of the group is that large
  int64_t max_tiles = 0;
  for (int s : g.slots) max_tiles = std::max<int64_t>(max_tiles, (int64_t)P.slots[s]->hp.tiles.size());
  const int split = max_tiles >= RED_SPLIT_MIN_TILES ? 1 : 0;
  auto red = [&](int op, int zsel) {
    ProfScope ps(P, KC_REDUCE, 0.0, st);
    op_reduce(st, IL, ni, D, op, zsel, R, (op == RDH_TRIAL_FUSED || op == RDH_YP_PROJ) ? split : 0);
  };
  auto sddmm = [&](int xrole, int msel, int wT, int wyp, int red_op, int zsel) {
    const double sbytes = B.sddmm + (msel >= 0 ? psum * sz : 0.0) + (wT ? 8 * msum : 0.0) + (wyp ? 8 * msum : 0.0);
    if (cdps.empty()) {
      ProfScope ps(P, KC_SDDMM, sbytes, st);
      if (any_lr) op_lr_dots(prec, R, st, T, nt, D, xrole);
      op_sddmm(prec, R, st, T, nt, D, xrole, msel, wT, wyp);
      if (gni > 0) {
        if (max_rk > 0) {
          // the constraints' low-rank parts of T (Algorithm 3) before the AL
          // epilogue of each constraint; their SpMM block after it, when the
          // pair values are formed for an SpMM (Algorithm 5)
          op_lc_kty(prec, R, st, T, nt, D, max_rk, xrole, 0);
          op_lc_sum(st, GL, gni, D, max_rk, R, 0);
          op_lc_red(st, GL, gni, D, LC_Y_T, R, zsel);
        }
        op_gen_constraints(prec, st, GL, gni, g.maxm, D, wT);
        if (max_rk > 0 && msel >= 0) {
          op_lc_red(st, GL, gni, D, LC_Z, R, zsel);
          op_lc_kz(prec, R, st, T, nt, D, zsel, 0);
        }
        if (msel >= 0) op_pairvals(prec, st, GL, gni, g.maxp, D, msel, nullptr, 1);
      }
    } else {
      // coded-diffraction instances (general mode): their constraint values
      // before the AL epilogue, their adjoint block after it when the pair
      // values are formed for an SpMM; timed as a class of their own
      {
        ProfScope ps(P, KC_SDDMM, sbytes, st);
        if (any_lr) op_lr_dots(prec, R, st, T, nt, D, xrole);
        op_sddmm(prec, R, st, T, nt, D, xrole, msel, wT, wyp);
        if (max_rk > 0) {
          op_lc_kty(prec, R, st, T, nt, D, max_rk, xrole, 0);
          op_lc_sum(st, GL, gni, D, max_rk, R, 0);
          op_lc_red(st, GL, gni, D, LC_Y_T, R, zsel);
        }
      }
      for (int q : cdps) {
        const HostProblem &h = P.slots[q]->hp;
        const int rq = live_cols(P, q, R);
        ProfScope pc(P, KC_CDP, cdp_bytes(h, sz, R, rq, 0) + cdp_bytes(h, sz, R, rq, 1), st);
        cdp_forward(P, q, st, xrole, 0, R, rq, 0);
      }
      {
        ProfScope po(P, KC_OTHER, 0.0, st);
        op_gen_constraints(prec, st, GL, gni, g.maxm, D, wT);
        if (max_rk > 0 && msel >= 0) {
          op_lc_red(st, GL, gni, D, LC_Z, R, zsel);
          op_lc_kz(prec, R, st, T, nt, D, zsel, 0);
        }
        if (msel >= 0) op_pairvals(prec, st, GL, gni, g.maxp, D, msel, nullptr, 1);
      }
      if (msel >= 0)
        for (int q : cdps) {
          const int rq = live_cols(P, q, R);
          ProfScope pc(P, KC_CDP, cdp_bytes(P.slots[q]->hp, sz, R, rq, 2), st);
          cdp_adjoint(P, q, st, R, rq, zsel, 0, nullptr);
        }
    }
    red(red_op, zsel);
  };
  switch (g.code) {
    case OP_TRIAL:
      {
        ProfScope ps(P, KC_VEC, 4 * B.urow, st);
        op_combo(prec, R, st, T, nt, D, nrows);
      }
      // partial sums go to disjoint slots so that one reduce serves several
      // kernels: the extrapolation's with the fused trial's, the
      // projection's with the SDDMM at y+
      if (fuse) {
        {
          ProfScope ps(P, KC_FUSED, B.fused + 3 * B.urow, st);
          op_trial_fused(prec, R, st, T, nt, D, RXT);
        }
        red(RDH_TRIAL_FUSED, 0);
      } else {
        red(RDH_COMBO, 0);
        sddmm(RXT, 0, 0, 0, RDH_SDDMM_XT, 0);
        {
          ProfScope ps(P, KC_SPMM, B.spmm_core + 3 * B.urow, st);
          op_spmm(prec, R, st, T, nt, D, RXT, 0, 0, 0, SPM_TRIAL);
        }
        red(RDH_TRIAL_PROJ, 0);
      }
      {
        ProfScope ps(P, KC_VEC, 5 * B.urow, st);
        op_proj(prec, R, st, T, nt, D, nrows);
      }
      // the AL value at y+ only: the pair values there are needed by the
      // gradient at the accepted trial, which forms them itself (OP_GRAD)
      sddmm(RZ, -1, 0, 0, RDH_YP_PROJ, 1);
      break;
    case OP_GRAD:
      sddmm(RZ, 1, 0, 0, RDH_SDDMM_YP, 1);
      {
        ProfScope ps(P, KC_SPMM, B.spmm_core + 3 * B.urow, st);
        op_spmm(prec, R, st, T, nt, D, RZ, 1, 1, 0, SPM_AIPP);
      }
      red(RDH_AIPP, 0);
      break;
    case OP_EVAL:
      sddmm(o.xrole, o.msel, o.wT, o.wyp, RDH_EVAL, o.zsel);
      break;
    case OP_COPY:
      {
        ProfScope ps(P, KC_VEC, 2 * B.urow, st);
        op_copy_scale(prec, R, st, T, nt, D, o.src, o.dst);
      }
      red(RDH_NORM, 0);
      break;
    case OP_PACK:
      {
        // the solve's first op: U0, and the caller's dual start p copied into
        // the pair-order and lower-order {p_l, b_l} operands
        ProfScope ps(P, KC_OTHER, 0.0, st);
        op_pack_f64(prec, R, st, T, nt, D, o.ext, o.ext_r, o.ext_ld, o.dst, 1.0);
        if (max_pb > 0) op_refresh_pb(st, IL, ni, max_pb, D);
      }
      red(RDH_NORM, 0);
      break;
    case OP_LZ_BEGIN:
      {
        ProfScope ps(P, KC_OTHER, 0.0, st);
        if (dni > 0) op_pairvals(prec, st, DL, dni, g.maxp, D, 2, nullptr, 0);
        if (gni > 0) op_pairvals(prec, st, GL, gni, g.maxp, D, 2, nullptr, 1);
        // the Lanczos matrix is fixed for the whole run: its lower half in
        // lower order once, so every SpMV reads it contiguously
        op_lower_copy(st, IL, ni, max_nl, D);
        op_lz_start(st, T, nt, D);
      }
      red(RDH_LZ_START, 0);
      {
        ProfScope ps(P, KC_LZ_ORTH, 2 * B.vec_n8, st);
        op_lz_first(st, T, nt, D);
      }
      break;
    case OP_LZ_STEPS:
      // instances with fewer steps skip the extra ones (their lz_steps counter reaches 0)
      for (int k = 0; k < g.steps; ++k) {
        // algorithmic bytes of one Gram-Schmidt pass: a sweep of the basis for
        // the dots (fused into the SpMV) and one for the update, plus w; a
        // second pass, when the device runs it, is overhead
        double vsweep = 0, wbytes = 0;
        if (P.profile)
          for (int s : g.slots) {
            const Slot &S = *P.slots[s];
            if (k < S.prm.lz_steps) {
              vsweep += (double)(S.prm.lz_j + k + 1) * S.hp.n * 8;
              wbytes += 3.0 * S.hp.n * 8;
            }
          }
        const double vb = vsweep + wbytes;
        if (max_rk > 0) {
          // K^T v_j and its coefficients for the SpMV's low-rank parts
          op_lc_kty(prec, R, st, T, nt, D, max_rk, 0, 1);
          op_lc_sum(st, IL, ni, D, max_rk, 1, 1);
          op_lc_red(st, IL, ni, D, LC_V_LZ, 1, 0);
          op_lc_kz(prec, 1, st, T, nt, D, 0, 1);
        }
        for (int q : cdps) {
          // the coded-diffraction part of G v_j
          const HostProblem &h = P.slots[q]->hp;
          ProfScope pc(P, KC_CDP, cdp_bytes(h, 8.0, 1, 1, 0) + cdp_bytes(h, 8.0, 1, 1, 2), st);
          cdp_forward(P, q, st, 0, 1, 1, 1, -1);
          cdp_adjoint(P, q, st, 1, 1, 0, 1, nullptr);
        }
        {
          // SpMV fused with the first Gram-Schmidt dots
          ProfScope ps(P, KC_LZ_SPMV, B.lz_spmv + vsweep, st);
          op_lz_spmv_dots(st, T, nt, D);
        }
        {
          // classical Gram-Schmidt against the whole basis; the second pass
          // runs only where the first removed most of w (the device decides
          // per instance, the skipped kernels return at once)
          ProfScope ps(P, KC_LZ_ORTH, vb, st);
          op_reduce(st, IL, ni, D, RDH_LZ_H1, 0, R, 0);
          op_lz_update(st, T, nt, D, 0);
          op_reduce(st, IL, ni, D, RDH_LZ_CHECKH2, 0, R, 0);
          op_lz_update(st, T, nt, D, 1);
          op_reduce(st, IL, ni, D, RDH_LZ_FINAL, 0, R, 0);
          op_lz_scale(st, T, nt, D);
        }
      }
      break;
    case OP_LZ_RITZ:
    case OP_LZ_RESTART:
      {
        ProfScope ps(P, KC_LZ_ORTH, 0.0, st);
        op_lz_combine(st, T, nt, D, g.code == OP_LZ_RITZ ? 1 : 0);
      }
      break;
    case OP_FW_PREP:
      for (int q : cdps) {
        // A(v v^T) of the Ritz vector for the step size
        const HostProblem &h = P.slots[q]->hp;
        ProfScope pc(P, KC_CDP, cdp_bytes(h, 8.0, 1, 1, 0) + cdp_bytes(h, 8.0, 1, 1, 1), st);
        cdp_forward(P, q, st, 0, 2, 1, 1, 1);
      }
      {
        ProfScope ps(P, KC_OTHER, 0.0, st);
        op_fw_den(st, T, nt, D);
        if (gni > 0 && max_rk > 0) {
          op_lc_kty(prec, R, st, T, nt, D, max_rk, 0, 2);
          op_lc_sum(st, GL, gni, D, max_rk, 1, 2);
          op_lc_red(st, GL, gni, D, LC_V_FW, 1, 0);
        }
        if (gni > 0) op_fw_den_gen(st, GL, gni, g.maxm, D);
      }
      red(RDH_FW_DEN, 0);
      break;
    case OP_FW_APPLY:
      {
        ProfScope ps(P, KC_VEC, 0.0, st);
        op_fw_apply(prec, g.R2, R, st, T, nt, D, o.src, o.dst);
      }
      break;
    case OP_SETP:
      {
        ProfScope ps(P, KC_VEC, 0.0, st);
        op_set_p(st, IL, ni, g.maxm, D);
        if (max_pb > 0) op_refresh_pb(st, IL, ni, max_pb, D);
      }
      red(RDH_SETP, 0);
      break;
    case OP_GRAM:
      {
        ProfScope ps(P, KC_OTHER, 0.0, st);
        op_gram(prec, R, st, T, nt, D, o.src);
      }
      red(RDH_GRAM, 0);
      break;
    case OP_ROTATE:
      {
        ProfScope ps(P, KC_VEC, 0.0, st);
        op_rotate(prec, g.R2, R, st, T, nt, D, o.src, o.dst);
      }
      break;
    default:
      break;
  }
}

static hallar_status run_round(Pool &P, bool &did_work) {
  did_work = false;
  const double tr0 = now_s();
  std::vector<int> ready;
  for (int s = 0; s < (int)P.slots.size(); ++s) {
    auto &sp = P.slots[s];
    if (sp && sp->used && sp->has_op && !sp->done) ready.push_back(s);
  }
  if (ready.empty()) return HALLAR_OK;
  std::stable_sort(ready.begin(), ready.end(), [&](int a, int b) { return group_key(P, a) < group_key(P, b); });
  int64_t up_used = 0, dl_used = 0, t_used = 0;
  std::vector<int> run;
  for (int s : ready) {
    Slot &S = *P.slots[s];
    const int64_t nup = (int64_t)S.op.upload.size(), ndl = S.op.dl_count, nt = (int64_t)S.hp.tiles.size();
    if (up_used + nup > P.up_cap || dl_used + ndl > P.dl_cap || t_used + nt > P.tiles_cap) {
      if (run.empty()) {
        P.err = "an operation exceeds the staging capacity";
        return HALLAR_E_UNSUPPORTED;
      }
      continue;
    }
    S.op.up_off = up_used;
    if (nup) std::memcpy(P.h_up + up_used, S.op.upload.data(), nup * sizeof(double));
    up_used += (nup + 7) & ~(int64_t)7;
    S.op.dl_off = dl_used;
    dl_used += (ndl + 7) & ~(int64_t)7;
    t_used += nt;
    run.push_back(s);
  }
  // groups
  std::vector<Group> groups;
  int64_t tpos = 0, ipos = 0;
  const bool same_tiles = run == P.tiles_run && P.tiles_epoch == P.tile_epoch;
  size_t q = 0;
  while (q < run.size()) {
    size_t e = q;
    const PendingOp &o = P.slots[run[q]]->op;
    const int64_t k0 = group_key(P, run[q]);
    while (e < run.size() && group_key(P, run[e]) == k0) ++e;
    Group g{};
    g.code = o.code;
    g.R = o.R;
    g.R2 = o.R2;
    g.op = &o;
    g.t0 = tpos;
    g.i0 = ipos;
    for (size_t u = q; u < e; ++u) {
      const int s = run[u];
      Slot &S = *P.slots[s];
      g.slots.push_back(s);
      g.steps = std::max(g.steps, S.op.steps);
      if (same_tiles) tpos += (int64_t)S.hp.tiles.size();
      else
        for (const Tile &t : S.hp.tiles) P.h_tiles[tpos++] = t;
      P.h_ilist[ipos++] = s;
      g.maxm = std::max(g.maxm, S.hp.m);
      g.maxp = std::max<int>(g.maxp, (int)S.hp.npairs);
    }
    g.nt = tpos - g.t0;
    g.ni = ipos - g.i0;
    g.gi0 = ipos;
    for (size_t u = q; u < e; ++u)
      if (!P.slots[run[u]]->hp.direct) P.h_ilist[ipos++] = run[u];
    g.gni = ipos - g.gi0;
    g.di0 = ipos;
    for (size_t u = q; u < e; ++u)
      if (P.slots[run[u]]->hp.direct) P.h_ilist[ipos++] = run[u];
    g.dni = ipos - g.di0;
    groups.push_back(g);
    q = e;
  }
  int maxs = 0;
  for (int s : run) {
    Slot &S = *P.slots[s];
    for (int r = 0; r < NROLE; ++r)
      if (S.prm.buf[r] < 0 || S.prm.buf[r] >= NBUF) {
        P.err = "internal error: work buffers exhausted";
        return HALLAR_E_UNSUPPORTED;
      }
    S.prm.up_off = S.op.up_off;
    S.prm.dl_off = S.op.dl_off;
    P.h_prm[s] = S.prm;
    maxs = std::max(maxs, s + 1);
  }
  hipStream_t st = P.stream;
  std::string &err = P.err;
  const double tr1 = now_s();
  if (P.insts_dirty) {
    HL_TRY(hipMemcpyAsync(P.d_insts, P.h_insts.data(), sizeof(InstDev) * P.max_slots, hipMemcpyHostToDevice, st),
           "upload descriptors");
    P.insts_dirty = false;
  }
  HL_TRY(hipMemcpyAsync(P.d_prm, P.h_prm, sizeof(InstParams) * maxs, hipMemcpyHostToDevice, st), "upload params");
  if (!same_tiles) {
    HL_TRY(hipMemcpyAsync(P.d_tiles, P.h_tiles, sizeof(Tile) * tpos, hipMemcpyHostToDevice, st), "upload tiles");
    P.tiles_run = run;
    P.tiles_epoch = P.tile_epoch;
  }
  if ((int64_t)P.ilist_dev.size() != ipos || !std::equal(P.ilist_dev.begin(), P.ilist_dev.end(), P.h_ilist)) {
    HL_TRY(hipMemcpyAsync(P.d_ilist, P.h_ilist, sizeof(int32_t) * ipos, hipMemcpyHostToDevice, st), "upload ilist");
    P.ilist_dev.assign(P.h_ilist, P.h_ilist + ipos);
  }
  if (up_used) HL_TRY(hipMemcpyAsync(P.d_up, P.h_up, sizeof(double) * up_used, hipMemcpyHostToDevice, st), "upload coef");
  auto launch_all = [&](hipStream_t ms) -> hallar_status {
    if (groups.size() == 1) {
      launch_group(P, groups[0], ms);
    } else {
      // groups touch disjoint instances: spread them over the main and side
      // streams, all after the uploads above, all joined before the downloads
      HL_TRY(hipEventRecord(P.ev_fork, ms), "fork");
      const int ns = std::min<int>((int)groups.size(), 1 + Pool::NSIDE);
      for (int q = 1; q < ns; ++q) HL_TRY(hipStreamWaitEvent(P.side[q - 1], P.ev_fork, 0), "fork wait");
      for (size_t gi = 0; gi < groups.size(); ++gi) {
        const int q = (int)(gi % ns);
        launch_group(P, groups[gi], q == 0 ? ms : P.side[q - 1]);
      }
      for (int q = 1; q < ns; ++q) {
        HL_TRY(hipEventRecord(P.ev_join[q - 1], P.side[q - 1]), "join");
        HL_TRY(hipStreamWaitEvent(ms, P.ev_join[q - 1], 0), "join wait");
      }
    }
    if (P.launch_err != HALLAR_OK) {
      const hallar_status e = P.launch_err;
      P.launch_err = HALLAR_OK;
      return e;
    }
    return HALLAR_OK;
  };
  // The kernel section of a round reads everything that changes from one
  // round to the next (parameters, tiles, instance lists, coefficients) from
  // device memory uploaded above, so a round whose launches are decided by
  // the same inputs (op codes and fields, groups, buckets, tile and instance
  // ranges, loaded instances) replays the graph captured from the first such
  // round instead of enqueuing its kernels one by one.  Captured on the second
  // occurrence; not used while kernel classes are timed (opts.profile).
  // Only rounds of one group are captured (a linear chain of kernels on the
  // graph stream, no events inside the graph): a batched solve whose
  // multi-group rounds were captured with their side-stream fork and join
  // ended in a host segmentation fault, cause not found, so that form is off.
  // Rounds of coded-diffraction instances are not captured: their FFTs are
  // enqueued by rocFFT, whose launches this library does not control.
  bool launched = false, direct_on_gst = false;
  bool any_cdp = false;
  for (const Group &g : groups)
    for (int q : g.slots) any_cdp = any_cdp || P.slots[q]->hp.cdp_L > 0;
  if (P.opts.graphs && !P.profile && P.gst && groups.size() == 1 && !any_cdp) {
    std::vector<int64_t> sig;
    sig.reserve(32 * groups.size() + 8);
    sig.push_back(P.tile_epoch);
    sig.push_back((int64_t)(uintptr_t)P.d_tiles);
    sig.push_back((int64_t)(uintptr_t)P.d_ilist);
    sig.push_back((int64_t)(uintptr_t)P.d_insts);
    for (const Group &g : groups) {
      const PendingOp &o = *g.op;
      const int64_t f[] = {g.code, g.R, g.R2, g.steps, g.t0, g.nt, g.i0, g.ni, g.gi0, g.gni, g.di0, g.dni, g.maxm,
                           g.maxp, o.xrole, o.msel, o.wT, o.wyp, o.zsel, o.src, o.dst,
                           (int64_t)(uintptr_t)o.ext, o.ext_r, o.ext_ld, (int64_t)g.slots.size()};
      sig.insert(sig.end(), std::begin(f), std::end(f));
      sig.insert(sig.end(), g.slots.begin(), g.slots.end());
    }
    uint64_t hsh = 1469598103934665603ull;
    for (int64_t v : sig) hsh = (hsh ^ (uint64_t)v) * 1099511628211ull;
    Pool::RoundGraph &rg = P.graphs[hsh];
    if (rg.sig != sig) {
      // a new signature (or a hash collision): start over for this key
      if (rg.exec) (void)hipGraphExecDestroy(rg.exec);
      rg = Pool::RoundGraph{};
      rg.sig = sig;
    }
    rg.last_use = P.rounds;
    const bool want = !rg.exec && !rg.failed && ++rg.seen >= 2;
    if (want || rg.exec) {
      // the graph runs on its own stream, after the uploads on `st`
      HL_TRY(hipEventRecord(P.ev_gfork, st), "graph fork");
      HL_TRY(hipStreamWaitEvent(P.gst, P.ev_gfork, 0), "graph fork wait");
    }
    if (want) {
      hipGraph_t graph = nullptr;
      bool ok = hipStreamBeginCapture(P.gst, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        const hallar_status ls = launch_all(P.gst);
        ok = hipStreamEndCapture(P.gst, &graph) == hipSuccess && ls == HALLAR_OK && graph;
      }
      if (ok) ok = hipGraphInstantiate(&rg.exec, graph, nullptr, nullptr, 0) == hipSuccess;
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      if (!ok) {
        rg.exec = nullptr;
        rg.failed = true;  // this signature launches directly from now on
      } else {
        P.graph_captures++;
      }
    }
    if (rg.exec) {
      HL_TRY(hipGraphLaunch(rg.exec, P.gst), "graph launch");
      P.graph_replays++;
      launched = true;
    } else if (want) {
      // capture failed: this round's kernels go directly onto the graph stream
      const hallar_status ls = launch_all(P.gst);
      if (ls != HALLAR_OK) return ls;
      launched = true;
      direct_on_gst = true;
    }
    if (launched) {
      HL_TRY(hipEventRecord(P.ev_gjoin, P.gst), "graph join");
      HL_TRY(hipStreamWaitEvent(st, P.ev_gjoin, 0), "graph join wait");
    }
    if (P.graphs.size() > 512) {
      // keep the cache bounded: drop the graphs unused for longest
      std::vector<std::pair<int64_t, uint64_t>> age;
      for (auto &kv : P.graphs) age.emplace_back(kv.second.last_use, kv.first);
      std::sort(age.begin(), age.end());
      for (size_t k = 0; k < age.size() / 2; ++k) {
        auto it = P.graphs.find(age[k].second);
        if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
        P.graphs.erase(it);
      }
    }
  }
  if (!launched) {
    const hallar_status ls = launch_all(st);
    if (ls != HALLAR_OK) return ls;
  }
  if (direct_on_gst) launched = false;  // counts replays only
  HL_TRY(hipGetLastError(), "kernel launch");
  HL_TRY(hipMemcpyAsync(P.h_res, P.d_res, sizeof(InstRes) * maxs, hipMemcpyDeviceToHost, st), "download results");
  if (dl_used) HL_TRY(hipMemcpyAsync(P.h_dl, P.d_dl, sizeof(double) * dl_used, hipMemcpyDeviceToHost, st), "download");
  const double tr2 = now_s();
  HL_TRY(hipStreamSynchronize(st), "round");
  // event times are read in batches, off most rounds' critical path (every
  // event of a finished round is complete)
  if (P.profile && P.ev_used + 512 > (int)P.events.size()) prof_flush(P);
  const double tr3 = now_s();
  P.rounds++;
  did_work = true;
  auto resume_one = [&](int i) {
    Slot &S = *P.slots[run[i]];
    S.has_op = false;
    S.result.n_rounds++;
    if (launched) S.result.n_graph_rounds++;
    if (S.op.dl_count) S.dl.assign(P.h_dl + S.op.dl_off, P.h_dl + S.op.dl_off + S.op.dl_count);
    auto h = S.resume;
    S.resume = {};
    h.resume();
  };
  if (run.size() >= 16) {
    if (!P.workers) P.workers = std::make_unique<ResumeWorkers>();
    P.workers->run((int)run.size(), resume_one);
  } else {
    for (int i = 0; i < (int)run.size(); ++i) resume_one(i);
  }
  const double tr4 = now_s();
  P.t_prep += tr1 - tr0;
  P.t_launch += tr2 - tr1;
  P.t_wait += tr3 - tr2;
  P.t_resume += tr4 - tr3;
  return HALLAR_OK;
}

// ------------------------------------------------------------------ solver
struct OpAwait {
  Slot &s;
  bool await_ready() { return false; }
  void await_suspend(std::coroutine_handle<> h) {
    s.resume = h;
    s.has_op = true;
  }
  void await_resume() {}
};

struct Ctx {
  Pool &P;
  Slot &S;
  int idx;
  const hallar_options &o;
  double res(int k) const { return P.h_res[idx].v[k]; }
  int alloc() {
    if (S.free_bufs.empty()) return -1;
    const int b = S.free_bufs.back();
    S.free_bufs.pop_back();
    return b;
  }
  void release(int b) {
    if (b >= 0) S.free_bufs.push_back(b);
  }
  PendingOp &op(OpCode c) {
    S.op = PendingOp{};
    S.op.code = c;
    // FP64 vector ops (Lanczos, step size, multipliers) do not depend on the U width
    const bool vec64 = c == OP_LZ_BEGIN || c == OP_LZ_STEPS || c == OP_LZ_RITZ || c == OP_LZ_RESTART ||
                       c == OP_FW_PREP || c == OP_SETP;
    S.op.R = vec64 ? 0 : S.cur_R;
    S.op.rlive = vec64 ? 0 : std::min(S.cur_r, S.cur_R);
    return S.op;
  }
};

static bool finite(double x) { return std::isfinite(x); }

struct FistaOut {
  int status = 0;  // 0 ok, 1 fail, 2 numerical, 3 no representable progress
  int W = -1;
  double L = 0, gW = 0, rl2 = 0, vdot = 0, dW2 = 0, wy = 0, gr2 = 0;
};

// Unit roundoff of the storage type of U and of the gradient buffer.  Function
// values and products are exact (FP64 accumulation) for the stored iterates,
// but (i) the stored gradient GR is rounded, so <GR, d> errs by up to
// u ||GR|| ||d||, and (ii) every new iterate is rounded on store, which moves
// it by up to u tau (||U|| <= tau) and psi by up to (||grad psi|| + L ||d||) u tau.
// The FISTA / AIPP inequalities below allow for these terms, and ADAP-AIPP's
// residual is resolved only down to u (||GR|| + L tau) / lam.  In FP64 all of
// them are below the 1e-13 relative slack; in FP32-mixed they keep rounding
// noise from reading as a failed descent (which would halve lam without end).
static double storage_eps(int prec) { return prec == 0 ? 0x1p-53 : 0x1p-24; }

// ADAP-FISTA (Appendix A.1) on psi_s = lam g + 1/2 ||. - x0||^2 over B_tau.
static Task fista(Ctx c, int x0, double lam, double L0, FistaOut &out) {
  const double mu = 0.5, chi = c.o.chi, sigma = c.o.sigma;
  double A = 0.0, tk = 1.0, L = L0;
  int y = x0, x = x0;
  const int xt = c.alloc(), gr = c.alloc();
  int z = c.alloc();
  bool pend = false;
  double u1 = 0, u2 = 0, u3 = 0;
  out = FistaOut{};
  for (int i = 0; i < c.o.fista_max_iter; ++i) {
    double a = 0, d2 = 0, ypw0 = 0, g_yp = 0;
    bool accepted = false;
    for (int bt = 0; bt < 80; ++bt) {
      a = (tk + std::sqrt(tk * tk + 4.0 * tk * A * (L - mu))) / (2.0 * (L - mu));
      InstParams &p = c.S.prm;
      p.cY = A / (A + a);
      p.cX = a / (A + a);
      p.lam = lam;
      p.L = L;
      p.invL = 1.0 / L;
      p.upd_x = pend ? 1 : 0;
      p.u1 = u1;
      p.u2 = u2;
      p.u3 = u3;
      int xn = -1;
      if (pend) xn = c.alloc();
      p.buf[RY] = y;
      p.buf[RX] = x;
      p.buf[RXT] = xt;
      p.buf[RW0] = x0;
      p.buf[RGR] = gr;
      p.buf[RZ] = z;
      p.buf[RU2] = pend ? xn : x;
      c.op(OP_TRIAL);
      c.S.result.n_fista_trials++;
      c.S.result.n_sddmm += 2;
      c.S.result.n_spmm += 1;
      co_await OpAwait{c.S};
      if (pend) {
        if (x != x0 && x != y) c.release(x);
        x = xn;
        pend = false;
      }
      const double g_xt = c.res(S_G_XT), xtw0 = c.res(S_XTW0), gr_d = c.res(S_GR_D);
      d2 = c.res(S_D2);
      ypw0 = c.res(S_YPW0);
      g_yp = c.res(S_G_YP);
      if (!finite(g_xt) || !finite(g_yp) || !finite(gr_d) || !finite(d2)) {
        out.status = 2;
        goto cleanup;
      }
      const double psx = lam * g_xt + 0.5 * xtw0, psy = lam * g_yp + 0.5 * ypw0;
      const double grn = std::sqrt(std::max(c.res(S_GR2T), 0.0)), dn = std::sqrt(std::max(d2, 0.0));
      const double slack = 4.0 * storage_eps(c.P.prec) * ((grn + L * dn) * c.S.prm.tau + grn * dn);
      if (psx + gr_d + 0.25 * (1.0 - chi) * L * d2 >= psy - slack) {
        accepted = true;
        break;
      }
      L *= 2.0;
    }
    if (!accepted) {
      out.status = 1;
      goto cleanup;
    }
    {
      const double A1 = A + a, tk1 = tk + a * mu;
      u1 = (mu * a + a * (L - mu)) / tk1;
      u2 = tk / tk1;
      u3 = -a * (L - mu) / tk1;
      if (ypw0 < chi * A1 * L * d2) {
        // y+ equal to x0 up to the storage rounding: no representable step
        const double ut = 4.0 * storage_eps(c.P.prec) * c.S.prm.tau;
        out.status = ypw0 <= ut * ut ? 3 : 1;
        goto cleanup;
      }
      if ((L - mu) * std::sqrt(d2) <= sigma * std::sqrt(ypw0)) {
        InstParams &p = c.S.prm;
        p.buf[RZ] = z;
        p.buf[RXT] = xt;
        p.buf[RGR] = gr;
        p.buf[RW0] = x0;
        p.lam = lam;
        p.L = L;
        c.op(OP_GRAD);
        c.S.result.n_spmm += 1;
        co_await OpAwait{c.S};
        out.status = 0;
        out.W = z;
        z = -1;
        out.L = L;
        out.gW = g_yp;
        out.rl2 = c.res(S_RL2);
        out.dW2 = ypw0;
        out.vdot = c.res(S_RL_W0) - ypw0;  // <V, x0 - y+> with V = Rl - (x0 - y+)
        out.wy = c.res(S_WY);
        out.gr2 = c.res(S_GR2A);
        goto cleanup;
      }
      if (y != x0) c.release(y);
      y = z;
      z = c.alloc();
      pend = true;
      A = A1;
      tk = tk1;
    }
  }
  out.status = 1;
cleanup:
  c.release(xt);
  c.release(gr);
  if (z >= 0) c.release(z);
  if (y != x0 && y != out.W) c.release(y);
  if (x != x0 && x != y && x != out.W) c.release(x);
  co_return;
}

struct AippOut {
  int status = 0;  // 0 ok, 1 iter limit, 2 numerical
  int W = -1;
  double lam = 0, g = 0;
};

// ADAP-AIPP (Appendix A): prox-point loop, halving lam on failure.
static Task aipp(Ctx c, int W0, double g0, double lam, double rho, AippOut &out) {
  int Wprev = W0;
  double gprev = g0, Mbar = 1.0;
  out = AippOut{};
  for (int j = 0; j < c.o.aipp_max_iter; ++j) {
    c.S.result.n_aipp_iters++;
    FistaOut fo;
    for (;;) {
      const double Mj = std::max(1.0, 0.5 * Mbar);
      co_await fista(c, Wprev, lam, Mj, fo);
      if (c.o.verbose >= 3 && fo.status != 0)
        fprintf(stderr, "[hallar]     aipp j=%d fista status=%d lam=%.3g\n", j, fo.status, lam);
      if (fo.status == 2) {
        out.status = 2;
        out.W = Wprev;
        co_return;
      }
      if (fo.status == 3) {
        // the prox step no longer moves the stored iterate: W_{j-1} is
        // stationary to the storage precision
        out.status = 0;
        out.W = Wprev;
        out.lam = lam;
        out.g = gprev;
        co_return;
      }
      if (fo.status == 0) {
        const double lhs = lam * gprev - (lam * fo.gW + 0.5 * fo.dW2);
        const double grn = std::sqrt(std::max(fo.gr2, 0.0)), dn = std::sqrt(std::max(fo.dW2, 0.0));
        const double slack = 1e-13 * (1.0 + std::fabs(lam * gprev)) +
                             4.0 * storage_eps(c.P.prec) * ((grn + dn) * c.S.prm.tau + grn * dn);
        if (lhs >= fo.vdot - slack) break;
        c.release(fo.W);
      }
      lam *= 0.5;
      if (lam < 1e-30) {
        out.status = 2;
        out.W = Wprev;
        co_return;
      }
    }
    const double Rn = std::sqrt(std::max(fo.rl2, 0.0)) / lam;
    // R_j is resolved only down to the rounding of the stored gradient
    const double Rfloor = 4.0 * storage_eps(c.P.prec) * (std::sqrt(std::max(fo.gr2, 0.0)) + fo.L * c.S.prm.tau) / lam;
    Mbar = fo.L;
    c.release(Wprev);
    Wprev = fo.W;
    gprev = fo.gW;
    if (c.o.verbose >= 3)
      fprintf(stderr, "[hallar]     aipp j=%d lam=%.3g Rn=%.3e rho=%.3e floor=%.3e L=%.3g g=%.12g\n", j, lam, Rn, rho,
              Rfloor, fo.L, gprev);
    if (Rn <= std::max(rho, Rfloor)) {
      out.status = 0;
      out.W = Wprev;
      out.lam = lam;
      out.g = gprev;
      co_return;
    }
  }
  out.status = 1;
  out.W = Wprev;
  out.lam = lam;
  out.g = gprev;
}

struct EigOut {
  double lam = 0, res = 0;
  int iters = 0, restarts = 0;
  bool converged = false;
};

// thick-restart Lanczos with full reorthogonalisation for lambda_min of
// G = C + A*(yp); the Ritz vector is left in lzv.
static Task lanczos(Ctx c, double tol_abs, int max_iter, int use_prev, EigOut &out) {
  Slot &S = c.S;
  const int kmax = S.kmax;
  const int LD = KMAX + 1;  // host H: column-major, H[j * LD + i]
  S.H.assign((size_t)LD * KMAX, 0.0);
  S.prm.lz_seed = S.seed * 0x9E3779B97F4A7C15ull + (uint64_t)(++S.result.n_eig_calls);
  S.prm.lz_use_prev = use_prev;
  S.prm.lz_basis = 0;
  c.op(OP_LZ_BEGIN);
  co_await OpAwait{S};
  int k = 0;
  out = EigOut{};
  std::vector<double> Hs, w, Q;
  // shift of the SpMV: the latest diagonal entry of the projected matrix
  // (a warm start begins near the previous smallest eigenvalue)
  double sigma = S.lz_sigma;
  int tri0 = 1;
  for (;;) {
    const int steps = std::min(8, kmax - k);
    S.prm.lz_j = k;
    S.prm.lz_j0 = k;
    S.prm.lz_steps = steps;
    S.prm.lz_shift = sigma;
    S.prm.lz_tri0 = tri0;
    PendingOp &op = c.op(OP_LZ_STEPS);
    op.steps = steps;
    op.dl_count = (int64_t)steps * (KMAX + 2);
    co_await OpAwait{S};
    for (int u = 0; u < steps; ++u) {
      const int col = k + u;
      const double *d = S.dl.data() + (size_t)u * (KMAX + 2);
      for (int i = 0; i <= col; ++i) S.H[(size_t)col * LD + i] = d[i];
      S.H[(size_t)col * LD + col + 1] = d[KMAX + 1];
      // undo the SpMV's shift and three-term subtraction
      S.H[(size_t)col * LD + col] += sigma;
      if (col >= tri0) S.H[(size_t)col * LD + col - 1] += S.H[(size_t)(col - 1) * LD + col];
    }
    sigma = S.H[(size_t)(k + steps - 1) * LD + (k + steps - 1)];
    k += steps;
    out.iters += steps;
    S.result.n_matvec += steps;
    // Rayleigh-Ritz on the symmetrised projected matrix
    Hs.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Hs[(size_t)i * k + j] = 0.5 * (S.H[(size_t)j * LD + i] + S.H[(size_t)i * LD + j]);
    w.assign(k, 0.0);
    Q.assign((size_t)k * k, 0.0);
    sym_eig(k, Hs.data(), w.data(), Q.data());
    const double bk = S.H[(size_t)(k - 1) * LD + k];
    const bool breakdown = !(bk > 1e-14 * std::max(1.0, std::fabs(w[0])));
    const double res = breakdown ? 0.0 : std::fabs(bk * Q[(size_t)(k - 1) * k + 0]);
    S.lz_sigma = w[0];
    out.lam = w[0];
    out.res = res;
    const bool conv = res <= std::max(tol_abs, c.o.eig_tol * std::max(1.0, std::fabs(w[0])));
    if (conv || out.iters >= max_iter || breakdown) {
      out.converged = conv || breakdown;
      S.prm.lz_j = k;
      PendingOp &r = c.op(OP_LZ_RITZ);
      r.upload.assign((size_t)KMAX * KMAX, 0.0);
      for (int q = 0; q < k; ++q) r.upload[(size_t)q * KMAX + 0] = Q[(size_t)q * k + 0];
      co_await OpAwait{S};
      co_return;
    }
    if (k == kmax) {
      const int qk = std::max(1, std::min(kmax / 2, 16));
      S.prm.lz_j = k;
      S.prm.lz_q = qk;
      PendingOp &r = c.op(OP_LZ_RESTART);
      r.upload.assign((size_t)KMAX * KMAX, 0.0);
      for (int q = 0; q < k; ++q)
        for (int cc = 0; cc < qk; ++cc) r.upload[(size_t)q * KMAX + cc] = Q[(size_t)q * k + cc];
      co_await OpAwait{S};
      S.prm.lz_basis ^= 1;
      std::fill(S.H.begin(), S.H.end(), 0.0);
      for (int cc = 0; cc < qk; ++cc) {
        S.H[(size_t)cc * LD + cc] = w[cc];
        S.H[(size_t)cc * LD + qk] = bk * Q[(size_t)(k - 1) * k + cc];
      }
      k = qk;
      tri0 = qk + 1;  // v_qk couples to every kept Ritz vector (arrowhead)
      out.restarts++;
    }
  }
}

// Rotate U onto the eigenvectors of U^T U and keep the directions with
// sigma^2 > drop_tol sigma_max^2 (at most keep_max of them, the largest).
static Task compress(Ctx c, int &buf, int &r, int keep_max, bool &truncated) {
  Slot &S = c.S;
  truncated = false;
  const int R = S.cur_R;
  PendingOp &op = c.op(OP_GRAM);
  op.src = RU;
  op.dl_count = (int64_t)R * R;
  S.prm.buf[RU] = buf;
  co_await OpAwait{S};
  std::vector<double> G((size_t)r * r), w(r), Q((size_t)r * r);
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) G[(size_t)a * r + b] = S.dl[(size_t)a * R + b];
  sym_eig(r, G.data(), w.data(), Q.data());
  const double wmax = std::max(w[r - 1], 0.0);
  std::vector<int> keep;
  // directions below the storage precision's noise floor are not resolved in
  // FP32 (sigma ~ 1e-7 sigma_max): drop below max(drop_tol, 1e-10) there
  const double dtol = c.P.prec == 0 ? c.o.drop_tol : std::max(c.o.drop_tol, 1e-10);
  for (int a = r - 1; a >= 0; --a)
    if (w[a] > dtol * wmax) keep.push_back(a);
  if (keep.empty()) keep.push_back(r - 1);
  if (keep_max > 0 && (int)keep.size() > keep_max) {
    keep.resize(keep_max);
    truncated = true;
  }
  if ((int)keep.size() == r && !truncated) co_return;
  const int rnew = (int)keep.size();
  const int RD = r_bucket(rnew, c.P.prec);
  const int dst = c.alloc();
  PendingOp &ro = c.op(OP_ROTATE);
  ro.R = RD;
  ro.R2 = R;
  ro.src = 0;
  ro.dst = 1;
  ro.upload.assign((size_t)R_MAX * R_MAX, 0.0);
  for (int a = 0; a < r; ++a)
    for (int cc = 0; cc < rnew; ++cc) ro.upload[(size_t)a * R_MAX + cc] = Q[(size_t)a * r + keep[cc]];
  S.prm.buf[0] = buf;  // role 0 (RX) = source, role 1 (RY) = destination
  S.prm.buf[1] = dst;
  S.prm.r = r;
  S.prm.rnew = rnew;
  co_await OpAwait{S};
  c.release(buf);
  buf = dst;
  r = rnew;
  S.cur_R = RD;
  S.cur_r = rnew;
}

static int map_status(int st) {
  return st;
}

static Task solve_main(Ctx c) {
  Slot &S = c.S;
  const hallar_options &o = c.o;
  HostProblem &hp = S.hp;
  const double tau2 = hp.tau2, tau = std::sqrt(tau2);
  const double t0 = now_s();
  S.t_start = t0;
  hallar_result &res = S.result;
  res.status = HALLAR_E_ITER_LIMIT;
  double beta = o.beta1;
  S.prm.beta = beta;
  // U0 (projected onto the ball B_tau)
  int U = c.alloc();
  int r = std::max(1, S.U0r);
  S.cur_R = r_bucket(r, c.P.prec);
  S.cur_r = r;
  {
    PendingOp &op = c.op(OP_PACK);
    op.ext = S.U0ext;
    op.ext_r = S.U0r;
    op.ext_ld = S.U0r;
    op.dst = 0;
    S.prm.buf[0] = U;
    co_await OpAwait{S};
    const double nrm2 = c.res(S_NZ);
    if (nrm2 > tau2) {
      S.prm.lz_scale = tau / std::sqrt(nrm2);
      PendingOp &cp = c.op(OP_COPY);
      cp.src = 0;
      cp.dst = 0;
      co_await OpAwait{S};
    }
  }
  auto eval = [&](int buf, int wT, int wyp) {
    PendingOp &op = c.op(OP_EVAL);
    op.xrole = RU;
    op.msel = -1;
    op.wT = wT;
    op.wyp = wyp;
    op.zsel = 0;
    S.prm.buf[RU] = buf;
    S.prm.beta = beta;
    S.result.n_sddmm++;
  };
  eval(U, 0, 0);
  co_await OpAwait{S};
  double pval_prev = c.res(S_T0);
  double rnorm_prev = std::sqrt(std::max(c.res(S_RR), 0.0));
  double lam = o.lam0;
  double theta = 0.0, pval = 0, dval = 0, pinf = 0, gapr = 0, dinf = 0;
  bool have_v = false;
  int t = 0;
  for (t = 1; t <= o.outer_max_iter; ++t) {
    eval(U, 0, 0);
    co_await OpAwait{S};
    double gY = c.res(S_G_EVAL);
    const double scale = 1.0 + std::max(std::fabs(pval_prev), std::fabs(gY));
    const double eps_t = std::max(o.eps1 * std::pow(o.eps_decay, t - 1), o.eps_floor * o.eps) * scale;
    // stationarity tolerance of ADAP-AIPP: G . YY^T = <grad g(Y), Y>/2 moves by
    // up to tau ||R|| / 2, so rho = eps_t / tau keeps it commensurate with the gap
    const double rho = eps_t / std::max(1.0, tau);
    bool hlr_ok = false;
    int Y = -1;
    double TYT0 = 0, lmin = 0, eres = 0;
    for (int it = 0; it < o.hlr_max_iter; ++it) {
      res.n_hlr_iters++;
      AippOut ao;
      co_await aipp(c, U, gY, std::min(lam, o.lam0), rho, ao);
      U = -1;
      Y = ao.W;
      lam = ao.lam;
      if (ao.status != 0 && o.verbose >= 2)
        fprintf(stderr, "[hallar]   aipp failed t=%d it=%d status=%d lam=%.3g rank=%d rho=%.3e\n", t, it, ao.status, ao.lam, r, rho);
      if (ao.status == 2) {
        res.status = HALLAR_E_NUMERICAL;
        break;
      }
      // ao.status == 1: ADAP-AIPP's iteration safeguard (the paper's method has
      // none) returns its last iterate; the Frank-Wolfe certificate judges it
      if (r > 1) {
        bool tr = false;
        co_await compress(c, Y, r, 0, tr);
      }
      // G = C + A*(p + beta (A(YY^T) - b)) (eq. Grad X Space): T(Y), y'' on device
      eval(Y, 1, 1);
      co_await OpAwait{S};
      TYT0 = c.res(S_T0);
      const double GYY = c.res(S_T0) + c.res(S_YT);
      EigOut eo;
      const double tol_abs = o.eig_frac * eps_t / tau2;
      co_await lanczos(c, tol_abs, o.eig_max_iter, have_v ? 1 : 0, eo);
      have_v = true;
      lmin = eo.lam;
      eres = eo.res;
      theta = std::max(-lmin, 0.0);
      const double gap = GYY + tau2 * theta;
      if (o.verbose >= 2)
        fprintf(stderr, "[hallar]   hlr t=%d it=%d rank=%d lam=%.3g aipp_g=%.10g gap=%.3e eps_t=%.3e theta=%.3e eig_it=%d res=%.2e trials=%lld\n",
                t, it, r, lam, ao.g, gap, eps_t, theta, eo.iters, eo.res, (long long)res.n_fista_trials);
      if (!finite(gap)) {
        res.status = HALLAR_E_NUMERICAL;
        break;
      }
      // the gap is the difference of G . YY^T and tau^2 theta, each of the
      // size of the objective; the stored iterate resolves it only to a few
      // units of its storage roundoff of their size (FP32-mixed: u = 2^-24;
      // in FP64 the allowance is far below eps_t)
      const double gap_floor = 4.0 * storage_eps(c.P.prec) * (std::fabs(GYY) + tau2 * theta);
      if (gap <= std::max(eps_t, gap_floor)) {
        hlr_ok = true;
        break;
      }
      // exact line search (eq. FW stepsize)
      S.prm.fw_v_on = theta > 0.0 ? 1 : 0;
      S.prm.tau2 = tau2;
      c.op(OP_FW_PREP);
      co_await OpAwait{S};
      const double den = beta * c.res(S_FWDEN);
      const double alpha = den > 0.0 ? std::min(gap / den, 1.0) : 1.0;
      int rnew;
      if (alpha >= 1.0) {
        S.prm.fw_col = 0;
        S.prm.fw_a = 0.0;
        S.prm.fw_b = theta > 0.0 ? tau : 0.0;
        rnew = 1;
      } else if (theta > 0.0) {
        S.prm.fw_col = r;
        S.prm.fw_a = std::sqrt(1.0 - alpha);
        S.prm.fw_b = std::sqrt(alpha) * tau;
        rnew = r + 1;
      } else {
        S.prm.fw_col = -1;
        S.prm.fw_a = std::sqrt(1.0 - alpha);
        S.prm.fw_b = 0.0;
        rnew = r;
      }
      const int RD = r_bucket(std::min(rnew, R_MAX), c.P.prec);
      const int Ynew = c.alloc();
      PendingOp &fa = c.op(OP_FW_APPLY);
      fa.R = RD;
      fa.R2 = S.cur_R;
      fa.src = 0;
      fa.dst = 1;
      S.prm.buf[0] = Y;
      S.prm.buf[1] = Ynew;
      S.prm.r = r;
      co_await OpAwait{S};
      const int r_prev = r, R_prev = S.cur_R;
      U = Ynew;
      r = rnew;
      S.cur_R = RD;
      S.cur_r = rnew;
      // at most R_MAX - 1 columns survive a step, so the next one fits R_MAX
      const int cap = o.rank_cap > 0 ? std::min(o.rank_cap, R_MAX - 1) : R_MAX - 1;
      if (r > cap) {
        // rank cap: drop the numerically null directions first; if the step
        // still needs more columns than the cap, stop with E_RANK_CAP and
        // return the iterate before the step (or, on request, keep the cap's
        // largest directions and count the truncation)
        bool tr = false;
        co_await compress(c, U, r, o.rank_cap_truncate ? cap : 0, tr);
        if (tr) res.n_truncations++;
        if (r > cap) {
          c.release(U);
          U = Y;
          Y = -1;
          r = r_prev;
          S.cur_R = R_prev;
          S.cur_r = r_prev;
          res.status = HALLAR_E_RANK_CAP;
          break;
        }
      }
      c.release(Y);
      Y = -1;
      eval(U, 0, 0);
      co_await OpAwait{S};
      gY = c.res(S_G_EVAL);
    }
    if (!hlr_ok) {
      if (Y >= 0) U = Y;
      if (res.status == HALLAR_E_ITER_LIMIT && (now_s() - t0) > o.time_limit) res.status = HALLAR_E_TIME_LIMIT;
      break;
    }
    U = Y;
    // p_t = p + beta (A(U U^T) - b) (eq. dual update SDP Algo 2)
    c.op(OP_SETP);
    co_await OpAwait{S};
    const double bp = c.res(S_BP), rr = c.res(S_RR), ptr = c.res(S_PTR);
    pval = TYT0;
    dval = -bp - tau2 * theta;
    const double rnorm = std::sqrt(std::max(rr, 0.0));
    pinf = rnorm / (1.0 + hp.b_l1);
    gapr = std::fabs(pval - dval) / (1.0 + std::fabs(pval) + std::fabs(dval));
    const double lamS = (lmin - eres) + theta;
    dinf = std::max(0.0, -lamS) / (1.0 + hp.c_l1);
    res.outer_iters = t;
    if (o.verbose)
      fprintf(stderr, "[hallar] t=%d beta=%.3g rank=%d pval=%.10g dval=%.10g pinf=%.2e gap=%.2e dinf=%.2e rounds=%lld\n",
              t, beta, r, pval, dval, pinf, gapr, dinf, (long long)res.n_rounds);
    // objective accuracy: the relative gap of eq. termination2 divides by
    // about twice the objective, so it alone admits an objective error near
    // 2 eps; weak duality puts P* above dval, pval above dval - |p^T r|, and
    // P* <= pval + p*^T r for an optimal multiplier p*, so with p_t near p*
    // |pval - dval| + |p_t^T r| bounds |pval - P*|
    auto obj_ok = [&]() {
      res.obj_bound = std::fabs(pval - dval) + std::fabs(ptr);
      return !o.obj_check || res.obj_bound <= o.eps * (1.0 + std::fabs(pval));
    };
    // the iteration's record (after the certification below, if it ran)
    auto record = [&]() {
      hallar_outer_record rec{};
      rec.t = t;
      rec.rank = r;
      rec.beta = beta;
      rec.pval = pval;
      rec.dval = dval;
      rec.theta = theta;
      rec.pinf = pinf;
      rec.gap = gapr;
      rec.dinf = dinf;
      rec.obj_bound = std::fabs(pval - dval) + std::fabs(ptr);
      rec.seconds = now_s() - t0;
      rec.n_fista_trials = res.n_fista_trials;
      rec.n_matvec = res.n_matvec;
      rec.n_hlr_iters = res.n_hlr_iters;
      S.history.push_back(rec);
    };
    if (std::max(pinf, std::max(gapr, dinf)) <= o.eps) {
      // Certification: the Ritz value bounds lambda_min from above, and near
      // the optimum a warm-started run can settle on a member of the cluster
      // of smallest eigenvalues (one per primal column) above the minimum.
      // A cold-started run of bounded length sees the whole cluster; its
      // Ritz value, if smaller, only tightens theta and the dual value.
      EigOut ec;
      co_await lanczos(c, o.eig_frac * eps_t / tau2, std::min(o.eig_max_iter, 400), 0, ec);
      if (ec.lam < lmin) {
        lmin = ec.lam;
        eres = ec.res;
        theta = std::max(-lmin, 0.0);
        dval = -bp - tau2 * theta;
        gapr = std::fabs(pval - dval) / (1.0 + std::fabs(pval) + std::fabs(dval));
        dinf = std::max(0.0, -((lmin - eres) + theta)) / (1.0 + hp.c_l1);
        if (o.verbose)
          fprintf(stderr, "[hallar] t=%d certification: lambda %.10g (cold) -> gap=%.2e dinf=%.2e\n", t, lmin, gapr, dinf);
      }
      if (std::max(pinf, std::max(gapr, dinf)) <= o.eps && obj_ok()) {
        res.status = HALLAR_OK;
        record();
        break;
      }
    }
    obj_ok();
    record();
    if (now_s() - t0 > o.time_limit) {
      res.status = HALLAR_E_TIME_LIMIT;
      break;
    }
    if (rnorm > o.infeas_ratio * rnorm_prev && pinf > o.pinf_gate * std::max(gapr, dinf))
      beta = std::min(beta * (rnorm > o.stall_ratio * rnorm_prev ? o.stall_growth : o.beta_growth), o.beta_max);
    S.prm.beta = beta;
    rnorm_prev = rnorm;
    pval_prev = pval;
  }
  if (t > o.outer_max_iter) res.status = HALLAR_E_ITER_LIMIT;
  res.rank = r;
  res.pval = pval;
  res.dval = dval;
  res.theta = theta;
  res.pinf = pinf;
  res.gap = gapr;
  res.dinf = dinf;
  res.beta = beta;
  res.seconds = now_s() - t0;
  S.final_buf = U;
  S.final_r = r;
  S.done = true;
  (void)map_status;
}

// coroutine holder so that Task lifetime matches the slot
void slot_start_solve(Pool &P, int s) {
  Slot &S = *P.slots[s];
  S.done = false;
  S.result = hallar_result{};
  // a solve starts from the instance alone: nothing a previous solve or
  // operator call on this slot left in the parameters (the Lanczos shift in
  // particular, which changes the rounding of every eigen solve) carries over
  {
    const double tau = S.prm.tau, tau2 = S.prm.tau2;
    S.prm = InstParams{};
    S.prm.tau = tau;
    S.prm.tau2 = tau2;
  }
  S.lz_sigma = 0.0;
  S.history.clear();
  S.free_bufs.clear();
  for (int q = NBUF - 1; q >= 0; --q) S.free_bufs.push_back(q);
  if (S.task) delete S.task;
  S.task = new Task(solve_main(Ctx{P, S, s, P.opts}));
  // start: runs until the first device op
  S.task->h.resume();
}

hallar_status pool_run(Pool &P, int max_rounds) {
  int done_rounds = 0;
  for (;;) {
    bool did = false;
    const hallar_status st = run_round(P, did);
    if (st != HALLAR_OK) {
      P.fatal = st;
      return st;
    }
    // collect finished
    for (int s = 0; s < (int)P.slots.size(); ++s) {
      auto &sp = P.slots[s];
      if (sp && sp->used && sp->done && sp->task && sp->ticket >= 0) {
        P.finished.emplace_back(sp->ticket, sp->result);
        sp->ticket = -2;  // reported
      }
    }
    if (!did) break;
    if (max_rounds > 0 && ++done_rounds >= max_rounds) break;
  }
  return HALLAR_OK;
}

// ------------------------------------------------------------------ standalone operator calls
// The standalone calls' parameters go down as a kernel argument (copied at
// enqueue time): consecutive asynchronous calls with different role tables
// cannot see each other's values, and the slot's own parameters are left as
// the solver set them.
static hallar_status upload_params(Pool &P, int s, const InstParams &prm, hipStream_t st, std::string &err) {
  op_put_params(st, P.d_prm + s, prm);
  if (P.insts_dirty) {
    HL_TRY(hipMemcpyAsync(P.d_insts, P.h_insts.data(), sizeof(InstDev) * P.max_slots, hipMemcpyHostToDevice, st),
           "descriptors");
    HL_TRY(hipStreamSynchronize(st), "descriptors");
    P.insts_dirty = false;
  }
  return HALLAR_OK;
}

static const Tile *slot_tiles(Pool &P, int s) {
  Slot &S = *P.slots[s];
  const Layout L = make_layout(S.hp, P.prec, S.Rcap, S.kmax);
  return (const Tile *)((char *)S.slab + L.tiles);
}
static const int32_t *slot_ilist(Pool &P, int s) {
  Slot &S = *P.slots[s];
  const Layout L = make_layout(S.hp, P.prec, S.Rcap, S.kmax);
  return (const int32_t *)((char *)S.slab + L.ilist);
}

// A caller buffer can stand in for a work buffer when its rows are exactly
// the bucket's rows (r = R, ld = R) and it is 16-byte aligned (the kernels
// move 16-byte chunks).
static bool in_place(const void *X, int r, int64_t ld, int R) {
  return r == R && ld == R && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
}

hallar_status op_eval_AUUt(Pool &P, int s, const void *U, int r, int64_t ldu, double *T, hipStream_t st) {
  Slot &S = *P.slots[s];
  std::string &err = P.err;
  const int R = r_bucket(r, P.prec);
  if (R > S.Rcap) {
    err = "r exceeds the handle's column capacity";
    return HALLAR_E_INVALID;
  }
  // the caller's U is read in place when its rows are the bucket's rows
  const bool u_direct = in_place(U, r, ldu, R);
  InstParams prm = S.prm;
  prm.buf[RU] = u_direct ? NBUF : 0;
  prm.ext[0] = u_direct ? const_cast<void *>(U) : nullptr;
  prm.beta = 0.0;
  if (upload_params(P, s, prm, st, err) != HALLAR_OK) return HALLAR_E_HIP;
  const Tile *T_ = slot_tiles(P, s);
  const int nt = (int)S.hp.tiles.size();
  const int32_t *IL = slot_ilist(P, s);
  const InstDev *D = P.d_insts;
  if (!u_direct) op_pack_op(P.prec, R, st, T_, nt, D, U, r, ldu, RU);
  // T does not depend on p: the epilogue's {p_l, b_l} reads (zeros at load,
  // else the last solve's) only feed scalars this call does not return
  op_lr_dots(P.prec, R, st, T_, nt, D, RU);
  // direct mode: each constrained pair's lane writes T_l into the caller's T
  op_sddmm(P.prec, R, st, T_, nt, D, RU, -1, 1, 0, S.hp.direct && S.hp.m > 0 ? T + 1 : nullptr);
  if (S.hp.rk > 0) {
    op_lc_kty(P.prec, R, st, T_, nt, D, S.hp.rk, RU, 0);
    op_lc_sum(st, IL, 1, D, S.hp.rk, R, 0);
    op_lc_red(st, IL, 1, D, LC_Y_T, R, 0);
  }
  if (S.hp.cdp_L > 0) {
    cdp_forward(P, s, st, RU, 0, R, r, 0);
    if (P.launch_err != HALLAR_OK) {
      const hallar_status e = P.launch_err;
      P.launch_err = HALLAR_OK;
      return e;
    }
  }
  if (!S.hp.direct) op_gen_constraints(P.prec, st, IL, 1, S.hp.m, D, 1);
  op_reduce(st, IL, 1, D, RDH_EVAL, 0, R, 0);
  HL_TRY(hipMemcpyAsync(T, &P.d_res[s].v[S_T0], sizeof(double), hipMemcpyDeviceToDevice, st), "T0");
  if (S.hp.m > 0 && !S.hp.direct)
    HL_TRY(hipMemcpyAsync(T + 1, S.dev.TY, sizeof(double) * S.hp.m, hipMemcpyDeviceToDevice, st), "T");
  HL_TRY(hipGetLastError(), "eval launch");
  return HALLAR_OK;
}

// The same evaluation with everything it writes besides T inside the
// scratch array (no allocation, nothing of the handle's workspace touched):
// the descriptor is copied on the device, so nothing host-side has to stay
// alive after the call returns.  Calls that overlap on one GPU share the
// array and race.
hallar_status op_eval_AUUt_noalloc(Pool &P, int s, const void *U, int r, int64_t ldu, double *T, hipStream_t st) {
  Slot &S = *P.slots[s];
  std::string &err = P.err;
  const int R = r_bucket(r, P.prec);
  if (R > S.Rcap) {
    err = "r exceeds the handle's column capacity";
    return HALLAR_E_INVALID;
  }
  if (!P.scratch) {
    err = "the scratch array's device address is unknown on this device";
    return HALLAR_E_HIP;
  }
  const HostProblem &h = S.hp;
  if (h.rk > 0 || h.cdp_L > 0) {
    err = "the allocation-free evaluation does not take low-rank or coded-diffraction constraints";
    return HALLAR_E_UNSUPPORTED;
  }
  const bool u_direct = in_place(U, r, ldu, R);
  const int nt = (int)h.tiles.size();
  const int prows = (int)prows_for(h);
  const int nslot = 4 + h.r0 * R;  // SDDMM sums, low-rank products
  // carve the scratch (256-byte aligned pieces)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t o_insts = take(sizeof(InstDev) * (size_t)(s + 1));
  const size_t o_prm = take(sizeof(InstParams));
  const size_t o_res = take(sizeof(InstRes));
  const size_t o_part = take(sizeof(double) * (size_t)nslot * prows);
  const size_t o_u = take(u_direct ? 0 : (size_t)h.n * R * (P.prec == 0 ? 8 : 4));
  const size_t o_z0 = take(sizeof(double) * 2 * LR_MAX * R_MAX);
  const size_t o_ty = take(h.direct ? 0 : sizeof(double) * (size_t)h.m);
  const size_t o_yp = take(h.direct ? 0 : sizeof(double) * (size_t)h.m);
  const size_t o_bp = take(h.direct ? 0 : sizeof(double) * (size_t)h.npairs);
  if (off > NOALLOC_SCRATCH_BYTES) {
    err = "the evaluation needs " + std::to_string(off) + " bytes of scratch, more than the " +
          std::to_string(NOALLOC_SCRATCH_BYTES) + " the allocation-free entry point has";
    return HALLAR_E_INVALID;
  }
  char *base = static_cast<char *>(P.scratch);
  NoallocViews v{};
  v.insts = reinterpret_cast<InstDev *>(base + o_insts);
  v.prm = reinterpret_cast<InstParams *>(base + o_prm);
  v.res = reinterpret_cast<InstRes *>(base + o_res);
  v.part = reinterpret_cast<double *>(base + o_part);
  v.prows = prows;
  v.ubuf = u_direct ? nullptr : base + o_u;
  v.u_ext = u_direct ? U : nullptr;
  v.Z0 = reinterpret_cast<double *>(base + o_z0);
  v.TY = h.direct ? nullptr : reinterpret_cast<double *>(base + o_ty);
  v.yp = h.direct ? nullptr : reinterpret_cast<double *>(base + o_yp);
  v.Bpair = h.direct ? nullptr : reinterpret_cast<double *>(base + o_bp);
  if (P.insts_dirty) {
    // the handle's own descriptor must be on the device before it is copied
    std::string e2;
    if (upload_params(P, s, S.prm, st, e2) != HALLAR_OK) {
      err = e2;
      return HALLAR_E_HIP;
    }
  }
  op_noalloc_setup(st, P.d_insts, s, v);
  const Tile *T_ = slot_tiles(P, s);
  const int32_t *IL = slot_ilist(P, s);
  const InstDev *D = v.insts;
  if (!u_direct) op_pack_op(P.prec, R, st, T_, nt, D, U, r, ldu, RU);
  op_lr_dots(P.prec, R, st, T_, nt, D, RU);
  op_sddmm(P.prec, R, st, T_, nt, D, RU, -1, 1, 0, h.direct && h.m > 0 ? T + 1 : nullptr);
  if (!h.direct) op_gen_constraints(P.prec, st, IL, 1, h.m, D, 1);
  op_reduce(st, IL, 1, D, RDH_EVAL, 0, R, 0);
  HL_TRY(hipMemcpyAsync(T, &v.res->v[S_T0], sizeof(double), hipMemcpyDeviceToDevice, st), "T0");
  if (h.m > 0 && !h.direct)
    HL_TRY(hipMemcpyAsync(T + 1, v.TY, sizeof(double) * h.m, hipMemcpyDeviceToDevice, st), "T");
  HL_TRY(hipGetLastError(), "eval launch");
  return HALLAR_OK;
}

hallar_status op_adjoint(Pool &P, int s, const double *p, const void *U, int r, int64_t ldu, void *W, int64_t ldw,
                         hipStream_t st) {
  Slot &S = *P.slots[s];
  std::string &err = P.err;
  const int R = r_bucket(r, P.prec);
  if (R > S.Rcap) {
    err = "r exceeds the handle's column capacity";
    return HALLAR_E_INVALID;
  }
  // U read and W written in place when their rows are the bucket's rows
  // (and W does not overlap U: the SpMM gathers rows of U while writing W)
  const bool u_direct = in_place(U, r, ldu, R);
  const size_t esz = P.prec == 0 ? 8 : 4;
  const uintptr_t u0 = reinterpret_cast<uintptr_t>(U), w0 = reinterpret_cast<uintptr_t>(W);
  const bool overlap = u0 < w0 + (size_t)S.hp.n * ldw * esz && w0 < u0 + (size_t)S.hp.n * ldu * esz;
  const bool w_direct = in_place(W, r, ldw, R) && !overlap;
  InstParams prm = S.prm;
  prm.buf[RU] = u_direct ? NBUF : 0;
  prm.buf[RU2] = w_direct ? NBUF + 1 : 1;
  prm.ext[0] = u_direct ? const_cast<void *>(U) : nullptr;
  prm.ext[1] = w_direct ? W : nullptr;
  if (upload_params(P, s, prm, st, err) != HALLAR_OK) return HALLAR_E_HIP;
  const Tile *T_ = slot_tiles(P, s);
  const int nt = (int)S.hp.tiles.size();
  const int32_t *IL = slot_ilist(P, s);
  const InstDev *D = P.d_insts;
  op_pairvals(P.prec, st, IL, 1, (int)S.hp.npairs, D, 0, p, S.hp.direct ? 0 : 1);
  if (!u_direct) op_pack_op(P.prec, R, st, T_, nt, D, U, r, ldu, RU);
  if (S.hp.r0 > 0) {
    op_lr_dots(P.prec, R, st, T_, nt, D, RU);
    op_reduce(st, IL, 1, D, RDH_LRONLY, 0, R, 0);
  }
  if (S.hp.rk > 0) {
    // blockdiag(p_l D_l) K^T U for the constraints' low-rank parts (Algorithm 5)
    op_lc_kty(P.prec, R, st, T_, nt, D, S.hp.rk, RU, 0);
    op_lc_sum(st, IL, 1, D, S.hp.rk, R, 0);
    op_lc_red(st, IL, 1, D, LC_Y_Z, R, 0, p);
    op_lc_kz(P.prec, R, st, T_, nt, D, 0, 0);
  }
  if (S.hp.cdp_L > 0) {
    // the coded-diffraction block D_l^H F^H (p_l * F D_l U)
    cdp_forward(P, s, st, RU, 0, R, r, -1);
    cdp_adjoint(P, s, st, R, r, 0, 0, p);
    if (P.launch_err != HALLAR_OK) {
      const hallar_status e = P.launch_err;
      P.launch_err = HALLAR_OK;
      return e;
    }
  }
  op_spmm(P.prec, R, st, T_, nt, D, RU, 0, 0, RU2, SPM_PLAIN);
  if (!w_direct) op_unpack_op(P.prec, R, st, T_, nt, D, W, r, ldw, RU2);
  HL_TRY(hipGetLastError(), "adjoint launch");
  return HALLAR_OK;
}

static Task eig_main(Ctx c, double tol, int max_iter, int use_prev, EigOut *out) {
  co_await lanczos(c, tol, max_iter, use_prev, *out);
  c.S.done = true;
}

hallar_status op_min_eig(Pool &P, int s, const double *p, const double *v0, double tol, int max_iter, double *lambda,
                         double *v, hallar_eig_info *info) {
  Slot &S = *P.slots[s];
  std::string &err = P.err;
  hipStream_t st = P.stream;
  if (S.hp.m > 0) HL_TRY(hipMemcpyAsync(S.dev.yp, p, sizeof(double) * S.hp.m, hipMemcpyDeviceToDevice, st), "p");
  if (v0) HL_TRY(hipMemcpyAsync(S.dev.lzv, v0, sizeof(double) * S.hp.n, hipMemcpyDeviceToDevice, st), "v0");
  HL_TRY(hipStreamSynchronize(st), "sync");
  EigOut eo;
  hallar_options o2 = P.opts;
  o2.eig_tol = tol;
  S.done = false;
  // the same call gives the same result: the start vector's seed and the
  // SpMV shift do not depend on earlier calls
  S.result.n_eig_calls = 0;
  S.lz_sigma = 0.0;
  if (S.task) delete S.task;
  S.free_bufs.clear();
  for (int q = NBUF - 1; q >= 0; --q) S.free_bufs.push_back(q);
  S.task = new Task(eig_main(Ctx{P, S, s, o2}, 0.0, max_iter, v0 ? 2 : 0, &eo));
  S.task->h.resume();
  const hallar_status rs = pool_run(P, 0);
  if (rs != HALLAR_OK) return rs;
  delete S.task;
  S.task = nullptr;
  *lambda = eo.lam;
  if (info) {
    info->iters = eo.iters;
    info->restarts = eo.restarts;
    info->residual = eo.res;
  }
  if (v) HL_TRY(hipMemcpyAsync(v, S.dev.lzv, sizeof(double) * S.hp.n, hipMemcpyDeviceToDevice, st), "v");
  HL_TRY(hipStreamSynchronize(st), "sync");
  return eo.converged ? HALLAR_OK : HALLAR_E_NOT_CONVERGED;
}

}  // namespace hl
