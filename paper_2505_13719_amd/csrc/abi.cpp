// extern "C" entry points declared in include/hallar.h.
#include <cmath>
#include <cstring>
#include <vector>
#include <mutex>
#include <random>

#include "engine.h"
#include "ops.h"

struct hallar_s {
  hl::Pool P;
  int prec = 0;
  std::string err;
};

struct hallar_pool_s {
  hl::Pool P;
  std::string err;
};

namespace {
thread_local std::string g_err;

hallar_status fail(hallar_t h, hallar_status st, const std::string &msg) {
  if (h) h->err = msg;
  g_err = msg;
  return st;
}
hallar_status failp(hallar_pool_t p, hallar_status st, const std::string &msg) {
  if (p) p->err = msg;
  g_err = msg;
  return st;
}

bool check_opts(const hallar_options &o, std::string &msg) {
  if (!(o.eps > 0)) { msg = "opts.eps must be > 0"; return false; }
  if (!(o.beta1 > 0) || !(o.beta_growth >= 1.0) || !(o.stall_growth >= 1.0)) {
    msg = "opts.beta1 > 0, beta_growth >= 1 and stall_growth >= 1 required";
    return false;
  }
  if (!(o.sigma > 0 && o.sigma < 0.5) || !(o.chi > 0 && o.chi < 1)) { msg = "opts.sigma in (0, 1/2), chi in (0, 1) required"; return false; }
  if (!(o.lam0 > 0)) { msg = "opts.lam0 must be > 0"; return false; }
  if (o.rank_cap < 0 || o.rank_cap > hl::R_MAX) { msg = "opts.rank_cap must be in [0, 64]"; return false; }
  if (o.eig_kmax < 0 || o.eig_kmax > hl::KMAX) { msg = "opts.eig_kmax must be in [0, 64]"; return false; }
  if (o.lower_gather != 0 && o.lower_gather != 1) { msg = "opts.lower_gather must be 0 or 1"; return false; }
  if (o.unfused_trial != 0 && o.unfused_trial != 1) { msg = "opts.unfused_trial must be 0 or 1"; return false; }
  if (o.obj_check != 0 && o.obj_check != 1) { msg = "opts.obj_check must be 0 or 1"; return false; }
  if (o.rank_cap_truncate != 0 && o.rank_cap_truncate != 1) { msg = "opts.rank_cap_truncate must be 0 or 1"; return false; }
  if (o.graphs != 0 && o.graphs != 1) { msg = "opts.graphs must be 0 or 1"; return false; }
  if (o.profile < 0 || o.profile > 2) { msg = "opts.profile must be 0, 1 or 2"; return false; }
  if (o.fista_max_iter < 1 || o.aipp_max_iter < 1 || o.hlr_max_iter < 1 || o.outer_max_iter < 1 || o.eig_max_iter < 1) {
    msg = "iteration caps must be >= 1";
    return false;
  }
  return true;
}

std::vector<double> gaussian(int64_t n, uint64_t seed) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> d(0.0, 1.0);
  std::vector<double> v(n);
  for (auto &x : v) x = d(g);
  return v;
}
}  // namespace

extern "C" {

void hallar_default_options(hallar_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps = 1e-5;
  o->beta1 = 1.0;
  o->beta_growth = 4.0;
  o->beta_max = 1e16;
  o->infeas_ratio = 0.5;
  o->pinf_gate = 0.1;
  o->stall_ratio = 0.9;
  o->stall_growth = 16.0;
  o->eps1 = 1e-2;
  o->eps_floor = 0.2;
  o->eps_decay = 0.5;
  o->sigma = 0.3;
  o->chi = 1e-3;
  o->lam0 = 10.0;
  o->fista_max_iter = 2000;
  o->aipp_max_iter = 500;
  o->hlr_max_iter = 1000;
  o->outer_max_iter = 300;
  o->eig_tol = 1e-13;
  o->eig_frac = 0.1;
  o->eig_kmax = 64;
  o->eig_max_iter = 20000;
  o->rank_cap = 0;
  o->drop_tol = 1e-14;
  o->time_limit = 3600.0;
  o->seed = 0;
  o->verbose = 0;
  o->obj_check = 1;
  o->rank_cap_truncate = 0;
  o->graphs = 0;
}

const char *hallar_last_error(hallar_t h) { return h ? h->err.c_str() : g_err.c_str(); }

namespace {

// Autotuner of the tile schedule: every candidate (minimum rows, entry cap)
// builds its tiles, loads the instance into a scratch pool and times the
// SDDMM (hallar_eval_AUUt) and SpMM (hallar_adjoint_spmm) entry points at two
// widths with HIP events; the fastest candidate wins (ties keep the earlier,
// the default comes first).
hallar_status tune_schedule(hl::HostProblem &hp, int prec, const hallar_options &o, hipStream_t st, std::string &msg) {
  struct Cand {
    int32_t min_rows, ent_cap;
  };
  static const Cand kCands[] = {{64, 2048}, {16, 2048}, {256, 2048}, {64, 1024}, {16, 512}, {256, 1024}};
  const size_t sz = prec == 0 ? 8 : 4;
  const int rcap = hl::rcap_for(o, prec);
  const int widths[2] = {std::min(4, rcap), std::min(16, rcap)};
  const size_t n = hp.n;
  void *dU = nullptr, *dW = nullptr;
  double *dT = nullptr, *dp = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&] {
    if (dU) (void)hipFree(dU);
    if (dW) (void)hipFree(dW);
    if (dT) (void)hipFree(dT);
    if (dp) (void)hipFree(dp);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&dU, n * 16 * sz) != hipSuccess || hipMalloc(&dW, n * 16 * sz) != hipSuccess ||
      hipMalloc((void **)&dT, (hp.m + 1) * 8) != hipSuccess || hipMalloc((void **)&dp, std::max(hp.m, 1) * 8) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    msg = "autotune: device allocation failed";
    return HALLAR_E_OOM;
  }
  {
    // deterministic operands: U entries in [-1, 1), p entries in [-1, 1)
    std::vector<float> uf;
    std::vector<double> ud, pv(std::max(hp.m, 1));
    uint64_t x = 0x9E3779B97F4A7C15ull;
    auto nxt = [&] {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    };
    if (prec == 0) {
      ud.resize(n * 16);
      for (auto &v : ud) v = nxt();
      (void)hipMemcpy(dU, ud.data(), ud.size() * 8, hipMemcpyHostToDevice);
    } else {
      uf.resize(n * 16);
      for (auto &v : uf) v = (float)nxt();
      (void)hipMemcpy(dU, uf.data(), uf.size() * 4, hipMemcpyHostToDevice);
    }
    for (auto &v : pv) v = nxt();
    (void)hipMemcpy(dp, pv.data(), pv.size() * 8, hipMemcpyHostToDevice);
  }
  hallar_options to = o;
  to.profile = 0;
  to.verbose = 0;
  int best = 0;
  float best_ms = 0.f;
  for (int c = 0; c < (int)(sizeof(kCands) / sizeof(kCands[0])); ++c) {
    hl::HostProblem h2 = hp;
    h2.tile_min_rows = kCands[c].min_rows;
    h2.tile_ent_cap = kCands[c].ent_cap;
    hl::build_tiles(h2);
    hl::Pool P;
    hallar_status s = hl::pool_init(P, 1, prec, to, st, 0, (int64_t)h2.tiles.size(), msg);
    if (s == HALLAR_OK) s = hl::slot_load(P, 0, std::move(h2), msg);
    float ms = -1.f;
    if (s == HALLAR_OK) {
      for (int rep = 0; rep < 4 && s == HALLAR_OK; ++rep) {
        if (rep == 1) (void)hipEventRecord(e0, st);
        for (int wi = 0; wi < 2 && s == HALLAR_OK; ++wi) {
          s = hl::op_eval_AUUt(P, 0, dU, widths[wi], widths[wi], dT, st);
          if (s == HALLAR_OK) s = hl::op_adjoint(P, 0, dp, dU, widths[wi], widths[wi], dW, widths[wi], st);
        }
      }
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      if (s == HALLAR_OK) (void)hipEventElapsedTime(&ms, e0, e1);
    }
    hl::pool_release(P);
    if (s != HALLAR_OK) {
      cleanup();
      return s;
    }
    if (o.verbose)
      fprintf(stderr, "[hallar] autotune: min_rows %d ent_cap %d: %.3f ms\n", kCands[c].min_rows, kCands[c].ent_cap, ms);
    if (c == 0 || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  cleanup();
  hp.tile_min_rows = kCands[best].min_rows;
  hp.tile_ent_cap = kCands[best].ent_cap;
  hl::build_tiles(hp);
  return HALLAR_OK;
}

}  // namespace

hallar_status hallar_create(const hallar_problem *prob, hallar_precision prec, const hallar_options *opts, void *stream,
                            hallar_t *out) {
  if (!out) return fail(nullptr, HALLAR_E_INVALID, "out is NULL");
  *out = nullptr;
  if (prec != HALLAR_FP64 && prec != HALLAR_FP32_MIXED) return fail(nullptr, HALLAR_E_INVALID, "bad precision");
  hallar_options o;
  if (opts) o = *opts;
  else hallar_default_options(&o);
  std::string msg;
  if (!check_opts(o, msg)) return fail(nullptr, HALLAR_E_INVALID, msg);
  hl::HostProblem hp;
  hallar_status code;
  msg = hl::build_host_problem(prob, hp, &code);
  if (code != HALLAR_OK) return fail(nullptr, code, msg);
  if (o.autotune) {
    code = tune_schedule(hp, (int)prec, o, (hipStream_t)stream, msg);
    if (code != HALLAR_OK) return fail(nullptr, code, msg);
  }
  auto h = new (std::nothrow) hallar_s;
  if (!h) return fail(nullptr, HALLAR_E_OOM, "out of host memory");
  h->prec = (int)prec;
  const int64_t nt = (int64_t)hp.tiles.size();
  hallar_status st = hl::pool_init(h->P, 1, (int)prec, o, (hipStream_t)stream, 0, nt, msg);
  if (st != HALLAR_OK) {
    hl::pool_release(h->P);
    delete h;
    return fail(nullptr, st, msg);
  }
  st = hl::slot_load(h->P, 0, std::move(hp), msg);
  if (st != HALLAR_OK) {
    hl::pool_release(h->P);
    delete h;
    return fail(nullptr, st, msg);
  }
  h->P.slots[0]->seed = o.seed;
  // the allocation-free evaluation's scratch: its device address on this
  // device, resolved once per device
  if (hl::noalloc_scratch(&h->P.scratch) != hipSuccess) h->P.scratch = nullptr;
  *out = h;
  return HALLAR_OK;
}

hallar_status hallar_destroy(hallar_t h) {
  if (!h) return HALLAR_E_INVALID;
  (void)hipStreamSynchronize(h->P.stream);
  hl::pool_release(h->P);
  delete h;
  return HALLAR_OK;
}

hallar_status hallar_schedule(hallar_t h, int32_t *min_rows, int32_t *ent_cap, int64_t *ntiles) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  const auto &hp = h->P.slots[0]->hp;
  if (min_rows) *min_rows = hp.tile_min_rows;
  if (ent_cap) *ent_cap = hp.tile_ent_cap;
  if (ntiles) *ntiles = (int64_t)hp.tiles.size();
  return HALLAR_OK;
}

hallar_status hallar_describe(hallar_t h, int64_t *pairs, int64_t *sym_nnz, int64_t *device_bytes) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  auto &S = *h->P.slots[0];
  if (pairs) *pairs = S.hp.npairs;
  if (sym_nnz) *sym_nnz = S.hp.npairs + S.hp.nlower;
  if (device_bytes) *device_bytes = (int64_t)S.slab_bytes;
  return HALLAR_OK;
}

hallar_status hallar_eval_AUUt(hallar_t h, const void *U, int32_t r, int64_t ldu, double *T, void *stream) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  if (!U || !T) return fail(h, HALLAR_E_INVALID, "U and T must be device pointers");
  if (r < 1 || r > hl::R_MAX || ldu < r) return fail(h, HALLAR_E_INVALID, "need 1 <= r <= 64 and ldu >= r");
  const hallar_status st = hl::op_eval_AUUt(h->P, 0, U, r, ldu, T, (hipStream_t)stream);
  if (st != HALLAR_OK) return fail(h, st, h->P.err);
  return HALLAR_OK;
}

hallar_status hallar_eval_AUUt_noalloc(hallar_t h, const void *U, int32_t r, int64_t ldu, double *T, void *stream) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  if (!U || !T) return fail(h, HALLAR_E_INVALID, "U and T must be device pointers");
  if (r < 1 || r > hl::R_MAX || ldu < r) return fail(h, HALLAR_E_INVALID, "need 1 <= r <= 64 and ldu >= r");
  const hallar_status st = hl::op_eval_AUUt_noalloc(h->P, 0, U, r, ldu, T, (hipStream_t)stream);
  if (st != HALLAR_OK) return fail(h, st, h->P.err);
  return HALLAR_OK;
}

hallar_status hallar_adjoint_spmm(hallar_t h, const double *p, const void *U, int32_t r, int64_t ldu, void *W,
                                  int64_t ldw, void *stream) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  if (!U || !W || (!p && h->P.slots[0]->hp.m > 0)) return fail(h, HALLAR_E_INVALID, "p, U and W must be device pointers");
  if (r < 1 || r > hl::R_MAX || ldu < r || ldw < r) return fail(h, HALLAR_E_INVALID, "need 1 <= r <= 64, ldu >= r, ldw >= r");
  const hallar_status st = hl::op_adjoint(h->P, 0, p, U, r, ldu, W, ldw, (hipStream_t)stream);
  if (st != HALLAR_OK) return fail(h, st, h->P.err);
  return HALLAR_OK;
}

hallar_status hallar_min_eig(hallar_t h, const double *p, const double *v0, double tol, int32_t max_iter, double *lambda,
                             double *v, hallar_eig_info *info, void *stream) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  if (!lambda || (!p && h->P.slots[0]->hp.m > 0)) return fail(h, HALLAR_E_INVALID, "p (device) and lambda (host) required");
  if (!(tol > 0) || max_iter < 1) return fail(h, HALLAR_E_INVALID, "tol > 0 and max_iter >= 1 required");
  hipStream_t keep = h->P.stream;
  if (stream) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    h->P.stream = (hipStream_t)stream;
  }
  const hallar_status st = hl::op_min_eig(h->P, 0, p, v0, tol, max_iter, lambda, v, info);
  h->P.stream = keep;
  if (st != HALLAR_OK && st != HALLAR_E_NOT_CONVERGED) return fail(h, st, h->P.err);
  return st;
}

static hallar_status prepare_solve(hl::Pool &P, int s, const double *U0, int32_t r0, const double *p0, std::string &msg) {
  hl::Slot &S = *P.slots[s];
  const int n = S.hp.n, m = S.hp.m;
  hipStream_t st = P.stream;
  if (m > 0) {
    if (p0) {
      if (hipMemcpyAsync(S.dev.p, p0, sizeof(double) * m, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        msg = "copy of p0 failed";
        return HALLAR_E_HIP;
      }
    } else if (hipMemsetAsync(S.dev.p, 0, sizeof(double) * m, st) != hipSuccess) {
      msg = "clearing p failed";
      return HALLAR_E_HIP;
    }
  }
  if (U0) {
    if (r0 < 1 || r0 > hl::R_MAX) {
      msg = "r0 must be in [1, 64]";
      return HALLAR_E_INVALID;
    }
    S.U0ext = U0;
    S.U0r = r0;
  } else {
    const auto g = gaussian(n, P.opts.seed * 1000003ull + 17);
    if (hipMemcpy(S.dev.lzv, g.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
      msg = "upload of U0 failed";
      return HALLAR_E_HIP;
    }
    S.U0ext = S.dev.lzv;
    S.U0r = 1;
  }
  S.seed = P.opts.seed;
  return HALLAR_OK;
}

hallar_status hallar_solve(hallar_t h, const double *U0, int32_t r0, const double *p0, hallar_result *res) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  if (!res) return fail(h, HALLAR_E_INVALID, "res is NULL");
  std::string msg;
  hallar_status st = prepare_solve(h->P, 0, U0, r0, p0, msg);
  if (st != HALLAR_OK) return fail(h, st, msg);
  h->P.slots[0]->ticket = -1;
  hl::slot_start_solve(h->P, 0);
  st = hl::pool_run(h->P, 0);
  if (st != HALLAR_OK) return fail(h, st, h->P.err);
  *res = h->P.slots[0]->result;
  return HALLAR_OK;
}

hallar_status hallar_get_solution(hallar_t h, double *U, int64_t ldu, double *p, void *stream) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  hl::Slot &S = *h->P.slots[0];
  if (S.final_buf < 0) return fail(h, HALLAR_E_INVALID, "no solution: call hallar_solve first");
  hipStream_t st = (hipStream_t)stream;
  if (U) {
    if (ldu < S.final_r) return fail(h, HALLAR_E_INVALID, "ldu < rank");
    // unpack the final factor through the standalone tile list
    S.prm.buf[hl::RU] = S.final_buf;
    hl::InstParams p2 = S.prm;
    (void)hipMemcpy(h->P.d_prm, &p2, sizeof(p2), hipMemcpyHostToDevice);
    std::vector<hl::Tile> tl = S.hp.tiles;
    hl::Tile *dt = nullptr;
    if (hipMalloc((void **)&dt, sizeof(hl::Tile) * tl.size()) != hipSuccess) return fail(h, HALLAR_E_OOM, "tiles");
    (void)hipMemcpy(dt, tl.data(), sizeof(hl::Tile) * tl.size(), hipMemcpyHostToDevice);
    if (h->P.insts_dirty) {
      (void)hipMemcpy(h->P.d_insts, h->P.h_insts.data(), sizeof(hl::InstDev) * h->P.max_slots, hipMemcpyHostToDevice);
      h->P.insts_dirty = false;
    }
    hl::op_unpack_f64(h->P.prec, S.cur_R, st, dt, (int)tl.size(), h->P.d_insts, U, S.final_r, ldu, hl::RU);
    (void)hipStreamSynchronize(st);
    (void)hipFree(dt);
  }
  if (p && S.hp.m > 0)
    if (hipMemcpyAsync(p, S.dev.p, sizeof(double) * S.hp.m, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(h, HALLAR_E_HIP, "copy of p failed");
  if (hipStreamSynchronize(st) != hipSuccess) return fail(h, HALLAR_E_HIP, "sync failed");
  return HALLAR_OK;
}

hallar_status hallar_get_history(hallar_t h, hallar_outer_record *out, int32_t cap, int32_t *total) {
  if (!h || !h->P.slots[0]) return fail(h, HALLAR_E_INVALID, "bad handle");
  if (!total || cap < 0 || (cap > 0 && !out)) return fail(h, HALLAR_E_INVALID, "total required; out required when cap > 0");
  const std::vector<hallar_outer_record> &hist = h->P.slots[0]->history;
  *total = (int32_t)hist.size();
  const size_t k = std::min(hist.size(), (size_t)cap);
  for (size_t i = 0; i < k; ++i) out[i] = hist[i];
  return HALLAR_OK;
}

hallar_status hallar_solve_batch(hallar_t *hs, int32_t count, const double *const *U0s, hallar_result *results) {
  if (!hs || count < 1 || !results) return fail(nullptr, HALLAR_E_INVALID, "hs, count >= 1 and results required");
  const int prec = hs[0] ? hs[0]->prec : 0;
  int64_t tiles = 0;
  for (int k = 0; k < count; ++k) {
    if (!hs[k] || !hs[k]->P.slots[0]) return fail(nullptr, HALLAR_E_INVALID, "bad handle in batch");
    if (hs[k]->prec != prec) return fail(nullptr, HALLAR_E_INVALID, "all handles must share the precision");
    tiles += (int64_t)hs[k]->P.slots[0]->hp.tiles.size();
  }
  hl::Pool B;
  std::string msg;
  hallar_status st = hl::pool_init(B, count, prec, hs[0]->P.opts, hs[0]->P.stream, 0, tiles, msg);
  if (st != HALLAR_OK) {
    hl::pool_release(B);
    return fail(nullptr, st, msg);
  }
  // attach every handle's instance as a view (no copy of device data)
  for (int k = 0; k < count; ++k) {
    hl::Slot &src = *hs[k]->P.slots[0];
    auto v = std::make_unique<hl::Slot>();
    // every scalar of the preprocessed problem the round executor reads
    // (the index arrays stay with the handle: the device copies are used)
    v->hp.n = src.hp.n;
    v->hp.m = src.hp.m;
    v->hp.tau2 = src.hp.tau2;
    v->hp.npairs = src.hp.npairs;
    v->hp.nlower = src.hp.nlower;
    v->hp.nentries = src.hp.nentries;
    v->hp.direct = src.hp.direct;
    v->hp.low_recompute = src.hp.low_recompute;
    v->hp.con_rule = src.hp.con_rule;
    v->hp.has_c = src.hp.has_c;
    v->hp.pa_uniform = src.hp.pa_uniform;
    v->hp.pa_const = src.hp.pa_const;
    v->hp.c_diag_only = src.hp.c_diag_only;
    v->hp.r0 = src.hp.r0;
    v->hp.rk = src.hp.rk;
    v->hp.nlc = src.hp.nlc;
    v->hp.cdp_L = src.hp.cdp_L;
    v->hp.cdp_nc = src.hp.cdp_nc;
    v->hp.b_l1 = src.hp.b_l1;
    v->hp.c_l1 = src.hp.c_l1;
    v->hp.tile_min_rows = src.hp.tile_min_rows;
    v->hp.tile_ent_cap = src.hp.tile_ent_cap;
    v->hp.tiles = src.hp.tiles;
    v->fft = src.fft;  // the handle's FFT plans, used through this view
    for (auto &t : v->hp.tiles) t.inst = k;
    v->Rcap = src.Rcap;
    v->kmax = src.kmax;
    v->used = true;
    v->slab = nullptr;  // owned by the handle
    hl::InstDev D = src.dev;
    D.up_base = B.d_up;
    D.dl_base = B.d_dl;
    D.prm = B.d_prm + k;
    D.res = B.d_res + k;
    v->dev = D;
    B.h_insts[k] = D;
    v->prm = hl::InstParams{};
    v->prm.tau2 = src.hp.tau2;
    v->prm.tau = std::sqrt(src.hp.tau2);
    B.slots[k] = std::move(v);
    st = prepare_solve(B, k, U0s ? U0s[k] : nullptr, 1, nullptr, msg);
    if (st != HALLAR_OK) {
      for (int q = 0; q <= k; ++q) {
        B.slots[q]->slab = nullptr;
        B.slots[q]->fft = nullptr;
      }
      hl::pool_release(B);
      return fail(nullptr, st, msg);
    }
    B.slots[k]->seed = hs[k]->P.opts.seed;
    B.slots[k]->ticket = -1;
  }
  B.insts_dirty = true;
  for (int k = 0; k < count; ++k) hl::slot_start_solve(B, k);
  st = hl::pool_run(B, 0);
  for (int k = 0; k < count; ++k) {
    hl::Slot &v = *B.slots[k];
    results[k] = v.result;
    hl::Slot &src = *hs[k]->P.slots[0];
    src.final_buf = v.final_buf;
    src.final_r = v.final_r;
    src.cur_R = v.cur_R;
    src.result = v.result;
    src.history = std::move(v.history);
    v.slab = nullptr;  // views: do not free
    v.fft = nullptr;
  }
  const std::string berr = B.err;
  hl::pool_release(B);
  if (st != HALLAR_OK) return fail(nullptr, st, berr);
  return HALLAR_OK;
}

// ------------------------------------------------------------------ serving pool
hallar_status hallar_footprint(const hallar_problem *prob, hallar_precision prec, const hallar_options *opts,
                               size_t *bytes) {
  if (!bytes) return fail(nullptr, HALLAR_E_INVALID, "bytes is NULL");
  hallar_options o;
  if (opts) o = *opts;
  else hallar_default_options(&o);
  hl::HostProblem hp;
  hallar_status code;
  std::string msg = hl::build_host_problem(prob, hp, &code);
  if (code != HALLAR_OK) return fail(nullptr, code, msg);
  *bytes = hl::instance_bytes(hp, (int)prec, hl::rcap_for(o, (int)prec), hl::kmax_for(o, hp.n));
  return HALLAR_OK;
}

hallar_status hallar_inspect(const hallar_problem *prob, hallar_structure *out, int64_t *tile_row0, int64_t cap) {
  if (!out) return fail(nullptr, HALLAR_E_INVALID, "out is NULL");
  hl::HostProblem hp;
  hallar_status code;
  std::string msg = hl::build_host_problem(prob, hp, &code);
  if (code != HALLAR_OK) return fail(nullptr, code, msg);
  out->pairs = hp.npairs;
  out->lower = hp.nlower;
  out->tiles = (int64_t)hp.tiles.size();
  out->direct = hp.direct ? 1 : 0;
  out->con_rule = hp.direct ? hp.con_rule : 0;
  out->lower_recompute = hp.low_recompute ? 1 : 0;
  out->pad_ = 0;
  if (tile_row0) {
    const int64_t nt = (int64_t)hp.tiles.size();
    for (int64_t t = 0; t < nt && t < cap; ++t) tile_row0[t] = hp.tiles[t].row0;
    if (nt < cap) tile_row0[nt] = hp.n;
  }
  return HALLAR_OK;
}

hallar_status hallar_pool_create(size_t hbm_budget, int32_t max_active, hallar_precision prec, const hallar_options *opts,
                                 void *stream, hallar_pool_t *out) {
  if (!out || max_active < 1 || hbm_budget < 4096) return fail(nullptr, HALLAR_E_INVALID, "bad pool arguments");
  hallar_options o;
  if (opts) o = *opts;
  else hallar_default_options(&o);
  std::string msg;
  if (!check_opts(o, msg)) return fail(nullptr, HALLAR_E_INVALID, msg);
  auto p = new (std::nothrow) hallar_pool_s;
  if (!p) return fail(nullptr, HALLAR_E_OOM, "host memory");
  const hallar_status st = hl::pool_init(p->P, max_active, (int)prec, o, (hipStream_t)stream, hbm_budget,
                                         (int64_t)max_active * 64, msg);
  if (st != HALLAR_OK) {
    hl::pool_release(p->P);
    delete p;
    return fail(nullptr, st, msg);
  }
  *out = p;
  return HALLAR_OK;
}

hallar_status hallar_pool_destroy(hallar_pool_t pool) {
  if (!pool) return HALLAR_E_INVALID;
  (void)hipStreamSynchronize(pool->P.stream);
  hl::pool_release(pool->P);
  delete pool;
  return HALLAR_OK;
}

hallar_status hallar_pool_admit(hallar_pool_t pool, const hallar_problem *prob, const double *U0, int64_t ticket) {
  if (!pool) return fail(nullptr, HALLAR_E_INVALID, "pool is NULL");
  if (ticket < 0) return failp(pool, HALLAR_E_INVALID, "ticket must be >= 0");
  hl::Pool &P = pool->P;
  int s = -1;
  for (int k = 0; k < P.max_slots; ++k)
    if (!P.slots[k]) {
      s = k;
      break;
    }
  if (s < 0) return failp(pool, HALLAR_E_BUSY, "no free slot");
  hl::HostProblem hp;
  hallar_status code;
  std::string msg = hl::build_host_problem(prob, hp, &code);
  if (code != HALLAR_OK) return failp(pool, code, msg);
  if (P.tiles_cap < (int64_t)hp.tiles.size()) return failp(pool, HALLAR_E_UNSUPPORTED, "instance has more tiles than the pool stages");
  const hallar_status st = hl::slot_load(P, s, std::move(hp), msg);
  if (st != HALLAR_OK) return failp(pool, st, msg);
  hl::Slot &S = *P.slots[s];
  const int n = S.hp.n;
  std::vector<double> u0 = U0 ? std::vector<double>(U0, U0 + n) : gaussian(n, P.opts.seed * 1000003ull + (uint64_t)ticket);
  if (hipMemcpy(S.dev.lzv, u0.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
    hl::slot_unload(P, s);
    return failp(pool, HALLAR_E_HIP, "upload of U0 failed");
  }
  S.U0ext = S.dev.lzv;
  S.U0r = 1;
  S.seed = P.opts.seed;  // same start vectors as a standalone solve of this request
  S.ticket = ticket;
  hl::slot_start_solve(P, s);
  return HALLAR_OK;
}

hallar_status hallar_pool_step(hallar_pool_t pool, int32_t rounds, int32_t *n_active) {
  if (!pool) return fail(nullptr, HALLAR_E_INVALID, "pool is NULL");
  hl::Pool &P = pool->P;
  const hallar_status st = hl::pool_run(P, rounds < 1 ? 1 : rounds);
  // release finished instances
  for (int s = 0; s < P.max_slots; ++s)
    if (P.slots[s] && P.slots[s]->done && P.slots[s]->ticket == -2) hl::slot_unload(P, s);
  if (n_active) *n_active = hl::pool_active(P);
  if (st != HALLAR_OK) return failp(pool, st, P.err);
  return HALLAR_OK;
}

hallar_status hallar_pool_poll(hallar_pool_t pool, int64_t *tickets, hallar_result *results, int32_t cap, int32_t *n_done) {
  if (!pool || !n_done || (cap > 0 && (!tickets || !results))) return fail(nullptr, HALLAR_E_INVALID, "bad poll arguments");
  int k = 0;
  auto &F = pool->P.finished;
  while (k < cap && !F.empty()) {
    tickets[k] = F.front().first;
    results[k] = F.front().second;
    F.pop_front();
    ++k;
  }
  *n_done = k;
  return HALLAR_OK;
}

static hallar_status profile_out(hl::Pool &P, double *ms, int64_t *launches, double *bytes, int32_t nc, int32_t reset) {
  if (nc < 0 || nc > hl::KC_N) return HALLAR_E_INVALID;
  if (P.profile) {
    if (hipStreamSynchronize(P.stream) != hipSuccess) return HALLAR_E_HIP;
    hl::prof_flush(P);
  }
  for (int c = 0; c < nc; ++c) {
    if (ms) ms[c] = P.prof_ms[c];
    if (launches) launches[c] = P.prof_n[c];
    if (bytes) bytes[c] = P.prof_bytes[c];
  }
  if (reset)
    for (int c = 0; c < hl::KC_N; ++c) {
      P.prof_ms[c] = 0;
      P.prof_n[c] = 0;
      P.prof_bytes[c] = 0;
    }
  return HALLAR_OK;
}

hallar_status hallar_profile(hallar_t h, double *ms, int64_t *launches, double *bytes, int32_t n_classes, int32_t reset) {
  if (!h) return fail(nullptr, HALLAR_E_INVALID, "bad handle");
  const hallar_status st = profile_out(h->P, ms, launches, bytes, n_classes, reset);
  return st == HALLAR_OK ? st : fail(h, st, "n_classes out of range");
}

hallar_status hallar_pool_profile(hallar_pool_t pool, double *ms, int64_t *launches, double *bytes, int32_t n_classes,
                                  int32_t reset) {
  if (!pool) return fail(nullptr, HALLAR_E_INVALID, "pool is NULL");
  const hallar_status st = profile_out(pool->P, ms, launches, bytes, n_classes, reset);
  return st == HALLAR_OK ? st : failp(pool, st, "n_classes out of range");
}

hallar_status hallar_pool_usage(hallar_pool_t pool, size_t *used, size_t *budget) {
  if (!pool) return fail(nullptr, HALLAR_E_INVALID, "pool is NULL");
  if (used) *used = pool->P.arena.used();
  if (budget) *budget = pool->P.arena.capacity();
  return HALLAR_OK;
}

}  // extern "C"
