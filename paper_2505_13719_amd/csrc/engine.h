// Batched round executor and the pool of resident instances.
#pragma once
#include <atomic>
#include <condition_variable>
#include <deque>
#include <unordered_map>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <functional>

#include "host.h"

namespace hl {

// First-fit sub-allocator over one device slab (no hipMalloc while serving).
class Arena {
 public:
  bool init(size_t bytes, std::string &err);
  void release();
  // returns offset or SIZE_MAX
  size_t alloc(size_t bytes);
  void free(size_t off, size_t bytes);
  char *base() const { return base_; }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }

 private:
  char *base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> size
};

// Host worker threads that resume the solver coroutines of a round in
// parallel (each coroutine touches only its own slot; the pool's shared
// state is read-only while they run).
class ResumeWorkers {
 public:
  ~ResumeWorkers();
  // run fn(i) for i in [0, n) on the workers and the calling thread
  void run(int n, const std::function<void(int)> &fn);

 private:
  struct Job {
    const std::function<void(int)> *fn;
    int n;
    std::atomic<int> next{0}, done{0};
  };
  void loop();
  static void work(Job &j);
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_;
  uint64_t gen_ = 0;
  bool stop_ = false;
  std::shared_ptr<Job> job_;  // a worker holds its own reference while it works on a job
};

// kernel classes of the profile
enum KClass : int { KC_SDDMM = 0, KC_SPMM, KC_LZ_SPMV, KC_LZ_ORTH, KC_VEC, KC_REDUCE, KC_OTHER, KC_FUSED, KC_CDP, KC_N };

struct ProfRec {
  int cls, e0, e1;
  double bytes;
};

struct Pool {
  int prec = 0;
  hallar_options opts{};
  hipStream_t stream = nullptr;
  size_t budget = 0;
  bool use_arena = false;  // serving pool: one slab for everything
  Arena arena;
  int max_slots = 0;
  std::vector<std::unique_ptr<Slot>> slots;
  // device / pinned arrays indexed by slot
  InstDev *d_insts = nullptr;
  InstParams *d_prm = nullptr, *h_prm = nullptr;
  InstRes *d_res = nullptr, *h_res = nullptr;
  std::vector<InstDev> h_insts;
  Tile *d_tiles = nullptr, *h_tiles = nullptr;
  int64_t tiles_cap = 0;
  // the slots whose tiles d_tiles holds, in order, and the load epoch they
  // were taken at: a round with the same slots in the same order (a
  // standalone solve, or a stable batch) skips rebuilding and uploading them
  std::vector<int> tiles_run;
  std::vector<int32_t> ilist_dev;  // the instance lists d_ilist holds (a round with the same lists skips the upload)
  int64_t tile_epoch = 0, tiles_epoch = -1;
  int32_t *d_ilist = nullptr, *h_ilist = nullptr;
  int64_t ilist_cap = 0;
  double *d_up = nullptr, *h_up = nullptr;
  int64_t up_cap = 0;
  double *d_dl = nullptr, *h_dl = nullptr;
  int64_t dl_cap = 0;
  bool insts_dirty = true;
  void *scratch = nullptr;  // device address of the allocation-free evaluation's scratch on this pool's device
  std::deque<std::pair<int64_t, hallar_result>> finished;
  int64_t rounds = 0;
  std::string err;
  hallar_status fatal = HALLAR_OK;
  hallar_status launch_err = HALLAR_OK;  // set by a launch helper that failed inside a round (err says why)
  // profiling (opts.profile)
  bool profile = false;
  int prof_level = 0;  // 1: every kernel class, 2: the sparse streaming classes only
  std::vector<hipEvent_t> events;
  int ev_used = 0;
  std::vector<ProfRec> recs;
  double prof_ms[KC_N] = {0}, prof_bytes[KC_N] = {0};
  int64_t prof_n[KC_N] = {0};
  // side streams (default priority) on which the groups of a round run
  // concurrently, joined to `stream` by events
  static constexpr int NSIDE = 3;
  hipStream_t side[NSIDE] = {};
  hipEvent_t ev_fork = nullptr, ev_join[NSIDE] = {};
  std::unique_ptr<ResumeWorkers> workers;
  // host-side seconds per round phase (reported at release when opts.verbose)
  double t_prep = 0, t_launch = 0, t_wait = 0, t_resume = 0;
  // captured rounds (opts.graphs): the kernel section of a round, keyed by
  // everything that decides its launches, replayed as one graph launch
  struct RoundGraph {
    std::vector<int64_t> sig;
    hipGraphExec_t exec = nullptr;
    int seen = 0;
    bool failed = false;
    int64_t last_use = 0;
  };
  std::unordered_map<uint64_t, RoundGraph> graphs;
  // stream the graphs are captured on and replayed from (the caller's stream
  // may be the null stream, which cannot be captured), forked from and
  // joined back to `stream` by events
  hipStream_t gst = nullptr;
  hipEvent_t ev_gfork = nullptr, ev_gjoin = nullptr;
  int64_t graph_replays = 0, graph_captures = 0;
};

// lifetime
hallar_status pool_init(Pool &P, int max_slots, int prec, const hallar_options &opts, hipStream_t stream,
                        size_t arena_bytes, int64_t tiles_cap, std::string &err);
void pool_release(Pool &P);

// footprint of an instance (bytes of its device slab)
size_t instance_bytes(const HostProblem &hp, int prec, int Rcap, int kmax);
int rcap_for(const hallar_options &o, int prec);
int kmax_for(const hallar_options &o, int n);

// upload a preprocessed problem into slot `s` (allocates the slab)
hallar_status slot_load(Pool &P, int s, HostProblem &&hp, std::string &err);
void slot_unload(Pool &P, int s);

// solver: start the coroutine of slot s (U0: device FP64 n x r0 or NULL)
void slot_start_solve(Pool &P, int s);
// adds the elapsed times of the recorded, completed profiling events to the per-class totals
void prof_flush(Pool &P);
// run rounds until no slot has work or `max_rounds` rounds (<=0: unlimited)
hallar_status pool_run(Pool &P, int max_rounds);
int pool_active(const Pool &P);

// standalone operator calls on slot s of P
hallar_status op_eval_AUUt(Pool &P, int s, const void *U, int r, int64_t ldu, double *T, hipStream_t st);
hallar_status op_eval_AUUt_noalloc(Pool &P, int s, const void *U, int r, int64_t ldu, double *T, hipStream_t st);
hallar_status op_adjoint(Pool &P, int s, const double *p, const void *U, int r, int64_t ldu, void *W, int64_t ldw,
                         hipStream_t st);
hallar_status op_min_eig(Pool &P, int s, const double *p, const double *v0, double tol, int max_iter, double *lambda,
                         double *v, hallar_eig_info *info);

}  // namespace hl
