// Host-side structures of the library: the preprocessed problem, the device
// slab allocator, pool slots and the per-instance solver state.
#pragma once
#include <coroutine>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hallar.h"
#include "internal.h"

namespace hl {

// ---------------------------------------------------------------- problem
// Preprocessed instance (Section 4.1): union support S of the upper-triangle
// entries, pair k = position in the row CSR; index lists L_ij; the
// strictly-lower transpose for the symmetric pattern S u S^T (Algorithm 4).
struct HostProblem {
  int32_t n = 0, m = 0;
  double tau2 = 1.0;
  int64_t npairs = 0, nlower = 0, nentries = 0;
  std::vector<int32_t> rowptr_u, col_u, pcon;  // pcon: 1..m or 0
  std::vector<double> c_u, pa;                 // C_ij and (A_l)_ij of the pair's constraint
  std::vector<int32_t> rowptr_l, col_l, pid_l;
  bool direct = true, has_c = false;
  bool pa_uniform = false;      // every constrained pair has the coefficient pa_const (direct mode)
  double pa_const = 0.0;
  bool c_diag_only = false;     // C's sparse part is diagonal: c_diag[i] = C_ii
  std::vector<double> c_diag;
  // every strictly-lower pair is constrained with coefficient pa_const and
  // has no sparse objective entry: the gradient SpMM recomputes the lower
  // half's values from (p_l, b_l) kept in lower order
  bool low_recompute = false;
  // direct mode: 1 if exactly the off-diagonal pairs are constrained (matrix
  // completion, theta), 2 if exactly the diagonal ones are (MaxCut), else 0;
  // kernels that only need to know whether a pair is constrained skip its
  // constraint id then
  int32_t con_rule = 0;
  // general mode (a constraint with several pairs or a pair in several constraints)
  std::vector<int32_t> eptr, econ, cptr, cent, epair;
  std::vector<double> ea, ew;
  // low-rank objective
  int32_t r0 = 0;
  std::vector<double> K0, D0;
  // low-rank parts of the constraints: terms merged per constraint (their K
  // columns side by side, their D blocks on the diagonal), K row-major n x rk
  int32_t rk = 0, nlc = 0;
  std::vector<double> Kc, Dc;
  std::vector<int32_t> lc_con, lc_off, lc_doff, lc_of_con;
  std::vector<int32_t> lc_term;  // term of each column of K (rk)
  // coded-diffraction constraints (Section 5.4) on the real form: L masks of
  // n_c = n / 2 complex entries, interleaved (re, im), pattern-major
  int32_t cdp_L = 0, cdp_nc = 0;
  std::vector<double> cdp_d;
  std::vector<double> b;
  double b_l1 = 0.0, c_l1 = 0.0;
  // tiles (row ranges) and their pair-stream choices; the schedule's two
  // parameters (defaults, or the autotuner's choice)
  std::vector<Tile> tiles;
  int32_t tile_min_rows = 64, tile_ent_cap = TILE_MAX_ENTRIES;
};

// Returns "" on success or an error message; *code receives the status.
std::string build_host_problem(const hallar_problem *p, HostProblem &out, hallar_status *code);
void build_tiles(HostProblem &hp);

// symmetric eigen decomposition (cyclic Jacobi): A (row-major n x n) ->
// ascending eigenvalues w and eigenvectors as columns of Q (row-major).
void sym_eig(int n, const double *A, double *w, double *Q);

inline int r_bucket(int r, int prec) {
  int R = prec == 0 ? 2 : 4;
  while (R < r) R *= 2;
  return R;
}

// ---------------------------------------------------------------- coroutine task
struct Task {
  struct promise_type {
    std::coroutine_handle<> cont;
    Task get_return_object() { return Task{std::coroutine_handle<promise_type>::from_promise(*this)}; }
    std::suspend_always initial_suspend() noexcept { return {}; }
    struct Final {
      bool await_ready() noexcept { return false; }
      std::coroutine_handle<> await_suspend(std::coroutine_handle<promise_type> h) noexcept {
        auto c = h.promise().cont;
        return c ? c : std::noop_coroutine();
      }
      void await_resume() noexcept {}
    };
    Final final_suspend() noexcept { return {}; }
    void return_void() {}
    void unhandled_exception() { std::terminate(); }
  };
  std::coroutine_handle<promise_type> h;
  explicit Task(std::coroutine_handle<promise_type> hh) : h(hh) {}
  Task(Task &&o) noexcept : h(o.h) { o.h = {}; }
  Task(const Task &) = delete;
  ~Task() {
    if (h) h.destroy();
  }
  bool await_ready() { return false; }
  std::coroutine_handle<> await_suspend(std::coroutine_handle<> c) {
    h.promise().cont = c;
    return h;
  }
  void await_resume() {}
};

// ---------------------------------------------------------------- device ops
enum OpCode : int {
  OP_NONE = 0, OP_TRIAL, OP_GRAD, OP_EVAL, OP_COPY, OP_PACK, OP_LZ_BEGIN, OP_LZ_STEPS, OP_LZ_RITZ, OP_LZ_RESTART,
  OP_FW_PREP, OP_FW_APPLY, OP_SETP, OP_GRAM, OP_ROTATE
};

struct PendingOp {
  OpCode code = OP_NONE;
  int R = 0, R2 = 0;        // bucket (destination) and source bucket
  int xrole = 0, msel = -1, wT = 0, wyp = 0, zsel = 0;
  int rlive = 0;            // columns of the operands that can be nonzero (<= R)
  int src = 0, dst = 0;
  const double *ext = nullptr;
  int ext_r = 0;
  int64_t ext_ld = 0;
  int steps = 0, use_prev = 0;
  uint64_t seed = 0;
  std::vector<double> upload;   // coefficients for this op
  int64_t dl_count = 0;         // doubles to download
  // filled by the engine
  int64_t up_off = 0, dl_off = 0;
  int key() const;
};

struct Pool;
struct CdpFft;  // FFT plans of a coded-diffraction instance (engine.cpp)

// per-instance solver state (one HALLaR solve)
struct Slot {
  bool used = false;
  int64_t ticket = -1;
  HostProblem hp;
  InstDev dev{};            // host copy of the device descriptor
  void *slab = nullptr;     // device memory of the instance
  size_t slab_bytes = 0;
  size_t slab_off = 0;      // offset in the pool arena (pool mode)
  int Rcap = 0;
  int kmax = 0;
  // solver
  Task *task = nullptr;
  std::coroutine_handle<> resume{};
  PendingOp op;
  bool has_op = false, done = false;
  hallar_result result{};
  std::vector<double> H;    // host Lanczos projected matrix
  double lz_sigma = 0.0;    // SpMV shift for the next Lanczos call (last smallest Ritz value)
  std::vector<double> dl;   // downloaded block of the last round
  // buffer bookkeeping
  std::vector<int> free_bufs;
  int cur_R = 0;            // bucket of live U-like buffers
  int cur_r = 1;            // columns of the iterate (the rest of the bucket is zero)
  InstParams prm{};
  const double *U0ext = nullptr;  // device FP64 U0
  int U0r = 0;
  const double *p0ext = nullptr;
  std::vector<double> U0host;
  int final_buf = -1, final_r = 0;
  double t_start = 0.0;
  uint64_t seed = 0;
  std::string err;
  CdpFft *fft = nullptr;    // owned; released by slot_unload
  std::vector<hallar_outer_record> history;  // one record per outer iteration of the solve
};

}  // namespace hl
