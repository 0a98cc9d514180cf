// Internal layout shared by the host engine and the HIP kernels.
//
// Every kernel is "segment indexed": its grid walks a list of Tiles, each a
// contiguous row range of one instance, and looks the instance up in a
// device array of InstDev descriptors.  One launch therefore serves one
// instance (a plain solve) or thousands of uneven ones (batched / served
// solves) with the same code.  Reductions are deterministic: every tile
// writes its partial sums to its own slot and a reduce kernel adds the
// slots of an instance in a fixed order, so an instance's results do not
// depend on which other instances share the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hl {

constexpr int BLOCK = 256;       // threads per workgroup (4 wave64)
constexpr int RBLOCK = 1024;     // threads of a reduce workgroup (16 wave64)
constexpr int LR_MAX = 2;        // rank of the low-rank objective term
constexpr int R_MAX = 64;        // columns of U
constexpr int RK_MAX = 4096;     // columns of the constraints' low-rank parts (all terms together)
constexpr int KMAX = 64;         // Lanczos basis vectors before a restart
constexpr int PSTRIDE = 144;     // partial-sum slots per tile (>= KMAX + 1 + LR_MAX, >= 3 + LR_MAX * R_MAX)
constexpr int LZ_W2_SLOT = PSTRIDE - 1;  // partial ||G v_j||^2 of the Lanczos SpMV
constexpr int LZ_WP_SLOT = PSTRIDE - 2;  // partial ||w'||^2 after the first Gram-Schmidt pass
constexpr int LZ_KV_SLOT = PSTRIDE - 4;  // partial K0^T w' (LR_MAX slots)
constexpr int RED_SPLIT = 16;            // workgroups per instance of the trial's reduces
constexpr int RED_SPLIT_MIN_TILES = 2048;  // instances with fewer tiles reduce in one workgroup
constexpr int FUSE_SLOT = PSTRIDE - 8;   // the fused trial kernel's SpMM partials (2 slots)
constexpr int COMBO_SLOT = PSTRIDE - 6;  // the extrapolation's ||XT - W0||^2 partial
constexpr int PROJ_SLOT = PSTRIDE - 12;  // the projection's three dot partials
static_assert(PROJ_SLOT >= 4 + LR_MAX * R_MAX && PROJ_SLOT + 3 <= FUSE_SLOT,
              "trial slots overlap the low-rank slots or each other");
static_assert(COMBO_SLOT == FUSE_SLOT + 2 && COMBO_SLOT < LZ_KV_SLOT, "one reduce reads FUSE_SLOT..COMBO_SLOT");
constexpr int NRES = 32;         // result scalars per instance
constexpr int TILE_MAX_ROWS = 1024;     // rows of a tile (row pointers staged in LDS)
constexpr int TILE_MAX_ENTRIES = 2048;  // entries of S u S^T staged per tile (longer tiles: single rows)

// Roles of the n x R work buffers (operator type).  The host maps roles to
// physical buffers per instance (InstParams::buf), so FISTA's y <- y+ and
// similar updates are pointer swaps, not copies.
enum Role : int { RX = 0, RY, RXT, RW0, RGR, RZ, RU, RU2, NROLE };
constexpr int NBUF = 8;

struct Tile {
  int32_t inst;     // index into the InstDev array
  int32_t row0, row1;
  int32_t lt;       // tile index inside its instance (partial slot)
  int8_t plog_u;    // log2 pair streams per row in the SDDMM
  int8_t plog_s;    // log2 pair streams per row in the SpMM / SpMV
  int8_t pad_[2];
};

// Per-instance scalars written by the host before a round.
struct InstParams {
  double beta;          // AL penalty
  double lam, L, invL;  // prox stepsize, FISTA curvature
  double tau, tau2;
  double cY, cX;        // x~ = cY * Y + cX * X
  double u1, u2, u3;    // X <- u1 * Z + u2 * X + u3 * XT (FISTA x update, Z = last y+)
  double fw_a, fw_b;    // FW: U~ = [fw_a * U, fw_b * v]
  double lz_scale;      // generic scale
  int32_t upd_x;
  int32_t r;            // columns in use
  int32_t buf[NROLE];   // role -> physical buffer
  int32_t lz_basis;     // 0: V is the basis, 1: V2
  int32_t lz_steps;     // Lanczos steps to run this round
  int32_t lz_j;         // index of the vector the next step multiplies
  int32_t lz_q;         // Ritz / restart columns
  int32_t fw_col;       // column receiving the FW direction (-1: none)
  int32_t fw_rnew;      // columns after the FW step
  int32_t rnew;         // columns after a rotation
  int32_t lz_j0;        // lz_j at the start of the round (download layout)
  int32_t lz_use_prev;  // Lanczos start: previous vector + small noise
  int32_t lz_skip;      // set on the device: this step's second Gram-Schmidt pass is not needed
  int32_t lz_tri0;      // from this basis index on, v_{j-1} is the previous vector of a three-term chain
  double lz_shift;      // the SpMV forms (G - lz_shift I) v_j - beta_{j-1} v_{j-1}
  int32_t fw_v_on;      // Frank-Wolfe direction present (theta > 0)
  uint64_t lz_seed;     // counter-based start-vector seed
  int64_t up_off;       // offset of this instance's coefficients in the upload buffer
  int64_t dl_off;       // offset of this instance's block in the download buffer
  void *ext[2];         // caller buffers addressed as roles NBUF, NBUF + 1 (standalone operator calls)
};

// Per-instance scalars written by the kernels, read back by the host.
struct InstRes {
  double v[NRES];
};

// Result slots.
enum ResSlot : int {
  S_G_XT = 0, S_G_YP, S_XTW0, S_GR_D, S_D2, S_YPW0, S_NZ, S_PROJC,
  S_RL2, S_RL_W0, S_WY, S_T0, S_PR, S_RR, S_G_EVAL, S_BP,
  S_FWDEN, S_LZ_BETA, S_LZ_NRM0, S_LZ_ALPHA, S_GRAM_OK, S_NAN,
  S_LZ_KV0, S_LZ_KV1,   // K0^T v for the next SpMV (low-rank term)
  S_YT,                 // sum_l y'_l T_l (G . XX^T = T_0 + sum_l y'_l T_l)
  S_GR2T,               // ||GR||^2 of a FISTA trial (rounding bound of <GR, d>)
  S_GR2A,               // ||GR||^2 at ADAP-FISTA's output (rounding bound of R_j)
  S_LZ_W2,              // ||G v_j||^2 before reorthogonalisation (second-pass test)
  S_PTR,                // p_t^T (A(X_t) - b) after the dual update (objective accuracy test)
  S_COUNT
};

// Device descriptor of one instance.
struct InstDev {
  int32_t n, m, npairs, nlower;
  int32_t r0;           // rank of the low-rank objective term (0: none)
  int32_t direct;       // every constraint has exactly one pair entry and every pair at most one constraint
  int32_t ntiles;
  int32_t prows;        // rows of the partial-sum matrix (slot q of row t at part[q * prows + t])
  // structure (device)
  const int32_t *rowptr_u, *col_u, *pcon;   // upper CSR over S (pair k = position), constraint of pair (0 = none)
  const int32_t *rowptr_l, *col_l, *pid_l;  // strictly-lower transpose of S with pair ids
  // lower-half recompute: every strictly-lower pair is constrained, with the
  // shared coefficient pa_const and no sparse objective entry, so the
  // gradient SpMM forms its values from (p_l, b_l) stored in lower order
  // instead of gathering the SDDMM's values through pid_l
  int32_t low_mode;
  double *low_pb;                           // nlower x {p_l, b_l} when low_mode
  // direct mode: {p_l, b_l} of each pair's constraint in pair order (zeros
  // for unconstrained pairs), so the SDDMM's loads of them do not wait for
  // the load of the pair's constraint id
  double *upb;
  const void *c_u, *pa;                     // operator type: C_ij per pair, (A_l)_ij of the pair's constraint
  int32_t pa_uniform, c_diag_only;          // the SDDMM reads pa_const / c_diag instead of pa / c_u
  int32_t con_rule;                         // 1: constrained <=> off-diagonal, 2: <=> diagonal, 0: read pcon
  double pa_const;
  const double *c_diag;                     // length n when c_diag_only
  const double *c64, *pa64, *b;             // FP64 copies, b (length m)
  const void *K0; const double *D0;         // low-rank objective: K0 n x r0 (op type), D0 r0 x r0
  const double *K064;                       // FP64 K0 for the Lanczos SpMV
  // general (multi-entry) constraints
  const int32_t *eptr, *econ;               // pair -> entries (constraint id 1..m)
  const double *ea64, *ew64;                // entry values (A_l)_ij and (2 - delta_ij)(A_l)_ij
  const int32_t *cptr, *cent;               // constraint -> entry ids (l - 1 indexing)
  const int32_t *epair;                     // entry -> pair
  // work buffers
  void *buf[NBUF];                          // n x R_cap, operator type
  void *m_xt, *m_yp;                        // pair values of M = C + A*(y') (operator type)
  double *Bpair;                            // general mode: <U_i,U_j> per pair
  double *p, *yp, *TY, *Ty;                 // length m
  double *m64;                              // pair values in FP64 (Lanczos)
  double *m64_low;                          // the same values in lower order (copied once per Lanczos start)
  double *V, *V2;                           // Lanczos bases, (KMAX + 1) x n
  double *w, *lzv;                          // Lanczos work vector, Ritz / start vector
  double *hcoef;                            // KMAX + 1 reorthogonalisation coefficients
  double *Z0;                               // 2 x LR_MAX x R_MAX low-rank products D0 K0^T X
  const double *up_base;                    // pool upload buffer (Ritz / restart coefficients, rotations)
  double *dl_base;                          // pool download buffer (Lanczos columns, Gram matrices)
  double *part;                             // PSTRIDE x prows partial sums, slot-major
  double *red_stage;                        // RED_SPLIT x RQ sums of the split trial reduces
  uint32_t *red_count;                      // blocks of a split reduce done (0 between launches)
  double *gram;                             // (R x R) x ntiles Gram partials, entry-major
  InstParams *prm;
  InstRes *res;
  // low-rank parts of the constraints (Section 3.2, eq. HSLR-rep-body): rk
  // columns K (n x rk row-major, operator type, and an FP64 copy for the
  // Lanczos SpMV), nlc terms, one per constraint that has one: term q sits on
  // constraint lc_con[q] (1..m), owns columns lc_off[q]..lc_off[q+1] and the
  // D block at Dc + lc_doff[q]; lc_of_con[l - 1] is constraint l's term or -1
  int32_t rk, nlc;
  const void *Kc;
  const double *Kc64, *Dc;
  const int32_t *lc_con, *lc_off, *lc_doff, *lc_of_con, *lc_term;  // lc_term: term of each column k
  double *lc_part;   // per tile: rk x R_MAX partial sums of K^T X (or K^T v)
  double *lc_Y;      // K^T X, rk x R_MAX
  double *lc_Z;      // 2 slots (zsel) of blockdiag(y'_l D_q) K^T X: rk x R (rows of stride R) in rk x R_MAX each
  double *lc_T;      // nlc: Tr(D_q (K_q^T X)(K_q^T X)^T), the low-rank part of A_l . X X^T
  double *lc_v;      // rk: K^T v for a vector v
  double *lc_zv;     // rk: blockdiag(y''_l D_q) K^T v (added by the Lanczos SpMV)
  double *lc_Tv;     // nlc: (K_q^T v)^T D_q (K_q^T v) (Frank-Wolfe step size)
  double *lc_W[2];   // per Z-slot: the adjoint's low-rank block K Z, n x R (rows of stride R)
  double *lc_wv;     // n: K lc_zv (the Lanczos product's low-rank part)
  // coded-diffraction constraints (Section 5.4) on the real form, n = 2 nc:
  // L masks d (nc complex each); spectra S of d_l * u_c, transform
  // (l R + c) contiguous (the FFTs' batch order), and their scaled copy S2;
  // cdp_T[l nc + k] = sum_c |S|^2 / nc (the constraint values); cdp_W[z] the
  // adjoint's n x R block added by the SpMM epilogue (z the Z-slot);
  // cdp_wv / cdp_Tv the Lanczos and Frank-Wolfe vector forms
  int32_t cdp_L, cdp_nc;
  const double2 *cdp_d;
  double2 *cdp_S, *cdp_S2;
  double *cdp_T, *cdp_Tv, *cdp_wv;
  double *cdp_W[2];
};

// Products of the constraints' low-rank parts (k_lc_red, after k_lc_sum has
// formed Y = K^T X or K^T v): lc_T from Y; lc_Z from Y with the multipliers
// (I.yp or given); both; lc_zv from K^T v (Lanczos, multipliers I.yp);
// lc_Tv from K^T v.
enum LcMode : int { LC_Y_T = 0, LC_Z, LC_Y_Z, LC_V_LZ, LC_V_FW };

// Scratch of the allocation-free evaluation: one static device array per GPU.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

// Where the allocation-free evaluation puts what it writes (all inside the
// scratch array): the descriptor array (instance s at insts[s]), parameters,
// result scalars, partial sums (prows rows per slot), the packed U (unless
// u_ext, the caller's U read in place), low-rank products and, in general
// mode, T, y' and the per-pair dot products.
struct NoallocViews {
  InstDev *insts;
  InstParams *prm;
  InstRes *res;
  double *part;
  int32_t prows;
  void *ubuf;
  const void *u_ext;
  double *Z0, *TY, *yp, *Bpair;
};

}  // namespace hl
