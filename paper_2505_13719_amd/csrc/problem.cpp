// Host preprocessing of an HSLR problem (Section 3.2) into the structures the
// kernels stream: the union support S and index lists L_ij (Section 4.1,
// eqs. def: support S ell and index list), the symmetric pattern S u S^T of
// the adjoint (Algorithm 4), and the tile schedule.
#include <algorithm>
#include <limits>
#include <cmath>
#include <cstring>
#include <numeric>

#include "host.h"

namespace hl {

namespace {
struct Ent {
  uint64_t key;  // (i << 32) | j
  int32_t l;
  int32_t idx;
};
}  // namespace

std::string build_host_problem(const hallar_problem *p, HostProblem &hp, hallar_status *code) {
  *code = HALLAR_E_INVALID;
  if (!p) return "problem is NULL";
  if (p->n < 1 || p->n >= (int64_t)1 << 31) return "n out of range";
  if (p->m < 0 || p->m >= (int64_t)1 << 31) return "m out of range";
  if (!(p->trace_bound > 0.0) || !std::isfinite(p->trace_bound)) return "trace_bound must be positive and finite";
  if (p->nnz < 0) return "nnz < 0";
  if (p->nnz > 0 && (!p->row || !p->col || !p->con || !p->val)) return "entry arrays are NULL";
  if (p->m > 0 && !p->b) return "b is NULL";
  const int32_t n = (int32_t)p->n, m = (int32_t)p->m;
  hp.n = n;
  hp.m = m;
  hp.tau2 = p->trace_bound;
  hp.b.assign(p->b, p->b + m);
  for (int l = 0; l < m; ++l)
    if (!std::isfinite(hp.b[l])) {
      *code = HALLAR_E_NUMERICAL;
      return "b has NaN/Inf";
    }
  if (p->n_lowrank < 0) return "n_lowrank < 0";
  if (p->n_lowrank > 0 && (!p->lr_con || !p->lr_rank || !p->K || !p->D)) return "low-rank arrays are NULL";
  bool has_lc = false;
  for (int32_t t = 0; t < p->n_lowrank; ++t) {
    if (p->lr_con[t] < 0 || p->lr_con[t] > m) return "lr_con out of range";
    if (p->lr_rank[t] < 1) return "lr_rank must be >= 1";
    if (p->lr_con[t] > 0) has_lc = true;
  }
  if (p->cdp_patterns < 0) return "cdp_patterns < 0";
  if (p->cdp_patterns > 0) {
    const int64_t L = p->cdp_patterns;
    if (!p->cdp_masks) return "cdp_masks is NULL";
    if (n % 2 != 0) return "coded-diffraction problems need an even n (the real form of n/2 complex entries)";
    if ((int64_t)m != L * (n / 2)) return "coded-diffraction problems need m = cdp_patterns * n / 2";
    if (p->n_lowrank > 0) {
      *code = HALLAR_E_UNSUPPORTED;
      return "coded-diffraction constraints cannot be combined with low-rank terms";
    }
    for (int64_t k = 0; k < p->nnz; ++k)
      if (p->con[k] != 0) {
        *code = HALLAR_E_UNSUPPORTED;
        return "coded-diffraction problems take sparse entries on the objective only";
      }
    hp.cdp_L = (int32_t)L;
    hp.cdp_nc = n / 2;
    hp.cdp_d.assign(p->cdp_masks, p->cdp_masks + 2 * L * (n / 2));
    for (double v : hp.cdp_d)
      if (!std::isfinite(v)) {
        *code = HALLAR_E_NUMERICAL;
        return "cdp_masks has NaN/Inf";
      }
  }
  std::vector<Ent> e((size_t)p->nnz);
  for (int64_t k = 0; k < p->nnz; ++k) {
    const int32_t i = p->row[k], j = p->col[k], l = p->con[k];
    if (i < 0 || j < 0 || i >= n || j >= n) return "entry index out of range";
    if (i > j) return "entries must be upper triangular (row <= col)";
    if (l < 0 || l > m) return "constraint index out of range";
    if (!std::isfinite(p->val[k])) {
      *code = HALLAR_E_NUMERICAL;
      return "val has NaN/Inf";
    }
    e[k] = Ent{((uint64_t)i << 32) | (uint32_t)j, l, (int32_t)k};
  }
  std::sort(e.begin(), e.end(), [](const Ent &a, const Ent &b) { return a.key != b.key ? a.key < b.key : (a.l != b.l ? a.l < b.l : a.idx < b.idx); });
  // merge duplicate (i, j, l) triples
  std::vector<uint64_t> keys;
  std::vector<int32_t> ls;
  std::vector<double> vs;
  keys.reserve(e.size());
  ls.reserve(e.size());
  vs.reserve(e.size());
  for (size_t k = 0; k < e.size();) {
    size_t q = k;
    double v = 0.0;
    while (q < e.size() && e[q].key == e[k].key && e[q].l == e[k].l) v += p->val[e[q++].idx];
    keys.push_back(e[k].key);
    ls.push_back(e[k].l);
    vs.push_back(v);
    k = q;
  }
  std::vector<Ent>().swap(e);
  // pairs
  std::vector<int64_t> pstart;
  for (size_t k = 0; k < keys.size(); ++k)
    if (k == 0 || keys[k] != keys[k - 1]) pstart.push_back((int64_t)k);
  const int64_t P = (int64_t)pstart.size();
  pstart.push_back((int64_t)keys.size());
  hp.npairs = P;
  hp.rowptr_u.assign(n + 1, 0);
  hp.col_u.resize(P);
  hp.c_u.assign(P, 0.0);
  hp.pcon.assign(P, 0);
  hp.pa.assign(P, 0.0);
  std::vector<int32_t> ccount(m, 0);
  int64_t nent = 0;
  bool direct = true, has_c = false;
  for (int64_t k = 0; k < P; ++k) {
    const uint64_t key = keys[pstart[k]];
    const int32_t i = (int32_t)(key >> 32), j = (int32_t)(key & 0xffffffffu);
    hp.rowptr_u[i + 1]++;
    hp.col_u[k] = j;
    int nc = 0;
    for (int64_t q = pstart[k]; q < pstart[k + 1]; ++q) {
      if (ls[q] == 0) {
        hp.c_u[k] += vs[q];
        has_c = true;
      } else {
        ++nc;
        ++nent;
        ccount[ls[q] - 1]++;
        hp.pcon[k] = ls[q];
        hp.pa[k] = vs[q];
      }
    }
    if (nc > 1) direct = false;
  }
  for (int l = 0; l < m; ++l)
    if (ccount[l] != 1) direct = false;
  // a constraint with a low-rank part sums more than its pairs
  if (has_lc || hp.cdp_L > 0) direct = false;
  for (int i = 0; i < n; ++i) hp.rowptr_u[i + 1] += hp.rowptr_u[i];
  hp.direct = direct;
  hp.has_c = has_c;
  hp.nentries = nent;
  // structure the SDDMM can exploit without reading per-pair arrays: one
  // coefficient shared by every constrained pair (MaxCut 1, theta and matrix
  // completion 1/2), and a sparse objective that lives on the diagonal only
  // (matrix completion's I/2)
  {
    bool uni = direct, first = true;
    double a0 = 0.0;
    for (int64_t k = 0; k < P && uni; ++k)
      if (hp.pcon[k] > 0) {
        if (first) {
          a0 = hp.pa[k];
          first = false;
        } else if (hp.pa[k] != a0) {
          uni = false;
        }
      }
    hp.pa_uniform = uni && !first;
    hp.pa_const = a0;
    bool off = direct, on = direct;
    for (int32_t i = 0; i < n && (off || on); ++i)
      for (int32_t k = hp.rowptr_u[i]; k < hp.rowptr_u[i + 1]; ++k) {
        const bool dg = hp.col_u[k] == i, con = hp.pcon[k] > 0;
        if (con == dg) off = false;
        if (con != dg) on = false;
      }
    hp.con_rule = off ? 1 : (on ? 2 : 0);
    bool diag = has_c;
    for (int32_t i = 0; i < n && diag; ++i)
      for (int32_t k = hp.rowptr_u[i]; k < hp.rowptr_u[i + 1]; ++k)
        if (hp.col_u[k] != i && hp.c_u[k] != 0.0) {
          diag = false;
          break;
        }
    hp.c_diag_only = diag;
    if (diag) {
      hp.c_diag.assign(n, 0.0);
      for (int32_t i = 0; i < n; ++i)
        for (int32_t k = hp.rowptr_u[i]; k < hp.rowptr_u[i + 1]; ++k)
          if (hp.col_u[k] == i) hp.c_diag[i] = hp.c_u[k];
    }
  }
  if (!direct) {
    hp.eptr.assign(P + 1, 0);
    hp.econ.resize(nent);
    hp.ea.resize(nent);
    hp.ew.resize(nent);
    hp.epair.resize(nent);
    int64_t t = 0;
    for (int64_t k = 0; k < P; ++k) {
      const uint64_t key = keys[pstart[k]];
      const bool diag = (key >> 32) == (key & 0xffffffffu);
      for (int64_t q = pstart[k]; q < pstart[k + 1]; ++q)
        if (ls[q] > 0) {
          hp.econ[t] = ls[q];
          hp.ea[t] = vs[q];
          hp.ew[t] = (diag ? 1.0 : 2.0) * vs[q];
          hp.epair[t] = (int32_t)k;
          ++t;
        }
      hp.eptr[k + 1] = (int32_t)t;
      hp.pcon[k] = 0;
      hp.pa[k] = 0.0;
    }
    hp.cptr.assign(m + 1, 0);
    for (int64_t q = 0; q < nent; ++q) hp.cptr[hp.econ[q]]++;
    for (int l = 0; l < m; ++l) hp.cptr[l + 1] += hp.cptr[l];
    std::vector<int32_t> fill(hp.cptr.begin(), hp.cptr.end() - 1);
    hp.cent.resize(nent);
    for (int64_t q = 0; q < nent; ++q) hp.cent[fill[hp.econ[q] - 1]++] = (int32_t)q;
  }
  // strictly-lower transpose: row j lists (i, pair) for pairs (i, j), i < j
  hp.rowptr_l.assign(n + 1, 0);
  int64_t nl = 0;
  for (int i = 0; i < n; ++i)
    for (int32_t k = hp.rowptr_u[i]; k < hp.rowptr_u[i + 1]; ++k)
      if (hp.col_u[k] != i) {
        hp.rowptr_l[hp.col_u[k] + 1]++;
        ++nl;
      }
  for (int i = 0; i < n; ++i) hp.rowptr_l[i + 1] += hp.rowptr_l[i];
  hp.nlower = nl;
  hp.col_l.resize(nl);
  hp.pid_l.resize(nl);
  {
    std::vector<int32_t> fill(hp.rowptr_l.begin(), hp.rowptr_l.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int32_t k = hp.rowptr_u[i]; k < hp.rowptr_u[i + 1]; ++k) {
        const int32_t j = hp.col_u[k];
        if (j != i) {
          const int32_t pos = fill[j]++;
          hp.col_l[pos] = i;
          hp.pid_l[pos] = k;
        }
      }
  }
  {
    bool low = direct && hp.pa_uniform && (!has_c || hp.c_diag_only) && nl > 0;
    for (int64_t e = 0; e < nl && low; ++e)
      if (hp.pcon[hp.pid_l[e]] <= 0) low = false;
    hp.low_recompute = low;
  }
  // low-rank parts (Section 3.2, eq. HSLR-rep-body, Algorithms 3 and 5): the
  // objective's (at most one term, rank <= LR_MAX) and the constraints' (any
  // number of terms of any rank; the terms of one constraint are merged)
  {
    std::vector<int32_t> obj;
    std::vector<std::vector<int32_t>> per(m);
    for (int32_t t = 0; t < p->n_lowrank; ++t) {
      if (p->lr_con[t] == 0) obj.push_back(t);
      else per[p->lr_con[t] - 1].push_back(t);
    }
    auto kof = [&](int32_t t) { return p->K_off ? p->K_off[t] : (int64_t)0; };
    auto dof = [&](int32_t t) { return p->D_off ? p->D_off[t] : (int64_t)0; };
    auto finite_block = [&](int32_t t) {
      const int r = p->lr_rank[t];
      for (int64_t q = 0; q < (int64_t)n * r; ++q)
        if (!std::isfinite(p->K[kof(t) + q])) return false;
      for (int64_t q = 0; q < (int64_t)r * r; ++q)
        if (!std::isfinite(p->D[dof(t) + q])) return false;
      return true;
    };
    for (int32_t t = 0; t < p->n_lowrank; ++t)
      if (!finite_block(t)) {
        *code = HALLAR_E_NUMERICAL;
        return "K or D has NaN/Inf";
      }
    if (obj.size() > 1) {
      *code = HALLAR_E_UNSUPPORTED;
      return "at most one low-rank objective term is supported";
    }
    if (obj.size() == 1) {
      const int32_t t = obj[0];
      const int r0 = p->lr_rank[t];
      if (r0 > LR_MAX) {
        *code = HALLAR_E_UNSUPPORTED;
        return "low-rank objective rank must be 1 or 2";
      }
      hp.r0 = r0;
      hp.K0.assign(p->K + kof(t), p->K + kof(t) + (int64_t)n * r0);
      hp.D0.assign(p->D + dof(t), p->D + dof(t) + r0 * r0);
    }
    int64_t rk = 0;
    for (int l = 0; l < m; ++l)
      for (int32_t t : per[l]) rk += p->lr_rank[t];
    if (rk > RK_MAX) {
      *code = HALLAR_E_UNSUPPORTED;
      return "the constraints' low-rank parts have more than " + std::to_string(RK_MAX) + " columns";
    }
    hp.rk = (int32_t)rk;
    hp.lc_of_con.assign(m, -1);
    if (rk > 0) {
      hp.Kc.assign((size_t)n * rk, 0.0);
      hp.lc_off.push_back(0);
      int32_t col = 0;
      int64_t doff = 0;
      for (int l = 0; l < m; ++l) {
        if (per[l].empty()) continue;
        int32_t rl = 0;
        for (int32_t t : per[l]) rl += p->lr_rank[t];
        hp.lc_of_con[l] = (int32_t)hp.lc_con.size();
        hp.lc_con.push_back(l + 1);
        hp.lc_doff.push_back((int32_t)doff);
        std::vector<double> Dl((size_t)rl * rl, 0.0);
        int32_t c0 = 0;
        for (int32_t t : per[l]) {
          const int r = p->lr_rank[t];
          for (int32_t i = 0; i < n; ++i)
            for (int a = 0; a < r; ++a) hp.Kc[(size_t)i * rk + col + c0 + a] = p->K[kof(t) + (int64_t)i * r + a];
          for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b) Dl[(size_t)(c0 + a) * rl + c0 + b] = p->D[dof(t) + a * r + b];
          c0 += r;
        }
        hp.Dc.insert(hp.Dc.end(), Dl.begin(), Dl.end());
        doff += (int64_t)rl * rl;
        col += rl;
        hp.lc_off.push_back(col);
        hp.lc_term.insert(hp.lc_term.end(), (size_t)rl, (int32_t)hp.lc_con.size() - 1);
      }
      hp.nlc = (int32_t)hp.lc_con.size();
    }
  }
  // norms for eq. termination2
  double bl1 = 0.0;
  for (double v : hp.b) bl1 += std::fabs(v);
  hp.b_l1 = bl1;
  double cl1 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int32_t k = hp.rowptr_u[i]; k < hp.rowptr_u[i + 1]; ++k)
      cl1 += (hp.col_u[k] == i ? 1.0 : 2.0) * std::fabs(hp.c_u[k]);
  if (hp.r0 > 0) {
    const int r0 = hp.r0;
    if (n <= 4096) {
      // exact entrywise l1 of C^sp + K D K^T
      std::vector<double> row(n);
      double tot = 0.0;
      for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
          double s = 0.0;
          for (int a = 0; a < r0; ++a)
            for (int c = 0; c < r0; ++c) s += hp.K0[(size_t)i * r0 + a] * hp.D0[a * r0 + c] * hp.K0[(size_t)j * r0 + c];
          row[j] = s;
        }
        for (int32_t k = hp.rowptr_u[i]; k < hp.rowptr_u[i + 1]; ++k) row[hp.col_u[k]] += hp.c_u[k];
        for (int32_t e2 = hp.rowptr_l[i]; e2 < hp.rowptr_l[i + 1]; ++e2) row[hp.col_l[e2]] += hp.c_u[hp.pid_l[e2]];
        for (int j = 0; j < n; ++j) tot += std::fabs(row[j]);
      }
      cl1 = tot;
    } else {
      // sum_ab |D_ab| (sum_i |K_ia|)(sum_j |K_jb|): exact for a constant K column, an upper bound otherwise
      std::vector<double> ks(r0, 0.0);
      for (int i = 0; i < n; ++i)
        for (int a = 0; a < r0; ++a) ks[a] += std::fabs(hp.K0[(size_t)i * r0 + a]);
      for (int a = 0; a < r0; ++a)
        for (int c = 0; c < r0; ++c) cl1 += std::fabs(hp.D0[a * r0 + c]) * ks[a] * ks[c];
    }
  }
  hp.c_l1 = cl1;
  build_tiles(hp);
  // the sparse kernels stage a tile's row pointers in LDS
  for (const Tile &t : hp.tiles)
    if (t.row1 - t.row0 > TILE_MAX_ROWS || t.row1 <= t.row0) {
      *code = HALLAR_E_INVALID;
      return "internal: tile row range outside the kernels' limits";
    }
  *code = HALLAR_OK;
  return "";
}

// Tile schedule: contiguous row ranges of at most TILE_MAX_ROWS rows and
// tile_ent_cap (<= TILE_MAX_ENTRIES) entries of S u S^T (a row longer than
// that is a tile of its own), aiming at about kMaxTiles tiles per large
// instance (8 workgroups per CU) and at least tile_min_rows rows per tile for
// small ones.  Per tile, the
// number of pair streams per row (power of two near the mean row length) is
// kept for the kernels that walk rows with teams.  The schedule depends on
// the instance only, so a batched instance reduces in the same order as a
// standalone one.
static int plog_for(double avg) {
  int pl = 0;
  while ((1 << pl) < avg && pl < 6) ++pl;
  return pl;
}

void build_tiles(HostProblem &hp) {
  constexpr int64_t kMaxTiles = 2048;
  const int32_t kMinRows = std::max<int32_t>(1, std::min<int32_t>(hp.tile_min_rows, TILE_MAX_ROWS));
  const int64_t kEntCap = std::max<int32_t>(1, std::min<int32_t>(hp.tile_ent_cap, TILE_MAX_ENTRIES));
  const int32_t n = hp.n;
  const int32_t row_target =
      std::min<int32_t>(TILE_MAX_ROWS, std::max<int32_t>(kMinRows, (int32_t)((n + kMaxTiles - 1) / kMaxTiles)));
  hp.tiles.clear();
  int32_t r0 = 0;
  while (r0 < n) {
    int64_t ent = 0;
    int32_t r1 = r0;
    bool capped = false;
    while (r1 < n && (r1 - r0) < row_target) {
      const int64_t e = (hp.rowptr_u[r1 + 1] - hp.rowptr_u[r1]) + (hp.rowptr_l[r1 + 1] - hp.rowptr_l[r1]);
      if (r1 > r0 && ent + e > kEntCap) {
        capped = true;
        break;
      }
      ent += e;
      ++r1;
    }
    // A tile closed by the entry cap has long rows, which the SpMM walks with
    // a power-of-two number of lanes per row: 4..128 rows are cut to a power
    // of two so that rows x lanes fill the workgroup (17 rows would leave
    // 120 of 256 lanes idle, 16 rows use all of them).
    if (capped && r1 - r0 >= 4 && r1 - r0 <= 128) {
      int32_t p2 = 1;
      while (p2 * 2 <= r1 - r0) p2 *= 2;
      r1 = r0 + p2;
    }
    const double rows = (double)(r1 - r0);
    const double up = (double)(hp.rowptr_u[r1] - hp.rowptr_u[r0]) / rows;
    const double sym = up + (double)(hp.rowptr_l[r1] - hp.rowptr_l[r0]) / rows;
    Tile t{};
    t.inst = 0;
    t.row0 = r0;
    t.row1 = r1;
    t.lt = (int32_t)hp.tiles.size();
    t.plog_u = (int8_t)plog_for(up);
    t.plog_s = (int8_t)plog_for(sym);
    hp.tiles.push_back(t);
    r0 = r1;
  }
}

// Symmetric eigen decomposition of a small dense matrix (the Rayleigh-Ritz
// matrices of the Lanczos solver and the Gram matrices of U): Householder
// reduction to tridiagonal form with the transformations accumulated, then
// implicit QL iterations with Wilkinson shifts on the tridiagonal matrix,
// rotating the accumulated basis; eigenpairs sorted ascending.  The QL sweep
// is the published method of Bowdler, Martin, Reinsch and Wilkinson ("The QR
// and QL algorithms for symmetric matrices", Numer. Math. 11, 1968; the tql2
// procedure of the Handbook for Automatic Computation, vol. II) and keeps its
// order of steps: the shift, the plane rotations chased upward, the
// deflation when a rotation's radius vanishes.
void sym_eig(int n, const double *A, double *w, double *Q) {
  if (n <= 0) return;
  std::vector<double> a(A, A + (size_t)n * n);
  std::vector<double> z((size_t)n * n, 0.0);  // accumulated orthogonal basis, row-major
  for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
  auto at = [&](int i, int j) -> double & { return a[(size_t)i * n + j]; };
  auto zt = [&](int i, int j) -> double & { return z[(size_t)i * n + j]; };
  std::vector<double> v(n), pv(n);
  // Householder: zero column k below the subdiagonal, k = 0 .. n-3
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += at(i, k) * at(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    const double x0 = at(k + 1, k);
    const double beta = x0 >= 0.0 ? -alpha : alpha;  // new subdiagonal entry
    // v = x - beta e1 (on indices k+1..n-1), tau = 2 / (v^T v)
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) {
      v[i] = at(i, k) - (i == k + 1 ? beta : 0.0);
      vv += v[i] * v[i];
    }
    if (vv == 0.0) continue;
    const double tau = 2.0 / vv;
    // p = tau A v (trailing block), K = tau/2 v^T p, q = p - K v
    for (int i = k + 1; i < n; ++i) {
      double sacc = 0.0;
      for (int j = k + 1; j < n; ++j) sacc += at(i, j) * v[j];
      pv[i] = tau * sacc;
    }
    double vp = 0.0;
    for (int i = k + 1; i < n; ++i) vp += v[i] * pv[i];
    const double K = 0.5 * tau * vp;
    for (int i = k + 1; i < n; ++i) pv[i] -= K * v[i];
    // A <- A - v q^T - q v^T on the trailing block; column / row k
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) at(i, j) -= v[i] * pv[j] + pv[i] * v[j];
    at(k + 1, k) = at(k, k + 1) = beta;
    for (int i = k + 2; i < n; ++i) at(i, k) = at(k, i) = 0.0;
    // Z <- Z (I - tau v v^T)
    for (int r = 0; r < n; ++r) {
      double sacc = 0.0;
      for (int j = k + 1; j < n; ++j) sacc += zt(r, j) * v[j];
      sacc *= tau;
      for (int j = k + 1; j < n; ++j) zt(r, j) -= sacc * v[j];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = at(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = at(i + 1, i);
  // implicit QL with Wilkinson shifts; e[i] couples d[i] and d[i+1]
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 60; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      // shift from the trailing 2x2 block of the unreduced part starting at l
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      for (; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // deflation inside the sweep
          d[i + 1] -= p;
          e[m] = 0.0;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {  // rotate basis columns i, i+1
          f = zt(k, i + 1);
          zt(k, i + 1) = s * zt(k, i) + c * f;
          zt(k, i) = c * zt(k, i) - s * f;
        }
      }
      if (r == 0.0 && i >= l) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int c = 0; c < n; ++c) {
    w[c] = d[idx[c]];
    for (int k = 0; k < n; ++k) Q[(size_t)k * n + c] = z[(size_t)k * n + idx[c]];
  }
}

}  // namespace hl
