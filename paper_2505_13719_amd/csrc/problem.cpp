// Host preprocessing of an HSLR problem (Section 3.2) into the structures the
// kernels stream: the union support S and index lists L_ij (Section 4.1,
// eqs. def: support S ell and index list), the symmetric pattern S u S^T of
// the adjoint (Algorithm 4), and the tile schedule.
#include <algorithm>
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
  for (int i = 0; i < n; ++i) hp.rowptr_u[i + 1] += hp.rowptr_u[i];
  hp.direct = direct;
  hp.has_c = has_c;
  hp.nentries = nent;
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
  // low-rank part (objective only)
  if (p->n_lowrank < 0) return "n_lowrank < 0";
  if (p->n_lowrank > 1) {
    *code = HALLAR_E_UNSUPPORTED;
    return "at most one low-rank term is supported";
  }
  if (p->n_lowrank == 1) {
    if (!p->lr_con || !p->lr_rank || !p->K || !p->D) return "low-rank arrays are NULL";
    if (p->lr_con[0] < 0 || p->lr_con[0] > m) return "lr_con out of range";
    if (p->lr_con[0] != 0) {
      *code = HALLAR_E_UNSUPPORTED;
      return "low-rank terms on constraints are not supported";
    }
    const int r0 = p->lr_rank[0];
    if (r0 < 1 || r0 > LR_MAX) {
      *code = HALLAR_E_UNSUPPORTED;
      return "low-rank objective rank must be 1 or 2";
    }
    const int64_t ko = p->K_off ? p->K_off[0] : 0, dof = p->D_off ? p->D_off[0] : 0;
    hp.r0 = r0;
    hp.K0.assign(p->K + ko, p->K + ko + (int64_t)n * r0);
    hp.D0.assign(p->D + dof, p->D + dof + r0 * r0);
    for (double v : hp.K0)
      if (!std::isfinite(v)) {
        *code = HALLAR_E_NUMERICAL;
        return "K has NaN/Inf";
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
// TILE_MAX_ENTRIES entries of S u S^T (a row longer than that is a tile of its
// own), aiming at about kMaxTiles tiles per large instance (8 workgroups per
// CU) and at least kMinRows rows per tile for small ones.  Per tile, the
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
  constexpr int32_t kMinRows = 16;
  const int32_t n = hp.n;
  const int32_t row_target =
      std::min<int32_t>(TILE_MAX_ROWS, std::max<int32_t>(kMinRows, (int32_t)((n + kMaxTiles - 1) / kMaxTiles)));
  hp.tiles.clear();
  int32_t r0 = 0;
  while (r0 < n) {
    int64_t ent = 0;
    int32_t r1 = r0;
    while (r1 < n && (r1 - r0) < row_target) {
      const int64_t e = (hp.rowptr_u[r1 + 1] - hp.rowptr_u[r1]) + (hp.rowptr_l[r1 + 1] - hp.rowptr_l[r1]);
      if (r1 > r0 && ent + e > TILE_MAX_ENTRIES) break;
      ent += e;
      ++r1;
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

// cyclic Jacobi eigen solver for small symmetric matrices
void sym_eig(int n, const double *A, double *w, double *Q) {
  std::vector<double> a(A, A + (size_t)n * n);
  std::vector<double> v((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - s * akq;
          a[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - s * aqk;
          a[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = c * vkp - s * vkq;
          v[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a[(size_t)x * n + x] < a[(size_t)y * n + y]; });
  for (int c = 0; c < n; ++c) {
    w[c] = a[(size_t)idx[c] * n + idx[c]];
    for (int k = 0; k < n; ++k) Q[(size_t)k * n + c] = v[(size_t)k * n + idx[c]];
  }
}

}  // namespace hl
