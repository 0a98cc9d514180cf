// Host-side checker of the problem preprocessing, built with the host
// address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py
// (test infrastructure: not part of the library).  For each problem file
// given on the command line it runs build_host_problem and build_tiles and
// prints one line: status npairs nlower nentries direct ntiles rk nlc cdp_L.
// It also runs sym_eig on a small symmetric matrix and checks Q^T A Q.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../paper_2505_13719_amd/csrc/host.h"

template <typename T>
static bool rd(std::FILE *f, std::vector<T> &v, int64_t n) {
  v.resize((size_t)n);
  return n == 0 || std::fread(v.data(), sizeof(T), (size_t)n, f) == (size_t)n;
}
template <typename T>
static bool rd1(std::FILE *f, T &x) {
  return std::fread(&x, sizeof(T), 1, f) == 1;
}

static int check_file(const char *path) {
  std::FILE *f = std::fopen(path, "rb");
  if (!f) return 2;
  int64_t n = 0, m = 0, nnz = 0, nK = 0, nD = 0, nmask = 0;
  double tau2 = 0;
  int32_t nl = 0, L = 0;
  std::vector<int32_t> row, col, con, lr_con, lr_rank;
  std::vector<int64_t> K_off, D_off;
  std::vector<double> val, b, K, D, masks;
  bool ok = rd1(f, n) && rd1(f, m) && rd1(f, tau2) && rd1(f, nnz) && rd(f, row, nnz) && rd(f, col, nnz) &&
            rd(f, con, nnz) && rd(f, val, nnz) && rd(f, b, m) && rd1(f, nl) && rd(f, lr_con, nl) &&
            rd(f, lr_rank, nl) && rd(f, K_off, nl) && rd(f, D_off, nl) && rd1(f, nK) && rd1(f, nD) && rd(f, K, nK) &&
            rd(f, D, nD) && rd1(f, L) && rd1(f, nmask) && rd(f, masks, nmask);
  std::fclose(f);
  if (!ok) return 3;
  hallar_problem p{};
  p.n = n;
  p.m = m;
  p.trace_bound = tau2;
  p.nnz = nnz;
  p.row = row.data();
  p.col = col.data();
  p.con = con.data();
  p.val = val.data();
  p.b = b.data();
  p.n_lowrank = nl;
  p.lr_con = lr_con.data();
  p.lr_rank = lr_rank.data();
  p.K_off = K_off.data();
  p.D_off = D_off.data();
  p.K = K.data();
  p.D = D.data();
  p.cdp_patterns = L;
  p.cdp_masks = masks.data();
  hl::HostProblem hp;
  hallar_status code = HALLAR_OK;
  const std::string err = hl::build_host_problem(&p, hp, &code);
  if (code == HALLAR_OK) hl::build_tiles(hp);
  std::printf("%d %lld %lld %lld %d %zu %d %d %d\n", (int)code, (long long)hp.npairs, (long long)hp.nlower,
              (long long)hp.nentries, hp.direct ? 1 : 0, hp.tiles.size(), hp.rk, hp.nlc, hp.cdp_L);
  return 0;
}

static int check_eig() {
  const int n = 6;
  std::vector<double> A(n * n), w(n), Q(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) A[i * n + j] = A[j * n + i] = std::sin(1.0 + i * 7 + j * 3);
  hl::sym_eig(n, A.data(), w.data(), Q.data());
  double off = 0, scale = 0;
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < n; ++c) {
      double s = 0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) s += Q[i * n + a] * A[i * n + j] * Q[j * n + c];
      if (a == c) scale = std::fmax(scale, std::fabs(s - w[a]));
      else off = std::fmax(off, std::fabs(s));
    }
  std::printf("eig %.3e %.3e\n", off, scale);
  return off < 1e-10 && scale < 1e-10 ? 0 : 4;
}

int main(int argc, char **argv) {
  int rc = check_eig();
  for (int k = 1; k < argc && rc == 0; ++k) rc = check_file(argv[k]);
  return rc;
}
