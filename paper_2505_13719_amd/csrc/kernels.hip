// HIP kernels of the HALLaR hot path for gfx950 (CDNA4, wave64).
//
// Data layout (per instance, see internal.h):
//   U-like buffers: n x R row-major, R in {2,4,...,64} zero padded, so one
//   row is G = R*sizeof(T)/16 aligned 16-byte chunks.  A "group" of G lanes
//   holds one row; a "team" of G << plog lanes works on one output row with
//   (1 << plog) pair streams.
//   Sparse structure: the union support S of the upper-triangle entries
//   (Section 4.1, eq. def: support S ell) as a row CSR (pair k = position),
//   and the strictly-lower transpose with pair ids for the symmetric SpMM
//   (Algorithm 4 uses the pattern S u S^T).
// Everything here is memory bound: no MFMA (no dense contraction).
#include <mutex>

#include "internal.h"

namespace hl {

template <typename T> struct NCh;
template <> struct NCh<float> { static constexpr int N = 4; };
template <> struct NCh<double> { static constexpr int N = 2; };

template <typename T>
struct alignas(16) Chunk {
  T v[NCh<T>::N];
};

// 16-byte chunk loads and stores through global-address-space pointers
// (global_load / global_store instead of the generic flat forms the
// compiler emits for pointers read from memory: no coupling with the LDS
// wait counter, scalar base + vector offset; measured 3% faster on the
// FP64 matrix-completion trial kernels).  Every chunk pointer addresses
// device global memory (factor buffers, or the caller's U and W).
#define HL_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ Chunk<T> ldc(const T *p) {
  typedef T vec __attribute__((ext_vector_type(NCh<T>::N)));
  const vec v = *(const HL_GLOBAL vec *)(p);
  Chunk<T> c;
#pragma unroll
  for (int e = 0; e < NCh<T>::N; ++e) c.v[e] = v[e];
  return c;
}
template <typename T>
__device__ __forceinline__ void stc(T *p, const Chunk<T> &c) {
  typedef T vec __attribute__((ext_vector_type(NCh<T>::N)));
  vec v;
#pragma unroll
  for (int e = 0; e < NCh<T>::N; ++e) v[e] = c.v[e];
  *(HL_GLOBAL vec *)(p) = v;
}

// Streamed operands (index lists, {p_l, b_l} pairs) of the trial kernels,
// loaded through global-address-space pointers as the chunks are.  (A
// non-temporal hint on them was measured slower: the next kernel of the
// trial reads the same arrays, and keeps finding them in the caches.)
typedef double dbl2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldg(const double2 *p) {
  const dbl2v v = *(const HL_GLOBAL dbl2v *)(p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ int32_t ldg(const int32_t *p) { return *(const HL_GLOBAL int32_t *)(p); }

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int m) {
  return __shfl_xor(v, m, 64);
}

// sum over aligned groups of W lanes
template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = W / 2; o >= 1; o >>= 1) v += shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

// <U_i, U_j> of one pair over one 16-byte chunk of each row: FP64 fused
// multiply-adds from zero.  A pair's product is the per-chunk partials
// combined in the xor-butterfly order of group_sum (chunk 0 alone for one
// chunk, d0 + d1 for two), whether one thread holds both chunks (the narrow
// SDDMM) or one lane per chunk does (the wide SDDMM and the SpMM), so every
// kernel that forms a pair value gets the same bits.
template <typename T>
__device__ __forceinline__ double chunk_dot(const Chunk<T> &a, const Chunk<T> &b) {
  double d = 0.0;
#pragma unroll
  for (int e = 0; e < NCh<T>::N; ++e) d = fma((double)a.v[e], (double)b.v[e], d);
  return d;
}

// Augmented-Lagrangian terms of one constrained pair (Section 2, eq. AL function: the
// multiplier estimate inside the gradient of the augmented Lagrangian):
// t = (2 - delta_ij) a B, r = t - b_l, y' = p_l + beta r and the pair value
// m = c + a y'.  Contraction is off and the fused steps are explicit, so the
// SDDMM and the SpMM's recomputed lower half round alike.
struct PairAL {
  double t, r, y, m;
};
__device__ __forceinline__ PairAL pair_al(double cv, double av, double bl, double pl, double beta, double B,
                                          double w2) {
#pragma clang fp contract(off)
  PairAL o;
  o.t = w2 * av * B;
  o.r = o.t - bl;
  o.y = fma(beta, o.r, pl);
  o.m = fma(av, o.y, cv);
  return o;
}

// Block reduction of NQ doubles per thread into partial row `row` of the
// instance (slot q at part[q * prows + row]).
template <int NQ, int BASE = 0>
__device__ __forceinline__ void block_partials(double (&acc)[NQ], const InstDev &I, int row) {
  __shared__ double red[BLOCK / 64][NQ > 0 ? NQ : 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = wave_sum(acc[q]);
    if (lane == 0) red[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) s += red[w][threadIdx.x];
    I.part[(size_t)(BASE + threadIdx.x) * I.prows + row] = s;
  }
}

// Buffer of a role: one of the instance's n x R_cap work buffers, or (index
// NBUF + k) the caller's buffer P.ext[k] that the standalone operator calls
// read or write in place when its layout is the bucket's (ld = R).
template <typename T>
__device__ __forceinline__ T *role_ptr(const InstDev &I, const InstParams &P, int role) {
  const int b = P.buf[role];
  return reinterpret_cast<T *>(b < NBUF ? I.buf[b] : P.ext[b - NBUF]);
}


// Tile of this workgroup.  The hardware deals workgroups to the 8 XCDs in
// turn (workgroup b to XCD b mod 8).  Tiles are grouped in chunks of 16
// consecutive tiles and XCD x takes chunks x, x + 8, x + 16, ...: neighbouring
// rows gathered by the sparse kernels stay in one XCD's L2 within a chunk,
// while every XCD gets chunks from the whole row range, so work stays
// balanced when it is concentrated in part of the rows (a bipartite pattern
// keeps all upper pairs in its first block).  Bijective: full groups of
// 8 x 16 tiles are permuted, the remainder maps to itself.
__device__ __forceinline__ int tile_index() {
  constexpr int C = 16;
  const int nb = gridDim.x, b = blockIdx.x;
  const int main = nb - nb % (8 * C);
  if (b >= main) return b;
  const int x = b & 7, k = b >> 3;
  return (x + 8 * (k / C)) * C + k % C;
}

// ---------------------------------------------------------------------------
// SDDMM: T_l = A_l . XX^T over the pairs of S (Algorithm 2, eq. omega:
// weight (2 - delta_ij) A_ij), T_0 = C . XX^T with the low-rank part
// Tr(D (K^T X)(K^T X)^T) (Algorithm 3), fused with the augmented-Lagrangian
// epilogue: r_l = T_l - b_l, y'_l = p_l + beta r_l, partial sums of T_0,
// p^T r, ||r||^2 and K^T X, and the pair values m_k = C_ij + sum_l y'_l (A_l)_ij
// of the matrix M = C + A*(y') that the following SpMM multiplies (Alg. 4).
// ---------------------------------------------------------------------------
struct SddmmArgs {
  int32_t xrole;     // input factor
  int32_t msel;      // 0: m_xt, 1: m_yp, -1: no pair values
  int32_t write_T;   // store T_l (l >= 1) in TY
  int32_t write_yp;  // store y'_l in yp
  double *tout;      // non-null (one instance only): T_l goes to tout[l - 1] instead of TY
};

// Narrow rows (at most two 16-byte chunks): one thread per pair holds both
// rows, all of a pair's loads are independent, no LDS round trip beyond the
// tile's row pointers (s_rp); two pairs per thread in flight.
template <typename T, int G>
__device__ __forceinline__ void sddmm_narrow_pairs(const Tile &tl, const InstDev &I, const InstParams &P,
                                                   const SddmmArgs &a, const T *__restrict__ X,
                                                   const int32_t *s_rp, int nrows, T *mout, double (&acc)[4]) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  constexpr int UP = 2;
  const T *__restrict__ cu = reinterpret_cast<const T *>(I.c_u);
  const T *__restrict__ pa = reinterpret_cast<const T *>(I.pa);
  const double beta = P.beta;
  const int direct = I.direct;
  const int kbeg = s_rp[0], kend = s_rp[nrows];
  for (int kb = kbeg + threadIdx.x; kb < kend; kb += BLOCK * UP) {
    int kk[UP], ii[UP], jj[UP], l[UP];
    double cv[UP], av[UP], bl[UP], pl[UP];
    Chunk<T> ci[UP][G], cj[UP][G];
#pragma unroll
    for (int u = 0; u < UP; ++u) {
      const int k = kb + u * BLOCK;
      kk[u] = k;
      l[u] = 0;
      cv[u] = av[u] = bl[u] = pl[u] = 0.0;
      ii[u] = jj[u] = 0;
      if (k < kend) {
        int lo = 0, hi = nrows - 1;  // last row whose first pair is <= k
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_rp[mid] <= k) lo = mid;
          else hi = mid - 1;
        }
        ii[u] = tl.row0 + lo;
        jj[u] = ldg(I.col_u + k);
        if (I.c_diag_only) cv[u] = ii[u] == jj[u] ? I.c_diag[ii[u]] : 0.0;
        else cv[u] = cu ? (double)cu[k] : 0.0;
        if (direct) {
          // the constraint id where T_l / y'_l are stored or no rule tells
          // which pairs are constrained; else a flag (1: constrained)
          if (a.write_T || a.write_yp || I.con_rule == 0) l[u] = ldg(I.pcon + k);
          else l[u] = (I.con_rule == 1) != (ii[u] == jj[u]) ? 1 : 0;
          const double2 v = ldg(reinterpret_cast<const double2 *>(I.upb) + k);
          if (l[u] > 0) {
            av[u] = I.pa_uniform ? I.pa_const : (double)pa[k];
            bl[u] = v.y;
            pl[u] = v.x;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < G; ++c) {
        ci[u][c] = ldc(X + (size_t)ii[u] * R + c * NC);
        cj[u][c] = ldc(X + (size_t)jj[u] * R + c * NC);
      }
    }
#pragma unroll
    for (int u = 0; u < UP; ++u) {
      const int k = kk[u];
      if (k >= kend) continue;
      // FP64 accumulation of the FP32 / FP64 products
      double B = chunk_dot(ci[u][0], cj[u][0]);
      if constexpr (G == 2) B = B + chunk_dot(ci[u][1], cj[u][1]);
      const double w2 = ii[u] == jj[u] ? 1.0 : 2.0;
      acc[0] += w2 * cv[u] * B;
      if (direct) {
        double mv = cv[u];
        if (l[u] > 0) {
          const PairAL q = pair_al(cv[u], av[u], bl[u], pl[u], beta, B, w2);
          acc[1] += pl[u] * q.r;
          acc[2] += q.r * q.r;
          acc[3] += q.y * q.t;
          if (a.write_T) (a.tout ? a.tout : I.TY)[l[u] - 1] = q.t;
          if (a.write_yp) I.yp[l[u] - 1] = q.y;
          mv = q.m;
        }
        if (mout) mout[k] = (T)mv;
      } else {
        I.Bpair[k] = B;
      }
    }
  }
}

template <typename T, int G>
__device__ __forceinline__ void sddmm_narrow(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                             const SddmmArgs &a) {
  __shared__ int32_t s_rp[TILE_MAX_ROWS + 1];
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *__restrict__ X = role_ptr<T>(I, P, a.xrole);
  T *mout = a.msel == 0 ? reinterpret_cast<T *>(I.m_xt) : (a.msel == 1 ? reinterpret_cast<T *>(I.m_yp) : nullptr);
  const int nrows = tl.row1 - tl.row0;
  for (int r = threadIdx.x; r <= nrows; r += BLOCK) s_rp[r] = I.rowptr_u[tl.row0 + r];
  __syncthreads();
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  sddmm_narrow_pairs<T, G>(tl, I, P, a, X, s_rp, nrows, mout, acc);
  block_partials<4>(acc, I, tl.lt);
}

template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_sddmm(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                 SddmmArgs a) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  constexpr int NQ = 4;          // T0, p^T r, ||r||^2, sum y' T
  if constexpr (G <= 2) {
    sddmm_narrow<T, G>(tiles, insts, a);
    return;
  }
  constexpr int PPP = BLOCK / G;           // pairs per pass (one G-lane group per pair)
  constexpr int PPT = G >= 4 ? 1 : 4 / G;  // pairs per thread in phases A and C
  constexpr int BB = BLOCK * PPT;          // pairs per batch
  constexpr int NP = BB / PPP;             // passes per batch (= G * PPT)
  constexpr int UN = NP < 4 ? NP : 4;
  // The tile's pairs are taken in batches of BB: (A) one thread per pair
  // (PPT pairs each) loads its row (search in the tile's row pointers),
  // column and epilogue operands; (B) G-lane groups form the dot products,
  // UN pairs per group in flight; (C) one thread per pair applies the
  // epilogue.
  __shared__ int32_t s_rp[TILE_MAX_ROWS + 1];
  __shared__ int32_t s_i[BB], s_j[BB];
  __shared__ double s_d[BB];
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *__restrict__ X = role_ptr<T>(I, P, a.xrole);
  const T *__restrict__ cu = reinterpret_cast<const T *>(I.c_u);
  const T *__restrict__ pa = reinterpret_cast<const T *>(I.pa);
  T *mout = a.msel == 0 ? reinterpret_cast<T *>(I.m_xt) : (a.msel == 1 ? reinterpret_cast<T *>(I.m_yp) : nullptr);
  const double beta = P.beta;
  const int direct = I.direct;
  const int nrows = tl.row1 - tl.row0;
  for (int r = threadIdx.x; r <= nrows; r += BLOCK) s_rp[r] = I.rowptr_u[tl.row0 + r];
  __syncthreads();
  const int kbeg = s_rp[0], kend = s_rp[nrows];
  const int ch = threadIdx.x % G, grp = threadIdx.x / G;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;

  for (int kb = kbeg; kb < kend; kb += BB) {
    int l[PPT];
    double cv[PPT], av[PPT], bl[PPT], pl[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int pb = threadIdx.x + u * BLOCK, k = kb + pb;
      l[u] = 0;
      cv[u] = av[u] = bl[u] = pl[u] = 0.0;
      if (k < kend) {
        int lo = 0, hi = nrows - 1;  // last row whose first pair is <= k
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_rp[mid] <= k) lo = mid;
          else hi = mid - 1;
        }
        s_i[pb] = tl.row0 + lo;
        const int jc = I.col_u[k];
        s_j[pb] = jc;
        if (I.c_diag_only) cv[u] = tl.row0 + lo == jc ? I.c_diag[jc] : 0.0;
        else cv[u] = cu ? (double)cu[k] : 0.0;
        if (direct) {
          if (a.write_T || a.write_yp || I.con_rule == 0) l[u] = I.pcon[k];
          else l[u] = (I.con_rule == 1) != (tl.row0 + lo == jc) ? 1 : 0;
          const double2 v = reinterpret_cast<const double2 *>(I.upb)[k];
          if (l[u] > 0) {
            av[u] = I.pa_uniform ? I.pa_const : (double)pa[k];
            bl[u] = v.y;
            pl[u] = v.x;
          }
        }
      }
    }
    __syncthreads();
    const int nb = min(BB, kend - kb);
    for (int ps = 0; ps < NP; ps += UN) {
      Chunk<T> ci[UN], cj[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int pb = (ps + u) * PPP + grp;
        if (pb < nb) {
          ci[u] = ldc(X + (size_t)s_i[pb] * R + ch * NC);
          cj[u] = ldc(X + (size_t)s_j[pb] * R + ch * NC);
        } else {
#pragma unroll
          for (int e = 0; e < NC; ++e) ci[u].v[e] = cj[u].v[e] = T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        // products accumulate in FP64 (also for FP32 U): the AL value that the
        // FISTA / AIPP tests compare must be exact for the stored iterate
        double d = chunk_dot(ci[u], cj[u]);
        d = group_sum<G>(d);
        const int pb = (ps + u) * PPP + grp;
        if (ch == 0 && pb < nb) s_d[pb] = d;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int pb = threadIdx.x + u * BLOCK, k = kb + pb;
      if (k >= kend) continue;
      const double B = s_d[pb];
      const double w2 = (s_i[pb] == s_j[pb]) ? 1.0 : 2.0;
      acc[0] += w2 * cv[u] * B;
      if (direct) {
        double mv = cv[u];
        if (l[u] > 0) {
          const PairAL q = pair_al(cv[u], av[u], bl[u], pl[u], beta, B, w2);
          acc[1] += pl[u] * q.r;
          acc[2] += q.r * q.r;
          acc[3] += q.y * q.t;
          if (a.write_T) (a.tout ? a.tout : I.TY)[l[u] - 1] = q.t;
          if (a.write_yp) I.yp[l[u] - 1] = q.y;
          mv = q.m;
        }
        if (mout) mout[k] = (T)mv;
      } else {
        I.Bpair[k] = B;
      }
    }
    __syncthreads();  // s_i, s_j, s_d are rewritten by the next batch
  }
  block_partials<NQ>(acc, I, tl.lt);
}

// K^T X for the low-rank objective term (Algorithm 3: Y_0 = K_0^T U), written
// to partial slots 4.. of the tile (slots 0..3 belong to k_sddmm).
template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_lr_dots(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                   int32_t xrole) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  __shared__ double lds[(BLOCK / 64) * PSTRIDE];
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *__restrict__ X = role_ptr<T>(I, P, xrole);
  const T *__restrict__ K0 = reinterpret_cast<const T *>(I.K0);
  const int r0 = I.r0;
  if (r0 == 0) return;  // no low-rank term: nothing to read (uniform per block)
  // thread -> (row offset, chunk); each thread accumulates LR_MAX x NC values
  double acc[LR_MAX * NC];
#pragma unroll
  for (int q = 0; q < LR_MAX * NC; ++q) acc[q] = 0.0;
  const int ch = threadIdx.x % G;
  const int rstep = BLOCK / G;
  for (int i = tl.row0 + threadIdx.x / G; i < tl.row1; i += rstep) {
    const Chunk<T> u = ldc(X + (size_t)i * R + ch * NC);
    for (int t = 0; t < r0; ++t) {
      const double kv = (double)K0[(size_t)i * r0 + t];
#pragma unroll
      for (int e = 0; e < NC; ++e) acc[t * NC + e] += kv * (double)u.v[e];
    }
  }
  // reduce lanes with equal chunk index: lanes l and l xor (multiples of G)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < LR_MAX * NC; ++q) {
    double s = acc[q];
    for (int o = 32; o >= G; o >>= 1) s += shfl_xor(s, o);
    acc[q] = s;
  }
  // lanes 0..G-1 of each wave hold the per-chunk sums
  if (lane < G) {
#pragma unroll
    for (int q = 0; q < LR_MAX * NC; ++q) {
      const int t = q / NC, e = q - (q / NC) * NC;
      lds[wave * PSTRIDE + t * R + lane * NC + e] = acc[q];
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < r0 * R; q += BLOCK) {
    double s = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) s += lds[w * PSTRIDE + q];
    I.part[(size_t)(4 + q) * I.prows + tl.lt] = s;
  }
}

// ---------------------------------------------------------------------------
// General constraints (a constraint with several pairs or a pair in several
// constraints): phase B sums the weighted pair products per constraint and
// applies the AL epilogue; phase C forms the pair values.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_constraints(const int32_t *__restrict__ ilist, const InstDev *__restrict__ insts,
                                                           SddmmArgs a) {
  const InstDev &I = insts[ilist[blockIdx.y]];
  const InstParams &P = *I.prm;
  const int l = blockIdx.x * BLOCK + threadIdx.x;  // 0-based constraint
  double acc[3] = {0.0, 0.0, 0.0};
  if (l < I.m) {
    double t = 0.0;
    for (int e = I.cptr[l]; e < I.cptr[l + 1]; ++e) {
      const int id = I.cent[e];
      t += I.ew64[id] * I.Bpair[I.epair[id]];  // (2 - delta_ij) (A_l)_ij <U_i, U_j>
    }
    if (I.nlc > 0) {
      const int q = I.lc_of_con[l];
      if (q >= 0) t += I.lc_T[q];  // + K_l D_l K_l^T . U U^T (Algorithm 3)
    }
    if (I.cdp_L > 0) t += I.cdp_T[l];  // coded-diffraction constraint value
    const double r = t - I.b[l];
    const double y = I.p[l] + P.beta * r;
    acc[0] = I.p[l] * r;
    acc[1] = r * r;
    acc[2] = y * t;
    if (a.write_T) I.TY[l] = t;
    I.yp[l] = y;
  }
  if (blockIdx.x * BLOCK < I.m) block_partials<3>(acc, I, I.ntiles + blockIdx.x);
}

// pair values m_k = C_ij + sum_{l in L_ij} y_l (A_l)_ij (Algorithm 4)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_pairvals(const int32_t *__restrict__ ilist, const InstDev *__restrict__ insts,
                                                        int32_t msel, int32_t use_yp_ext, const double *__restrict__ yext) {
  const InstDev &I = insts[ilist[blockIdx.y]];
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= I.npairs) return;
  const double *y = use_yp_ext ? yext : I.yp;
  double mv = I.c64 ? I.c64[k] : 0.0;
  for (int e = I.eptr[k]; e < I.eptr[k + 1]; ++e) mv += y[I.econ[e] - 1] * I.ea64[e];
  if (msel == 2) {
    I.m64[k] = mv;
  } else {
    T *m = reinterpret_cast<T *>(msel == 0 ? I.m_xt : I.m_yp);
    m[k] = (T)mv;
  }
}

// Direct-mode pair values from an external or internal multiplier vector
// (used by the adjoint call and to build the FP64 Lanczos matrix).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_pairvals(const int32_t *__restrict__ ilist, const InstDev *__restrict__ insts,
                                                    int32_t msel, const double *__restrict__ yext) {
  const InstDev &I = insts[ilist[blockIdx.y]];
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= I.npairs) return;
  const double *y = yext ? yext : I.yp;
  double mv = I.c64 ? I.c64[k] : 0.0;
  const int l = I.pcon[k];
  if (l > 0) mv += I.pa64[k] * y[l - 1];
  if (msel == 2) {
    I.m64[k] = mv;
  } else {
    T *m = reinterpret_cast<T *>(msel == 0 ? I.m_xt : I.m_yp);
    m[k] = (T)mv;
  }
}

// ---------------------------------------------------------------------------
// SpMM: W = M X + K0 (D0 K0^T X) on the symmetric pattern S u S^T
// (Algorithms 4 and 5) with epilogues:
//   PLAIN: store W (role out).
//   TRIAL: GR = 2 lam W + X - W0 (grad of psi_s = lam g + 1/2||. - W0||^2,
//          eq. Grad U Space), Z = X - GR / L, partial ||Z||^2, ||GR||^2.
//   AIPP:  X = y+, GR = grad psi_s(x~): Rl = 2 lam W - GR + L (XT - X)
//          = V + W0 - y+ (V of ADAP-FISTA's output), partial ||Rl||^2,
//          <Rl, W0 - X>, <W, X> (= G . XX^T), ||GR||^2.
// ---------------------------------------------------------------------------
enum SpmmMode : int { SP_PLAIN = 0, SP_TRIAL = 1, SP_AIPP = 2 };

struct SpmmArgs {
  int32_t xrole;
  int32_t msel;   // 0: m_xt, 1: m_yp
  int32_t zsel;   // low-rank product slot
  int32_t outrole;
};

// Stage a tile's entries of S u S^T into LDS: columns and pair values of the
// upper CSR (coalesced), then the lower transpose, whose values come from a
// lower-order copy (m_low, coalesced) or are gathered through the pair ids,
// unless the caller recomputes them (lower_vals false: columns only); SU
// entries per thread are loaded before any is stored, so the gathers of a
// thread are in flight together.
template <typename T>
__device__ __forceinline__ void stage_entries(const InstDev &I, const T *__restrict__ m, int ku0, int nu, int kl0,
                                              int nl, bool lower_vals, int32_t *s_col, T *s_m,
                                              const T *__restrict__ m_low = nullptr) {
  constexpr int SU = 8;
  for (int e0 = threadIdx.x; e0 < nu; e0 += BLOCK * SU) {
    int c[SU];
    T v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = e0 + u * BLOCK;
      if (e < nu) {
        c[u] = I.col_u[ku0 + e];
        v[u] = m[ku0 + e];
      }
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = e0 + u * BLOCK;
      if (e < nu) {
        s_col[e] = c[u];
        s_m[e] = v[u];
      }
    }
  }
  for (int e0 = threadIdx.x; e0 < nl; e0 += BLOCK * SU) {
    int c[SU], id[SU];
    T v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = e0 + u * BLOCK;
      if (e < nl) {
        c[u] = I.col_l[kl0 + e];
        if (lower_vals && !m_low) id[u] = I.pid_l[kl0 + e];
      }
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = e0 + u * BLOCK;
      v[u] = T(0);
      if (lower_vals && e < nl) v[u] = m_low ? m_low[kl0 + e] : m[id[u]];
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = e0 + u * BLOCK;
      if (e < nl) {
        s_col[nu + e] = c[u];
        s_m[nu + e] = v[u];
      }
    }
  }
  __syncthreads();
}

// operands of the row epilogue, loaded before the row's products so that
// their latency overlaps the gathers
template <typename T>
struct EpiIn {
  Chunk<T> x, a, b, c;
};

template <typename T, int G, int MODE>
__device__ __forceinline__ EpiIn<T> spmm_epi_load(const InstDev &I, const InstParams &P, const T *X, size_t off) {
  EpiIn<T> in;
  if (MODE == SP_TRIAL) {
    in.x = ldc(X + off);
    in.a = ldc(role_ptr<T>(I, P, RW0) + off);
  } else if (MODE == SP_AIPP) {
    in.x = ldc(X + off);
    in.a = ldc(role_ptr<T>(I, P, RGR) + off);
    in.b = ldc(role_ptr<T>(I, P, RXT) + off);
    in.c = ldc(role_ptr<T>(I, P, RW0) + off);
  }
  return in;
}

template <typename T, int G, int MODE, int NQ>
__device__ __forceinline__ void spmm_epi_apply(const InstDev &I, const InstParams &P, const SpmmArgs &a, int i, int ch,
                                               double (&w)[NCh<T>::N], const EpiIn<T> &in, double (&acc)[NQ]) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const int r0 = I.r0;
  const T *__restrict__ K0 = reinterpret_cast<const T *>(I.K0);
  const double *Z0 = I.Z0 + a.zsel * LR_MAX * R_MAX;
  for (int t = 0; t < r0; ++t) {
    const double kv = (double)K0[(size_t)i * r0 + t];
#pragma unroll
    for (int e = 0; e < NC; ++e) w[e] += kv * Z0[t * R_MAX + ch * NC + e];
  }
  if (I.rk > 0) {
    // constraints' low-rank parts: K_i . (blockdiag(y_l D_l) K^T X) (Algorithm 5), formed by k_lc_kz
    const double *__restrict__ Wc = I.lc_W[a.zsel] + (size_t)i * R + ch * NC;
#pragma unroll
    for (int e = 0; e < NC; ++e) w[e] += Wc[e];
  }
  if (I.cdp_L > 0) {
    // coded-diffraction constraints: their adjoint block, formed by the FFTs
    const double *__restrict__ Wc = I.cdp_W[a.zsel] + (size_t)i * R + ch * NC;
#pragma unroll
    for (int e = 0; e < NC; ++e) w[e] += Wc[e];
  }
  const size_t off = (size_t)i * R + ch * NC;
  if (MODE == SP_PLAIN) {
    Chunk<T> o;
#pragma unroll
    for (int e = 0; e < NC; ++e) o.v[e] = (T)w[e];
    stc(role_ptr<T>(I, P, a.outrole) + off, o);
  } else if (MODE == SP_TRIAL) {
    const double lam2 = 2.0 * P.lam, invL = P.invL;
    Chunk<T> gr, z;
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      const double g = lam2 * w[e] + ((double)in.x.v[e] - (double)in.a.v[e]);
      gr.v[e] = (T)g;
      z.v[e] = (T)((double)in.x.v[e] - g * invL);
      acc[0] += (double)z.v[e] * (double)z.v[e];
      acc[1] += (double)gr.v[e] * (double)gr.v[e];
    }
    stc(role_ptr<T>(I, P, RGR) + off, gr);
    stc(role_ptr<T>(I, P, RZ) + off, z);
  } else {
    const double lam2 = 2.0 * P.lam, Lc = P.L;
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      const double rl = lam2 * w[e] - (double)in.a.v[e] + Lc * ((double)in.b.v[e] - (double)in.x.v[e]);
      acc[0] += rl * rl;
      acc[1] += rl * ((double)in.c.v[e] - (double)in.x.v[e]);
      acc[2] += w[e] * (double)in.x.v[e];
      acc[3] += (double)in.a.v[e] * (double)in.a.v[e];
    }
  }
}

// Rows of a staged tile (columns and, unless recomputed, pair values of
// S u S^T in LDS): a team of G * S lanes per row walks the upper entries,
// then the lower ones, and applies the row epilogue.
template <typename T, int G, int MODE, int NQ>
__device__ __forceinline__ void spmm_staged_rows(const Tile &tl, const InstDev &I, const InstParams &P,
                                                 const SpmmArgs &a, const T *__restrict__ X, const int32_t *s_ru,
                                                 const int32_t *s_rl, const int32_t *s_col, const T *s_m, int nrows,
                                                 int ku0, int nu, int kl0, bool rec, double (&acc)[NQ]) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  constexpr int UN = 4;  // gathers in flight per lane (measured: 4 beats 8 on the torus and MC)
  const double beta = P.beta, a_low = I.pa_const;
  const double2 *__restrict__ low_pb = reinterpret_cast<const double2 *>(I.low_pb);
  // a team of G * S lanes per row: S pair streams (power of two) when the
  // tile has fewer rows than the block has G-lane groups (long rows); stream
  // s takes the row's entries s, s + S, s + 2S, ..., UN at a time, so the
  // streams of a team read consecutive entries together
  int S = 1;
  while (S * 2 * G <= 64 && nrows * S * 2 * G <= BLOCK) S *= 2;
  const int TS = G * S;
  const int team = threadIdx.x / TS, lt = threadIdx.x - team * TS;
  const int strm = lt / G, ch = lt - strm * G;
  const int nteams = BLOCK / TS;
  for (int rb = 0; rb < nrows; rb += nteams) {
    const int r = rb + team;
    if (r >= nrows) continue;
    const int i = tl.row0 + r;
    EpiIn<T> in;
    if (strm == 0) in = spmm_epi_load<T, G, MODE>(I, P, X, (size_t)i * R + ch * NC);
    const int a0 = s_ru[r] - ku0, cu = s_ru[r + 1] - s_ru[r];
    const int b0 = nu + s_rl[r] - kl0 - cu, cnt = cu + s_rl[r + 1] - s_rl[r];
    // own row (chunk ch) and the row's (p_l, b_l) for recomputed values
    Chunk<T> xo;
    if (rec && cnt > cu) xo = ldc(X + (size_t)i * R + ch * NC);
    const double2 *__restrict__ pbr = rec ? low_pb + (s_rl[r] - cu) : nullptr;
    // FP64 accumulation (also for FP32 data): near a stationary point the
    // row sum cancels, and the FISTA / AIPP tests need the gradient to
    // relative accuracy, not to the size of its terms
    double w[NC];
#pragma unroll
    for (int e = 0; e < NC; ++e) w[e] = 0.0;
    for (int q = strm; q < cnt; q += S * UN) {
      Chunk<T> x[UN];
      T mv[UN];
      double2 pb[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int idx = q + u * S;
        if (idx < cnt) {
          const int pos = idx < cu ? a0 + idx : b0 + idx;
          if (rec && idx >= cu) pb[u] = pbr[idx];
          else mv[u] = s_m[pos];
          x[u] = ldc(X + (size_t)s_col[pos] * R + ch * NC);
        } else {
          mv[u] = T(0);
#pragma unroll
          for (int e = 0; e < NC; ++e) x[u].v[e] = T(0);
        }
      }
      if (rec) {
        // lanes of a G-group share idx, so the butterfly stays inside
        // lanes that take this branch together
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int idx = q + u * S;
          if (idx >= cu && idx < cnt) {
            const double B = group_sum<G>(chunk_dot(x[u], xo));
            mv[u] = (T)pair_al(0.0, a_low, pb[u].y, pb[u].x, beta, B, 2.0).m;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int e = 0; e < NC; ++e) w[e] += (double)mv[u] * (double)x[u].v[e];
    }
    for (int o = TS / 2; o >= G; o >>= 1) {
#pragma unroll
      for (int e = 0; e < NC; ++e) w[e] += shfl_xor(w[e], o);
    }
    if (strm == 0) spmm_epi_apply<T, G, MODE, NQ>(I, P, a, i, ch, w, in, acc);
  }
}

template <typename T, int G, int MODE>
__global__ __launch_bounds__(BLOCK) void k_spmm(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                SpmmArgs a) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  constexpr int NQ = MODE == SP_AIPP ? 4 : (MODE == SP_TRIAL ? 2 : 1);
  __shared__ int32_t s_ru[TILE_MAX_ROWS + 1], s_rl[TILE_MAX_ROWS + 1];
  __shared__ int32_t s_col[TILE_MAX_ENTRIES];
  __shared__ T s_m[TILE_MAX_ENTRIES];
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *__restrict__ X = role_ptr<T>(I, P, a.xrole);
  const T *__restrict__ m = reinterpret_cast<const T *>(a.msel ? I.m_yp : I.m_xt);
  const int nrows = tl.row1 - tl.row0;
  for (int r = threadIdx.x; r <= nrows; r += BLOCK) {
    s_ru[r] = I.rowptr_u[tl.row0 + r];
    s_rl[r] = I.rowptr_l[tl.row0 + r];
  }
  __syncthreads();
  const int ku0 = s_ru[0], nu = s_ru[nrows] - ku0;
  const int kl0 = s_rl[0], nl = s_rl[nrows] - kl0;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;

  if (nu + nl <= TILE_MAX_ENTRIES) {
    // The gradient SpMMs follow an SDDMM on the same factor, dual iterate and
    // penalty.  Where every lower pair is a constrained pair with the shared
    // coefficient and no sparse objective entry, a lower entry's value is
    // recomputed from the two factor rows (the neighbour row is gathered for
    // the product anyway) and (p_l, b_l) read in lower order, with the
    // SDDMM's arithmetic: no gather of the SDDMM's values through the pair
    // ids, which would cost a cache line per 4- or 8-byte value.
    const bool rec = MODE != SP_PLAIN && I.low_mode != 0;
    // stage the tile's columns and pair values of S u S^T (upper part, then
    // the lower transpose through its pair ids) with coalesced loads
    stage_entries<T>(I, m, ku0, nu, kl0, nl, !rec, s_col, s_m);
    spmm_staged_rows<T, G, MODE, NQ>(tl, I, P, a, X, s_ru, s_rl, s_col, s_m, nrows, ku0, nu, kl0, rec, acc);
  } else {
    // a tile too long to stage (one row of very high degree): teams of
    // G << plog lanes, 2^plog pair streams per row, read from HBM
    constexpr int LOGG = G >= 32 ? 5 : G >= 16 ? 4 : G >= 8 ? 3 : G >= 4 ? 2 : G >= 2 ? 1 : 0;
    const int plog = min((int)tl.plog_s, 6 - LOGG);
    const int TS = G << plog;
    const int team = threadIdx.x / TS;
    const int lt = threadIdx.x - team * TS;
    const int strm = lt / G, ch = lt - (lt / G) * G;
    const int nteams = BLOCK / TS;
    for (int i = tl.row0 + team; i < tl.row1; i += nteams) {
      double w[NC];
#pragma unroll
      for (int e = 0; e < NC; ++e) w[e] = 0.0;
      const int k0 = I.rowptr_u[i], k1 = I.rowptr_u[i + 1];
      for (int k = k0 + strm; k < k1; k += (1 << plog)) {
        const double mv = (double)m[k];
        const Chunk<T> x = ldc(X + (size_t)I.col_u[k] * R + ch * NC);
#pragma unroll
        for (int e = 0; e < NC; ++e) w[e] += mv * (double)x.v[e];
      }
      const int e0 = I.rowptr_l[i], e1 = I.rowptr_l[i + 1];
      for (int e2 = e0 + strm; e2 < e1; e2 += (1 << plog)) {
        const double mv = (double)m[I.pid_l[e2]];
        const Chunk<T> x = ldc(X + (size_t)I.col_l[e2] * R + ch * NC);
#pragma unroll
        for (int e = 0; e < NC; ++e) w[e] += mv * (double)x.v[e];
      }
      for (int o = TS / 2; o >= G; o >>= 1) {
#pragma unroll
        for (int e = 0; e < NC; ++e) w[e] += shfl_xor(w[e], o);
      }
      if (strm == 0) {
        const EpiIn<T> in = spmm_epi_load<T, G, MODE>(I, P, X, (size_t)i * R + ch * NC);
        spmm_epi_apply<T, G, MODE, NQ>(I, P, a, i, ch, w, in, acc);
      }
    }
  }
  if (MODE != SP_PLAIN) block_partials<NQ>(acc, I, tl.lt);
}

// FISTA trial point (Appendix A.1, ADAP-FISTA): the SDDMM at XT and the
// gradient SpMM at XT in one pass, for direct instances whose lower half is
// recomputed, with no low-rank objective term and narrow rows (G <= 2).  The
// row walk of the SpMM recomputes every entry's value from the two factor
// rows -- the neighbour row is gathered once for the product and for the
// accumulation -- and {p_l, b_l} in pair order (upper entries) or lower order
// (lower entries), and the upper entries, which are the pairs of the tile's
// own rows, also feed the SDDMM's partial sums (slots 0..3).  Per pair that
// is one gather of a factor row instead of three (SDDMM, SpMM upper and
// lower), and no pair values written or read.  The pair values and the
// SpMM's sums are bit-identical to the separate kernels'; the SDDMM's partial
// sums are formed in walk order instead of pair order.
// LATE: the epilogue operands are loaded after the row's walk (fewer live
// registers during the walk).
template <typename T, int G, bool LATE>
__device__ __forceinline__ void trial_fused_body(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                 int32_t xrole) {
  static_assert(G <= 2, "the fused trial kernel takes narrow rows");
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  // entries per step and lane: two for one-chunk rows, one for two-chunk
  // rows, with the next step's index loads issued before this step's rows
  // are gathered (software pipeline).  Measured on matrix completion rank 4:
  // FP64 340 -> 300 us and FP32 252 -> 217 us against the unpipelined walk
  // with two / four entries in flight; the pipelined walk with twice the
  // entries per step is slower (302 / 224 us: registers), with four
  // slower still (329 us FP64)
  constexpr int UN = G == 1 ? 2 : 1;
  __shared__ int32_t s_ru[TILE_MAX_ROWS + 1], s_rl[TILE_MAX_ROWS + 1];
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *__restrict__ X = role_ptr<T>(I, P, xrole);
  const int nrows = tl.row1 - tl.row0;
  for (int r = threadIdx.x; r <= nrows; r += BLOCK) {
    s_ru[r] = I.rowptr_u[tl.row0 + r];
    s_rl[r] = I.rowptr_l[tl.row0 + r];
  }
  __syncthreads();
  const double beta = P.beta, a_low = I.pa_const;
  const T *__restrict__ cuv = reinterpret_cast<const T *>(I.c_u);
  const T *__restrict__ pav = reinterpret_cast<const T *>(I.pa);
  const double2 *__restrict__ upb = reinterpret_cast<const double2 *>(I.upb);
  const double2 *__restrict__ low_pb = reinterpret_cast<const double2 *>(I.low_pb);
  const SpmmArgs sa{xrole, 0, 0, 0};
  // teams as in the staged SpMM: G * S lanes per row
  int S = 1;
  while (S * 2 * G <= 64 && nrows * S * 2 * G <= BLOCK) S *= 2;
  const int TS = G * S;
  const int team = threadIdx.x / TS, lt = threadIdx.x - team * TS;
  const int strm = lt / G, ch = lt - strm * G;
  const int nteams = BLOCK / TS;
  double acc4[4] = {0.0, 0.0, 0.0, 0.0};  // T0, p^T r, ||r||^2, sum y' T
  double acc2[2] = {0.0, 0.0};            // ||Z||^2, ||GR||^2
  for (int rb = 0; rb < nrows; rb += nteams) {
    const int r = rb + team;
    if (r >= nrows) continue;
    const int i = tl.row0 + r;
    EpiIn<T> in;
    if (!LATE && strm == 0) in = spmm_epi_load<T, G, SP_TRIAL>(I, P, X, (size_t)i * R + ch * NC);
    const int ku = s_ru[r], cu = s_ru[r + 1] - ku;
    const int kl = s_rl[r], cnt = cu + s_rl[r + 1] - kl;
    const Chunk<T> xo = ldc(X + (size_t)i * R + ch * NC);
    double w[NC];
#pragma unroll
    for (int e = 0; e < NC; ++e) w[e] = 0.0;
    // software pipeline: the next step's columns and {p_l, b_l} are loaded
    // while this step's factor rows are gathered
    double2 pb[UN], pbn[UN];
    int col[UN], lk[UN], coln[UN], lkn[UN];
    auto idx_load = [&](int q0, int (&cl)[UN], double2 (&pv)[UN], int (&lv)[UN]) {
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int idx = q0 + u * S;
        lv[u] = 0;
        cl[u] = i;
        if (idx < cnt) {
          if (idx < cu) {
            const int k = ku + idx;
            cl[u] = ldg(I.col_u + k);
            if (!I.con_rule) lv[u] = ldg(I.pcon + k);
            pv[u] = ldg(upb + k);
          } else {
            const int e = kl + idx - cu;
            cl[u] = ldg(I.col_l + e);
            pv[u] = ldg(low_pb + e);
          }
        }
      }
    };
    idx_load(strm, col, pb, lk);
    for (int q = strm; q < cnt; q += S * UN) {
      Chunk<T> x[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u)
        if (q + u * S < cnt) x[u] = ldc(X + (size_t)col[u] * R + ch * NC);
      if (q + S * UN < cnt) idx_load(q + S * UN, coln, pbn, lkn);
      // lanes of a G-group share idx: the butterfly stays inside lanes that
      // take the branch together, and one lane of the group adds the SDDMM
      // sums
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int idx = q + u * S;
        if (idx >= cnt) continue;
        const double B = group_sum<G>(chunk_dot(x[u], xo));
        double mv;
        if (idx < cu) {
          const int k = ku + idx;
          const bool dg = col[u] == i;
          const double w2 = dg ? 1.0 : 2.0;
          const double cv = I.c_diag_only ? (dg ? I.c_diag[i] : 0.0) : (cuv ? (double)cuv[k] : 0.0);
          if (ch == 0) acc4[0] += w2 * cv * B;
          mv = cv;
          if (I.con_rule ? (I.con_rule == 1) != dg : lk[u] > 0) {
            const double av = I.pa_uniform ? I.pa_const : (double)pav[k];
            const PairAL qv = pair_al(cv, av, pb[u].y, pb[u].x, beta, B, w2);
            if (ch == 0) {
              acc4[1] += pb[u].x * qv.r;
              acc4[2] += qv.r * qv.r;
              acc4[3] += qv.y * qv.t;
            }
            mv = qv.m;
          }
        } else {
          mv = pair_al(0.0, a_low, pb[u].y, pb[u].x, beta, B, 2.0).m;
        }
        const double mt = (double)(T)mv;
#pragma unroll
        for (int e = 0; e < NC; ++e) w[e] += mt * (double)x[u].v[e];
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        col[u] = coln[u];
        lk[u] = lkn[u];
        pb[u] = pbn[u];
      }
    }
    for (int o = TS / 2; o >= G; o >>= 1) {
#pragma unroll
      for (int e = 0; e < NC; ++e) w[e] += shfl_xor(w[e], o);
    }
    if (strm == 0) {
      if (LATE) in = spmm_epi_load<T, G, SP_TRIAL>(I, P, X, (size_t)i * R + ch * NC);
      spmm_epi_apply<T, G, SP_TRIAL, 2>(I, P, sa, i, ch, w, in, acc2);
    }
  }
  block_partials<4>(acc4, I, tl.lt);
  block_partials<2, FUSE_SLOT>(acc2, I, tl.lt);
}

template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_trial_fused(const Tile *__restrict__ tiles,
                                                       const InstDev *__restrict__ insts, int32_t xrole) {
  trial_fused_body<T, G, false>(tiles, insts, xrole);
}
// FP64 rank-4 rows (the matrix-completion headline): capped at 80 VGPRs for
// six waves per SIMD, with the epilogue loaded late so that nothing spills
// (measured 300 -> 286 us per launch; the same cap spills in the other
// instantiations)
template <>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_trial_fused<double, 2>(
    const Tile *__restrict__ tiles, const InstDev *__restrict__ insts, int32_t xrole) {
  trial_fused_body<double, 2, true>(tiles, insts, xrole);
}

// ---------------------------------------------------------------------------
// Vector kernels over the rows of a tile (G chunks per row).
// ---------------------------------------------------------------------------
// The trial's two vector kernels stream a few bytes per row.  For tiles of
// few chunks (the short tiles of long rows) a workgroup takes VT tiles at
// once, VL lanes each (strided over the tile's chunks), and each tile's
// partial sums are formed by a butterfly inside its VL lanes -- no LDS, no
// barrier, and VT times fewer workgroups than tiles; tiles of many chunks
// take one workgroup each (k_combo_tile, k_proj_tile below).
constexpr int VT = 16;
constexpr int VL = BLOCK / VT;
static_assert(VL <= 64 && (VL & (VL - 1)) == 0, "a tile's lanes sit inside one wave");

// FISTA extrapolation: optionally X <- u1 Y + u2 X + u3 XT (x_{i+1} of the
// previous accepted trial, Y = y_{i+1}, s = (L - mu)(x~ - y+) folded in), then
// XT = cY Y + cX X; partial ||XT - W0||^2.
template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_combo(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                 int nt) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const int tix = blockIdx.x * VT + threadIdx.x / VL, sl = threadIdx.x % VL;
  if (tix >= nt) return;  // whole VL-lane groups leave together
  const Tile tl = tiles[tix];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *Xp = role_ptr<T>(I, P, RX);
  T *XNp = role_ptr<T>(I, P, RU2);  // updated x (a different buffer than RX)
  const T *Yp = role_ptr<T>(I, P, RY);
  T *XTp = role_ptr<T>(I, P, RXT);
  const T *W0p = role_ptr<T>(I, P, RW0);
  const T cY = (T)P.cY, cX = (T)P.cX, u1 = (T)P.u1, u2 = (T)P.u2, u3 = (T)P.u3;
  const int upd = P.upd_x;
  double acc = 0.0;
  const int total = (tl.row1 - tl.row0) * G;
  const size_t base = (size_t)tl.row0 * R;
  for (int t = sl; t < total; t += VL) {
    const size_t off = base + (size_t)t * NC;
    Chunk<T> x = ldc(Xp + off);
    const Chunk<T> y = ldc(Yp + off), w0 = ldc(W0p + off);
    if (upd) {
      const Chunk<T> xt = ldc(XTp + off);
#pragma unroll
      for (int e = 0; e < NC; ++e) x.v[e] = u1 * y.v[e] + u2 * x.v[e] + u3 * xt.v[e];
      stc(XNp + off, x);
    }
    Chunk<T> o;
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      o.v[e] = cY * y.v[e] + cX * x.v[e];
      const double d = (double)o.v[e] - (double)w0.v[e];
      acc += d * d;
    }
    stc(XTp + off, o);
  }
  acc = group_sum<VL>(acc);
  if (sl == 0) I.part[(size_t)COMBO_SLOT * I.prows + tl.lt] = acc;
}

// y+ = c Z (projection onto the Frobenius ball, c from the reduce kernel),
// partials <GR, y+ - XT>, ||y+ - XT||^2, ||y+ - W0||^2.
template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_proj(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                int nt) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const int tix = blockIdx.x * VT + threadIdx.x / VL, sl = threadIdx.x % VL;
  if (tix >= nt) return;
  const Tile tl = tiles[tix];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  T *Zp = role_ptr<T>(I, P, RZ);
  const T *XTp = role_ptr<T>(I, P, RXT);
  const T *GRp = role_ptr<T>(I, P, RGR);
  const T *W0p = role_ptr<T>(I, P, RW0);
  const T c = (T)I.res->v[S_PROJC];
  double acc[3] = {0.0, 0.0, 0.0};
  const int total = (tl.row1 - tl.row0) * G;
  const size_t base = (size_t)tl.row0 * R;
  for (int t = sl; t < total; t += VL) {
    const size_t off = base + (size_t)t * NC;
    Chunk<T> z = ldc(Zp + off);
    const Chunk<T> xt = ldc(XTp + off), gr = ldc(GRp + off), w0 = ldc(W0p + off);
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      z.v[e] = c * z.v[e];
      const double d = (double)z.v[e] - (double)xt.v[e];
      const double f = (double)z.v[e] - (double)w0.v[e];
      acc[0] += (double)gr.v[e] * d;
      acc[1] += d * d;
      acc[2] += f * f;
    }
    stc(Zp + off, z);
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double v = group_sum<VL>(acc[q]);
    if (sl == 0) I.part[(size_t)(PROJ_SLOT + q) * I.prows + tl.lt] = v;
  }
}

// The same two steps with one workgroup per tile, for tiles of many chunks
// (long row ranges or wide rows), where sixteen lanes per tile would leave
// the chip short of loads in flight.
template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_combo_tile(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *Xp = role_ptr<T>(I, P, RX);
  T *XNp = role_ptr<T>(I, P, RU2);  // updated x (a different buffer than RX)
  const T *Yp = role_ptr<T>(I, P, RY);
  T *XTp = role_ptr<T>(I, P, RXT);
  const T *W0p = role_ptr<T>(I, P, RW0);
  const T cY = (T)P.cY, cX = (T)P.cX, u1 = (T)P.u1, u2 = (T)P.u2, u3 = (T)P.u3;
  const int upd = P.upd_x;
  double acc[1] = {0.0};
  const int total = (tl.row1 - tl.row0) * G;
  const size_t base = (size_t)tl.row0 * R;
  for (int t = threadIdx.x; t < total; t += BLOCK) {
    const size_t off = base + (size_t)t * NC;
    Chunk<T> x = ldc(Xp + off);
    const Chunk<T> y = ldc(Yp + off), w0 = ldc(W0p + off);
    if (upd) {
      const Chunk<T> xt = ldc(XTp + off);
#pragma unroll
      for (int e = 0; e < NC; ++e) x.v[e] = u1 * y.v[e] + u2 * x.v[e] + u3 * xt.v[e];
      stc(XNp + off, x);
    }
    Chunk<T> o;
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      o.v[e] = cY * y.v[e] + cX * x.v[e];
      const double d = (double)o.v[e] - (double)w0.v[e];
      acc[0] += d * d;
    }
    stc(XTp + off, o);
  }
  block_partials<1, COMBO_SLOT>(acc, I, tl.lt);
}

// y+ = c Z (projection onto the Frobenius ball, c from the reduce kernel),
// partials <GR, y+ - XT>, ||y+ - XT||^2, ||y+ - W0||^2.
template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_proj_tile(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  T *Zp = role_ptr<T>(I, P, RZ);
  const T *XTp = role_ptr<T>(I, P, RXT);
  const T *GRp = role_ptr<T>(I, P, RGR);
  const T *W0p = role_ptr<T>(I, P, RW0);
  const T c = (T)I.res->v[S_PROJC];
  double acc[3] = {0.0, 0.0, 0.0};
  const int total = (tl.row1 - tl.row0) * G;
  const size_t base = (size_t)tl.row0 * R;
  for (int t = threadIdx.x; t < total; t += BLOCK) {
    const size_t off = base + (size_t)t * NC;
    Chunk<T> z = ldc(Zp + off);
    const Chunk<T> xt = ldc(XTp + off), gr = ldc(GRp + off), w0 = ldc(W0p + off);
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      z.v[e] = c * z.v[e];
      const double d = (double)z.v[e] - (double)xt.v[e];
      const double f = (double)z.v[e] - (double)w0.v[e];
      acc[0] += (double)gr.v[e] * d;
      acc[1] += d * d;
      acc[2] += f * f;
    }
    stc(Zp + off, z);
  }
  block_partials<3, PROJ_SLOT>(acc, I, tl.lt);
}

// Copy role src -> role dst (scaled), optional partial ||dst||^2.
template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_copy_scale(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                      int32_t src, int32_t dst) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *S = role_ptr<T>(I, P, src);
  T *D = role_ptr<T>(I, P, dst);
  const T c = (T)P.lz_scale;
  double acc[1] = {0.0};
  const int total = (tl.row1 - tl.row0) * G;
  const size_t base = (size_t)tl.row0 * R;
  for (int t = threadIdx.x; t < total; t += BLOCK) {
    const size_t off = base + (size_t)t * NC;
    Chunk<T> x = ldc(S + off);
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      x.v[e] *= c;
      acc[0] += (double)x.v[e] * (double)x.v[e];
    }
    stc(D + off, x);
  }
  block_partials<1>(acc, I, tl.lt);
}

// Pack an external n x r (ld) FP64/op-type matrix into role dst (R columns,
// zero padded) and optionally scale; partial ||dst||^2.
template <typename T, int G, typename S>
__global__ __launch_bounds__(BLOCK) void k_pack(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                const S *__restrict__ src, int32_t r, int64_t ld, int32_t dst, double scale) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  T *D = role_ptr<T>(I, P, dst);
  double acc[1] = {0.0};
  const int total = (tl.row1 - tl.row0) * R;
  for (int t = threadIdx.x; t < total; t += BLOCK) {
    const int i = tl.row0 + t / R, c = t % R;
    const T v = c < r ? (T)(scale * (double)src[(size_t)i * ld + c]) : T(0);
    D[(size_t)i * R + c] = v;
    acc[0] += (double)v * (double)v;
  }
  block_partials<1>(acc, I, tl.lt);
}

template <typename T, int G, typename S>
__global__ __launch_bounds__(BLOCK) void k_unpack(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                  S *__restrict__ out, int32_t r, int64_t ld, int32_t src) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *Sx = role_ptr<T>(I, P, src);
  const int total = (tl.row1 - tl.row0) * r;
  for (int t = threadIdx.x; t < total; t += BLOCK) {
    const int i = tl.row0 + t / r, c = t % r;
    out[(size_t)i * ld + c] = (S)Sx[(size_t)i * R + c];
  }
}

// Frank-Wolfe update in U-space (eq. tilde Y Algo 2): dst[:, :r] = fw_a src,
// dst[:, fw_col] = fw_b v, zero padding up to the destination width RD.
template <typename T, int GS, int GD>
__global__ __launch_bounds__(BLOCK) void k_fw_apply(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                    int32_t src, int32_t dst) {
  constexpr int NC = NCh<T>::N;
  constexpr int RS = GS * NC, RD = GD * NC;
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *S = role_ptr<T>(I, P, src);
  T *D = role_ptr<T>(I, P, dst);
  const T fa = (T)P.fw_a;
  const double fb = P.fw_b;
  const int r = P.r, col = P.fw_col;
  const double *v = I.lzv;
  const int total = (tl.row1 - tl.row0) * RD;
  for (int t = threadIdx.x; t < total; t += BLOCK) {
    const int i = tl.row0 + t / RD, c = t % RD;
    T val = T(0);
    if (c == col) val = (T)(fb * v[i]);
    else if (c < r && c < RS && col != 0) val = fa * S[(size_t)i * RS + c];
    D[(size_t)i * RD + c] = val;
  }
}

// Gram partials X^T X (compression of U, R x R per tile).
template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_gram(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                int32_t src) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  constexpr int RB = 16;  // rows staged per step
  __shared__ double rows[RB][R];
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *S = role_ptr<T>(I, P, src);
  constexpr int PER = (R * R + BLOCK - 1) / BLOCK;
  double acc[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) acc[q] = 0.0;
  for (int i0 = tl.row0; i0 < tl.row1; i0 += RB) {
    const int nr = min(RB, tl.row1 - i0);
    for (int t = threadIdx.x; t < RB * R; t += BLOCK) {
      const int rr = t / R, c = t % R;
      rows[rr][c] = rr < nr ? (double)S[(size_t)(i0 + rr) * R + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + q * BLOCK;
      if (idx < R * R) {
        const int a = idx / R, b = idx % R;
        double s = 0.0;
        for (int rr = 0; rr < RB; ++rr) s += rows[rr][a] * rows[rr][b];
        acc[q] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = threadIdx.x + q * BLOCK;
    if (idx < R * R) I.gram[(size_t)idx * I.ntiles + tl.lt] = acc[q];
  }
}

// dst[:, :rnew] = src[:, :r] Q (Q: R_MAX stride, column c of the new basis).
template <typename T, int GS, int GD>
__global__ __launch_bounds__(BLOCK) void k_rotate(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                  int32_t src, int32_t dst) {
  constexpr int NC = NCh<T>::N;
  constexpr int RS = GS * NC, RD = GD * NC;
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const T *S = role_ptr<T>(I, P, src);
  T *D = role_ptr<T>(I, P, dst);
  const int r = P.r, rnew = P.rnew;
  const double *Q = I.up_base + P.up_off;
  const int total = (tl.row1 - tl.row0) * RD;
  for (int t = threadIdx.x; t < total; t += BLOCK) {
    const int i = tl.row0 + t / RD, c = t % RD;
    double s = 0.0;
    if (c < rnew)
      for (int a = 0; a < r; ++a) s += (double)S[(size_t)i * RS + a] * Q[a * R_MAX + c];
    D[(size_t)i * RD + c] = (T)s;
  }
}

// ---------------------------------------------------------------------------
// Frank-Wolfe step size: T(v v^T)_l for the constraints and the partial
// sum of (T(YY^T)_l - tau^2 T(vv^T)_l)^2 (denominator of eq. FW stepsize).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_fw_den(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts) {
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const double *v = I.lzv;
  const double tau2 = P.tau2;
  double acc[1] = {0.0};
  const int k0 = I.rowptr_u[tl.row0], k1 = I.rowptr_u[tl.row1];
  // pair -> row by a per-row walk: each thread takes pairs of rows
  for (int i = tl.row0 + threadIdx.x; i < tl.row1; i += BLOCK) {
    const double vi = v[i];
    for (int k = I.rowptr_u[i]; k < I.rowptr_u[i + 1]; ++k) {
      const int j = I.col_u[k];
      const double w2 = (i == j) ? 1.0 : 2.0;
      if (I.direct) {
        const int l = I.pcon[k];
        if (l > 0) {
          const double t = P.fw_v_on ? w2 * I.pa64[k] * vi * v[j] : 0.0;
          I.Ty[l - 1] = t;
          const double d = I.TY[l - 1] - tau2 * t;
          acc[0] += d * d;
        }
      } else {
        I.Bpair[k] = P.fw_v_on ? vi * v[j] : 0.0;
      }
    }
  }
  (void)k0; (void)k1;
  block_partials<1>(acc, I, tl.lt);
}

// general-mode denominator (per constraint)
__global__ __launch_bounds__(BLOCK) void k_fw_den_gen(const int32_t *__restrict__ ilist, const InstDev *__restrict__ insts) {
  const InstDev &I = insts[ilist[blockIdx.y]];
  const InstParams &P = *I.prm;
  const int l = blockIdx.x * BLOCK + threadIdx.x;
  double acc[1] = {0.0};
  if (l < I.m) {
    double t = 0.0;
    for (int e = I.cptr[l]; e < I.cptr[l + 1]; ++e) {
      const int id = I.cent[e];
      t += I.ew64[id] * I.Bpair[I.epair[id]];
    }
    if (I.nlc > 0) {
      const int q = I.lc_of_con[l];
      if (q >= 0) t += I.lc_Tv[q];
    }
    if (I.cdp_L > 0) t += I.cdp_Tv[l];
    I.Ty[l] = t;
    const double d = I.TY[l] - P.tau2 * t;
    acc[0] = d * d;
  }
  if (blockIdx.x * BLOCK < I.m) block_partials<1>(acc, I, I.ntiles + blockIdx.x);
}

// p <- y'(Y) and partial b^T p (dual value), ||T(Y) - b||^2 and p^T (T(Y) - b)
// with the new p (the objective accuracy estimate |pval - dval| + |p^T r|).
__global__ __launch_bounds__(BLOCK) void k_set_p(const int32_t *__restrict__ ilist, const InstDev *__restrict__ insts) {
  const InstDev &I = insts[ilist[blockIdx.y]];
  const int l = blockIdx.x * BLOCK + threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  if (l < I.m) {
    const double y = I.yp[l];
    I.p[l] = y;
    acc[0] = I.b[l] * y;
    const double r = I.TY[l] - I.b[l];
    acc[1] = r * r;
    acc[2] = y * r;
  }
  if (blockIdx.x * BLOCK < I.m) block_partials<3>(acc, I, I.ntiles + blockIdx.x);
}

// {p_l, b_l} per pair in pair order (direct mode, zeros for unconstrained
// pairs) for the SDDMM, and per strictly-lower pair in lower order for the
// gradient SpMM's recomputed lower half; rerun whenever p changes.
__global__ __launch_bounds__(BLOCK) void k_refresh_pb(const int32_t *__restrict__ ilist,
                                                      const InstDev *__restrict__ insts) {
  const InstDev &I = insts[ilist[blockIdx.y]];
  if (I.upb) {
    double2 *out = reinterpret_cast<double2 *>(I.upb);
    for (int k = blockIdx.x * BLOCK + threadIdx.x; k < I.npairs; k += gridDim.x * BLOCK) {
      const int l = I.pcon[k];
      out[k] = l > 0 ? make_double2(I.p[l - 1], I.b[l - 1]) : make_double2(0.0, 0.0);
    }
  }
  if (I.low_mode) {
    double2 *out = reinterpret_cast<double2 *>(I.low_pb);
    for (int e = blockIdx.x * BLOCK + threadIdx.x; e < I.nlower; e += gridDim.x * BLOCK) {
      const int l = I.pcon[I.pid_l[e]];  // >= 1: every lower pair is constrained in this mode
      out[e] = make_double2(I.p[l - 1], I.b[l - 1]);
    }
  }
}

// FP64 pair values of the strictly-lower pairs in lower order (the Lanczos
// matrix, fixed for a run).
__global__ __launch_bounds__(BLOCK) void k_lower_copy(const int32_t *__restrict__ ilist,
                                                      const InstDev *__restrict__ insts) {
  const InstDev &I = insts[ilist[blockIdx.y]];
  for (int e = blockIdx.x * BLOCK + threadIdx.x; e < I.nlower; e += gridDim.x * BLOCK) I.m64_low[e] = I.m64[I.pid_l[e]];
}

// ---------------------------------------------------------------------------
// Lanczos (FP64).  Basis rows V[q * n + i]; w is the work vector.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double *lz_basis(const InstDev &I, const InstParams &P) { return P.lz_basis ? I.V2 : I.V; }

// Partial dots <V_q, w> over the rows of a tile for q < nq, w given for the
// tile's rows in LDS: each wave takes groups of 8 basis vectors, lanes stride
// over rows; written to partial slots 0..nq-1 of the tile.
__device__ __forceinline__ void lz_tile_dots(const InstDev &I, const double *V, int nq, const Tile &tl,
                                             const double *s_w, double *lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t n = I.n;
  const int nrows = tl.row1 - tl.row0;
  constexpr int QB = 8;
  for (int q0 = wave * QB; q0 < nq; q0 += (BLOCK / 64) * QB) {
    double acc[QB];
#pragma unroll
    for (int u = 0; u < QB; ++u) acc[u] = 0.0;
    for (int r = lane; r < nrows; r += 64) {
      const double wi = s_w[r];
      const size_t i = (size_t)tl.row0 + r;
#pragma unroll
      for (int u = 0; u < QB; ++u)
        if (q0 + u < nq) acc[u] += V[(size_t)(q0 + u) * n + i] * wi;
    }
#pragma unroll
    for (int u = 0; u < QB; ++u) {
      const double sum = wave_sum(acc[u]);
      if (lane == 0 && q0 + u < nq) lds[q0 + u] = sum;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nq; q += BLOCK) I.part[(size_t)q * I.prows + tl.lt] = lds[q];
}

// One Lanczos step, first half: w = (G - s I) v_j - beta_{j-1} v_{j-1} with
// G = C + A*(y) in FP64 (pair values m64) plus the low-rank term
// K0 D0 (K0^T v_j) and the host's shift s, partial ||w||^2, then
// (fused) the first Gram-Schmidt dots <V_q, w>, q <= j, from the tile's w
// kept in LDS.  The tile's columns and pair values are staged in LDS (as in
// the SpMM); teams of 2^max(0, plog - 2) lanes share a row, so each lane
// gathers about four entries of v at once.
__global__ __launch_bounds__(BLOCK) void k_lz_spmv_dots(const Tile *__restrict__ tiles,
                                                        const InstDev *__restrict__ insts) {
  // staging area of the SpMV, reused for w and the dot partials afterwards
  __shared__ int32_t s_ru[TILE_MAX_ROWS + 1], s_rl[TILE_MAX_ROWS + 1];
  __shared__ int32_t s_col[TILE_MAX_ENTRIES];
  __shared__ double s_m[TILE_MAX_ENTRIES];
  __shared__ double s_w[TILE_MAX_ROWS];
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  if (P.lz_steps <= 0) return;
  const double *V = lz_basis(I, P);
  const double *v = V + (size_t)P.lz_j * I.n;
  double kd[LR_MAX] = {0.0, 0.0};
  for (int t = 0; t < I.r0; ++t) {
    double sacc = 0.0;
    for (int u = 0; u < I.r0; ++u) sacc += I.D0[t * I.r0 + u] * I.res->v[S_LZ_KV0 + u];
    kd[t] = sacc;
  }
  const int nrows = tl.row1 - tl.row0;
  for (int r = threadIdx.x; r <= nrows; r += BLOCK) {
    s_ru[r] = I.rowptr_u[tl.row0 + r];
    s_rl[r] = I.rowptr_l[tl.row0 + r];
  }
  __syncthreads();
  const int ku0 = s_ru[0], nu = s_ru[nrows] - ku0;
  const int kl0 = s_rl[0], nl = s_rl[nrows] - kl0;
  const bool staged = nu + nl <= TILE_MAX_ENTRIES;
  if (staged) stage_entries<double>(I, I.m64, ku0, nu, kl0, nl, true, s_col, s_m, I.m64_low);
  const int plog = staged ? max(0, (int)tl.plog_s - 2) : (int)tl.plog_s;
  const int TS = 1 << plog;
  const int team = threadIdx.x >> plog;
  const int strm = threadIdx.x & (TS - 1);
  const int nteams = BLOCK >> plog;
  double acc[1] = {0.0};
  for (int r = team; r < nrows; r += nteams) {
    const int i = tl.row0 + r;
    double w = 0.0;
    if (staged) {
      const int a0 = s_ru[r] - ku0, cu = s_ru[r + 1] - s_ru[r];
      const int b0 = nu + s_rl[r] - kl0 - cu, cnt = cu + s_rl[r + 1] - s_rl[r];
      constexpr int UN = 4;
      for (int q = strm * UN; q < cnt; q += TS * UN) {
        double mv[UN], x[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int idx = q + u;
          if (idx < cnt) {
            const int pos = idx < cu ? a0 + idx : b0 + idx;
            mv[u] = s_m[pos];
            x[u] = v[s_col[pos]];
          } else {
            mv[u] = 0.0;
            x[u] = 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) w += mv[u] * x[u];
      }
    } else {
      for (int k = I.rowptr_u[i] + strm; k < I.rowptr_u[i + 1]; k += TS) w += I.m64[k] * v[I.col_u[k]];
      for (int e = I.rowptr_l[i] + strm; e < I.rowptr_l[i + 1]; e += TS) w += I.m64_low[e] * v[I.col_l[e]];
    }
    for (int o = TS / 2; o >= 1; o >>= 1) w += shfl_xor(w, o);
    if (strm == 0) {
      for (int t = 0; t < I.r0; ++t) w += I.K064[(size_t)i * I.r0 + t] * kd[t];
      if (I.rk > 0) w += I.lc_wv[i];  // constraints' low-rank parts of G v (k_lc_kz)
      if (I.cdp_L > 0) w += I.cdp_wv[i];  // coded-diffraction part of G v
      // shifted three-term form: the Gram-Schmidt dots then see only the
      // small remainder, so the DGKS test can skip the second pass (the
      // host adds the shift and beta back into the projected matrix)
      w -= P.lz_shift * v[i];
      if (P.lz_j >= P.lz_tri0) w -= I.res->v[S_LZ_BETA] * V[(size_t)(P.lz_j - 1) * I.n + i];
      I.w[i] = w;
      s_w[r] = w;
      acc[0] += w * w;
    }
  }
  block_partials<1, LZ_W2_SLOT>(acc, I, tl.lt);  // (its barrier also publishes s_w)
  lz_tile_dots(I, V, P.lz_j + 1, tl, s_w, s_m);
}

// w -= sum_q V_q h_q with partial ||w||^2 and K0^T w.  First pass: the
// partials go to LZ_WP_SLOT / LZ_KV_SLOT (they decide whether a second pass
// is needed) and the second pass's dots <V_q, w'> follow from the tile's w'
// in LDS, re-reading V from L2 right after the update read it.  Second pass
// (skipped where the first sufficed): partials to slots 0..LR_MAX.
__global__ __launch_bounds__(BLOCK) void k_lz_update(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                     int32_t final_pass) {
  __shared__ double h[KMAX + 1];
  __shared__ double s_w[TILE_MAX_ROWS];
  __shared__ double lds[(BLOCK / 64) * PSTRIDE];
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  if (P.lz_steps <= 0 || (final_pass && P.lz_skip)) return;
  const double *V = lz_basis(I, P);
  const int nq = P.lz_j + 1;
  const size_t n = I.n;
  for (int q = threadIdx.x; q < nq; q += BLOCK) h[q] = I.hcoef[q];
  __syncthreads();
  double acc[1 + LR_MAX] = {0.0, 0.0, 0.0};
  for (int i = tl.row0 + threadIdx.x; i < tl.row1; i += BLOCK) {
    double wi = I.w[i];
    for (int q = 0; q < nq; ++q) wi -= V[(size_t)q * n + i] * h[q];
    I.w[i] = wi;
    s_w[i - tl.row0] = wi;
    acc[0] += wi * wi;
    for (int t = 0; t < I.r0; ++t) acc[1 + t] += I.K064[(size_t)i * I.r0 + t] * wi;
  }
  if (final_pass) {
    block_partials<1 + LR_MAX>(acc, I, tl.lt);
  } else {
    double a0[1] = {acc[0]};
    double akv[LR_MAX] = {acc[1], acc[2]};
    block_partials<1, LZ_WP_SLOT>(a0, I, tl.lt);
    block_partials<LR_MAX, LZ_KV_SLOT>(akv, I, tl.lt);  // (its barrier also publishes s_w)
    lz_tile_dots(I, V, nq, tl, s_w, lds);
  }
}

// v_{j+1} = w / beta_j (beta from the reduce kernel)
__global__ __launch_bounds__(BLOCK) void k_lz_scale(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts) {
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  if (P.lz_steps < 0) return;
  // the reduce kernel already advanced lz_j; the new vector index is lz_j
  double *V = lz_basis(I, P);
  const double b = I.res->v[S_LZ_BETA];
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  const int j = P.lz_j;
  if (j > KMAX) return;
  for (int i = tl.row0 + threadIdx.x; i < tl.row1; i += BLOCK) V[(size_t)j * I.n + i] = I.w[i] * inv;
}

// start vector: w = lzv (written by the host-side generator kernel), partial
// ||w||^2 and K0^T w.
__global__ __launch_bounds__(BLOCK) void k_lz_start(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts) {
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const uint64_t seed = P.lz_seed;
  const int use_prev = P.lz_use_prev;
  double acc[1 + LR_MAX] = {0.0, 0.0, 0.0};
  for (int i = tl.row0 + threadIdx.x; i < tl.row1; i += BLOCK) {
    // counter-based Gaussian: splitmix64 of (seed, i), Box-Muller
    uint64_t z = seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(i + 1));
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u1 = ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    uint64_t z2 = z * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z2 = (z2 ^ (z2 >> 30)) * 0xBF58476D1CE4E5B9ull;
    z2 = (z2 ^ (z2 >> 27)) * 0x94D049BB133111EBull;
    z2 ^= z2 >> 31;
    const double u2 = ((z2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    const double wi = use_prev == 2 ? I.lzv[i] : (use_prev ? I.lzv[i] + 1e-2 * g / sqrt((double)I.n) : g);
    I.w[i] = wi;
    acc[0] += wi * wi;
    for (int t = 0; t < I.r0; ++t) acc[1 + t] += I.K064[(size_t)i * I.r0 + t] * wi;
  }
  block_partials<1 + LR_MAX>(acc, I, tl.lt);
}

// V[dst] = sum_{q < nq} Vsrc_q S[q, c] for c < ncol (Ritz vectors / thick restart),
// writing either the other basis (restart) or lzv (single Ritz vector).
__global__ __launch_bounds__(BLOCK) void k_lz_combine(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                      int32_t to_lzv) {
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  const double *Vs = lz_basis(I, P);
  double *Vd = P.lz_basis ? I.V : I.V2;
  const int nq = P.lz_j;  // basis vectors v_0..v_{k-1}
  const int ncol = to_lzv ? 1 : P.lz_q;
  const size_t n = I.n;
  const double *S = I.up_base + P.up_off;
  for (int i = tl.row0 + threadIdx.x; i < tl.row1; i += BLOCK) {
    for (int c = 0; c < ncol; ++c) {
      double s = 0.0;
      for (int q = 0; q < nq; ++q) s += Vs[(size_t)q * n + i] * S[q * KMAX + c];
      if (to_lzv) I.lzv[i] = s;
      else Vd[(size_t)c * n + i] = s;
    }
    if (!to_lzv) Vd[(size_t)ncol * n + i] = Vs[(size_t)nq * n + i];  // residual direction v_k
  }
}

// ---------------------------------------------------------------------------
// Reductions: one block per instance sums that instance's tile partials in a
// fixed order and applies the op's scalar epilogue.
// ---------------------------------------------------------------------------
enum RedOp : int {
  RD_COMBO = 0,    // ||XT - W0||^2
  RD_SDDMM_XT,     // g(XT), Z0 slot 0
  RD_TRIAL_PROJ,   // ||Z||^2 -> projection factor
  RD_PROJ_DOTS,    // <GR, d>, ||d||^2, ||y+ - W0||^2
  RD_SDDMM_YP,     // g(y+), Z0 slot 1
  RD_AIPP,         // ||Rl||^2, <Rl, W0 - y+>, <W, y+>
  RD_EVAL,         // g at an evaluation point, T0, p^T r, ||r||^2
  RD_LRONLY,       // K0^T X -> Z0 slot (zsel 0)
  RD_LZ_START,     // ||w||, K0^T w -> normalise into V_0
  RD_LZ_H1,        // h1 -> hcoef, H column
  RD_LZ_H2,        // h2 -> hcoef, H column += h2
  RD_LZ_FINAL,     // beta_j, K0^T v_{j+1}, j++
  RD_FW_DEN,       // sum (T_Y - tau2 T_v)^2
  RD_SETP,         // b^T p, ||r||^2 (constraint-major partials)
  RD_NORM,         // ||.||^2 of a pack / copy
  RD_GEN_EXTRA,    // general mode: add constraint-major p^T r, ||r||^2 rows
  RD_GRAM,         // sum gram partials
  RD_LZ_CHECKH2,   // after the first Gram-Schmidt pass: skip the second if ||w'|| >= ||w|| / sqrt(2),
                   // else h2 -> hcoef, H column += h2
  RD_TRIAL_FUSED,  // RD_SDDMM_XT, RD_TRIAL_PROJ (from FUSE_SLOT) and RD_COMBO after the fused trial kernel
  RD_YP_PROJ       // RD_SDDMM_YP and RD_PROJ_DOTS
};

struct RedArgs {
  int32_t op;
  int32_t zsel;
  int32_t R;      // current width (for K^T X slots / gram)
  int32_t extra;  // RD_TRIAL_FUSED / RD_YP_PROJ: 1 = split over RED_SPLIT workgroups per instance
};

// Sums of slots [q0, q1) and then [q2, q3) over partial rows [row0, row0 +
// nrows) into out[0..): slots in batches of RQ; every thread adds rows t,
// t + blockDim, ... of each slot of the batch (all loads of the batch in
// flight together, the next row's issued before the current one is added),
// then a fixed wave and cross-wave reduction -- a fixed order for every
// instance, whichever batch a slot falls in.
constexpr int RQ = 8;
__device__ void reduce_slots(const InstDev &I, int q0, int q1, int row0, int nrows, double *out, int q2 = 0,
                             int q3 = 0) {
  __shared__ double red[RBLOCK / 64][RQ];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, nw = blockDim.x >> 6;
  const int n1 = q1 - q0, ntot = n1 + (q3 - q2);
  for (int qb = 0; qb < ntot; qb += RQ) {
    const int nq = min(RQ, ntot - qb);
    const double *src[RQ];
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      const int j = qb + u, q = j < n1 ? q0 + j : q2 + (j - n1);
      src[u] = I.part + (size_t)(u < nq ? q : q0) * I.prows + row0;
    }
    double s[RQ];
#pragma unroll
    for (int u = 0; u < RQ; ++u) s[u] = 0.0;
    double cur[RQ];
    int t = tid;
#pragma unroll
    for (int u = 0; u < RQ; ++u) cur[u] = (u < nq && t < nrows) ? src[u][t] : 0.0;
    for (; t < nrows; t += blockDim.x) {
      const int tn = t + blockDim.x;
      double nxt[RQ];
#pragma unroll
      for (int u = 0; u < RQ; ++u) nxt[u] = (u < nq && tn < nrows) ? src[u][tn] : 0.0;
#pragma unroll
      for (int u = 0; u < RQ; ++u) s[u] += cur[u];
#pragma unroll
      for (int u = 0; u < RQ; ++u) cur[u] = nxt[u];
    }
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      const double v = wave_sum(s[u]);
      if (lane == 0) red[wave][u] = v;
    }
    __syncthreads();
    if (tid < nq) {
      double v = 0.0;
      for (int w = 0; w < nw; ++w) v += red[w][tid];
      out[qb + tid] = v;
    }
    __syncthreads();
  }
  __syncthreads();
}

// Y0 (r0 x R) = K0^T X from slots 4.. (already summed in y0), Z0 = D0 Y0,
// returns Tr(D0 Y0 Y0^T) (Algorithms 3 and 5 for the objective).
__device__ double lowrank_finish(const InstDev &I, int R, int zsel, const double *y0) {
  const int r0 = I.r0;
  double *Z0 = I.Z0 + zsel * LR_MAX * R_MAX;
  for (int q = threadIdx.x; q < r0 * R_MAX; q += blockDim.x) {
    const int t = q / R_MAX, c = q % R_MAX;
    double s = 0.0;
    if (c < R)
      for (int u = 0; u < r0; ++u) s += I.D0[t * r0 + u] * y0[u * R + c];
    Z0[q] = s;
  }
  double tr = 0.0;
  for (int t = 0; t < r0; ++t)
    for (int u = 0; u < r0; ++u) {
      double d = 0.0;
      for (int c = 0; c < R; ++c) d += y0[t * R + c] * y0[u * R + c];
      tr += I.D0[t * r0 + u] * d;
    }
  return tr;
}

__global__ __launch_bounds__(RBLOCK) void k_reduce(const int32_t *__restrict__ ilist, const InstDev *__restrict__ insts,
                                                   RedArgs a) {
  __shared__ double S[PSTRIDE];
  __shared__ double E[4];
  const InstDev &I = insts[ilist[blockIdx.x]];
  InstParams &P = *I.prm;
  double *res = I.res->v;
  const int nt = I.ntiles;
  const int tid = threadIdx.x;
  // The trial's two reduces are split over RED_SPLIT workgroups per
  // instance (one workgroup alone is bound by its own load latency over
  // thousands of tile rows): workgroup y sums its contiguous share of the
  // rows, writes its sums, and the workgroup that finishes last -- counted
  // with one device-scope atomic, no waiting -- adds the RED_SPLIT rows in y
  // order and goes on with the op.  The order of every sum is fixed.
  const bool split = (a.op == RD_TRIAL_FUSED || a.op == RD_YP_PROJ) && gridDim.y == RED_SPLIT && I.direct &&
                     4 + I.r0 * a.R + 3 <= RQ && nt >= RED_SPLIT_MIN_TILES;
  if (split) {
    __shared__ int s_last;
    const int nlr = I.r0 * a.R, nq = 4 + nlr + 3;
    const int x0 = a.op == RD_TRIAL_FUSED ? FUSE_SLOT : PROJ_SLOT;
    const int chunk = (nt + RED_SPLIT - 1) / RED_SPLIT;
    const int y0 = blockIdx.y * chunk, y1 = min(nt, y0 + chunk);
    reduce_slots(I, 0, 4 + nlr, y0, max(0, y1 - y0), S, x0, x0 + 3);
    if (tid == 0) {
      for (int q = 0; q < nq; ++q) I.red_stage[blockIdx.y * RQ + q] = S[q];
      __threadfence();
      s_last = atomicAdd(I.red_count, 1u) == RED_SPLIT - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (tid < nq) {
      double v = 0.0;
      for (int y = 0; y < RED_SPLIT; ++y) v += I.red_stage[y * RQ + tid];
      S[tid] = v;
    }
    if (tid == 0) *I.red_count = 0u;  // every workgroup of this launch has counted
    __syncthreads();
  } else if (blockIdx.y > 0 && a.op != RD_LZ_H1 && a.op != RD_LZ_CHECKH2 && a.op != RD_GRAM) {
    return;
  }
  switch (a.op) {
    case RD_COMBO:
    case RD_NORM:
    case RD_TRIAL_PROJ: {
      const int q0 = a.op == RD_COMBO ? COMBO_SLOT : 0;
      reduce_slots(I, q0, q0 + (a.op == RD_TRIAL_PROJ ? 2 : 1), 0, nt, S);
      if (tid == 0) {
        if (a.op == RD_COMBO) res[S_XTW0] = S[0];
        else if (a.op == RD_NORM) res[S_NZ] = S[0];
        else {
          res[S_NZ] = S[0];
          res[S_PROJC] = S[0] > P.tau2 ? P.tau / sqrt(S[0]) : 1.0;
          res[S_GR2T] = S[1];
        }
      }
      break;
    }
    case RD_SDDMM_XT:
    case RD_TRIAL_FUSED:
    case RD_SDDMM_YP:
    case RD_YP_PROJ:
    case RD_EVAL: {
      const int nlr = I.r0 * a.R;
      // the trial's second kernel's three slots ride in the same pass when
      // they fit its batch
      const int x0 = a.op == RD_TRIAL_FUSED ? FUSE_SLOT : (a.op == RD_YP_PROJ ? PROJ_SLOT : -1);
      const bool one_pass = x0 >= 0 && 4 + nlr + 3 <= RQ;
      if (split) {
        // S holds the sums already
      } else if (one_pass) {
        reduce_slots(I, 0, 4 + nlr, 0, nt, S, x0, x0 + 3);
      } else {
        reduce_slots(I, 0, 4 + nlr, 0, nt, S);
      }
      double X3[3];
      if (one_pass)
        for (int q = 0; q < 3; ++q) X3[q] = S[4 + nlr + q];
      const int ex = I.direct ? 0 : (I.m + BLOCK - 1) / BLOCK;
      if (ex > 0) reduce_slots(I, 0, 3, nt, ex, E);
      else if (tid < 4) E[tid] = 0.0;
      __syncthreads();
      const int zsel = a.op == RD_SDDMM_YP || a.op == RD_YP_PROJ ? 1 : a.zsel;
      double tr = 0.0;
      if (I.r0 > 0) tr = lowrank_finish(I, a.R, zsel, S + 4);
      if (tid == 0) {
        const double t0 = S[0] + tr, pr = S[1] + E[0], rr = S[2] + E[1], yt = S[3] + E[2];
        const double g = t0 + pr + 0.5 * P.beta * rr;
        const int slot = a.op == RD_SDDMM_XT || a.op == RD_TRIAL_FUSED
                             ? S_G_XT
                             : (a.op == RD_SDDMM_YP || a.op == RD_YP_PROJ ? S_G_YP : S_G_EVAL);
        res[slot] = g;
        if (a.op == RD_EVAL) {
          res[S_T0] = t0;
          res[S_PR] = pr;
          res[S_RR] = rr;
          res[S_YT] = yt;
        }
        if (!(g == g) || g - g != 0.0) res[S_NAN] = 1.0;
      }
      if (x0 >= 0 && !one_pass) {
        __syncthreads();
        reduce_slots(I, x0, x0 + 3, 0, nt, S);  // FUSE_SLOT + 2 = COMBO_SLOT
        for (int q = 0; q < 3; ++q) X3[q] = S[q];
      }
      if (tid == 0) {
        if (a.op == RD_TRIAL_FUSED) {
          res[S_NZ] = X3[0];
          res[S_PROJC] = X3[0] > P.tau2 ? P.tau / sqrt(X3[0]) : 1.0;
          res[S_GR2T] = X3[1];
          res[S_XTW0] = X3[2];
        } else if (a.op == RD_YP_PROJ) {
          res[S_GR_D] = X3[0];
          res[S_D2] = X3[1];
          res[S_YPW0] = X3[2];
        }
      }
      break;
    }
    case RD_PROJ_DOTS:
    case RD_AIPP: {
      const int q0 = a.op == RD_PROJ_DOTS ? PROJ_SLOT : 0;
      reduce_slots(I, q0, q0 + (a.op == RD_AIPP ? 4 : 3), 0, nt, S);
      if (tid == 0) {
        if (a.op == RD_PROJ_DOTS) {
          res[S_GR_D] = S[0];
          res[S_D2] = S[1];
          res[S_YPW0] = S[2];
        } else {
          res[S_RL2] = S[0];
          res[S_RL_W0] = S[1];
          res[S_WY] = S[2];
          res[S_GR2A] = S[3];
        }
      }
      break;
    }
    case RD_LRONLY: {
      reduce_slots(I, 4, 4 + I.r0 * a.R, 0, nt, S);
      if (I.r0 > 0) (void)lowrank_finish(I, a.R, a.zsel, S);
      break;
    }
    case RD_LZ_START:
    case RD_LZ_FINAL: {
      // (P.lz_skip and P.lz_steps are read by every thread before the
      // barriers in reduce_slots; thread 0 writes them after)
      if (a.op != RD_LZ_START && P.lz_steps <= 0) break;
      if (a.op == RD_LZ_FINAL && P.lz_skip) {
        // one pass sufficed: beta and K0^T w from the first pass's partials
        reduce_slots(I, LZ_WP_SLOT, LZ_WP_SLOT + 1, 0, nt, S);
        reduce_slots(I, LZ_KV_SLOT, LZ_KV_SLOT + I.r0, 0, nt, S + 1);
      } else {
        reduce_slots(I, 0, 1 + I.r0, 0, nt, S);
      }
      if (tid == 0) {
        const double b = sqrt(S[0]);
        res[S_LZ_BETA] = b;
        for (int t = 0; t < I.r0; ++t) res[S_LZ_KV0 + t] = b > 0 ? S[1 + t] / b : 0.0;
        if (a.op == RD_LZ_START) {
          res[S_LZ_NRM0] = b;
          P.lz_j = 0;
        } else {
          I.dl_base[P.dl_off + (size_t)(P.lz_j - P.lz_j0) * (KMAX + 2) + KMAX + 1] = b;
          P.lz_j += 1;
          P.lz_steps -= 1;
        }
      }
      break;
    }
    case RD_LZ_H1:
    case RD_LZ_CHECKH2: {
      // slots split over blockIdx.y in runs of RQ (independent coefficients)
      if (P.lz_steps <= 0) break;
      const int nq = P.lz_j + 1;
      if (a.op == RD_LZ_CHECKH2) {
        // DGKS criterion (every block decides alike): one classical
        // Gram-Schmidt pass suffices unless it removed most of w, eta = 1/sqrt(2)
        reduce_slots(I, LZ_WP_SLOT, LZ_WP_SLOT + 1, 0, nt, E);
        const bool skip = 2.0 * E[0] >= res[S_LZ_W2];
        if (blockIdx.y == 0 && tid == 0) P.lz_skip = skip ? 1 : 0;
        if (skip) break;
      }
      if (a.op == RD_LZ_H1 && blockIdx.y == 0) {
        reduce_slots(I, LZ_W2_SLOT, LZ_W2_SLOT + 1, 0, nt, E);
        if (tid == 0) res[S_LZ_W2] = E[0];
      }
      const int qa = blockIdx.y * RQ, qe = min(nq, qa + RQ);
      if (qa >= nq) break;
      reduce_slots(I, qa, qe, 0, nt, S);
      double *Hc = I.dl_base + P.dl_off + (size_t)(P.lz_j - P.lz_j0) * (KMAX + 2);
      for (int q = qa + tid; q < qe; q += blockDim.x) {
        I.hcoef[q] = S[q - qa];
        if (a.op == RD_LZ_H1) Hc[q] = S[q - qa];
        else Hc[q] += S[q - qa];
      }
      break;
    }
    case RD_FW_DEN: {
      reduce_slots(I, 0, 1, 0, nt, S);
      const int ex = I.direct ? 0 : (I.m + BLOCK - 1) / BLOCK;
      if (ex > 0) reduce_slots(I, 0, 1, nt, ex, E);
      if (tid == 0) res[S_FWDEN] = S[0] + (ex > 0 ? E[0] : 0.0);
      break;
    }
    case RD_SETP: {
      const int ex = (I.m + BLOCK - 1) / BLOCK;
      if (ex > 0) reduce_slots(I, 0, 3, nt, ex, E);
      if (tid == 0) {
        res[S_BP] = ex > 0 ? E[0] : 0.0;
        res[S_RR] = ex > 0 ? E[1] : 0.0;
        res[S_PTR] = ex > 0 ? E[2] : 0.0;
      }
      break;
    }
    case RD_GRAM: {
      // entries split over blockIdx.y in runs of 64
      const int R = a.R;
      const int wave = tid >> 6, lane = tid & 63, nw = blockDim.x >> 6;
      const int qe = min(R * R, (int)(blockIdx.y + 1) * 64);
      for (int q = blockIdx.y * 64 + wave; q < qe; q += nw) {
        const double *src = I.gram + (size_t)q * nt;
        double s = 0.0;
        for (int t = lane; t < nt; t += 64) s += src[t];
        s = wave_sum(s);
        if (lane == 0) I.dl_base[P.dl_off + q] = s;  // Gram matrix, row-major R x R
      }
      break;
    }
    default:
      break;
  }
}

// Lanczos start: V_0 = w / ||w||
__global__ __launch_bounds__(BLOCK) void k_lz_first(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts) {
  const Tile tl = tiles[tile_index()];
  const InstDev &I = insts[tl.inst];
  const InstParams &P = *I.prm;
  double *V = lz_basis(I, P);
  const double b = I.res->v[S_LZ_BETA];
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  for (int i = tl.row0 + threadIdx.x; i < tl.row1; i += BLOCK) V[i] = I.w[i] * inv;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T>
constexpr int g_of(int R) {
  return R * (int)sizeof(T) / 16;
}

#define HL_DISPATCH_G(T, R, FN, ...)                        \
  do {                                                      \
    switch (g_of<T>(R)) {                                   \
      case 1: FN<T, 1>(__VA_ARGS__); break;                 \
      case 2: FN<T, 2>(__VA_ARGS__); break;                 \
      case 4: FN<T, 4>(__VA_ARGS__); break;                 \
      case 8: FN<T, 8>(__VA_ARGS__); break;                 \
      case 16: FN<T, 16>(__VA_ARGS__); break;               \
      case 32: if constexpr (sizeof(T) == 8) { FN<T, 32>(__VA_ARGS__); } break; \
      default: break;                                       \
    }                                                       \
  } while (0)

template <typename T, int G>
static void l_sddmm(hipStream_t s, const Tile *t, int nt, const InstDev *d, SddmmArgs a) {
  hipLaunchKernelGGL((k_sddmm<T, G>), dim3(nt), dim3(BLOCK), 0, s, t, d, a);
}
template <typename T, int G>
static void l_lrdots(hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole) {
  hipLaunchKernelGGL((k_lr_dots<T, G>), dim3(nt), dim3(BLOCK), 0, s, t, d, xrole);
}
template <typename T, int G>
static void l_spmm(hipStream_t s, const Tile *t, int nt, const InstDev *d, SpmmArgs a, int mode) {
  if (mode == SP_PLAIN) hipLaunchKernelGGL((k_spmm<T, G, SP_PLAIN>), dim3(nt), dim3(BLOCK), 0, s, t, d, a);
  else if (mode == SP_TRIAL) hipLaunchKernelGGL((k_spmm<T, G, SP_TRIAL>), dim3(nt), dim3(BLOCK), 0, s, t, d, a);
  else hipLaunchKernelGGL((k_spmm<T, G, SP_AIPP>), dim3(nt), dim3(BLOCK), 0, s, t, d, a);
}
template <typename T, int G>
static void l_combo(hipStream_t s, const Tile *t, int nt, const InstDev *d, bool grouped) {
  if (grouped) hipLaunchKernelGGL((k_combo<T, G>), dim3((nt + VT - 1) / VT), dim3(BLOCK), 0, s, t, d, nt);
  else hipLaunchKernelGGL((k_combo_tile<T, G>), dim3(nt), dim3(BLOCK), 0, s, t, d);
}
template <typename T, int G>
static void l_proj(hipStream_t s, const Tile *t, int nt, const InstDev *d, bool grouped) {
  if (grouped) hipLaunchKernelGGL((k_proj<T, G>), dim3((nt + VT - 1) / VT), dim3(BLOCK), 0, s, t, d, nt);
  else hipLaunchKernelGGL((k_proj_tile<T, G>), dim3(nt), dim3(BLOCK), 0, s, t, d);
}
template <typename T, int G>
static void l_copy(hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst) {
  hipLaunchKernelGGL((k_copy_scale<T, G>), dim3(nt), dim3(BLOCK), 0, s, t, d, src, dst);
}
template <typename T, int G>
static void l_gram(hipStream_t s, const Tile *t, int nt, const InstDev *d, int src) {
  hipLaunchKernelGGL((k_gram<T, G>), dim3(nt), dim3(BLOCK), 0, s, t, d, src);
}

}  // namespace hl

// Host-visible launch API (ops.h declares these)
#include "ops.h"

namespace hl {

static bool is64(int prec) { return prec == 0; }

void op_sddmm(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole, int msel, int wT,
              int wyp, double *tout) {
  if (nt <= 0) return;
  SddmmArgs a{xrole, msel, wT, wyp, tout};
  if (is64(prec)) HL_DISPATCH_G(double, R, l_sddmm, s, t, nt, d, a);
  else HL_DISPATCH_G(float, R, l_sddmm, s, t, nt, d, a);
}
void op_lr_dots(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole) {
  if (nt <= 0) return;
  if (is64(prec)) HL_DISPATCH_G(double, R, l_lrdots, s, t, nt, d, xrole);
  else HL_DISPATCH_G(float, R, l_lrdots, s, t, nt, d, xrole);
}
void op_spmm(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole, int msel, int zsel,
             int outrole, int mode) {
  if (nt <= 0) return;
  SpmmArgs a{xrole, msel, zsel, outrole};
  if (is64(prec)) HL_DISPATCH_G(double, R, l_spmm, s, t, nt, d, a, mode);
  else HL_DISPATCH_G(float, R, l_spmm, s, t, nt, d, a, mode);
}
bool trial_fusable(int prec, int R) {
  const int G = is64(prec) ? g_of<double>(R) : g_of<float>(R);
  return G == 1 || G == 2;
}
void op_trial_fused(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole) {
  if (nt <= 0) return;
  const int G = is64(prec) ? g_of<double>(R) : g_of<float>(R);
  if (is64(prec)) {
    if (G == 1) hipLaunchKernelGGL((k_trial_fused<double, 1>), dim3(nt), dim3(BLOCK), 0, s, t, d, xrole);
    else if (G == 2) hipLaunchKernelGGL((k_trial_fused<double, 2>), dim3(nt), dim3(BLOCK), 0, s, t, d, xrole);
  } else {
    if (G == 1) hipLaunchKernelGGL((k_trial_fused<float, 1>), dim3(nt), dim3(BLOCK), 0, s, t, d, xrole);
    else if (G == 2) hipLaunchKernelGGL((k_trial_fused<float, 2>), dim3(nt), dim3(BLOCK), 0, s, t, d, xrole);
  }
}
// tiles of at most 64 chunks on average take the grouped vector kernels
static bool vec_grouped(int prec, int R, int nt, int64_t rows) {
  const int G = is64(prec) ? g_of<double>(R) : g_of<float>(R);
  return rows * G <= (int64_t)64 * nt;
}
void op_combo(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int64_t rows) {
  if (nt <= 0) return;
  const bool gr = vec_grouped(prec, R, nt, rows);
  if (is64(prec)) HL_DISPATCH_G(double, R, l_combo, s, t, nt, d, gr);
  else HL_DISPATCH_G(float, R, l_combo, s, t, nt, d, gr);
}
void op_proj(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int64_t rows) {
  if (nt <= 0) return;
  const bool gr = vec_grouped(prec, R, nt, rows);
  if (is64(prec)) HL_DISPATCH_G(double, R, l_proj, s, t, nt, d, gr);
  else HL_DISPATCH_G(float, R, l_proj, s, t, nt, d, gr);
}
void op_copy_scale(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst) {
  if (nt <= 0) return;
  if (is64(prec)) HL_DISPATCH_G(double, R, l_copy, s, t, nt, d, src, dst);
  else HL_DISPATCH_G(float, R, l_copy, s, t, nt, d, src, dst);
}
void op_gram(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src) {
  if (nt <= 0) return;
  if (is64(prec)) HL_DISPATCH_G(double, R, l_gram, s, t, nt, d, src);
  else HL_DISPATCH_G(float, R, l_gram, s, t, nt, d, src);
}

template <typename T, int G, typename S>
static void l_pack(hipStream_t s, const Tile *t, int nt, const InstDev *d, const S *src, int r, int64_t ld, int dst,
                   double scale) {
  hipLaunchKernelGGL((k_pack<T, G, S>), dim3(nt), dim3(BLOCK), 0, s, t, d, src, r, ld, dst, scale);
}
template <typename T, int G>
static void l_pack_d(hipStream_t s, const Tile *t, int nt, const InstDev *d, const double *src, int r, int64_t ld,
                     int dst, double scale) {
  l_pack<T, G, double>(s, t, nt, d, src, r, ld, dst, scale);
}
template <typename T, int G>
static void l_pack_o(hipStream_t s, const Tile *t, int nt, const InstDev *d, const T *src, int r, int64_t ld, int dst,
                     double scale) {
  l_pack<T, G, T>(s, t, nt, d, src, r, ld, dst, scale);
}

void op_pack_f64(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, const double *src, int r,
                 int64_t ld, int dst, double scale) {
  if (nt <= 0) return;
  if (is64(prec)) HL_DISPATCH_G(double, R, l_pack_d, s, t, nt, d, src, r, ld, dst, scale);
  else HL_DISPATCH_G(float, R, l_pack_d, s, t, nt, d, src, r, ld, dst, scale);
}
void op_pack_op(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, const void *src, int r,
                int64_t ld, int dst) {
  if (nt <= 0) return;
  if (is64(prec)) HL_DISPATCH_G(double, R, l_pack_o, s, t, nt, d, (const double *)src, r, ld, dst, 1.0);
  else HL_DISPATCH_G(float, R, l_pack_o, s, t, nt, d, (const float *)src, r, ld, dst, 1.0);
}

template <typename T, int G, typename S>
static void l_unpack(hipStream_t s, const Tile *t, int nt, const InstDev *d, S *out, int r, int64_t ld, int src) {
  hipLaunchKernelGGL((k_unpack<T, G, S>), dim3(nt), dim3(BLOCK), 0, s, t, d, out, r, ld, src);
}
template <typename T, int G>
static void l_unpack_d(hipStream_t s, const Tile *t, int nt, const InstDev *d, double *out, int r, int64_t ld, int src) {
  l_unpack<T, G, double>(s, t, nt, d, out, r, ld, src);
}
template <typename T, int G>
static void l_unpack_o(hipStream_t s, const Tile *t, int nt, const InstDev *d, T *out, int r, int64_t ld, int src) {
  l_unpack<T, G, T>(s, t, nt, d, out, r, ld, src);
}
void op_unpack_f64(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, double *out, int r,
                   int64_t ld, int src) {
  if (nt <= 0) return;
  if (is64(prec)) HL_DISPATCH_G(double, R, l_unpack_d, s, t, nt, d, out, r, ld, src);
  else HL_DISPATCH_G(float, R, l_unpack_d, s, t, nt, d, out, r, ld, src);
}
void op_unpack_op(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, void *out, int r,
                  int64_t ld, int src) {
  if (nt <= 0) return;
  if (is64(prec)) HL_DISPATCH_G(double, R, l_unpack_o, s, t, nt, d, (double *)out, r, ld, src);
  else HL_DISPATCH_G(float, R, l_unpack_o, s, t, nt, d, (float *)out, r, ld, src);
}

template <typename T, int GS, int GD>
static void l_fw2(hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst) {
  hipLaunchKernelGGL((k_fw_apply<T, GS, GD>), dim3(nt), dim3(BLOCK), 0, s, t, d, src, dst);
}
template <typename T, int GS, int GD>
static void l_rot2(hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst) {
  hipLaunchKernelGGL((k_rotate<T, GS, GD>), dim3(nt), dim3(BLOCK), 0, s, t, d, src, dst);
}

template <typename T, int GS>
static void l_fw_gd(int GD, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst, bool rot) {
  switch (GD) {
    case 1: rot ? l_rot2<T, GS, 1>(s, t, nt, d, src, dst) : l_fw2<T, GS, 1>(s, t, nt, d, src, dst); break;
    case 2: rot ? l_rot2<T, GS, 2>(s, t, nt, d, src, dst) : l_fw2<T, GS, 2>(s, t, nt, d, src, dst); break;
    case 4: rot ? l_rot2<T, GS, 4>(s, t, nt, d, src, dst) : l_fw2<T, GS, 4>(s, t, nt, d, src, dst); break;
    case 8: rot ? l_rot2<T, GS, 8>(s, t, nt, d, src, dst) : l_fw2<T, GS, 8>(s, t, nt, d, src, dst); break;
    case 16: rot ? l_rot2<T, GS, 16>(s, t, nt, d, src, dst) : l_fw2<T, GS, 16>(s, t, nt, d, src, dst); break;
    case 32:
      if constexpr (sizeof(T) == 8) { rot ? l_rot2<T, GS, 32>(s, t, nt, d, src, dst) : l_fw2<T, GS, 32>(s, t, nt, d, src, dst); }
      break;
    default: break;
  }
}
template <typename T>
static void l_fw_gs(int GS, int GD, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst, bool rot) {
  switch (GS) {
    case 1: l_fw_gd<T, 1>(GD, s, t, nt, d, src, dst, rot); break;
    case 2: l_fw_gd<T, 2>(GD, s, t, nt, d, src, dst, rot); break;
    case 4: l_fw_gd<T, 4>(GD, s, t, nt, d, src, dst, rot); break;
    case 8: l_fw_gd<T, 8>(GD, s, t, nt, d, src, dst, rot); break;
    case 16: l_fw_gd<T, 16>(GD, s, t, nt, d, src, dst, rot); break;
    case 32:
      if constexpr (sizeof(T) == 8) l_fw_gd<T, 32>(GD, s, t, nt, d, src, dst, rot);
      break;
    default: break;
  }
}
void op_fw_apply(int prec, int RS, int RD, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst) {
  if (nt <= 0) return;
  if (is64(prec)) l_fw_gs<double>(g_of<double>(RS), g_of<double>(RD), s, t, nt, d, src, dst, false);
  else l_fw_gs<float>(g_of<float>(RS), g_of<float>(RD), s, t, nt, d, src, dst, false);
}
void op_rotate(int prec, int RS, int RD, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst) {
  if (nt <= 0) return;
  if (is64(prec)) l_fw_gs<double>(g_of<double>(RS), g_of<double>(RD), s, t, nt, d, src, dst, true);
  else l_fw_gs<float>(g_of<float>(RS), g_of<float>(RD), s, t, nt, d, src, dst, true);
}

void op_gen_constraints(int prec, hipStream_t s, const int32_t *ilist, int ni, int maxm, const InstDev *d, int wT) {
  if (ni <= 0 || maxm <= 0) return;
  SddmmArgs a{0, -1, wT, 1};
  dim3 g((maxm + BLOCK - 1) / BLOCK, ni);
  if (is64(prec)) hipLaunchKernelGGL(k_gen_constraints<double>, g, dim3(BLOCK), 0, s, ilist, d, a);
  else hipLaunchKernelGGL(k_gen_constraints<float>, g, dim3(BLOCK), 0, s, ilist, d, a);
}
void op_pairvals(int prec, hipStream_t s, const int32_t *ilist, int ni, int maxpairs, const InstDev *d, int msel,
                 const double *yext, int general) {
  if (ni <= 0 || maxpairs <= 0) return;
  dim3 g((maxpairs + BLOCK - 1) / BLOCK, ni);
  if (general) {
    if (is64(prec)) hipLaunchKernelGGL(k_gen_pairvals<double>, g, dim3(BLOCK), 0, s, ilist, d, msel, yext ? 1 : 0, yext);
    else hipLaunchKernelGGL(k_gen_pairvals<float>, g, dim3(BLOCK), 0, s, ilist, d, msel, yext ? 1 : 0, yext);
  } else {
    if (is64(prec)) hipLaunchKernelGGL(k_pairvals<double>, g, dim3(BLOCK), 0, s, ilist, d, msel, yext);
    else hipLaunchKernelGGL(k_pairvals<float>, g, dim3(BLOCK), 0, s, ilist, d, msel, yext);
  }
}
void op_fw_den(hipStream_t s, const Tile *t, int nt, const InstDev *d) {
  if (nt > 0) hipLaunchKernelGGL(k_fw_den, dim3(nt), dim3(BLOCK), 0, s, t, d);
}
void op_fw_den_gen(hipStream_t s, const int32_t *ilist, int ni, int maxm, const InstDev *d) {
  if (ni <= 0 || maxm <= 0) return;
  hipLaunchKernelGGL(k_fw_den_gen, dim3((maxm + BLOCK - 1) / BLOCK, ni), dim3(BLOCK), 0, s, ilist, d);
}
void op_set_p(hipStream_t s, const int32_t *ilist, int ni, int maxm, const InstDev *d) {
  if (ni <= 0 || maxm <= 0) return;
  hipLaunchKernelGGL(k_set_p, dim3((maxm + BLOCK - 1) / BLOCK, ni), dim3(BLOCK), 0, s, ilist, d);
}
void op_lower_copy(hipStream_t s, const int32_t *ilist, int ni, int64_t maxnl, const InstDev *d) {
  if (ni <= 0 || maxnl <= 0) return;
  const int64_t nb = (maxnl + BLOCK - 1) / BLOCK;
  const int gx = nb < 4096 ? (int)nb : 4096;
  hipLaunchKernelGGL(k_lower_copy, dim3(gx, ni), dim3(BLOCK), 0, s, ilist, d);
}
void op_refresh_pb(hipStream_t s, const int32_t *ilist, int ni, int64_t maxcount, const InstDev *d) {
  if (ni <= 0 || maxcount <= 0) return;
  const int64_t nb = (maxcount + BLOCK - 1) / BLOCK;
  const int gx = nb < 4096 ? (int)nb : 4096;
  hipLaunchKernelGGL(k_refresh_pb, dim3(gx, ni), dim3(BLOCK), 0, s, ilist, d);
}
void op_reduce(hipStream_t s, const int32_t *ilist, int ni, const InstDev *d, int op, int zsel, int R, int extra) {
  if (ni <= 0) return;
  RedArgs a{op, zsel, R, extra};
  int ny = 1;
  if (op == RD_LZ_H1 || op == RD_LZ_CHECKH2) ny = (KMAX + 1 + RQ - 1) / RQ;
  else if ((op == RD_TRIAL_FUSED || op == RD_YP_PROJ) && extra) ny = RED_SPLIT;
  else if (op == RD_GRAM) ny = (R * R + 63) / 64;
  hipLaunchKernelGGL(k_reduce, dim3(ni, ny), dim3(RBLOCK), 0, s, ilist, d, a);
}
// ---------------------------------------------------------------------------
// Low-rank parts of the constraints (Section 3.2, eq. HSLR-rep-body;
// Algorithm 3 for A~(XX^T) and Algorithm 5 for the adjoint): the dense
// contraction K^T X over the rows of each tile, its fixed-order sum per
// instance, then per term Tr(D_q Y_q Y_q^T), or the coefficients
// blockdiag(y_l D_q) K^T X that the SpMM epilogue multiplies by K's rows.
// ---------------------------------------------------------------------------
// Per tile and group of 64 columns of K: partial K^T X (vsrc 0: the factor
// of role xrole, R columns) or K^T v (vsrc 1: the Lanczos vector being
// multiplied; 2: the Ritz vector lzv), into lc_part[tile][k][c].
// Per tile and group of 64 columns of K: partial K^T X (vsrc 0: the factor
// of role xrole, R columns, K in the operator type) or K^T v (vsrc 1: the
// Lanczos vector being multiplied; 2: the Ritz vector lzv; R = 1, K in
// FP64), into lc_part[tile][k][c] (rows of stride R).  Lane = column k of
// K (coalesced reads of each row of K); the four waves take every fourth
// row of the tile and their sums are added in wave order through LDS.
template <typename T, int RC>
__device__ __forceinline__ void lc_kty_tile(const Tile &tl, const InstDev &I, const T *__restrict__ K,
                                            const T *__restrict__ X, const double *__restrict__ v, int rk, int k,
                                            double *out) {
  __shared__ double s_red[BLOCK / 64][64];
  // the rows of X (or v) staged in LDS, 64 rows at a time: every lane reads
  // the same row, so LDS broadcasts it instead of per-lane vector loads
  constexpr int RB = 64;
  __shared__ double s_x[RB * RC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[RC];
#pragma unroll
  for (int c = 0; c < RC; ++c) acc[c] = 0.0;
  for (int i0 = tl.row0; i0 < tl.row1; i0 += RB) {
    const int nr = min(RB, tl.row1 - i0);
    __syncthreads();  // the previous block's reads of s_x are done
    for (int e = threadIdx.x; e < nr * RC; e += BLOCK) s_x[e] = X ? (double)X[(size_t)i0 * RC + e] : v[i0 + e];
    __syncthreads();
    // wave w takes rows w, w + 4, ... of the tile, in order (RB is a
    // multiple of the wave count)
    if (k < rk)
      for (int r = wave; r < nr; r += BLOCK / 64) {
        const double kv = (double)K[(size_t)(i0 + r) * rk + k];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] += kv * s_x[r * RC + c];
      }
  }
  for (int c = 0; c < RC; ++c) {
    s_red[wave][lane] = acc[c];
    __syncthreads();
    if (wave == 0 && k < rk) {
      double t = s_red[0][lane];
      for (int w = 1; w < BLOCK / 64; ++w) t += s_red[w][lane];
      out[(size_t)k * RC + c] = t;
    }
    __syncthreads();
  }
}

template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_lc_kty(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                  int32_t xrole, int32_t vsrc) {
  constexpr int NC = NCh<T>::N;
  constexpr int R = G * NC;
  const Tile tl = tiles[blockIdx.x];
  const InstDev &I = insts[tl.inst];
  const int rk = I.rk;
  if (rk == 0 || (int)blockIdx.y * 64 >= rk) return;  // uniform per block
  const InstParams &P = *I.prm;
  if (vsrc == 1 && P.lz_steps <= 0) return;
  const int k = blockIdx.y * 64 + (threadIdx.x & 63);
  if (vsrc == 0) {
    double *out = I.lc_part + (size_t)tl.lt * rk * R;
    lc_kty_tile<T, R>(tl, I, reinterpret_cast<const T *>(I.Kc), role_ptr<T>(I, P, xrole), nullptr, rk, k, out);
  } else {
    double *out = I.lc_part + (size_t)tl.lt * rk;
    const double *v = vsrc == 1 ? lz_basis(I, P) + (size_t)P.lz_j * I.n : I.lzv;
    lc_kty_tile<double, 1>(tl, I, I.Kc64, nullptr, v, rk, k, out);
  }
}

// sum_ab D_q[a][b] <Y_a, Y_b> over c < R for term q (Y rows of stride ld)
__device__ double lc_quad(const InstDev &I, int q, const double *Y, int ld, int R, int a0, int astep) {
  const int o = I.lc_off[q], rl = I.lc_off[q + 1] - o;
  const double *Dq = I.Dc + I.lc_doff[q];
  double s = 0.0;
  for (int a = a0; a < rl; a += astep)
    for (int c = 0; c < R; ++c) {
      double dy = 0.0;
      for (int b = 0; b < rl; ++b) dy += Dq[(size_t)a * rl + b] * Y[(size_t)(o + b) * ld + c];
      s += Y[(size_t)(o + a) * ld + c] * dy;
    }
  return s;
}

struct LcArgs {
  int32_t mode;   // LcMode
  int32_t R;      // columns of X
  int32_t zsel;   // lc_Z slot
  const double *mult;  // multipliers y_l of the coefficients (null: I.yp)
};

// One 1024-thread block per instance: the fixed-order sum of the tiles'
// partials, then the mode's products.
__global__ __launch_bounds__(RBLOCK) void k_lc_red(const int32_t *__restrict__ ilist, const InstDev *__restrict__ insts,
                                                   LcArgs a) {
  const InstDev &I = insts[ilist[blockIdx.x]];
  const int rk = I.rk;
  if (rk == 0) return;
  const InstParams &P = *I.prm;
  if (a.mode == LC_V_LZ && P.lz_steps <= 0) return;
  const bool vec = a.mode == LC_V_LZ || a.mode == LC_V_FW;
  const int R = vec ? 1 : a.R, ld = vec ? 1 : R_MAX;
  const double *Y = vec ? I.lc_v : I.lc_Y;  // summed over the tiles by k_lc_sum
  if (a.mode == LC_Y_T || a.mode == LC_V_FW) {
    double *out = a.mode == LC_Y_T ? I.lc_T : I.lc_Tv;
    // small terms: one thread each; larger ones: the whole block, in turn
    for (int q = threadIdx.x; q < I.nlc; q += blockDim.x)
      if (I.lc_off[q + 1] - I.lc_off[q] <= 8) out[q] = lc_quad(I, q, Y, ld, R, 0, 1);
    __shared__ double red[RBLOCK / 64];
    __shared__ int s_any;
    // the terms checked a block at a time (one flag per block of terms), so
    // that only blocks holding a larger term are walked term by term
    for (int q0 = 0; q0 < I.nlc; q0 += blockDim.x) {
      if (threadIdx.x == 0) s_any = 0;
      __syncthreads();
      const int qt = q0 + threadIdx.x;
      if (qt < I.nlc && I.lc_off[qt + 1] - I.lc_off[qt] > 8) s_any = 1;
      __syncthreads();
      const bool any = s_any != 0;
      __syncthreads();  // every thread has read the flag before it is reset
      if (!any) continue;
      for (int q = q0; q < min(I.nlc, q0 + (int)blockDim.x); ++q) {
        if (I.lc_off[q + 1] - I.lc_off[q] <= 8) continue;
        double v = wave_sum(lc_quad(I, q, Y, ld, R, threadIdx.x, blockDim.x));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
          double s = 0.0;
          for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
          out[q] = s;
        }
        __syncthreads();
      }
    }
    return;
  }
  // coefficients blockdiag(y_l D_q) Y: lc_Z slot zsel (rk x R, rows of
  // stride R) or lc_zv (vector)
  const double *y = a.mult ? a.mult : I.yp;
  double *Z = vec ? I.lc_zv : I.lc_Z + (size_t)a.zsel * rk * R_MAX;
  for (int q2 = threadIdx.x; q2 < rk * R; q2 += blockDim.x) {
    const int k = q2 / R, c = q2 - (q2 / R) * R;
    const int q = I.lc_term[k];
    const int o = I.lc_off[q], rl = I.lc_off[q + 1] - o, ai = k - o;
    const double *Dq = I.Dc + I.lc_doff[q];
    double s = 0.0;
    for (int b = 0; b < rl; ++b) s += Dq[(size_t)ai * rl + b] * Y[(size_t)(o + b) * ld + c];
    Z[(size_t)k * R + c] = y[I.lc_con[q] - 1] * s;
  }
}

// K^T X (or K^T v) summed over the tiles: a wave per 8 consecutive (k, c)
// entries, its lanes in 8 groups taking every eighth tile (each load reads
// 8 consecutive entries of one tile), then the groups added by a butterfly
// in fixed order.  Many workgroups per instance.
constexpr int LC_QW = 8;
__global__ __launch_bounds__(BLOCK) void k_lc_sum(const int32_t *__restrict__ ilist,
                                                  const InstDev *__restrict__ insts, int32_t R, int32_t vec) {
  const InstDev &I = insts[ilist[blockIdx.x]];
  const int rk = I.rk;
  if (rk == 0) return;
  const InstParams &P = *I.prm;
  if (vec == 1 && P.lz_steps <= 0) return;
  const int Rn = vec ? 1 : R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qq = lane % LC_QW, tq = lane / LC_QW;
  const int q = (blockIdx.y * (BLOCK / 64) + wave) * LC_QW + qq;
  const int total = rk * Rn;
  if ((blockIdx.y * (BLOCK / 64) + wave) * LC_QW >= total) return;  // whole wave
  const int nt = I.ntiles;
  const size_t stride = (size_t)total;
  double s = 0.0;
  if (q < total)
    for (int t = tq; t < nt; t += 64 / LC_QW) s += I.lc_part[(size_t)t * stride + q];
  for (int o = LC_QW; o < 64; o <<= 1) s += shfl_xor(s, o);
  if (tq == 0 && q < total) {
    const int k = q / Rn, c = q - k * Rn;
    if (vec) I.lc_v[k] = s;
    else I.lc_Y[(size_t)k * R_MAX + c] = s;
  }
}

// The constraints' low-rank block of the adjoint, K (blockdiag(y_l D_l) K^T X)
// (Algorithm 5), for the rows of each tile: a wave per row, its lanes over
// the columns k of K (coalesced reads of the row of K), a wave reduction per
// output column.  vec 0: R columns from the Z-slot zsel into lc_W[zsel]
// (rows of stride R), K in the operator type -- launched for R = 2 only, the
// tiled form below takes R >= 4; vec 1: the Lanczos vector's coefficients
// lc_zv into lc_wv, K in FP64.
template <typename T, int R>
__global__ __launch_bounds__(BLOCK) void k_lc_kz(const Tile *__restrict__ tiles, const InstDev *__restrict__ insts,
                                                 int32_t zsel, int32_t vec) {
  const Tile tl = tiles[blockIdx.x];
  const InstDev &I = insts[tl.inst];
  const int rk = I.rk;
  if (rk == 0) return;
  const InstParams &P = *I.prm;
  if (vec && P.lz_steps <= 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = tl.row0 + wave; i < tl.row1; i += BLOCK / 64) {
    double acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = 0.0;
    if (vec) {
      const double *__restrict__ Krow = I.Kc64 + (size_t)i * rk;
      for (int k = lane; k < rk; k += 64) acc[0] += Krow[k] * I.lc_zv[k];
    } else {
      const T *__restrict__ Krow = reinterpret_cast<const T *>(I.Kc) + (size_t)i * rk;
      const double *__restrict__ Z = I.lc_Z + (size_t)zsel * rk * R_MAX;
#pragma unroll 4
      for (int k = lane; k < rk; k += 64) {
        const double kv = (double)Krow[k];
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] += kv * Z[(size_t)k * R + c];
      }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = wave_sum(acc[c]);
    if (lane == 0) {
      if (vec) I.lc_wv[i] = acc[0];
      else
#pragma unroll
        for (int c = 0; c < R; ++c) I.lc_W[zsel][(size_t)i * R + c] = acc[c];
    }
  }
}

// The same two contractions tiled through LDS, so that a row of X or of Z
// is read once per block of rows rather than once per row.  K^T X for wide
// factors (R >= 16) per tile: the block's rows of X staged in LDS, lane =
// column k of K, wave = a group of R/4 output columns (no cross-wave sums),
// each (k, c) summed over the tile's rows in row order; into
// lc_part[tile][k][c] as above.
template <typename T, int R>
__global__ __launch_bounds__(BLOCK) void k_lc_kty_wide(const Tile *__restrict__ tiles,
                                                       const InstDev *__restrict__ insts, int32_t xrole) {
  static_assert(R >= 16 && R % (BLOCK / 64) == 0, "wide factors only");
  constexpr int CW = R / (BLOCK / 64);
  constexpr int RB = 64;
  __shared__ double sX[RB * R];
  const Tile tl = tiles[blockIdx.x];
  const InstDev &I = insts[tl.inst];
  const int rk = I.rk;
  if (rk == 0 || (int)blockIdx.y * 64 >= rk) return;  // uniform per block
  const InstParams &P = *I.prm;
  const T *__restrict__ K = reinterpret_cast<const T *>(I.Kc);
  const T *__restrict__ X = role_ptr<T>(I, P, xrole);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = blockIdx.y * 64 + lane;
  double acc[CW];
#pragma unroll
  for (int j = 0; j < CW; ++j) acc[j] = 0.0;
  for (int i0 = tl.row0; i0 < tl.row1; i0 += RB) {
    const int nr = min(RB, tl.row1 - i0);
    __syncthreads();  // the previous block's reads of sX are done
    for (int e = threadIdx.x; e < nr * R; e += BLOCK) sX[e] = (double)X[(size_t)i0 * R + e];
    __syncthreads();
    if (k < rk) {
#pragma unroll 4
      for (int r = 0; r < nr; ++r) {
        const double kv = (double)K[(size_t)(i0 + r) * rk + k];
#pragma unroll
        for (int j = 0; j < CW; ++j) acc[j] += kv * sX[r * R + wave * CW + j];
      }
    }
  }
  if (k < rk) {
    double *out = I.lc_part + (size_t)tl.lt * rk * R + (size_t)k * R + wave * CW;
#pragma unroll
    for (int j = 0; j < CW; ++j) out[j] = acc[j];
  }
}

// K Z for R >= 4 columns: per block of 64 rows of the tile, the columns of
// K in chunks of 32 -- the chunk of K (transposed, padded) and the matching
// 32 rows of Z staged in LDS -- lane = row, wave = a group of R/4 output
// columns, each output summed over k in order; into lc_W[zsel].  (A wave per
// row re-read all of Z, rk x R, from the L2 for every row of K: 244 KB per
// row at R = 8.)
template <typename T, int R>
__global__ __launch_bounds__(BLOCK) void k_lc_kz_tiled(const Tile *__restrict__ tiles,
                                                      const InstDev *__restrict__ insts, int32_t zsel) {
  static_assert(R >= 4 && R % (BLOCK / 64) == 0, "four or more columns");
  constexpr int CW = R / (BLOCK / 64);
  constexpr int RB = 64, KC = 32;
  __shared__ double sK[KC * (RB + 1)];
  __shared__ double sZ[KC * R];
  const Tile tl = tiles[blockIdx.x];
  const InstDev &I = insts[tl.inst];
  const int rk = I.rk;
  if (rk == 0) return;
  const T *__restrict__ K = reinterpret_cast<const T *>(I.Kc);
  const double *__restrict__ Z = I.lc_Z + (size_t)zsel * rk * R_MAX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i0 = tl.row0; i0 < tl.row1; i0 += RB) {
    const int nr = min(RB, tl.row1 - i0);
    double acc[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) acc[j] = 0.0;
    for (int k0 = 0; k0 < rk; k0 += KC) {
      const int kn = min(KC, rk - k0);
      __syncthreads();  // the previous chunk's reads are done
      // K[i0 + rr][k0 + kk] -> sK[kk][rr]: consecutive threads read along a row of K
      for (int e = threadIdx.x; e < RB * KC; e += BLOCK) {
        const int rr = e / KC, kk = e - rr * KC;
        sK[kk * (RB + 1) + rr] = (rr < nr && kk < kn) ? (double)K[(size_t)(i0 + rr) * rk + k0 + kk] : 0.0;
      }
      for (int e = threadIdx.x; e < kn * R; e += BLOCK) sZ[e] = Z[(size_t)k0 * R + e];
      __syncthreads();
      for (int kk = 0; kk < kn; ++kk) {
        const double kv = sK[kk * (RB + 1) + lane];
#pragma unroll
        for (int j = 0; j < CW; ++j) acc[j] += kv * sZ[kk * R + wave * CW + j];
      }
    }
    if (lane < nr) {
      double *o = I.lc_W[zsel] + (size_t)(i0 + lane) * R + wave * CW;
#pragma unroll
      for (int j = 0; j < CW; ++j) o[j] = acc[j];
    }
  }
}

// Parameters of a standalone operator call, passed by value as the kernel's
// argument (captured when the launch is enqueued, so nothing host-side has to
// stay unchanged until the stream reaches it).
__global__ void k_put_params(InstParams *dst, InstParams v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = v;
}
template <typename T, int G>
static void l_lc_kty(hipStream_t s, const Tile *t, int nt, const InstDev *d, int ncg, int xrole, int vsrc) {
  hipLaunchKernelGGL((k_lc_kty<T, G>), dim3(nt, ncg), dim3(BLOCK), 0, s, t, d, xrole, vsrc);
}
void op_lc_kty(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int max_rk, int xrole, int vsrc) {
  if (nt <= 0 || max_rk <= 0) return;
  const int ncg = (max_rk + 63) / 64;
  if (vsrc == 0 && R >= 16) {
    switch (R) {
#define HL_KTYW(RR)                                                                                              \
  case RR:                                                                                                     \
    if (is64(prec)) hipLaunchKernelGGL((k_lc_kty_wide<double, RR>), dim3(nt, ncg), dim3(BLOCK), 0, s, t, d, xrole); \
    else hipLaunchKernelGGL((k_lc_kty_wide<float, RR>), dim3(nt, ncg), dim3(BLOCK), 0, s, t, d, xrole);            \
    return;
      HL_KTYW(16) HL_KTYW(32) HL_KTYW(64)
#undef HL_KTYW
      default: break;
    }
  }
  if (vsrc != 0) R = is64(prec) ? 2 : 4;  // the vector forms read FP64 K and v: any instantiation
  if (is64(prec)) HL_DISPATCH_G(double, R, l_lc_kty, s, t, nt, d, ncg, xrole, vsrc);
  else HL_DISPATCH_G(float, R, l_lc_kty, s, t, nt, d, ncg, xrole, vsrc);
}
void op_lc_sum(hipStream_t s, const int32_t *ilist, int ni, const InstDev *d, int max_rk, int R, int vec) {
  if (ni <= 0 || max_rk <= 0) return;
  const int Rn = vec ? 1 : R;
  const int per_block = (BLOCK / 64) * LC_QW;
  hipLaunchKernelGGL(k_lc_sum, dim3(ni, (max_rk * Rn + per_block - 1) / per_block), dim3(BLOCK), 0, s, ilist, d, R,
                     vec);
}
template <typename T, int R>
static void l_lc_kz(hipStream_t s, const Tile *t, int nt, const InstDev *d, int zsel, int vec) {
  hipLaunchKernelGGL((k_lc_kz<T, R>), dim3(nt), dim3(BLOCK), 0, s, t, d, zsel, vec);
}
void op_lc_kz(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int zsel, int vec) {
  if (nt <= 0) return;
  if (vec) {
    l_lc_kz<double, 1>(s, t, nt, d, 0, 1);
    return;
  }
  switch (R) {
#define HL_KZ(RR)                                                  \
  case RR:                                                         \
    if (is64(prec)) l_lc_kz<double, RR>(s, t, nt, d, zsel, 0);     \
    else l_lc_kz<float, RR>(s, t, nt, d, zsel, 0);                 \
    break;
#define HL_KZW(RR)                                                                                            \
  case RR:                                                                                                  \
    if (is64(prec)) hipLaunchKernelGGL((k_lc_kz_tiled<double, RR>), dim3(nt), dim3(BLOCK), 0, s, t, d, zsel); \
    else hipLaunchKernelGGL((k_lc_kz_tiled<float, RR>), dim3(nt), dim3(BLOCK), 0, s, t, d, zsel);            \
    break;
    HL_KZ(2) HL_KZW(4) HL_KZW(8) HL_KZW(16) HL_KZW(32) HL_KZW(64)
#undef HL_KZ
#undef HL_KZW
    default: break;
  }
}
void op_lc_red(hipStream_t s, const int32_t *ilist, int ni, const InstDev *d, int mode, int R, int zsel,
               const double *mult) {
  if (ni <= 0) return;
  LcArgs a{mode, R, zsel, mult};
  hipLaunchKernelGGL(k_lc_red, dim3(ni), dim3(RBLOCK), 0, s, ilist, d, a);
}
// ---------------------------------------------------------------------------
// Coded-diffraction constraints (Section 5.4, eq. phase retrieval SDP) on the
// real form, n = 2 nc: constraint l nc + k is sum_c |(F (d_l * u_c))_k|^2
// with u_c = X[0:nc, c] + i X[nc:n, c] and F the unitary DFT; the adjoint
// block is sum_l conj(d_l) * F^H (y_l * F (d_l * u_c)), split back into
// real and imaginary rows.  The transforms run in rocFFT, unnormalised both
// ways; the 1/nc of the unitary pair is applied by k_cdp_abs2 / k_cdp_scale.
// Launched per instance (the instance's FFT plans are its own).
// ---------------------------------------------------------------------------
// S[(l Rc + c) nc + j] = d_l[j] u_c[j] for the first Rc columns (the ones
// that can be nonzero: the iterate's rank; the rest of the bucket's R are
// zero).  vsrc 0: role xrole, rows of stride R; 1: the Lanczos vector v_j
// (zeros once the instance takes no more steps); 2: the Ritz vector lzv
// (R = Rc = 1 for both vector forms).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cdp_pack(const InstDev *__restrict__ insts, int s, int xrole, int vsrc,
                                                    int R, int Rc) {
  const InstDev &I = insts[s];
  const InstParams &P = *I.prm;
  const int nc = I.cdp_nc;
  const size_t total = (size_t)I.cdp_L * Rc * nc;
  const bool idle = vsrc == 1 && P.lz_steps <= 0;
  const T *__restrict__ X = vsrc == 0 ? role_ptr<T>(I, P, xrole) : nullptr;
  const double *__restrict__ v = vsrc == 1 ? lz_basis(I, P) + (size_t)P.lz_j * I.n : I.lzv;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t t = e / nc;
    const int j = (int)(e - t * nc), c = (int)(t % Rc), l = (int)(t / Rc);
    double re = 0.0, im = 0.0;
    if (!idle) {
      if (vsrc == 0) {
        re = (double)X[(size_t)j * R + c];
        im = (double)X[(size_t)(nc + j) * R + c];
      } else {
        re = v[j];
        im = v[nc + j];
      }
    }
    const double2 d = I.cdp_d[(size_t)l * nc + j];
    I.cdp_S[e] = make_double2(d.x * re - d.y * im, d.x * im + d.y * re);
  }
}

// The same packing for the columns of a role (vsrc 0), through LDS: a
// workgroup takes CDP_TJ consecutive rows and CDP_CW columns, reads the
// rows' real and imaginary halves with coalesced loads (each row's columns
// are contiguous), and writes, for every mask and column, CDP_TJ consecutive
// spectra entries (the transforms' contiguous layout).
constexpr int CDP_TJ = 64, CDP_CW = 16;
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cdp_pack_cols(const InstDev *__restrict__ insts, int s, int xrole, int R,
                                                         int Rc) {
  __shared__ double s_re[CDP_TJ][CDP_CW + 1], s_im[CDP_TJ][CDP_CW + 1];
  const InstDev &I = insts[s];
  const InstParams &P = *I.prm;
  const int nc = I.cdp_nc, L = I.cdp_L;
  const int j0 = blockIdx.x * CDP_TJ, c0 = blockIdx.y * CDP_CW;
  const int tj = min(CDP_TJ, nc - j0), cw = min(CDP_CW, Rc - c0);
  const T *__restrict__ X = role_ptr<T>(I, P, xrole);
  for (int t = threadIdx.x; t < CDP_TJ * CDP_CW; t += BLOCK) {
    const int jj = t / CDP_CW, cc = t - jj * CDP_CW;
    if (jj < tj && cc < cw) {
      s_re[jj][cc] = (double)X[(size_t)(j0 + jj) * R + c0 + cc];
      s_im[jj][cc] = (double)X[(size_t)(nc + j0 + jj) * R + c0 + cc];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < L * CDP_CW * CDP_TJ; t += BLOCK) {
    const int jj = t % CDP_TJ, q = t / CDP_TJ, cc = q % CDP_CW, l = q / CDP_CW;
    if (jj >= tj || cc >= cw) continue;
    const double2 d = I.cdp_d[(size_t)l * nc + j0 + jj];
    const double re = s_re[jj][cc], im = s_im[jj][cc];
    I.cdp_S[((size_t)l * Rc + c0 + cc) * nc + j0 + jj] = make_double2(d.x * re - d.y * im, d.x * im + d.y * re);
  }
}

// out[l nc + k] = sum_c |S[(l Rc + c) nc + k]|^2 / nc, c in column order
// (out 0: the constraint values cdp_T; 1: the Frank-Wolfe vector's cdp_Tv)
__global__ __launch_bounds__(BLOCK) void k_cdp_abs2(const InstDev *__restrict__ insts, int s, int Rc, int out) {
  const InstDev &I = insts[s];
  const int nc = I.cdp_nc;
  const size_t total = (size_t)I.cdp_L * nc;
  double *__restrict__ o = out ? I.cdp_Tv : I.cdp_T;
  const double inv = 1.0 / (double)nc;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t l = e / nc, k = e - l * nc;
    const double2 *__restrict__ S = I.cdp_S + l * Rc * nc + k;
    double acc = 0.0;
    for (int c = 0; c < Rc; ++c) {
      const double2 z = S[(size_t)c * nc];
      acc += z.x * z.x + z.y * z.y;
    }
    o[e] = acc * inv;
  }
}

// S2 = S * y_{l nc + k} / nc with the multipliers y (null: the instance's y')
__global__ __launch_bounds__(BLOCK) void k_cdp_scale(const InstDev *__restrict__ insts, int s, int Rc,
                                                     const double *__restrict__ mult) {
  const InstDev &I = insts[s];
  const int nc = I.cdp_nc;
  const size_t total = (size_t)I.cdp_L * Rc * nc;
  const double *__restrict__ y = mult ? mult : I.yp;
  const double inv = 1.0 / (double)nc;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t t = e / nc, k = e - t * nc, l = t / Rc;
    const double f = y[l * nc + k] * inv;
    const double2 z = I.cdp_S[e];
    I.cdp_S2[e] = make_double2(z.x * f, z.y * f);
  }
}

// sum_l conj(d_l[j]) S2[(l Rc + c) nc + j], l in order, into row j (real
// part) and row nc + j (imaginary part), column c < Rc of the adjoint block;
// columns Rc..R-1 are zero (vec 0: cdp_W[zsel], rows of stride R; vec 1: the
// Lanczos vector's cdp_wv, R = Rc = 1)
__global__ __launch_bounds__(BLOCK) void k_cdp_gather(const InstDev *__restrict__ insts, int s, int R, int Rc,
                                                      int zsel, int vec) {
  const InstDev &I = insts[s];
  const int nc = I.cdp_nc, L = I.cdp_L;
  const size_t total = (size_t)R * nc;
  double *__restrict__ W = vec ? I.cdp_wv : I.cdp_W[zsel];
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t c = e / nc, j = e - c * nc;
    double re = 0.0, im = 0.0;
    if ((int)c < Rc)
      for (int l = 0; l < L; ++l) {
        const double2 d = I.cdp_d[(size_t)l * nc + j];
        const double2 z = I.cdp_S2[((size_t)l * Rc + c) * nc + j];
        re += d.x * z.x + d.y * z.y;
        im += d.x * z.y - d.y * z.x;
      }
    W[j * R + c] = re;
    W[(nc + j) * R + c] = im;
  }
}

// The gather for a block of columns (vec 0), through LDS: a workgroup takes
// CDP_TJ rows and CDP_CW of the bucket's R columns, forms the sums with
// coalesced reads of S2 (rows fastest), and writes the block's rows of W
// with coalesced stores; columns from Rc on are zero.
__global__ __launch_bounds__(BLOCK) void k_cdp_gather_cols(const InstDev *__restrict__ insts, int s, int R, int Rc,
                                                           int zsel) {
  __shared__ double s_re[CDP_TJ][CDP_CW + 1], s_im[CDP_TJ][CDP_CW + 1];
  const InstDev &I = insts[s];
  const int nc = I.cdp_nc, L = I.cdp_L;
  const int j0 = blockIdx.x * CDP_TJ, c0 = blockIdx.y * CDP_CW;
  const int tj = min(CDP_TJ, nc - j0), cw = min(CDP_CW, R - c0);
  for (int t = threadIdx.x; t < CDP_TJ * CDP_CW; t += BLOCK) {
    const int jj = t % CDP_TJ, cc = t / CDP_TJ;
    const int j = j0 + jj, c = c0 + cc;
    double re = 0.0, im = 0.0;
    if (jj < tj && c < Rc)
      for (int l = 0; l < L; ++l) {
        const double2 d = I.cdp_d[(size_t)l * nc + j];
        const double2 z = I.cdp_S2[((size_t)l * Rc + c) * nc + j];
        re += d.x * z.x + d.y * z.y;
        im += d.x * z.y - d.y * z.x;
      }
    s_re[jj][cc] = re;
    s_im[jj][cc] = im;
  }
  __syncthreads();
  double *__restrict__ W = I.cdp_W[zsel];
  for (int t = threadIdx.x; t < CDP_TJ * CDP_CW; t += BLOCK) {
    const int jj = t / CDP_CW, cc = t - jj * CDP_CW;
    if (jj < tj && cc < cw) {
      W[(size_t)(j0 + jj) * R + c0 + cc] = s_re[jj][cc];
      W[(size_t)(nc + j0 + jj) * R + c0 + cc] = s_im[jj][cc];
    }
  }
}

static unsigned cdp_grid(size_t total) {
  const size_t g = (total + BLOCK - 1) / BLOCK;
  return (unsigned)std::max<size_t>(1, std::min<size_t>(g, 16384));
}
void op_cdp_pack(int prec, hipStream_t st, const InstDev *d, int s, int xrole, int vsrc, int R, int Rc,
                 size_t total, int nc) {
  if (vsrc == 0) {
    const dim3 grid((nc + CDP_TJ - 1) / CDP_TJ, (Rc + CDP_CW - 1) / CDP_CW);
    if (is64(prec)) hipLaunchKernelGGL(k_cdp_pack_cols<double>, grid, dim3(BLOCK), 0, st, d, s, xrole, R, Rc);
    else hipLaunchKernelGGL(k_cdp_pack_cols<float>, grid, dim3(BLOCK), 0, st, d, s, xrole, R, Rc);
    return;
  }
  if (is64(prec) || vsrc != 0)
    hipLaunchKernelGGL(k_cdp_pack<double>, dim3(cdp_grid(total)), dim3(BLOCK), 0, st, d, s, xrole, vsrc, R, Rc);
  else
    hipLaunchKernelGGL(k_cdp_pack<float>, dim3(cdp_grid(total)), dim3(BLOCK), 0, st, d, s, xrole, vsrc, R, Rc);
}
void op_cdp_abs2(hipStream_t st, const InstDev *d, int s, int Rc, int out, size_t total) {
  hipLaunchKernelGGL(k_cdp_abs2, dim3(cdp_grid(total)), dim3(BLOCK), 0, st, d, s, Rc, out);
}
void op_cdp_scale(hipStream_t st, const InstDev *d, int s, int Rc, const double *mult, size_t total) {
  hipLaunchKernelGGL(k_cdp_scale, dim3(cdp_grid(total)), dim3(BLOCK), 0, st, d, s, Rc, mult);
}
void op_cdp_gather(hipStream_t st, const InstDev *d, int s, int R, int Rc, int zsel, int vec, size_t total, int nc) {
  if (!vec) {
    const dim3 grid((nc + CDP_TJ - 1) / CDP_TJ, (R + CDP_CW - 1) / CDP_CW);
    hipLaunchKernelGGL(k_cdp_gather_cols, grid, dim3(BLOCK), 0, st, d, s, R, Rc, zsel);
    return;
  }
  hipLaunchKernelGGL(k_cdp_gather, dim3(cdp_grid(total)), dim3(BLOCK), 0, st, d, s, R, Rc, zsel, vec);
}

void op_put_params(hipStream_t s, InstParams *dst, const InstParams &v) {
  hipLaunchKernelGGL(k_put_params, dim3(1), dim3(64), 0, s, dst, v);
}
void op_lz_start(hipStream_t s, const Tile *t, int nt, const InstDev *d) {
  if (nt > 0) hipLaunchKernelGGL(k_lz_start, dim3(nt), dim3(BLOCK), 0, s, t, d);
}
void op_lz_first(hipStream_t s, const Tile *t, int nt, const InstDev *d) {
  if (nt > 0) hipLaunchKernelGGL(k_lz_first, dim3(nt), dim3(BLOCK), 0, s, t, d);
}
void op_lz_spmv_dots(hipStream_t s, const Tile *t, int nt, const InstDev *d) {
  if (nt > 0) hipLaunchKernelGGL(k_lz_spmv_dots, dim3(nt), dim3(BLOCK), 0, s, t, d);
}
void op_lz_update(hipStream_t s, const Tile *t, int nt, const InstDev *d, int final_pass) {
  if (nt > 0) hipLaunchKernelGGL(k_lz_update, dim3(nt), dim3(BLOCK), 0, s, t, d, final_pass);
}
void op_lz_scale(hipStream_t s, const Tile *t, int nt, const InstDev *d) {
  if (nt > 0) hipLaunchKernelGGL(k_lz_scale, dim3(nt), dim3(BLOCK), 0, s, t, d);
}
void op_lz_combine(hipStream_t s, const Tile *t, int nt, const InstDev *d, int to_lzv) {
  if (nt > 0) hipLaunchKernelGGL(k_lz_combine, dim3(nt), dim3(BLOCK), 0, s, t, d, to_lzv);
}

// ---------------------------------------------------------------------------
// Allocation-free evaluation of A~(UU^T): its scratch (descriptor copy,
// parameters, result scalars, partial sums, packed U, general-mode per-pair
// and per-constraint vectors) lives in one file-scope device array per GPU,
// held until the process ends.  Host code never passes the array's name to
// a kernel: it takes the device address once per device from
// hipGetSymbolAddress and uses that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void **ptr) {
  static std::mutex mu;
  static void *addr[NOALLOC_MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = q;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// One thread copies the handle's descriptor and parameters into the scratch
// and points every buffer the evaluation writes at the scratch.
__global__ void k_noalloc_setup(const InstDev *__restrict__ src, int s, NoallocViews v) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  InstDev I = src[s];
  InstParams P = *I.prm;
  P.beta = 0.0;
  P.buf[RU] = v.u_ext ? NBUF : 0;
  P.ext[0] = const_cast<void *>(v.u_ext);
  I.prm = v.prm;
  I.res = v.res;
  I.part = v.part;
  I.prows = v.prows;
  I.buf[0] = v.ubuf;
  I.Z0 = v.Z0;
  if (!I.direct) {
    I.TY = v.TY;
    I.yp = v.yp;
    I.Bpair = v.Bpair;
  }
  for (int q = 0; q < NRES; ++q) v.res->v[q] = 0.0;
  *v.prm = P;
  v.insts[s] = I;
}
void op_noalloc_setup(hipStream_t st, const InstDev *src, int s, const NoallocViews &v) {
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(64), 0, st, src, s, v);
}

}  // namespace hl
