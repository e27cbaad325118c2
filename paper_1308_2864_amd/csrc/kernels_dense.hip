// Tall-skinny dense products of the Stiefel step (Section 3), FP64 on the matrix cores.
//
//  * Gram blocks  [A^T A, A^T B, B^T B]  of two n x p blocks (A = X, B = G or D): the
//    "X^T G" products of the gradient (eq. (def-nablaE)), of Y^T Y for the Cholesky QR
//    (Alg. 2) and of V^T U for the Cayley/SMW system (eq. (WY3)).
//  * Combine  out = C0 + X A + Y B  with small p x p weights: the retraction update
//    X+ = X A + D B (QR) or X A + G B (WY), and the gradient D = G - X (G^T X).
//    Fused epilogues: the density of the new block, and the Frobenius sums of the
//    Barzilai-Borwein step (eq. (bb-1)) and of ||grad E||_F.
//
// Both use v_mfma_f64_16x16x4f64: per wavefront a 16x16 FP64 tile accumulates the
// product of a 16x4 and a 4x16 fragment, one element per lane:
//   A fragment: lane l holds A[l % 16][l / 16]
//   B fragment: lane l holds B[l / 16][l % 16]
//   C/D tile:   lane l, register r holds D[(l / 16) + 4 r][l % 16]
// (for the FP64 variant each 64-bit register holds the rows congruent to l / 16 mod 4).
// Columns beyond p and rows beyond n are read as zero, so any p and ld work; the small
// matrices are padded to pp = round_up(p, 16).  All sums use a fixed order (per-lane,
// then fixed-order cross-wave and cross-block reductions), so results are bitwise
// reproducible run to run.
#include <algorithm>
#include <cstring>

#include <hip/hip_ext.h>
#include <type_traits>

#include "ks_common.h"

namespace ks {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGramMaxChunks = 512;
// One resident wave of blocks on 256 CUs at three blocks per CU keeps every wavefront
// streaming several 16-row tiles (measured against 256 - 4096 blocks on a 64^3 grid).
constexpr int kCombineMaxBlocks = 512;

// Product bits of a Gram launch: A^T A, A^T B, B^T B.  Symmetric products store only the
// tiles ti <= tj; the reduction mirrors them.
constexpr int kPAA = 1, kPAB = 2, kPBB = 4;

template <int kT, int kMask>
struct GramTiles {
  static constexpr int kSym = kT * (kT + 1) / 2;
  static constexpr int kAll = kT * kT;
  static constexpr int kN = ((kMask & kPAA) ? kSym : 0) + ((kMask & kPAB) ? kAll : 0) +
                            ((kMask & kPBB) ? kSym : 0);
};

// Fixed-order sum of one 16x16 tile over the four waves of a block: waves 1..3 park it in
// LDS (6 KiB) and wave 0 adds them in wave order.
__device__ inline void wave_reduce_tile(d4& v, double* lds, int w, int lane) {
  if (w > 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) lds[((w - 1) * 4 + r) * 64 + lane] = v[r];
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int ww = 0; ww < 3; ++ww)
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] += lds[(ww * 4 + r) * 64 + lane];
  }
  __syncthreads();
}

// Writes the tile (ti, tj) of product prod of this block's partial (wave 0 only).
template <int kPP>
__device__ inline void put_tile(double* part, int blk, int prod, int ti, int tj, const d4& v,
                                int lr, int lc) {
  double* o = part + ((size_t)blk * 3 + prod) * kPP * kPP;
#pragma unroll
  for (int r = 0; r < 4; ++r) o[(ti * 16 + lr + 4 * r) * kPP + tj * 16 + lc] = v[r];
}

// ---- Gram: per-chunk partials -------------------------------------------------------
template <typename T, int kT, int kMask>
__device__ inline void k_gram_body(const GramArgs<T>& ka, int ks_bid, int ks_nb) {
  const T* __restrict__ A = ka.A;
  const T* __restrict__ B = ka.B;
  int ld = ka.ld;
  int n = ka.n;
  int p = ka.p;
  const int pb = ka.pb ? ka.pb : ka.p;  // columns of B (a sub-block of a wider block)
  double* __restrict__ part = ka.part;
  (void)ks_bid;
  (void)ks_nb;

  constexpr int kPP = kT * 16;
  constexpr int kAcc = GramTiles<kT, kMask>::kN;
  extern __shared__ double lds[];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  const int chunk = ks_bid, nchunks = ks_nb;
  const int ngroups = (n + 3) / 4;
  const int per = (ngroups + nchunks - 1) / nchunks;
  const int g_beg = chunk * per, g_end = min(ngroups, g_beg + per);

  d4 acc[kAcc];
#pragma unroll
  for (int t = 0; t < kAcc; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  // Software pipeline over batches of kU row groups: the loads of the next batch
  // (branch-free, clamped addresses) are issued before the products of the current one,
  // so memory and matrix cores overlap.  The accumulation order per wavefront (groups
  // g_beg + w, + 4, + 8, ...) is that of one group at a time.
  constexpr int kU = kT <= 2 ? 4 : 2;
  // raw storage values: converting at load time would wait for the loads of the next
  // batch before the products of the current one
  struct Batch {
    T a[kU][kT], b[kU][kT];
  };
  auto load = [&](Batch& f, int grp0) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int row = (grp0 + 4 * u) * 4 + lr;
      const bool rok = grp0 + 4 * u < g_end && row < n;
      const size_t roff = (size_t)(rok ? row : 0) * ld;
#pragma unroll
      for (int t = 0; t < kT; ++t) {
        const int col = t * 16 + lc;
        const bool ok = rok && col < p, okb = rok && col < pb;
        const size_t idx = ok ? roff + col : 0, idxb = okb ? roff + col : 0;
        f.a[u][t] = ok ? A[idx] : T(0);
        f.b[u][t] = T(0);
        if (kMask & (kPAB | kPBB)) f.b[u][t] = okb ? B[idxb] : T(0);
      }
    }
  };
  auto products = [&](const Batch& f, int grp0) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (grp0 + 4 * u >= g_end) break;
      double fa[kT], fb[kT];
#pragma unroll
      for (int t = 0; t < kT; ++t) {
        fa[t] = (double)f.a[u][t];
        fb[t] = (double)f.b[u][t];
      }
      int a = 0;
      if (kMask & kPAA) {
#pragma unroll
        for (int ti = 0; ti < kT; ++ti)
#pragma unroll
          for (int tj = ti; tj < kT; ++tj, ++a) acc[a] = mfma16(fa[ti], fa[tj], acc[a]);
      }
      if (kMask & kPAB) {
#pragma unroll
        for (int ti = 0; ti < kT; ++ti)
#pragma unroll
          for (int tj = 0; tj < kT; ++tj, ++a) acc[a] = mfma16(fa[ti], fb[tj], acc[a]);
      }
      if (kMask & kPBB) {
#pragma unroll
        for (int ti = 0; ti < kT; ++ti)
#pragma unroll
          for (int tj = ti; tj < kT; ++tj, ++a) acc[a] = mfma16(fb[ti], fb[tj], acc[a]);
      }
    }
  };
  constexpr int kStep = 4 * kU;  // groups per batch of one wavefront
  int grp0 = g_beg + w;
  Batch f0, f1;
  if (grp0 < g_end) load(f0, grp0);
  while (grp0 < g_end) {
    if (grp0 + kStep < g_end) load(f1, grp0 + kStep);
    products(f0, grp0);
    grp0 += kStep;
    if (grp0 >= g_end) break;
    if (grp0 + kStep < g_end) load(f0, grp0 + kStep);
    products(f1, grp0);
    grp0 += kStep;
  }
#pragma unroll
  for (int t = 0; t < kAcc; ++t) wave_reduce_tile(acc[t], lds, w, lane);
  if (w == 0) {
    int a = 0;
    if (kMask & kPAA) {
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = ti; tj < kT; ++tj) put_tile<kPP>(part, chunk, 0, ti, tj, acc[a++], lr, lc);
    }
    if (kMask & kPAB) {
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = 0; tj < kT; ++tj) put_tile<kPP>(part, chunk, 1, ti, tj, acc[a++], lr, lc);
    }
    if (kMask & kPBB) {
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = ti; tj < kT; ++tj) put_tile<kPP>(part, chunk, 2, ti, tj, acc[a++], lr, lc);
    }
  }
}

template <typename T, int kT, int kMask>
__global__ __launch_bounds__(256) void k_gram(GramArgs<T> ka) {
  k_gram_body<T, kT, kMask>(ka, blockIdx.x, gridDim.x);
}

template <typename T, int kT, int kMask>
__global__ __launch_bounds__(256) void k_gram_batch(BatchPtrs<GramArgs<T>> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_gram_body<T, kT, kMask>(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// out[prod][i][j] = sum over the chunk partials, for the products in mask; the other
// products are left untouched.  Block = kRedCols consecutive entries of one row of one
// product x kRedGroups chunk groups: a wavefront's load covers whole 128-byte lines of
// four chunks.  Group g sums chunks g, g + kRedGroups, ... (loaded kRedU at a time, all in
// flight together) and the group sums are added in group order, so the result is the same
// on every run.  Symmetric products are summed on their upper 16 x 16 tiles (and the
// diagonal tiles) and written to both mirrored places.  With W != nullptr also
// W = -(product 1)^T.
constexpr int kRedCols = 16;
constexpr int kRedGroups = 64;
constexpr int kRedU = 8;

__device__ inline void k_gram_reduce_body(const GramReduceArgs& ka, int ks_bid, int ks_nb) {
  const int pp = ka.pp, nchunks = ka.nchunks;
  (void)ks_nb;
  const int per = pp * pp;
  const int e0 = ks_bid * kRedCols;  // first entry of the block (pp is a multiple of 16)
  if (e0 >= 3 * per) return;
  const int prod = e0 / per, ij0 = e0 % per, i = ij0 / pp, j0 = ij0 % pp;
  if (!((ka.mask >> prod) & 1)) return;
  const bool sym = prod != 1;
  if (sym && i / 16 > j0 / 16) return;  // a lower tile: written as the mirror
  __shared__ double red[kRedGroups][kRedCols + 1];
  const int c = threadIdx.x % kRedCols, g = threadIdx.x / kRedCols;
  const double* __restrict__ q = ka.part + (size_t)prod * per + ij0 + c;
  const size_t cs = (size_t)3 * per;
  double sum = 0.0;
  const bool formula = prod == 1 && ka.xd_xx != nullptr;  // X^T G + (X^T X) W, group g: k = g
  if (formula && g < pp) sum = ka.xd_xx[i * pp + g] * ka.xd_W[g * pp + j0 + c];
  for (int c0 = g; !formula && c0 < nchunks; c0 += kRedGroups * kRedU) {
    double v[kRedU];
#pragma unroll
    for (int u = 0; u < kRedU; ++u) {
      const int ch = c0 + kRedGroups * u;
      v[u] = q[(size_t)(ch < nchunks ? ch : 0) * cs];
    }
#pragma unroll
    for (int u = 0; u < kRedU; ++u)
      if (c0 + kRedGroups * u < nchunks) sum += v[u];
  }
  red[g][c] = sum;
  __syncthreads();
  if (g == 0) {
    double t = 0.0;
    for (int k = 0; k < kRedGroups; ++k) t += red[k][c];
    const int j = j0 + c;
    if (formula) t += ka.xd_xg[i * pp + j];
    double* out = ka.out + (size_t)prod * per;
    out[i * pp + j] = t;
    if (sym && i / 16 < j / 16) out[j * pp + i] = t;
    if (ka.W && prod == 1) ka.W[j * pp + i] = -t;
  }
}

__global__ __launch_bounds__(kRedCols * kRedGroups) void k_gram_reduce(GramReduceArgs ka) {
  k_gram_reduce_body(ka, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kRedCols * kRedGroups) void k_gram_reduce_batch(
    BatchPtrs<GramReduceArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_gram_reduce_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// ---- combine ------------------------------------------------------------------------
// out[g][:] = C0[g][:] + X[g][:] A + Y[g][:] B  (A, B: pp x pp, staged in LDS).
//
// The product is formed transposed, out^T = A^T X^T, so that the rows of X enter the
// matrix cores as B fragments (lane l holds X[row l % 16][k]) and the result tile comes
// back one grid row per lane as well.  The contraction index k and the output column
// are both free to be permuted (the weights in LDS are permuted to match), which is used
// to give every operand and the result one common register layout:
//   lane (q = l / 16, c = l % 16) of a wavefront owning rows g0 .. g0 + 15 holds row
//   g0 + c, columns 8 j + 2 q + e (j < 2 kT, e < 2): element s = 2 j + e.
// Each lane therefore reads and writes column pairs (one 16-byte load or store for FP64
// when p and ld are even), four lanes cover 64 contiguous bytes of a row, and X, C0, Xk
// and Dk are each read exactly once.  For MFMA step s (contraction indices
// k(s, q) = 8 (s >> 1) + 2 q + (s & 1)) the B fragment is element s of X; the A fragment
// of output tile t is Wp[4 s + q][16 t + c] with Wp[4 s + q][16 t + m] = A[k(s, q)][16 t +
// pi(m)], pi(m) = 8 (m >> 3) + 2 (m & 3) + ((m >> 2) & 1); register r of output tile t is
// then element 4 t + r.  Each wavefront owns 16-row tiles.  Epilogues:
//   kRho   density of out (row sums across the four lanes of a row),
//   kGrad  out is D = grad E; Frobenius sums ||D||^2 and the BB sums against (Xk, Dk).
template <int kT>
struct CombineFrag {
  static constexpr int kE = 4 * kT;  // elements per lane
  double v[kE];
};

__device__ inline int comb_col(int s, int q) { return 8 * (s >> 1) + 2 * q + (s & 1); }

// Loads the lane's elements of rows g0 + c (zero outside n x p).  kVec: column pairs as
// one load (p, ld even, 2-element aligned base).
// kNT: a stream read here for the last time (non-temporal: it should not displace blocks
// the next kernels read again from the last-level cache)
template <typename T, int kT, bool kVec, bool kNT = false>
__device__ inline void comb_load(const T* __restrict__ base, int ld, int n, int p, int row,
                                 int q, CombineFrag<kT>& f) {
  const bool rok = row < n;
  const size_t roff = (size_t)(rok ? row : 0) * ld;
#pragma unroll
  for (int j = 0; j < 2 * kT; ++j) {
    const int c0 = 8 * j + 2 * q;
    if constexpr (kVec) {
      const bool ok = rok && c0 < p;
      typedef T t2 __attribute__((ext_vector_type(2)));
      const t2* src = reinterpret_cast<const t2*>(base + (ok ? roff + c0 : 0));
      t2 w;
      if constexpr (kNT) w = __builtin_nontemporal_load(src);
      else w = *src;
      f.v[2 * j] = ok ? (double)w[0] : 0.0;
      f.v[2 * j + 1] = ok ? (double)w[1] : 0.0;
    } else {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const bool ok = rok && c0 + e < p;
        const T w = base[ok ? roff + c0 + e : 0];
        f.v[2 * j + e] = ok ? (double)w : 0.0;
      }
    }
  }
}

// Permuted weights Wp = [A; B] (kK x kPP) into LDS.
template <int kT, bool kHasY>
__device__ inline void comb_stage(const CombineArgs& a, double* lds) {
  constexpr int kPP = kT * 16;
  constexpr int kK = kHasY ? 2 * kPP : kPP;
  const int lda = a.lda ? a.lda : kPP;  // row stride of A and B (a sub-block of larger weights)
  const int pk = a.pk ? a.pk : a.p;
  lds_stage<kK * kPP / kBlock>(
      kK * kPP,
      [&](int e) {
        const int r = e / kPP, col = e % kPP;
        const int rr = r % kPP, s = rr >> 2, qq = rr & 3;
        const int t = col >> 4, m = col & 15;
        const int kr = comb_col(s, qq), kc = 16 * t + 8 * (m >> 3) + 2 * (m & 3) + ((m >> 2) & 1);
        // rows past the contraction width and columns past the output width are zero
        // (a sub-block of wider weights may end inside the tile)
        const bool ok = kr < pk && kc < a.p;
        const int src = ok ? kr * lda + kc : 0;
        const double v = (kHasY && r >= kPP) ? a.B[src] : a.A[src];
        return ok ? v : 0.0;
      },
      [&](int e, double v) { lds[e] = v; });
}

// The first tile's loads are issued before the weights are staged, so they overlap the
// staging and the barrier.
// Gram tiles accumulated by the gradient combine with kGram2: X^T D (kT^2 tiles) and the
// upper tiles of D^T D.
template <int kT>
struct Gram2Acc {
  static constexpr int kN = kT * kT + kT * (kT + 1) / 2;
  d4 t[kN];
};

template <typename T, int kT, bool kVec, bool kHasY, bool kHasC0, bool kRho, bool kGrad,
          bool kGram2, bool kUpper, bool kBBR>
__device__ inline void combine_tiles(const CombineArgs& a, double* lds, int t_beg, int t_end,
                                     d4& sums, Gram2Acc<kT>& g2) {
  const T* aX = static_cast<const T*>(a.X);
  const T* aY = static_cast<const T*>(a.Y);
  const T* aC0 = static_cast<const T*>(a.C0);
  const T* aXk = static_cast<const T*>(a.Xk);
  const T* aDk = static_cast<const T*>(a.Dk);
  T* aout = static_cast<T*>(a.out);
  constexpr int kPP = kT * 16;
  constexpr int kS = 4 * kT;  // MFMA steps per operand (= elements per lane)
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int q = lane / 16, c = lane % 16;
  const int ld = a.ld, p = a.p, n = a.n;
  const int pk = a.pk ? a.pk : a.p;  // columns of X and Y (the contraction) to read

  // operands of one tile (v0: the warm start and its six neighbours at the lane's row)
  struct Tile {
    CombineFrag<kT> x, y, c0, xk, dk;
    double v0[7];
  };
  const bool resid = kRho && a.resid != nullptr;
  auto load_v0 = [&](Tile& f, int row) {
    // x0 at row and its neighbours in the order of the Laplacian's sum (-x, +x, -y, +y,
    // -z, +z); a neighbour outside the grid is not summed (zero Dirichlet values)
    const int r = row < n ? row : n - 1;
    const int nx = a.gnx, ny = a.gny, sy = nx, sz = nx * ny;
    const int i = r % nx, j = (r / nx) % ny, k = r / sz;
    const double* x0 = a.resid_x0;
    f.v0[0] = x0[r];
    f.v0[1] = i > 0 ? x0[r - 1] : 0.0;
    f.v0[2] = i < nx - 1 ? x0[r + 1] : 0.0;
    f.v0[3] = j > 0 ? x0[r - sy] : 0.0;
    f.v0[4] = j < ny - 1 ? x0[r + sy] : 0.0;
    f.v0[5] = k > 0 ? x0[r - sz] : 0.0;
    f.v0[6] = k < a.gnz - 1 ? x0[r + sz] : 0.0;
  };
  auto load = [&](Tile& f, int tile) {
    const int row = tile * 16 + c;
    comb_load<T, kT, kVec>(aX, ld, n, pk, row, q, f.x);
    if constexpr (kHasY) comb_load<T, kT, kVec>(aY, ld, n, pk, row, q, f.y);
    // the gradient form reads G, X_k and D_k for the last time in the trial
    if constexpr (kHasC0) comb_load<T, kT, kVec, kGrad>(aC0, ld, n, p, row, q, f.c0);
    if constexpr (kGrad) {
      if constexpr (!kBBR) comb_load<T, kT, kVec, true>(aXk, ld, n, p, row, q, f.xk);
      comb_load<T, kT, kVec, true>(aDk, ld, n, p, row, q, f.dk);
    }
    if constexpr (kRho) {
      if (resid) load_v0(f, row);
    }
  };
  auto compute = [&](const Tile& f, int tile) {
    const int row = tile * 16 + c;
    d4 acc[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    // kUpper: A and B are upper triangular (the QR weights R^{-1}, -tau R^{-1}), so output
    // tile t only needs the steps whose rows 8 (s >> 1) .. + 7 reach its columns
    // 16 t .. 16 t + 15, i.e. s < 4 (t + 1); the skipped products are exact zeros.
#pragma unroll
    for (int s = 0; s < kS; ++s) {
#pragma unroll
      for (int t = 0; t < kT; ++t)
        if (!kUpper || s < 4 * (t + 1))
          acc[t] = mfma16(lds[(4 * s + q) * kPP + t * 16 + c], f.x.v[s], acc[t]);
    }
    if constexpr (kHasY) {
#pragma unroll
      for (int s = 0; s < kS; ++s) {
#pragma unroll
        for (int t = 0; t < kT; ++t)
          if (!kUpper || s < 4 * (t + 1))
            acc[t] = mfma16(lds[kPP * kPP + (4 * s + q) * kPP + t * 16 + c], f.y.v[s], acc[t]);
      }
    }
    const bool rok = row < n;
    const size_t roff = (size_t)(rok ? row : 0) * ld;
    double sq = 0.0;
    double dv[kS];  // the stored values (kGram2)
#pragma unroll
    for (int j = 0; j < 2 * kT; ++j) {
      double v[2];
      bool ok[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int s = 2 * j + e;
        ok[e] = rok && comb_col(s, q) < p;
        double x = acc[s / 4][s % 4];
        if constexpr (kHasC0) x += f.c0.v[s];
        x = ok[e] ? (double)(T)x : 0.0;  // the epilogues see the stored value
        v[e] = x;
        dv[s] = x;
        if constexpr (kRho) sq += x * x;
        if constexpr (kGrad && kBBR) {
          sums[0] += x * x;
          sums[3] += f.dk.v[s] * x;  // <D_k, D_t>
        } else if constexpr (kGrad) {
          const double sd = f.x.v[s] - f.xk.v[s];
          const double yd = x - f.dk.v[s];
          sums[0] += x * x;
          sums[1] += sd * sd;
          sums[2] += sd * yd;
          sums[3] += yd * yd;
        } else if constexpr (kHasY && !kHasC0) {
          if (a.bbr) {  // the retraction's part of the BB sums: s = X_t - X_k, <s, D_k>
            const double sd = x - f.x.v[s];
            sums[1] += sd * sd;
            sums[2] += sd * f.y.v[s];
          }
        }
      }
      const int c0 = 8 * j + 2 * q;
      if constexpr (kVec) {
        typedef T t2 __attribute__((ext_vector_type(2)));
        if (ok[0]) {
          t2 o;
          o[0] = (T)v[0];
          o[1] = (T)v[1];
          *reinterpret_cast<t2*>(aout + roff + c0) = o;
        }
      } else {
        if (ok[0]) aout[roff + c0] = (T)v[0];
        if (ok[1]) aout[roff + c0 + 1] = (T)v[1];
      }
    }
    if constexpr (kRho) {
      sq += __shfl_xor(sq, 16, kWave);
      sq += __shfl_xor(sq, 32, kWave);
      const double rv = a.rho_scale * sq;
      if (q == 0 && rok) a.rho[row] = rv;
      if (resid && q == 0 && rok) {
        // b - L x0 with the CG start's arithmetic: b = 4 pi rhs_scale rho,
        // L x0 = (6 x0 - sum of neighbours) / h^2
        // (a neighbour outside the grid was loaded as 0.0, and adding it changes no sum)
        const double* v = f.v0;
        double nb = 0.0;
#pragma unroll
        for (int e = 1; e < 7; ++e) nb += v[e];
        const double b = 4.0 * kPi * a.rhs_scale * rv;
        a.resid[row] = b - (6.0 * v[0] - nb) * a.inv_h2;
      }
    }
    if constexpr (kGram2) {
      // X^T D and D^T D of the tile: the grid rows must be the contraction index, so the
      // X and D tiles go through a wavefront-private LDS patch (row stride kPP + 1) and come
      // back as Gram fragments (lane l: row 4 kk + l / 16, column 16 t + l % 16).
      constexpr int kGS = kPP + 1;
      double* xs = lds + (kHasY ? 2 : 1) * kPP * kPP + w * 2 * 16 * kGS;
      double* ds = xs + 16 * kGS;
#pragma unroll
      for (int s2 = 0; s2 < kS; ++s2) {
        if constexpr (!kBBR) xs[c * kGS + comb_col(s2, q)] = f.x.v[s2];
        ds[c * kGS + comb_col(s2, q)] = dv[s2];
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        double fa[kT], fd[kT];
#pragma unroll
        for (int t = 0; t < kT; ++t) {
          if constexpr (!kBBR) fa[t] = xs[(4 * kk + q) * kGS + 16 * t + c];
          fd[t] = ds[(4 * kk + q) * kGS + 16 * t + c];
        }
        int g = 0;
        // kBBR: X^T D is formed from X^T G, X^T X and W by the reduction instead
        if constexpr (!kBBR) {
#pragma unroll
          for (int ti = 0; ti < kT; ++ti)
#pragma unroll
            for (int tj = 0; tj < kT; ++tj, ++g) g2.t[g] = mfma16(fa[ti], fd[tj], g2.t[g]);
        } else {
          g = kT * kT;
        }
#pragma unroll
        for (int ti = 0; ti < kT; ++ti)
#pragma unroll
          for (int tj = ti; tj < kT; ++tj, ++g) g2.t[g] = mfma16(fd[ti], fd[tj], g2.t[g]);
      }
    }
  };

  int tile = t_beg + w;
  Tile f0;
  if (tile < t_end) load(f0, tile);
  comb_stage<kT, kHasY>(a, lds);
  __syncthreads();
  for (; tile < t_end; tile += 4) {
    if (tile > t_beg + w) load(f0, tile);
    compute(f0, tile);
  }
}

template <typename T, int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad,
          bool kGram2 = false, bool kUpper = false, bool kBBR = false>
__device__ inline void k_combine_body(const CombineArgs& a, int ks_bid, int ks_nb) {
  extern __shared__ double lds[];            // permuted weights Wp = [A; B]: kK x kPP
  __shared__ double sh[kBlock / kWave];

  const int ntiles = (a.n + 15) / 16;
  const int lb = xcd_remap(ks_bid, ks_nb);
  const int per = (ntiles + ks_nb - 1) / ks_nb;
  const int t_beg = lb * per, t_end = min(ntiles, t_beg + per);
  // column pairs can be moved as one load or store when every block is pair-aligned
  constexpr uintptr_t kAl = 2 * sizeof(T) - 1;
  const bool vec = ((a.ld | a.p | a.pk) & 1) == 0 &&
                   ((reinterpret_cast<uintptr_t>(a.X) | reinterpret_cast<uintptr_t>(a.Y) |
                     reinterpret_cast<uintptr_t>(a.C0) | reinterpret_cast<uintptr_t>(a.out) |
                     reinterpret_cast<uintptr_t>(a.Xk) | reinterpret_cast<uintptr_t>(a.Dk)) &
                    kAl) == 0;
  d4 sums = {0.0, 0.0, 0.0, 0.0};
  Gram2Acc<kT> g2;
#pragma unroll
  for (int t = 0; t < Gram2Acc<kT>::kN; ++t) g2.t[t] = d4{0.0, 0.0, 0.0, 0.0};
  if (vec)
    combine_tiles<T, kT, true, kHasY, kHasC0, kRho, kGrad, kGram2, kUpper, kBBR>(a, lds, t_beg, t_end, sums,
                                                                   g2);
  else
    combine_tiles<T, kT, false, kHasY, kHasC0, kRho, kGrad, kGram2, kUpper, kBBR>(a, lds, t_beg, t_end, sums,
                                                                    g2);
  if constexpr (kGram2) {
    // fixed-order sum over the block's waves, then this block's partial tiles (chunk lb)
    constexpr int kPP = kT * 16;
    double* red = lds + (kHasY ? 2 : 1) * kPP * kPP;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    __syncthreads();  // every wave is done with its LDS patch
#pragma unroll
    for (int t = kBBR ? kT * kT : 0; t < Gram2Acc<kT>::kN; ++t)
      wave_reduce_tile(g2.t[t], red, w, lane);
    if (w == 0) {
      const int lr = lane / 16, lc = lane % 16;
      int g = 0;
      if constexpr (!kBBR) {
#pragma unroll
        for (int ti = 0; ti < kT; ++ti)
#pragma unroll
          for (int tj = 0; tj < kT; ++tj)
            put_tile<kPP>(a.gram_part, lb, 1, ti, tj, g2.t[g++], lr, lc);
      } else {
        g = kT * kT;
      }
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = ti; tj < kT; ++tj) put_tile<kPP>(a.gram_part, lb, 2, ti, tj, g2.t[g++], lr, lc);
    }
  }
  // the block sums with one barrier (block_sum_n: each in block_sum's order)
  __shared__ double shn[4 * (kBlock / kWave)];
  if (kGrad && kBBR) {
    double v[2] = {sums[0], sums[3]};
    block_sum_n<2>(v, shn);
    if (threadIdx.x == 0) {
      const int st = a.pt.stride;
      a.pt.buf[(size_t)SL_DD * st + lb] = v[0];
      a.pt.buf[(size_t)SL_YY * st + lb] = v[1];
    }
  } else if (kGrad) {
    double v[4] = {sums[0], sums[1], sums[2], sums[3]};
    block_sum_n<4>(v, shn);
    if (threadIdx.x == 0) {
      const int st = a.pt.stride;
      a.pt.buf[(size_t)SL_DD * st + lb] = v[0];
      a.pt.buf[(size_t)SL_SS * st + lb] = v[1];
      a.pt.buf[(size_t)SL_SY * st + lb] = v[2];
      a.pt.buf[(size_t)SL_YY * st + lb] = v[3];
    }
  } else if (kHasY && !kHasC0 && a.bbr) {
    double v[2] = {sums[1], sums[2]};
    block_sum_n<2>(v, shn);
    if (threadIdx.x == 0) {
      const int st = a.pt.stride;
      a.pt.buf[(size_t)SL_SS * st + lb] = v[0];
      a.pt.buf[(size_t)SL_SY * st + lb] = v[1];
    }
  }
  (void)sh;
}

template <typename T, int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad,
          bool kGram2 = false, bool kUpper = false, bool kBBR = false>
__global__ __launch_bounds__(256) void k_combine(CombineArgs a) {
  k_combine_body<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2, kUpper, kBBR>(a, blockIdx.x, gridDim.x);
}

template <typename T, int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad,
          bool kGram2 = false, bool kUpper = false, bool kBBR = false>
__global__ __launch_bounds__(256) void k_combine_batch(BatchPtrs<CombineArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_combine_body<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2, kUpper, kBBR>(batch_arg(b, s), blockIdx.x - b.off[s],
                                                            b.off[s + 1] - b.off[s]);
}

// LDS of a combine block: the weights, and with kGram2 the wavefronts' X and D patches (the
// Gram reduction reuses them).
template <int kT, bool kHasY, bool kGram2>
constexpr size_t combine_lds_bytes() {
  constexpr size_t kPP = kT * 16;
  return ((kHasY ? 2 : 1) * kPP * kPP + (kGram2 ? 4 * 2 * 16 * (kPP + 1) : 0)) * sizeof(double);
}

void set_lds_attr(const void* k, size_t bytes) {
  if (bytes > 32768) set_dyn_lds_once(k, (int)bytes);
}

template <typename T, int kT, int kMask>
void launch_gram_m(const T* A, const T* B, int ld, int n, int p, double* part, int nchunks,
                   hipStream_t st) {
  const size_t lds = (size_t)3 * 4 * 64 * sizeof(double);
  hipLaunchKernelGGL((k_gram<T, kT, kMask>), dim3(nchunks), dim3(256), lds, st,
                     GramArgs<T>{A, B, ld, n, p, part});
}

// Up to 32 columns all requested products run in one pass; wider blocks run one product
// per pass to bound the accumulator registers.
template <typename T, int kT>
void launch_gram_t(const T* A, const T* B, int ld, int n, int p, int mask, double* part,
                   int nchunks, hipStream_t st) {
  if constexpr (kT <= 2) {
    if (mask == (kPAA | kPAB | kPBB))
      return launch_gram_m<T, kT, 7>(A, B, ld, n, p, part, nchunks, st);
    if (mask == (kPAA | kPAB)) return launch_gram_m<T, kT, 3>(A, B, ld, n, p, part, nchunks, st);
    if (mask == (kPAB | kPBB)) return launch_gram_m<T, kT, 6>(A, B, ld, n, p, part, nchunks, st);
  }
  if (mask & kPAA) launch_gram_m<T, kT, 1>(A, B, ld, n, p, part, nchunks, st);
  if (mask & kPAB) launch_gram_m<T, kT, 2>(A, B, ld, n, p, part, nchunks, st);
  if (mask & kPBB) launch_gram_m<T, kT, 4>(A, B, ld, n, p, part, nchunks, st);
}

// set_launch_events: per host thread, consumed by the next single-kernel combine launch
thread_local hipEvent_t g_launch_start = nullptr, g_launch_stop = nullptr;

template <typename T, int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad,
          bool kGram2 = false, bool kUpper = false, bool kBBR = false>
void launch_combine_t(const CombineArgs& a, hipStream_t st) {
  constexpr size_t lds = combine_lds_bytes<kT, kHasY, kGram2>();
  // function-local static initialisation runs once even when several host threads launch
  static const bool attr = (set_lds_attr(reinterpret_cast<const void*>(
                                k_combine<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2, kUpper, kBBR>),
                                lds),
                            true);
  (void)attr;
  if (g_launch_start) {
    // the dispatch itself records the events: the kernel's own start and end
    hipEvent_t e0 = g_launch_start, e1 = g_launch_stop;
    g_launch_start = g_launch_stop = nullptr;
    hipExtLaunchKernelGGL((k_combine<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2, kUpper, kBBR>),
                          dim3(combine_blocks(a.n)), dim3(256), (std::uint32_t)lds, st, e0, e1,
                          0u, a);
    return;
  }
  hipLaunchKernelGGL((k_combine<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2, kUpper, kBBR>),
                     dim3(combine_blocks(a.n)), dim3(256), lds, st, a);
}

template <typename T, int kT>
void launch_combine_tt(const CombineArgs& a, hipStream_t st) {
  const bool y = a.Y != nullptr, c0 = a.C0 != nullptr, rho = a.rho != nullptr,
             gr = a.Xk != nullptr;
  // the combinations the library uses
  if (y && !c0 && rho && !gr && a.upper)
    return launch_combine_t<T, kT, true, false, true, false, false, true>(a, st);
  if (y && !c0 && rho && !gr) return launch_combine_t<T, kT, true, false, true, false>(a, st);
  if (y && !c0 && !rho && !gr) return launch_combine_t<T, kT, true, false, false, false>(a, st);
  if constexpr (kT <= 2) {
    if constexpr (std::is_same<T, double>::value) {
      if (!y && c0 && !rho && gr && a.gram_part && a.bbr)
        return launch_combine_t<T, kT, false, true, false, true, true, false, true>(a, st);
    }
    if (!y && c0 && !rho && gr && a.gram_part)
      return launch_combine_t<T, kT, false, true, false, true, true>(a, st);
  }
  if (!y && c0 && !rho && gr) return launch_combine_t<T, kT, false, true, false, true>(a, st);
  if (!y && c0 && !rho && !gr) return launch_combine_t<T, kT, false, true, false, false>(a, st);
  if (!y && !c0 && rho && !gr) return launch_combine_t<T, kT, false, false, true, false>(a, st);
  if (y && c0 && !rho && !gr) return launch_combine_t<T, kT, true, true, false, false>(a, st);
  launch_combine_t<T, kT, false, false, false, false>(a, st);
}

template <typename T>
void launch_combine_p(const CombineArgs& a, hipStream_t st) {
  const int pp = round_up(a.p, 16);
  switch (pp / 16) {
    case 1: launch_combine_tt<T, 1>(a, st); break;
    case 2: launch_combine_tt<T, 2>(a, st); break;
    case 3: launch_combine_tt<T, 3>(a, st); break;
    case 4: launch_combine_tt<T, 4>(a, st); break;
    default: break;
  }
}

template <typename T>
void launch_gram_p(const T* A, const T* B, int ld, int n, int p, int mask, double* partials,
                   int nchunks, hipStream_t st) {
  const int pp = round_up(p, 16);
  switch (pp / 16) {
    case 1: launch_gram_t<T, 1>(A, B, ld, n, p, mask, partials, nchunks, st); break;
    case 2: launch_gram_t<T, 2>(A, B, ld, n, p, mask, partials, nchunks, st); break;
    case 3: launch_gram_t<T, 3>(A, B, ld, n, p, mask, partials, nchunks, st); break;
    case 4: launch_gram_t<T, 4>(A, B, ld, n, p, mask, partials, nchunks, st); break;
    default: break;
  }
}

}  // namespace

int gram_chunks(int n, int pp) {
  (void)pp;
  int c = (n + 63) / 64;
  if (c > kGramMaxChunks) c = kGramMaxChunks;
  return c < 1 ? 1 : c;
}

// partial tiles of the Gram launches and of the gradient combine's fused Gram tiles (blocks
// wider than 64 columns: the partial 128 x 128 tiles of the wide Gram)
size_t wide_gram_part_doubles(int n);

size_t gram_part_doubles(int n, int pp) {
  const size_t w = std::min(pp, 64);
  const size_t sub = (size_t)std::max(gram_chunks(n, pp), combine_blocks(n)) * 3 * w * w;
  return pp > 64 ? std::max(sub, wide_gram_part_doubles(n)) : sub;
}

void launch_gram(const void* A, const void* B, bool f32, int ld, int n, int p, int mask,
                 double* partials, int nchunks, hipStream_t st) {
  if (f32)
    launch_gram_p<float>(static_cast<const float*>(A), static_cast<const float*>(B), ld, n, p,
                         mask, partials, nchunks, st);
  else
    launch_gram_p<double>(static_cast<const double*>(A), static_cast<const double*>(B), ld, n, p,
                          mask, partials, nchunks, st);
}

void launch_gram_reduce(const double* partials, int nchunks, int pp, int mask, double* out,
                        double* W, hipStream_t st, const double* xd_xg, const double* xd_xx,
                        const double* xd_W) {
  hipLaunchKernelGGL(k_gram_reduce, dim3(gram_reduce_blocks(pp)), dim3(kRedCols * kRedGroups), 0,
                     st,
                     GramReduceArgs{partials, nchunks, pp, mask, out, W, xd_xg, xd_xx, xd_W});
}

int combine_blocks(int n) {
  int tiles = (n + 15) / 16;
  int b = (tiles + 3) / 4;
  if (b > kCombineMaxBlocks) b = kCombineMaxBlocks;
  return b < 1 ? 1 : b;
}


// ---- blocks wider than 64 columns ------------------------------------------------------
// Output tiles of 128 x 128, so that every operand value loaded feeds 128 products (the
// 64-column products feed 64, which leaves a p = 512 product bound by HBM).
//
// Gram: one launch forms every requested product.  Block b owns one output tile of one
// product over one chunk of grid rows; its four wavefronts own the four 64 x 64 quarters
// of the tile and walk the same rows (4 per MFMA step).  The partial tiles are summed over
// the chunks in a fixed order by a second kernel, which also mirrors the symmetric
// products (only their tiles I <= J are formed) and writes W = -(A^T B)^T.
//
// Combine: persistent blocks.  A unit is one row tile (128 grid rows) times one output
// column tile; block g takes one unit per round.  Within a round the units of one row tile
// sit on the same XCD (blocks g = x mod 8 share XCD x), so a row of X and Y is fetched from
// HBM about once per round and served to its column tiles from that XCD's L2.  Each
// wavefront owns a 32-row strip of the unit (two 16-row MFMA tiles by eight 16-column
// tiles); the weights go through LDS in slabs of 16 contraction rows x 128 columns, double
// buffered, one barrier per slab.  The contraction index of MFMA step s in lane group q is
// comb_col(s, q), so each lane reads column pairs of its row.
constexpr int kWT = 128;             // edge of an output tile
constexpr int kWK = 16;              // contraction rows of a combine weight slab
constexpr int kWideResident = 512;   // blocks of a wide launch (two per CU)
constexpr int kWideMaxTiles = 48;    // 3 products x 4 x 4 tiles (p <= 512)

struct WideGramArgs {
  const void* A;
  const void* B;
  int ld, n, p;
  int nch, ntiles;
  double* part;  // [nch][ntiles][128][128]
  signed char tp[kWideMaxTiles], ti[kWideMaxTiles], tj[kWideMaxTiles];
};

typedef float fx4 __attribute__((ext_vector_type(4)));

__device__ inline fx4 mfma16f(float a, float b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// FP32 matrix-core combine (kMc, float storage only): the MFMA sums run in fp32 over a
// chain of 64 contraction indices and are added into FP64 accumulators after it, so a
// rounding error is at most (64 + 4) 2^-24 of the chain's sum of |products|.  The fp32
// result tile is laid out as lane l, register r = row 4 (l / 16) + r, column l % 16 (the
// FP64 tile has row l / 16 + 4 r).  (An fp32 Gram with FP64 chain sums was measured
// slower than the FP64 one on float data: its FP64 accumulators leave too few registers
// for the loads in flight.)
constexpr int kMcSlabs = 4;  // 4 weight slabs = 64 contraction indices per fp32 chain

// The block stages slabs of kGramSlab rows of its two column blocks (L[:, I], R[:, J]:
// 16 x 256 values) in LDS, double buffered: thread t loads column t of every row of the
// next slab (coalesced, 16 loads in flight per thread) while the wavefronts multiply the
// current one from LDS, so a whole slab's MFMA time covers the loads.
constexpr int kGramSlab = 16;

template <typename T>
__global__ __launch_bounds__(256, 2) void k_gram_wide(WideGramArgs a) {
  __shared__ double sl[2][kGramSlab][2 * kWT];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);  // the tiles of one chunk share an XCD
  const int chunk = lb / a.ntiles, tile = lb % a.ntiles;
  const int prod = a.tp[tile];
  const T* __restrict__ L = static_cast<const T*>(prod == 2 ? a.B : a.A);
  const T* __restrict__ R = static_cast<const T*>(prod == 0 ? a.A : a.B);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int q = lane / 16, c = lane % 16;
  const int ld = a.ld, n = a.n, p = a.p;
  const int ngroups = (n + 3) / 4;
  const int per = (ngroups + a.nch - 1) / a.nch;
  const int r_beg = 4 * min(ngroups, chunk * per);
  const int r_end = min(n, 4 * min(ngroups, chunk * per + per));
  const int nslab = (r_end - r_beg + kGramSlab - 1) / kGramSlab;
  // staging: thread t owns slab column t (L side below 128, R side above)
  const int t = threadIdx.x;
  const T* __restrict__ S = t < kWT ? L : R;
  const int scol = (t < kWT ? a.ti[tile] : a.tj[tile]) * kWT + (t % kWT);
  const bool cok = scol < p;
  const int scl = cok ? scol : 0;
  auto load = [&](T (&v)[kGramSlab], int sidx) {
    const int r0 = r_beg + sidx * kGramSlab;
#pragma unroll
    for (int u = 0; u < kGramSlab; ++u) {
      const int row = r0 + u;
      v[u] = S[(size_t)(row < r_end ? row : r_beg) * ld + scl];  // raw, clamped
    }
  };
  auto store = [&](const T (&v)[kGramSlab], int sidx, int buf) {
    const int r0 = r_beg + sidx * kGramSlab;
#pragma unroll
    for (int u = 0; u < kGramSlab; ++u)
      sl[buf][u][t] = (cok && r0 + u < r_end) ? (double)v[u] : 0.0;
  };
  d4 acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  const int li = 64 * (w >> 1) + c, rj = kWT + 64 * (w & 1) + c;
  if (nslab > 0) {
    T v[kGramSlab];
    load(v, 0);
    store(v, 0, 0);
    __syncthreads();
    for (int si = 0; si < nslab; ++si) {
      const int sn = si + 1 < nslab ? si + 1 : si;  // the last slab reloads itself
      load(v, sn);
      __builtin_amdgcn_sched_barrier(0);
      const double(*b)[2 * kWT] = sl[si & 1];
#pragma unroll
      for (int g = 0; g < kGramSlab / 4; ++g) {
        const int row = 4 * g + q;
        double fl[4], fr[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          fl[f] = b[row][li + 16 * f];
          fr[f] = b[row][rj + 16 * f];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[4 * x + y] = mfma16(fl[x], fr[y], acc[4 * x + y]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (si + 1 < nslab) store(v, sn, (si + 1) & 1);
      __syncthreads();
    }
  }
  double* o = a.part + (size_t)lb * kWT * kWT;
  const int r0 = 64 * (w >> 1), c0 = 64 * (w & 1);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        o[(size_t)(r0 + 16 * x + q + 4 * r) * kWT + c0 + 16 * y + c] = acc[4 * x + y][r];
}

// Row chunks of a wide Gram launch: one block per (chunk, tile) and at most
// kWideResident blocks, each chunk at least 16 row groups.
int wide_gram_nch(int n, int ntiles) {
  const int ngroups = (n + 3) / 4;
  const int nch = std::max(1, kWideResident / std::max(1, ntiles));
  return std::min(nch, std::max(1, (ngroups + 15) / 16));
}

size_t wide_gram_part_doubles(int n) {
  const int ngroups = (n + 3) / 4;
  const size_t units = std::min<size_t>(kWideResident,
                                        (size_t)kWideMaxTiles * std::max(1, (ngroups + 15) / 16));
  return std::max<size_t>(units, kWideMaxTiles) * kWT * kWT;
}

struct WideReduceArgs {
  const double* part;
  int nch, ntiles, pp, mask, sym;  // sym: bit per product, only its tiles I <= J exist
  double* out;                     // [3][pp][pp]
  double* W;                       // optional: -(A^T B)^T
  signed char lut[3][4][4];        // tile index of (product, I, J)
};

__global__ __launch_bounds__(256) void k_gram_wide_reduce(WideReduceArgs a) {
  const int pp = a.pp, per = pp * pp;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * per) return;
  const int prod = e / per, ij = e % per, i = ij / pp, j = ij % pp;
  if (!((a.mask >> prod) & 1)) return;
  const bool mir = ((a.sym >> prod) & 1) && i > j;
  const int si = mir ? j : i, sj = mir ? i : j;
  const int tile = a.lut[prod][si / kWT][sj / kWT];
  const double* src = a.part + (size_t)tile * kWT * kWT + (si % kWT) * kWT + sj % kWT;
  const size_t cs = (size_t)a.ntiles * kWT * kWT;
  constexpr int kU = 8;
  double s = 0.0;
  for (int c0 = 0; c0 < a.nch; c0 += kU) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = c0 + u < a.nch ? src[(size_t)(c0 + u) * cs] : 0.0;
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (c0 + u < a.nch) s += v[u];
  }
  a.out[e] = s;
  if (a.W && prod == 1) a.W[(size_t)j * pp + i] = -s;
}

// Two blocks per CU (256 registers per lane) so that one block's epilogue and slab loads
// overlap the other's products; the gradient form (four more operands in its epilogue)
// and the fp32-matrix-core form (fp32 and FP64 accumulators) do not fit and run one
// block per CU.
template <typename T, bool kHasY, bool kHasC0, bool kGrad, bool kVec, bool kMc = false>
__global__ __launch_bounds__(256, (kMc || kGrad) ? 1 : 2) void k_combine_wide(CombineArgs a,
                                                                             int nct) {
  static_assert(!kMc || std::is_same<T, float>::value, "fp32 matrix cores take float data");
  using WT = typename std::conditional<kMc, float, double>::type;  // staged weights
  __shared__ WT wl[2][kWK * kWT];
  __shared__ double sh[kBlock / kWave];
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const T* __restrict__ Y = static_cast<const T*>(a.Y);
  const T* __restrict__ C0 = static_cast<const T*>(a.C0);
  const T* __restrict__ Xk = static_cast<const T*>(a.Xk);
  const T* __restrict__ Dk = static_cast<const T*>(a.Dk);
  T* __restrict__ out = static_cast<T*>(a.out);
  const int ld = a.ld, n = a.n, p = a.p, pp = round_up(p, 16);
  const int pk = a.pk ? a.pk : p, lda = a.lda ? a.lda : pp;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int q = lane / 16, c = lane % 16;
  const int nrt = (n + kWT - 1) / kWT;
  const int G = gridDim.x, xcd = blockIdx.x % kXcds, m = blockIdx.x / kXcds;
  const int R = G / nct;  // row tiles per round (G is a multiple of 8 nct)
  d4 sums = {0.0, 0.0, 0.0, 0.0};

  for (int round = 0; round * R < nrt; ++round) {
    const int rt = round * R + (m / nct) * kXcds + xcd;
    const int J = (m % nct + round) % nct;  // rotates, so upper-triangular work balances
    if (rt >= nrt) continue;
    const int roww = rt * kWT + 32 * w;  // first row of this wavefront's strip
    const int J0 = J * kWT;
    const int kmax = a.upper ? min(pk, J0 + kWT) : pk;
    const int nsx = (kmax + kWK - 1) / kWK;
    const int ns = kHasY ? 2 * nsx : nsx;

    // Operand loads are branch-free and select nothing: a select right after a load makes
    // the compiler wait for it before the products of the current slab.  Rows past n are
    // read from row 0 (their outputs are never stored); columns past the contraction read
    // the row's first element and meet zero weights (finite x 0 = 0).
    auto load_x = [&](T (&dst)[2][4], int si) {
      const T* src = (kHasY && si >= nsx) ? Y : X;
      const int k0 = (si % nsx) * kWK;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int row = roww + 16 * t + c;
        const size_t roff = (size_t)(row < n ? row : 0) * ld;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = k0 + 8 * j + 2 * q;
          if constexpr (kVec) {
            typedef T t2 __attribute__((ext_vector_type(2)));
            const t2 v = *reinterpret_cast<const t2*>(src + roff + (col < pk ? col : 0));
            dst[t][2 * j] = v[0];
            dst[t][2 * j + 1] = v[1];
          } else {
#pragma unroll
            for (int e = 0; e < 2; ++e) dst[t][2 * j + e] = src[roff + (col + e < pk ? col + e : 0)];
          }
        }
      }
    };
    constexpr int kWPer = kWK * kWT / kBlock;  // weight values per thread and slab
    // weights: raw values now, the zero padding is applied when they go to LDS
    auto load_w = [&](double (&dst)[kWPer], int si) {
      const double* src = (kHasY && si >= nsx) ? a.B : a.A;
      const int k0 = (si % nsx) * kWK;
#pragma unroll
      for (int u = 0; u < kWPer; ++u) {
        const int e = threadIdx.x + kBlock * u;
        const int kk = k0 + e / kWT, col = J0 + e % kWT;
        dst[u] = src[kk < pk && col < p ? (size_t)kk * lda + col : 0];
      }
    };
    auto store_w = [&](const double (&src)[kWPer], int si, int buf) {
      const int k0 = (si % nsx) * kWK;
#pragma unroll
      for (int u = 0; u < kWPer; ++u) {
        const int e = threadIdx.x + kBlock * u;
        const bool ok = k0 + e / kWT < pk && J0 + e % kWT < p;
        wl[buf][e] = ok ? (WT)src[u] : WT(0);
      }
    };

    d4 acc[2][8];
    fx4 acc32[2][8];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
        acc32[t][u] = fx4{0.f, 0.f, 0.f, 0.f};
      }
    // Slab si + 1 is loaded while slab si is multiplied.  The loads are unconditional (the
    // last slab reloads itself) so that the compiler can count them exactly and wait only
    // for the older ones; the scheduling barriers keep the loads ahead of the products and
    // the LDS stores and register moves (which wait for the new loads) behind them.
    T xc[2][4];
    {
      double w0[kWPer];
      load_x(xc, 0);
      load_w(w0, 0);
      store_w(w0, 0, 0);
    }
    __syncthreads();
    for (int si = 0; si < ns; ++si) {
      const int sn = si + 1 < ns ? si + 1 : si;
      T xn[2][4];
      double wn[kWPer];
      load_x(xn, sn);
      load_w(wn, sn);
      __builtin_amdgcn_sched_barrier(0);
      const WT* wb = wl[si & 1];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kr = comb_col(s, q);
        WT bw[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) bw[u] = wb[kr * kWT + 16 * u + c];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if constexpr (kMc) {
#pragma unroll
            for (int u = 0; u < 8; ++u) acc32[t][u] = mfma16f(xc[t][s], bw[u], acc32[t][u]);
          } else {
            const double xa = (double)xc[t][s];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[t][u] = mfma16(xa, bw[u], acc[t][u]);
          }
        }
      }
      if constexpr (kMc) {
        // chains end at fixed slabs (and at the last one)
        if ((si + 1) % kMcSlabs == 0 || si + 1 == ns) {
#pragma unroll
          for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[t][u][r] += (double)acc32[t][u][r];
              acc32[t][u] = fx4{0.f, 0.f, 0.f, 0.f};
            }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      store_w(wn, sn, (si + 1) & 1);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) xc[t][e] = xn[t][e];
      __syncthreads();
    }

    // epilogue: lane (q, c), register r of tile (t, u) is row roww + 16 t + q + 4 r
    // (fp32 tiles: + 4 q + r), column J0 + 16 u + c
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = roww + 16 * t + (kMc ? 4 * q + r : q + 4 * r);
        const bool rok = row < n;
        const size_t roff = (size_t)(rok ? row : 0) * ld;
        // the row's operands are all loaded before its first store (a store between loads
        // would make each load wait for the one before)
        T c0v[8], xv[8], xkv[8], dkv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int col = J0 + 16 * u + c;
          const size_t idx = rok && col < p ? roff + col : 0;
          if constexpr (kHasC0) c0v[u] = C0[idx];
          if constexpr (kGrad) {
            xv[u] = X[idx];
            xkv[u] = Xk[idx];
            dkv[u] = Dk[idx];
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int col = J0 + 16 * u + c;
          const bool ok = rok && col < p;
          double x = acc[t][u][r];
          if constexpr (kHasC0) x += (double)c0v[u];
          x = ok ? (double)(T)x : 0.0;  // the epilogue sees the stored value
          if (ok) out[roff + col] = (T)x;
          if constexpr (kGrad) {
            const double sd = ok ? (double)xv[u] - (double)xkv[u] : 0.0;
            const double yd = ok ? x - (double)dkv[u] : 0.0;
            sums[0] += x * x;
            sums[1] += sd * sd;
            sums[2] += sd * yd;
            sums[3] += yd * yd;
          }
        }
      }
  }
  if constexpr (kGrad) {
    const double dd = block_sum(sums[0], sh);
    const double ss = block_sum(sums[1], sh);
    const double sy = block_sum(sums[2], sh);
    const double yy = block_sum(sums[3], sh);
    if (threadIdx.x == 0) {
      const int st = a.pt.stride;
      a.pt.buf[(size_t)SL_DD * st + blockIdx.x] = dd;
      a.pt.buf[(size_t)SL_SS * st + blockIdx.x] = ss;
      a.pt.buf[(size_t)SL_SY * st + blockIdx.x] = sy;
      a.pt.buf[(size_t)SL_YY * st + blockIdx.x] = yy;
    }
  }
}

// Blocks of a wide combine: a multiple of 8 x (column tiles), at most kWideResident, and
// no more row tiles per round than there are.
int wide_combine_grid(int n, int p) {
  const int nct = (round_up(p, 16) + kWT - 1) / kWT;
  const int nrt = (n + kWT - 1) / kWT;
  const int k = std::max(1, std::min(kWideResident / (kXcds * nct), (nrt + kXcds - 1) / kXcds));
  return kXcds * nct * k;
}

template <typename T, bool kHasY, bool kHasC0, bool kGrad, bool kMc>
void launch_combine_wide_m(const CombineArgs& a, hipStream_t st) {
  const int nct = (round_up(a.p, 16) + kWT - 1) / kWT;
  const int G = wide_combine_grid(a.n, a.p);
  constexpr uintptr_t kAl = 2 * sizeof(T) - 1;
  const bool vec = ((a.ld | (a.pk ? a.pk : a.p)) & 1) == 0 &&
                   ((reinterpret_cast<uintptr_t>(a.X) | reinterpret_cast<uintptr_t>(a.Y)) &
                    kAl) == 0;
  if (vec)
    hipLaunchKernelGGL((k_combine_wide<T, kHasY, kHasC0, kGrad, true, kMc>), dim3(G),
                       dim3(kBlock), 0, st, a, nct);
  else
    hipLaunchKernelGGL((k_combine_wide<T, kHasY, kHasC0, kGrad, false, kMc>), dim3(G),
                       dim3(kBlock), 0, st, a, nct);
}

template <typename T, bool kHasY, bool kHasC0, bool kGrad>
void launch_combine_wide_v(const CombineArgs& a, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (a.mc) return launch_combine_wide_m<T, kHasY, kHasC0, kGrad, true>(a, st);
  }
  launch_combine_wide_m<T, kHasY, kHasC0, kGrad, false>(a, st);
}

template <typename T>
void launch_combine_wide(const CombineArgs& a, hipStream_t st) {
  const bool y = a.Y != nullptr, c0 = a.C0 != nullptr, gr = a.Xk != nullptr;
  if (y && !c0 && !gr) launch_combine_wide_v<T, true, false, false>(a, st);
  else if (!y && c0 && gr) launch_combine_wide_v<T, false, true, true>(a, st);
  else if (!y && c0 && !gr) launch_combine_wide_v<T, false, true, false>(a, st);
  else if (y && c0 && !gr) launch_combine_wide_v<T, true, true, false>(a, st);
  else launch_combine_wide_v<T, false, false, false>(a, st);
  if (a.rho)
    launch_density<T>(static_cast<const T*>(a.out), a.ld, a.n, a.p, a.rho_scale, a.rho, st);
}

// The 64-column sub-product path remains for the bf16 products (KS_PREC_MIXED_BF16): their
// matrix cores are fast enough that the re-reads are all the time they take.
constexpr int kSubCols = 64;

__global__ void k_gram_place(const double* __restrict__ sub, double* __restrict__ out, int pp,
                             int i0, int j0, int mirror, double* __restrict__ W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kSubCols * kSubCols) return;
  const int i = e / kSubCols, j = e % kSubCols;
  if (i0 + i >= pp || j0 + j >= pp) return;
  const double v = sub[e];
  out[(size_t)(i0 + i) * pp + j0 + j] = v;
  if (mirror) out[(size_t)(j0 + j) * pp + i0 + i] = v;
  if (W) W[(size_t)(j0 + j) * pp + i0 + i] = -v;
}

int sub_blocks(int p) { return (p + kSubCols - 1) / kSubCols; }

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_launch_start = start;
  g_launch_stop = stop;
}

void launch_combine(const CombineArgs& a, hipStream_t st) {
  if (round_up(a.p, 16) > kSubCols) {
    if (a.f32) launch_combine_wide<float>(a, st);
    else launch_combine_wide<double>(a, st);
    return;
  }
  if (a.f32) launch_combine_p<float>(a, st);
  else launch_combine_p<double>(a, st);
}

int combine_partial_blocks(int n, int p) {
  return round_up(p, 16) > kSubCols ? wide_combine_grid(n, p) : combine_blocks(n);
}

// ---- BF16 Gram sub-product (KS_PREC_MIXED_BF16) ---------------------------------------
// L[:, 0:pa]^T R[:, 0:pb] over one chunk of rows on the bf16 matrix cores (16 x 16 x 16,
// fp32 accumulation); L and R are stored in float and rounded to nearest-even bf16 in
// registers.  Lane l of a wavefront on the rows g0 .. g0 + 15 holds rows g0 + 4 (l / 16) + e
// (e < 4) of column 16 t + l % 16: the A operand of tile t of L^T and the B operand of tile
// t of R alike.  A wavefront sums its 16-row groups in fp32; the four wavefronts are added
// in a fixed order in fp64, and the 64 x 64 tile goes to the slot of the fp64 kernel's
// A^T B partial, so the reduction and placement that follow are shared.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline short bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ __launch_bounds__(256) void k_gram_bf16(GramArgs<float> ka) {
  const float* __restrict__ L = ka.A;
  const float* __restrict__ R = ka.B;
  const int ld = ka.ld, n = ka.n, pa = ka.p, pb = ka.pb ? ka.pb : ka.p;
  extern __shared__ double lds[];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  const int ngroups = (n + 15) / 16;
  const int per = (ngroups + (int)gridDim.x - 1) / (int)gridDim.x;
  const int g_beg = (int)blockIdx.x * per, g_end = min(ngroups, g_beg + per);
  f32x4 acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  struct Raw {
    float a[4][4], b[4][4];  // [tile][row e]
  };
  auto load = [&](Raw& f, int grp) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = grp * 16 + 4 * lr + e;
      const bool rok = grp < g_end && row < n;
      const size_t roff = (size_t)(rok ? row : 0) * ld;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = 16 * t + lc;
        f.a[t][e] = (rok && col < pa) ? L[roff + col] : 0.f;
        f.b[t][e] = (rok && col < pb) ? R[roff + col] : 0.f;
      }
    }
  };
  auto products = [&](const Raw& f) {
    bf16x4 a[4], b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[t][e] = bf16_rne(f.a[t][e]);
        b[t][e] = bf16_rne(f.b[t][e]);
      }
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
        acc[ti * 4 + tj] =
            __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[ti], b[tj], acc[ti * 4 + tj], 0, 0, 0);
  };
  int grp = g_beg + w;
  Raw f0, f1;
  if (grp < g_end) load(f0, grp);
  while (grp < g_end) {
    if (grp + 4 < g_end) load(f1, grp + 4);
    products(f0);
    grp += 4;
    if (grp >= g_end) break;
    if (grp + 4 < g_end) load(f0, grp + 4);
    products(f1);
    grp += 4;
  }
  double* o = ka.part + ((size_t)blockIdx.x * 3 + 1) * kSubCols * kSubCols;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    d4 v = d4{acc[t][0], acc[t][1], acc[t][2], acc[t][3]};
    wave_reduce_tile(v, lds, w, lane);
    if (w == 0) {
      const int ti = t / 4, tj = t % 4;
      // fp32 result layout: register r of lane l is row 4 (l / 16) + r, column l % 16
#pragma unroll
      for (int r = 0; r < 4; ++r) o[(ti * 16 + 4 * lr + r) * kSubCols + tj * 16 + lc] = v[r];
    }
  }
}

template <typename T>
void launch_gram_full_t(const T* A, const T* B, int ld, int n, int p, int mask,
                        double* partials, double* sub, double* out, double* W, hipStream_t st,
                        bool sym_ab, int bf16_mask) {
  const int pp = round_up(p, 16);
  // A^T A and B^T B, and A^T B when the caller knows it is symmetric (X^T B X, D^T B D
  // in the B metric): the tiles I <= J only, mirrored
  const int wide = mask & ~bf16_mask;
  if (wide) {
    WideGramArgs ga{};
    WideReduceArgs ra{};
    std::memset(ra.lut, -1, sizeof(ra.lut));
    const int nb = (pp + kWT - 1) / kWT;
    int nt = 0;
    for (int prod = 0; prod < 3; ++prod) {
      if (!((wide >> prod) & 1)) continue;
      const bool sym = prod != 1 || sym_ab;
      if (sym) ra.sym |= 1 << prod;
      for (int I = 0; I < nb; ++I)
        for (int J = sym ? I : 0; J < nb; ++J) {
          ga.tp[nt] = (signed char)prod;
          ga.ti[nt] = (signed char)I;
          ga.tj[nt] = (signed char)J;
          ra.lut[prod][I][J] = (signed char)nt;
          ++nt;
        }
    }
    ga.A = A;
    ga.B = B;
    ga.ld = ld;
    ga.n = n;
    ga.p = p;
    ga.ntiles = nt;
    ga.nch = wide_gram_nch(n, nt);
    ga.part = partials;
    hipLaunchKernelGGL(k_gram_wide<T>, dim3(ga.nch * nt), dim3(kBlock), 0, st, ga);
    ra.part = partials;
    ra.nch = ga.nch;
    ra.ntiles = nt;
    ra.pp = pp;
    ra.mask = wide;
    ra.out = out;
    ra.W = (wide & kPAB) ? W : nullptr;
    hipLaunchKernelGGL(k_gram_wide_reduce, dim3((3 * pp * pp + kBlock - 1) / kBlock),
                       dim3(kBlock), 0, st, ra);
  }
  if constexpr (std::is_same<T, float>::value) {
    const int nsb = sub_blocks(p), nch = gram_chunks(n, kSubCols);
    const size_t lds = (size_t)3 * 4 * 64 * sizeof(double);
    for (int prod = 0; prod < 3; ++prod) {
      if (!((mask & bf16_mask) >> prod & 1)) continue;
      const float* L = prod == 2 ? B : A;
      const float* R = prod == 0 ? A : B;
      const bool sym = prod != 1 || sym_ab;
      for (int I = 0; I < nsb; ++I)
        for (int J = sym ? I : 0; J < nsb; ++J) {
          const int pa = std::min(kSubCols, p - kSubCols * I);
          const int pb = std::min(kSubCols, p - kSubCols * J);
          hipLaunchKernelGGL(k_gram_bf16, dim3(nch), dim3(256), lds, st,
                             GramArgs<float>{L + kSubCols * I, R + kSubCols * J, ld, n, pa,
                                             partials, pb});
          launch_gram_reduce(partials, nch, kSubCols, kPAB, sub, nullptr, st);
          hipLaunchKernelGGL(k_gram_place, dim3(kSubCols * kSubCols / 256), dim3(256), 0, st,
                             sub + kSubCols * kSubCols, out + (size_t)prod * pp * pp, pp,
                             kSubCols * I, kSubCols * J, sym && I != J ? 1 : 0,
                             prod == 1 ? W : nullptr);
        }
    }
  }
}

void launch_gram_full(const void* A, const void* B, bool f32, int ld, int n, int p, int mask,
                      double* partials, double* sub, double* out, double* W, hipStream_t st,
                      bool sym_ab, int bf16_mask) {
  if (f32)
    launch_gram_full_t<float>(static_cast<const float*>(A), static_cast<const float*>(B), ld, n,
                              p, mask, partials, sub, out, W, st, sym_ab, bf16_mask);
  else
    launch_gram_full_t<double>(static_cast<const double*>(A), static_cast<const double*>(B), ld,
                               n, p, mask, partials, sub, out, W, st, sym_ab, 0);
}

// ---- batched launches ------------------------------------------------------------------

template <typename T>
void launch_gram_batch(const BatchPtrs<GramArgs<T>>& b, int pp, int mask, int blocks,
                       hipStream_t st) {
  const size_t lds = (size_t)3 * 4 * 64 * sizeof(double);
  const bool t1 = pp <= 16;
  if (mask == (kPAA | kPAB)) {
    if (t1) hipLaunchKernelGGL((k_gram_batch<T, 1, 3>), dim3(blocks), dim3(256), lds, st, b);
    else hipLaunchKernelGGL((k_gram_batch<T, 2, 3>), dim3(blocks), dim3(256), lds, st, b);
  } else {
    if (t1) hipLaunchKernelGGL((k_gram_batch<T, 1, 6>), dim3(blocks), dim3(256), lds, st, b);
    else hipLaunchKernelGGL((k_gram_batch<T, 2, 6>), dim3(blocks), dim3(256), lds, st, b);
  }
}
template void launch_gram_batch<double>(const BatchPtrs<GramArgs<double>>&, int, int, int,
                                        hipStream_t);
template void launch_gram_batch<float>(const BatchPtrs<GramArgs<float>>&, int, int, int,
                                       hipStream_t);

int gram_reduce_blocks(int pp) { return 3 * pp * pp / kRedCols; }

void launch_gram_reduce_batch(const BatchPtrs<GramReduceArgs>& b, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_reduce_batch, dim3(blocks), dim3(kRedCols * kRedGroups), 0, st,
                     b);
}

template <typename T, int kT>
void combine_batch_retract_t(const BatchPtrs<CombineArgs>& b, int blocks, hipStream_t st) {
  constexpr size_t lds = combine_lds_bytes<kT, true, false>();
  // batches run the QR retraction: upper triangular weights
  hipLaunchKernelGGL((k_combine_batch<T, kT, true, false, true, false, false, true>),
                     dim3(blocks), dim3(256), lds, st, b);
}

// FP64 batches take the BB sums without X_k (CombineArgs::bbr), as lone FP64 runs do
template <typename T, int kT>
void combine_batch_grad_t(const BatchPtrs<CombineArgs>& b, int blocks, hipStream_t st) {
  constexpr size_t lds = combine_lds_bytes<kT, false, true>();
  constexpr bool kB = std::is_same<T, double>::value;
  static const bool attr =
      (set_lds_attr(reinterpret_cast<const void*>(
                        k_combine_batch<T, kT, false, true, false, true, true, false, kB>),
                    lds),
       true);
  (void)attr;
  hipLaunchKernelGGL((k_combine_batch<T, kT, false, true, false, true, true, false, kB>),
                     dim3(blocks), dim3(256), lds, st, b);
}

template <typename T>
void launch_combine_retract_batch(const BatchPtrs<CombineArgs>& b, int pp, int blocks,
                                  hipStream_t st) {
  if (pp <= 16) combine_batch_retract_t<T, 1>(b, blocks, st);
  else combine_batch_retract_t<T, 2>(b, blocks, st);
}

template <typename T>
void launch_combine_grad_batch(const BatchPtrs<CombineArgs>& b, int pp, int blocks,
                               hipStream_t st) {
  if (pp <= 16) combine_batch_grad_t<T, 1>(b, blocks, st);
  else combine_batch_grad_t<T, 2>(b, blocks, st);
}
template void launch_combine_retract_batch<double>(const BatchPtrs<CombineArgs>&, int, int,
                                                   hipStream_t);
template void launch_combine_retract_batch<float>(const BatchPtrs<CombineArgs>&, int, int,
                                                  hipStream_t);
template void launch_combine_grad_batch<double>(const BatchPtrs<CombineArgs>&, int, int,
                                                hipStream_t);
template void launch_combine_grad_batch<float>(const BatchPtrs<CombineArgs>&, int, int,
                                               hipStream_t);

}  // namespace ks
