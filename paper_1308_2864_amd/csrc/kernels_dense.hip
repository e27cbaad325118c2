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

#include "ks_common.h"

namespace ks {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGramMaxChunks = 512;
constexpr int kGradMaxBlocks = 512;
constexpr bool kFuseGram = false;

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

  for (int grp = g_beg + w; grp < g_end; grp += 4) {
    const int row = grp * 4 + lr;
    const bool rok = row < n;
    double fa[kT], fb[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      const int col = t * 16 + lc;
      const bool ok = rok && col < p;
      fa[t] = ok ? (double)A[(size_t)row * ld + col] : 0.0;
      fb[t] = ((kMask & (kPAB | kPBB)) && ok) ? (double)B[(size_t)row * ld + col] : 0.0;
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
  k_gram_body<T, kT, kMask>(*b.a[s], blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// out[prod][i][j] = sum over chunks in increasing order, for the products in mask; the
// other products are zero.  Block = 16 output slots x 16 chunk lanes; chunk lane c sums
// chunks c, c+16, ... and the 16 lane sums are added in lane order.  Symmetric products
// read the mirrored upper tile.  With W != nullptr also W = -(product 1)^T.
__device__ inline void k_gram_reduce_body(const GramReduceArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ part = ka.part;
  int nchunks = ka.nchunks;
  int pp = ka.pp;
  int mask = ka.mask;
  double* __restrict__ out = ka.out;
  double* __restrict__ W = ka.W;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double red[16][17];
  const int sl = threadIdx.x % 16, cl = threadIdx.x / 16;
  const int per = pp * pp;
  const int e = ks_bid * 16 + sl;
  double s = 0.0;
  int prod = 0, i = 0, j = 0;
  bool live = false;
  if (e < 3 * per) {
    prod = e / per;
    const int ij = e % per;
    i = ij / pp;
    j = ij % pp;
    live = (mask >> prod) & 1;
    if (live) {
      const int src = (prod != 1 && (i / 16) > (j / 16)) ? j * pp + i : ij;
      const double* q = part + (size_t)prod * per + src;
      for (int c = cl; c < nchunks; c += 16) s += q[(size_t)c * 3 * per];
    }
  }
  red[sl][cl] = s;
  __syncthreads();
  // products outside the mask are left untouched in out
  if (cl == 0 && e < 3 * per && live) {
    double t = 0.0;
    for (int c = 0; c < 16; ++c) t += red[sl][c];
    out[e] = t;
    if (W && prod == 1) W[j * pp + i] = -t;
  }
}

__global__ __launch_bounds__(256) void k_gram_reduce(GramReduceArgs ka) {
  k_gram_reduce_body(ka, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_gram_reduce_batch(BatchPtrs<GramReduceArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_gram_reduce_body(*b.a[s], blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// ---- combine ------------------------------------------------------------------------
// out[g][:] = C0[g][:] + X[g][:] A + Y[g][:] B  (A, B: pp x pp, staged in LDS).
// Each wavefront owns a 16-row tile and all column tiles of it.  Epilogues:
//   kRho   density of out,
//   kGrad  out is D = grad E; Frobenius sums ||D||^2 and the BB sums against (Xk, Dk),
//          and, with kGram2, the Gram tiles X^T D and D^T D: an FP64 MFMA result tile of
//          a 4-row group (register r) is laid out exactly as an MFMA input fragment, so
//          D goes from the accumulators straight back into the matrix cores.
template <typename T, int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad, bool kGram2>
__device__ inline void k_combine_body(const CombineArgs& a, int ks_bid, int ks_nb) {
  (void)ks_bid;
  (void)ks_nb;

  const T* aX = static_cast<const T*>(a.X);
  const T* aY = static_cast<const T*>(a.Y);
  const T* aC0 = static_cast<const T*>(a.C0);
  const T* aXk = static_cast<const T*>(a.Xk);
  const T* aDk = static_cast<const T*>(a.Dk);
  T* aout = static_cast<T*>(a.out);
  constexpr int kPP = kT * 16;
  constexpr int kK = kHasY ? 2 * kPP : kPP;  // contraction length
  constexpr int kG2 = kGram2 ? (kT * kT + kT * (kT + 1) / 2) : 1;
  extern __shared__ double lds[];            // W = [A; B] : kK x kPP (+ 6 KiB reduction)
  __shared__ double sh[kBlock / kWave];

  for (int e = threadIdx.x; e < kPP * kPP; e += blockDim.x) {
    lds[e] = a.A[e];
    if (kHasY) lds[kPP * kPP + e] = a.B[e];
  }
  __syncthreads();

  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  const int ntiles = (a.n + 15) / 16;
  const int lb = xcd_remap(ks_bid, ks_nb);
  const int per = (ntiles + ks_nb - 1) / ks_nb;
  const int t_beg = lb * per, t_end = min(ntiles, t_beg + per);
  const int ld = a.ld, p = a.p;
  double dd = 0.0, ss = 0.0, sy = 0.0, yy = 0.0;
  d4 g2[kG2];
#pragma unroll
  for (int t = 0; t < kG2; ++t) g2[t] = d4{0.0, 0.0, 0.0, 0.0};

  for (int tile = t_beg + w; tile < t_end; tile += 4) {
    const int g0 = tile * 16;
    d4 acc[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    // A-fragment rows: g0 + lc ; columns k0 + lr
    const int arow = g0 + lc;
    const bool arok = arow < a.n;
    const T* xr = aX + (size_t)arow * ld;
    const T* yr = kHasY ? aY + (size_t)arow * ld : nullptr;
#pragma unroll 4
    for (int k0 = 0; k0 < kK; k0 += 4) {
      const int k = k0 + lr;
      double av;
      if (!kHasY || k < kPP) {
        av = (arok && k < p) ? (double)xr[k] : 0.0;
      } else {
        const int ky = k - kPP;
        av = (arok && ky < p) ? (double)yr[ky] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < kT; ++t) {
        const double bv = lds[k * kPP + t * 16 + lc];
        acc[t] = mfma16(av, bv, acc[t]);
      }
    }
    // epilogue: lane holds rows g0 + lr + 4 r, column t*16 + lc
    double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      const int col = t * 16 + lc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = g0 + lr + 4 * r;
        const bool ok = row < a.n && col < p;
        double v = 0.0;
        if (ok) {
          const size_t off = (size_t)row * ld + col;
          v = acc[t][r];
          if (kHasC0) v += (double)aC0[off];
          const T vs = (T)v;
          aout[off] = vs;
          v = (double)vs;  // the epilogues see the stored value
          if (kRho) sq[r] += v * v;
          if (kGrad) {
            const double s = (double)aX[off] - (double)aXk[off];
            const double y = v - (double)aDk[off];
            dd += v * v;
            ss += s * s;
            sy += s * y;
            yy += y * y;
          }
        }
        acc[t][r] = v;  // masked D, reused as an MFMA fragment below
      }
    }
    if (kGram2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = g0 + 4 * r + lr;
        double fx[kT];
#pragma unroll
        for (int t = 0; t < kT; ++t) {
          const int col = t * 16 + lc;
          fx[t] = (row < a.n && col < p) ? (double)aX[(size_t)row * ld + col] : 0.0;
        }
        int q = 0;
#pragma unroll
        for (int ti = 0; ti < kT; ++ti)
#pragma unroll
          for (int tj = 0; tj < kT; ++tj, ++q) g2[q] = mfma16(fx[ti], acc[tj][r], g2[q]);
#pragma unroll
        for (int ti = 0; ti < kT; ++ti)
#pragma unroll
          for (int tj = ti; tj < kT; ++tj, ++q) g2[q] = mfma16(acc[ti][r], acc[tj][r], g2[q]);
      }
    }
    if (kRho) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = sq[r];
        v += __shfl_xor(v, 8, 16);
        v += __shfl_xor(v, 4, 16);
        v += __shfl_xor(v, 2, 16);
        v += __shfl_xor(v, 1, 16);
        const int row = g0 + lr + 4 * r;
        if (lc == 0 && row < a.n) a.rho[row] = a.rho_scale * v;
      }
    }
  }
  if (kGrad) {
    dd = block_sum(dd, sh);
    ss = block_sum(ss, sh);
    sy = block_sum(sy, sh);
    yy = block_sum(yy, sh);
    if (threadIdx.x == 0) {
      const int st = a.pt.stride;
      a.pt.buf[(size_t)SL_DD * st + lb] = dd;
      a.pt.buf[(size_t)SL_SS * st + lb] = ss;
      a.pt.buf[(size_t)SL_SY * st + lb] = sy;
      a.pt.buf[(size_t)SL_YY * st + lb] = yy;
    }
  }
  if (kGram2) {
    double* red = lds + kK * kPP;
#pragma unroll
    for (int t = 0; t < kG2; ++t) wave_reduce_tile(g2[t], red, w, lane);
    if (w == 0) {
      int q = 0;
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = 0; tj < kT; ++tj) put_tile<kPP>(a.gram_part, lb, 1, ti, tj, g2[q++], lr, lc);
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = ti; tj < kT; ++tj) put_tile<kPP>(a.gram_part, lb, 2, ti, tj, g2[q++], lr, lc);
    }
  }
}

template <typename T, int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad, bool kGram2>
__global__ __launch_bounds__(256) void k_combine(CombineArgs a) {
  k_combine_body<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2>(a, blockIdx.x, gridDim.x);
}

template <typename T, int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad, bool kGram2>
__global__ __launch_bounds__(256) void k_combine_batch(BatchPtrs<CombineArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_combine_body<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2>(*b.a[s], blockIdx.x - b.off[s],
                                                             b.off[s + 1] - b.off[s]);
}


void set_lds_attr(const void* k, size_t bytes) {
  if (bytes > 32768)
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
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

template <typename T, int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad, bool kGram2>
void launch_combine_t(const CombineArgs& a, hipStream_t st) {
  constexpr int kPP = kT * 16;
  const size_t lds = (size_t)(kHasY ? 2 : 1) * kPP * kPP * sizeof(double) +
                     (kGram2 ? (size_t)3 * 4 * 64 * sizeof(double) : 0);
  // function-local static initialisation runs once even when several host threads launch
  static const bool attr = (set_lds_attr(reinterpret_cast<const void*>(
                                k_combine<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2>),
                                lds),
                            true);
  (void)attr;
  const int nb = kGram2 ? combine_blocks_gram(a.n) : combine_blocks(a.n);
  hipLaunchKernelGGL((k_combine<T, kT, kHasY, kHasC0, kRho, kGrad, kGram2>), dim3(nb), dim3(256),
                     lds, st, a);
}

template <typename T, int kT>
void launch_combine_tt(const CombineArgs& a, hipStream_t st) {
  const bool y = a.Y != nullptr, c0 = a.C0 != nullptr, rho = a.rho != nullptr,
             gr = a.Xk != nullptr, g2 = a.gram_part != nullptr;
  // the combinations the library uses
  if (y && !c0 && rho && !gr)
    return launch_combine_t<T, kT, true, false, true, false, false>(a, st);
  if (y && !c0 && !rho && !gr)
    return launch_combine_t<T, kT, true, false, false, false, false>(a, st);
  if constexpr (kT <= 2) {
    if (!y && c0 && !rho && gr && g2)
      return launch_combine_t<T, kT, false, true, false, true, true>(a, st);
  }
  if (!y && c0 && !rho && gr)
    return launch_combine_t<T, kT, false, true, false, true, false>(a, st);
  if (!y && c0 && !rho && !gr)
    return launch_combine_t<T, kT, false, true, false, false, false>(a, st);
  if (!y && !c0 && rho && !gr)
    return launch_combine_t<T, kT, false, false, true, false, false>(a, st);
  launch_combine_t<T, kT, false, false, false, false, false>(a, st);
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

size_t gram_part_doubles(int n, int pp) {
  const int c = std::max(gram_chunks(n, pp), combine_blocks_gram(n));
  return (size_t)c * 3 * pp * pp;
}

bool combine_fuses_gram(int p) { return round_up(p, 16) <= 32 && kFuseGram; }

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
                        double* W, hipStream_t st) {
  const int total = 3 * pp * pp;
  hipLaunchKernelGGL(k_gram_reduce, dim3((total + 15) / 16), dim3(256), 0, st,
                     GramReduceArgs{partials, nchunks, pp, mask, out, W});
}

int combine_blocks(int n) {
  int tiles = (n + 15) / 16;
  int b = (tiles + 3) / 4;
  if (b > 4096) b = 4096;
  return b < 1 ? 1 : b;
}

int combine_blocks_gram(int n) {
  int b = combine_blocks(n);
  return b > kGradMaxBlocks ? kGradMaxBlocks : b;
}

void launch_combine(const CombineArgs& a, hipStream_t st) {
  if (a.f32) launch_combine_p<float>(a, st);
  else launch_combine_p<double>(a, st);
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

int gram_reduce_blocks(int pp) { return (3 * pp * pp + 15) / 16; }

void launch_gram_reduce_batch(const BatchPtrs<GramReduceArgs>& b, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_reduce_batch, dim3(blocks), dim3(256), 0, st, b);
}

template <typename T, int kT>
void combine_batch_retract_t(const BatchPtrs<CombineArgs>& b, int blocks, hipStream_t st) {
  constexpr int kPP = kT * 16;
  const size_t lds = (size_t)2 * kPP * kPP * sizeof(double);
  hipLaunchKernelGGL((k_combine_batch<T, kT, true, false, true, false, false>), dim3(blocks),
                     dim3(256), lds, st, b);
}

template <typename T, int kT>
void combine_batch_grad_t(const BatchPtrs<CombineArgs>& b, int blocks, hipStream_t st) {
  constexpr int kPP = kT * 16;
  const size_t lds = (size_t)kPP * kPP * sizeof(double);
  hipLaunchKernelGGL((k_combine_batch<T, kT, false, true, false, true, false>), dim3(blocks),
                     dim3(256), lds, st, b);
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
