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
#include "ks_common.h"

namespace ks {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGramMaxChunks = 512;

// ---- Gram: per-chunk partials -------------------------------------------------------
// grid.x = chunks of rows; grid.y = product index when kAll3 == false.
// kT = pp / 16 tiles per dimension.  Symmetric products (A^T A, B^T B) compute only the
// tiles ti <= tj; the reduction mirrors them.
template <int kT, bool kAll3>
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A,
                                              const double* __restrict__ B, int ld, int n,
                                              int p, int nprod, double* __restrict__ part) {
  constexpr int kPP = kT * 16;
  constexpr int kTilesSym = kT * (kT + 1) / 2;
  constexpr int kTilesAll = kT * kT;
  // tiles held per wave
  constexpr int kAcc = kAll3 ? (2 * kTilesSym + kTilesAll) : kTilesAll;
  extern __shared__ double lds[];

  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int chunk = blockIdx.x, nchunks = gridDim.x;
  const int prod_y = (nprod == 1) ? 1 : (int)blockIdx.y;  // product when !kAll3
  // row range of this chunk, in groups of 4 rows
  const int ngroups = (n + 3) / 4;
  const int per = (ngroups + nchunks - 1) / nchunks;
  const int g_beg = chunk * per;
  const int g_end = min(ngroups, g_beg + per);

  d4 acc[kAcc];
#pragma unroll
  for (int t = 0; t < kAcc; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  const int lr = lane / 16, lc = lane % 16;
  for (int grp = g_beg + w; grp < g_end; grp += 4) {
    const int row = grp * 4 + lr;
    const bool rok = row < n;
    double fa[kT], fb[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      const int col = t * 16 + lc;
      const bool ok = rok && col < p;
      fa[t] = ok ? A[(size_t)row * ld + col] : 0.0;
      fb[t] = ok ? B[(size_t)row * ld + col] : 0.0;
    }
    if (kAll3) {
      int a = 0;
      // A^T A (upper tiles)
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = ti; tj < kT; ++tj, ++a) acc[a] = mfma16(fa[ti], fa[tj], acc[a]);
      // A^T B (all tiles)
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = 0; tj < kT; ++tj, ++a) acc[a] = mfma16(fa[ti], fb[tj], acc[a]);
      // B^T B (upper tiles)
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = ti; tj < kT; ++tj, ++a) acc[a] = mfma16(fb[ti], fb[tj], acc[a]);
    } else {
      int a = 0;
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = 0; tj < kT; ++tj) {
          const double x = (prod_y == 2) ? fb[ti] : fa[ti];
          const double y = (prod_y == 0) ? fa[tj] : fb[tj];
          acc[a] = mfma16(x, y, acc[a]);
          ++a;
        }
    }
  }

  // fixed-order sum over the four waves, one tile at a time: waves 1..3 park the tile
  // in LDS and wave 0 adds them in wave order
#pragma unroll
  for (int t = 0; t < kAcc; ++t) {
    if (w > 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) lds[((w - 1) * 4 + r) * 64 + lane] = acc[t][r];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int ww = 0; ww < 3; ++ww)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] += lds[(ww * 4 + r) * 64 + lane];
    }
    __syncthreads();
  }
  if (w == 0) {
    // write this chunk's partial tiles: part[chunk][prod][pp][pp]
    double* out = part + (size_t)chunk * 3 * kPP * kPP;
    auto put = [&](int prod, int ti, int tj, const d4& v) {
      double* o = out + (size_t)prod * kPP * kPP;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ti * 16 + lr + 4 * r, j = tj * 16 + lc;
        o[i * kPP + j] = v[r];
      }
    };
    int a = 0;
    if (kAll3) {
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = ti; tj < kT; ++tj) put(0, ti, tj, acc[a++]);
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = 0; tj < kT; ++tj) put(1, ti, tj, acc[a++]);
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = ti; tj < kT; ++tj) put(2, ti, tj, acc[a++]);
    } else {
#pragma unroll
      for (int ti = 0; ti < kT; ++ti)
#pragma unroll
        for (int tj = 0; tj < kT; ++tj) put(prod_y, ti, tj, acc[a++]);
    }
  }
}

// out[prod][i][j] = sum over chunks, fixed order; symmetric products are mirrored from
// their upper tiles.  Entries with i >= p or j >= p are zero (the loads were masked).
__global__ void k_gram_reduce(const double* __restrict__ part, int nchunks, int pp, int nprod,
                              int sym_only_upper, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = pp * pp;
  if (e >= 3 * per) return;
  const int prod = e / per, ij = e % per, i = ij / pp, j = ij % pp;
  if (nprod == 1 && prod != 1) {
    out[e] = 0.0;
    return;
  }
  int src = ij;
  if (prod != 1 && sym_only_upper && (i / 16) > (j / 16)) src = j * pp + i;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * 3 * per + (size_t)prod * per + src];
  out[e] = s;
}

// ---- combine ------------------------------------------------------------------------
// out[g][:] = C0[g][:] + X[g][:] A + Y[g][:] B  (A, B: pp x pp, staged in LDS).
// Each wavefront owns a 16-row tile and all column tiles of it.
template <int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad>
__global__ __launch_bounds__(256) void k_combine(CombineArgs a) {
  constexpr int kPP = kT * 16;
  constexpr int kK = kHasY ? 2 * kPP : kPP;  // contraction length
  extern __shared__ double lds[];            // W = [A; B] : kK x kPP
  __shared__ double sh[kBlock / kWave];

  for (int e = threadIdx.x; e < kPP * kPP; e += blockDim.x) {
    lds[e] = a.A[e];
    if (kHasY) lds[kPP * kPP + e] = a.B[e];
  }
  __syncthreads();

  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  const int ntiles = (a.n + 15) / 16;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int t_beg = lb * per, t_end = min(ntiles, t_beg + per);
  const int ld = a.ld, p = a.p;
  double dd = 0.0, ss = 0.0, sy = 0.0, yy = 0.0;

  for (int tile = t_beg + w; tile < t_end; tile += 4) {
    const int g0 = tile * 16;
    d4 acc[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    // A-fragment rows: g0 + lc ; columns k0 + lr
    const int arow = g0 + lc;
    const bool arok = arow < a.n;
    const double* xr = a.X + (size_t)arow * ld;
    const double* yr = kHasY ? a.Y + (size_t)arow * ld : nullptr;
#pragma unroll 4
    for (int k0 = 0; k0 < kK; k0 += 4) {
      const int k = k0 + lr;
      double av;
      if (!kHasY || k < kPP) {
        av = (arok && k < p) ? xr[k] : 0.0;
      } else {
        const int ky = k - kPP;
        av = (arok && ky < p) ? yr[ky] : 0.0;
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
        if (row < a.n && col < p) {
          const size_t off = (size_t)row * ld + col;
          double v = acc[t][r];
          if (kHasC0) v += a.C0[off];
          a.out[off] = v;
          if (kRho) sq[r] += v * v;
          if (kGrad) {
            const double s = a.X[off] - a.Xk[off];
            const double y = v - a.Dk[off];
            dd += v * v;
            ss += s * s;
            sy += s * y;
            yy += y * y;
          }
        }
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
}

template <int kT>
void launch_gram_t(const double* A, const double* B, int ld, int n, int p, int nprod,
                   double* partials, int nchunks, hipStream_t st) {
  constexpr int kTilesSym = kT * (kT + 1) / 2, kTilesAll = kT * kT;
  (void)kTilesSym;
  (void)kTilesAll;
  const size_t lds = (size_t)3 * 4 * 64 * sizeof(double);
  if constexpr (kT <= 2) {
    if (nprod == 3) {
      hipLaunchKernelGGL((k_gram<kT, true>), dim3(nchunks), dim3(256), lds, st, A, B, ld, n, p,
                         nprod, partials);
      return;
    }
  }
  hipLaunchKernelGGL((k_gram<kT, false>), dim3(nchunks, nprod == 1 ? 1 : 3), dim3(256), lds, st,
                     A, B, ld, n, p, nprod, partials);
}

template <int kT, bool kHasY, bool kHasC0, bool kRho, bool kGrad>
void launch_combine_t(const CombineArgs& a, hipStream_t st) {
  constexpr int kPP = kT * 16;
  const size_t lds = (size_t)(kHasY ? 2 : 1) * kPP * kPP * sizeof(double);
  static bool attr = false;
  if (!attr && lds > 32768) {
    (void)hipFuncSetAttribute(
        reinterpret_cast<const void*>(k_combine<kT, kHasY, kHasC0, kRho, kGrad>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL((k_combine<kT, kHasY, kHasC0, kRho, kGrad>), dim3(combine_blocks(a.n)),
                     dim3(256), lds, st, a);
}

template <int kT>
void launch_combine_tt(const CombineArgs& a, hipStream_t st) {
  const bool y = a.Y != nullptr, c0 = a.C0 != nullptr, rho = a.rho != nullptr,
             gr = a.Xk != nullptr;
  // the combinations the library uses
  if (y && !c0 && rho && !gr) return launch_combine_t<kT, true, false, true, false>(a, st);
  if (y && !c0 && !rho && !gr) return launch_combine_t<kT, true, false, false, false>(a, st);
  if (!y && c0 && !rho && gr) return launch_combine_t<kT, false, true, false, true>(a, st);
  if (!y && c0 && !rho && !gr) return launch_combine_t<kT, false, true, false, false>(a, st);
  if (!y && !c0 && rho && !gr) return launch_combine_t<kT, false, false, true, false>(a, st);
  if (!y && !c0 && !rho && !gr) return launch_combine_t<kT, false, false, false, false>(a, st);
  // unreachable for the library's call sites
  launch_combine_t<kT, true, true, true, true>(a, st);
}

}  // namespace

int gram_chunks(int n, int pp) {
  (void)pp;
  int c = (n + 63) / 64;
  if (c > kGramMaxChunks) c = kGramMaxChunks;
  return c < 1 ? 1 : c;
}

void launch_gram(const double* A, const double* B, int ld, int n, int p, int nprod,
                 double* partials, int nchunks, hipStream_t st) {
  const int pp = round_up(p, 16);
  switch (pp / 16) {
    case 1: launch_gram_t<1>(A, B, ld, n, p, nprod, partials, nchunks, st); break;
    case 2: launch_gram_t<2>(A, B, ld, n, p, nprod, partials, nchunks, st); break;
    case 3: launch_gram_t<3>(A, B, ld, n, p, nprod, partials, nchunks, st); break;
    case 4: launch_gram_t<4>(A, B, ld, n, p, nprod, partials, nchunks, st); break;
    default: break;
  }
}

void launch_gram_reduce(const double* partials, int nchunks, int pp, int nprod, int p,
                        double* out, hipStream_t st) {
  (void)p;
  const int total = 3 * pp * pp;
  // the all-in-one kernel (pp <= 32, three products) stores only upper tiles of the
  // symmetric products; the per-product kernel stores every tile
  const int upper = (pp <= 32 && nprod == 3) ? 1 : 0;
  hipLaunchKernelGGL(k_gram_reduce, dim3((total + 255) / 256), dim3(256), 0, st, partials,
                     nchunks, pp, nprod, upper, out);
}

int combine_blocks(int n) {
  int tiles = (n + 15) / 16;
  int b = (tiles + 3) / 4;
  if (b > 4096) b = 4096;
  return b < 1 ? 1 : b;
}

void launch_combine(const CombineArgs& a, hipStream_t st) {
  const int pp = round_up(a.p, 16);
  switch (pp / 16) {
    case 1: launch_combine_tt<1>(a, st); break;
    case 2: launch_combine_tt<2>(a, st); break;
    case 3: launch_combine_tt<3>(a, st); break;
    case 4: launch_combine_tt<4>(a, st); break;
    default: break;
  }
}

}  // namespace ks
