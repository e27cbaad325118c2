// Trilinear (Q1) finite elements on the uniform hexahedral mesh (Section 2.3, the
// finite-element form with the mass matrix B and the constraint X^T B X = I).
//
// On a uniform mesh the element matrices are tensor products of the 1D linear-element
// matrices K = (1/h) tridiag(-1, 2, -1) and M = (h/6) tridiag(1, 4, 1):
//   B = M x M x M,   A = K x M x M + M x K x M + M x M x K.
// Both are 27-point stencils with one coefficient per neighbour class (centre, face,
// edge, corner): A = (8h/3, 0, -h/6, -h/12) (the face couplings cancel exactly) and
// B = (8h^3/27, 2h^3/27, h^3/54, h^3/216).  The kernels apply them as stencils over the
// grid-major orbital block instead of as CSR matrices: no index arrays to stream, and
// both products come out of one pass over X.
//
// B^{-1} is exact through the tensor structure: three sweeps of the constant-coefficient
// tridiagonal solve with M, one per axis.  A thread owns one (line, orbital) pair and
// keeps the whole line in registers, so each sweep reads and writes the block once.
#include "ks_common.h"

namespace ks {

namespace {

__device__ inline void write_partial(Partials pt, int slot, int b, double v) {
  if (threadIdx.x == 0) pt.buf[(size_t)slot * pt.stride + b] = v;
}

struct Q1Coef {
  double a0, a2, a3;      // A: centre, edge, corner (faces are zero)
  double b0, b1, b2, b3;  // B: centre, face, edge, corner
};

Q1Coef q1_coef(double h) {
  const double h3 = h * h * h;
  return Q1Coef{8.0 * h / 3.0, -h / 6.0, -h / 12.0,
                8.0 * h3 / 27.0, 2.0 * h3 / 27.0, h3 / 54.0, h3 / 216.0};
}

// Y = scale ((1/2) A X + h3 veff X) and BX = B X.  Per plane the 3 x 3 in-plane
// neighbourhood of a point reduces to three partial sums (centre P0, in-plane faces P1,
// in-plane corners P2); the 3-D neighbour classes of plane k are then
//   centre P0(k), faces P1(k) + P0(k-1) + P0(k+1), edges P2(k) + P1(k-1) + P1(k+1),
//   corners P2(k-1) + P2(k+1).
// A block owns a tile of kQ1Tx x-points, kQ1Ty y-rows and kQ1Tc orbitals and marches
// along z over kQ1Chunk planes: each plane of the tile, with its one-point x/y halo, is
// staged once in LDS (double-buffered, one barrier per plane; each 16-orbital run is one
// 128-byte segment; the next plane is fetched into registers meanwhile), and a thread
// forms the partial sums of its point in its kQ1Ty rows from LDS, keeping P(k-1) and P(k)
// in registers.  Global reads per plane are
// (kQ1Tx + 2)(kQ1Ty + 2) / (kQ1Tx kQ1Ty) = 1.7 times the tile.  Blocks loop over tiles
// (at most kQ1ApplyMaxBlocks blocks, so the energy partials fit their slots).
constexpr int kQ1Chunk = 16;
constexpr int kQ1Tx = 16, kQ1Ty = 4, kQ1Tc = 16;
constexpr int kQ1ApplyMaxBlocks = 2048;
static_assert(kQ1Tx * kQ1Tc == kBlock, "one thread per (x-point, orbital) of the tile");

struct Q1Tiles {
  int tx, ty, tc, tz;
  __host__ __device__ size_t total() const { return (size_t)tx * ty * tc * tz; }
};

__host__ __device__ inline Q1Tiles q1_tiles(const Grid& g, int p) {
  return Q1Tiles{(g.nx + kQ1Tx - 1) / kQ1Tx, (g.ny + kQ1Ty - 1) / kQ1Ty,
                 (p + kQ1Tc - 1) / kQ1Tc, (g.nz + kQ1Chunk - 1) / kQ1Chunk};
}

typedef double Q1Plane[kQ1Ty + 2][kQ1Tx + 2][kQ1Tc];

constexpr int kQ1Stage = (kQ1Ty + 2) * (kQ1Tx + 2) * kQ1Tc;  // values of one staged plane
constexpr int kQ1StagePer = (kQ1Stage + kBlock - 1) / kBlock;  // per thread

// The thread's share of a staged plane: offsets within plane 0 and the mask of entries
// inside the grid (computed once per tile); q1_fetch then loads plane k into registers,
// so the loads of the next plane fly while the current one is used.
struct Q1Share {
  size_t off[kQ1StagePer];
  unsigned mask;
};

__device__ inline Q1Share q1_share(const Grid& gr, int p, int i0, int j0, int c0) {
  Q1Share sh{};
#pragma unroll
  for (int q = 0; q < kQ1StagePer; ++q) {
    const int e = threadIdx.x + q * kBlock;
    const int cc = e % kQ1Tc, xx = (e / kQ1Tc) % (kQ1Tx + 2), yy = e / (kQ1Tc * (kQ1Tx + 2));
    const int gi = i0 + xx - 1, gj = j0 + yy - 1, c = c0 + cc;
    const bool ok = e < kQ1Stage && gi >= 0 && gi < gr.nx && gj >= 0 && gj < gr.ny && c < p;
    sh.off[q] = ok ? ((size_t)gi + (size_t)gr.nx * gj) * p + c : 0;
    sh.mask |= ok ? 1u << q : 0u;
  }
  return sh;
}

// (storage type: a conversion here would wait for the loads at once)
template <typename T>
__device__ inline void q1_fetch(T v[kQ1StagePer], const T* __restrict__ X, const Grid& gr,
                                int p, const Q1Share& sh, int k) {
  const bool kin = k >= 0 && k < gr.nz;
  const T* plane = X + (kin ? (size_t)k * gr.nx * gr.ny * p : 0);
#pragma unroll
  for (int q = 0; q < kQ1StagePer; ++q)
    v[q] = (kin && ((sh.mask >> q) & 1u)) ? plane[sh.off[q]] : T(0);
}

template <typename T>
__device__ inline void q1_put(Q1Plane& L, const T v[kQ1StagePer]) {
#pragma unroll
  for (int q = 0; q < kQ1StagePer; ++q) {
    const int e = threadIdx.x + q * kBlock;
    if (e < kQ1Stage) {
      const int cc = e % kQ1Tc, xx = (e / kQ1Tc) % (kQ1Tx + 2), yy = e / (kQ1Tc * (kQ1Tx + 2));
      L[yy][xx][cc] = (double)v[q];
    }
  }
}

// partial sums of row r at x-point lx, orbital lc (the halo is zero outside the grid);
// neighbours in the order dy = -1, 0, 1 and dx = -1, 0, 1
__device__ inline void q1_sums(const Q1Plane& L, int r, int lx, int lc, double P[3]) {
  P[0] = L[r + 1][lx + 1][lc];
  P[1] = ((L[r][lx + 1][lc] + L[r + 1][lx][lc]) + L[r + 1][lx + 2][lc]) + L[r + 2][lx + 1][lc];
  P[2] = ((L[r][lx][lc] + L[r][lx + 2][lc]) + L[r + 2][lx][lc]) + L[r + 2][lx + 2][lc];
}

template <typename T, bool kG, bool kEnergy>
__global__ __launch_bounds__(256) void k_q1_apply(const T* __restrict__ X, T* __restrict__ Y,
                                                  T* __restrict__ BX,
                                                  const double* __restrict__ veff, Grid gr,
                                                  int p, double scale, Q1Coef cf,
                                                  Partials pt) {
  __shared__ Q1Plane L[2];
  __shared__ double sh[kBlock / kWave];
  const int lc = threadIdx.x % kQ1Tc, lx = threadIdx.x / kQ1Tc;
  const Q1Tiles nt = q1_tiles(gr, p);
  const size_t total = nt.total();
  const double h3 = gr.dV;
  double kin = 0.0;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  for (size_t tile = lb; tile < total; tile += gridDim.x) {
    // tile -> (orbital tile, x tile, y tile, z chunk), orbital tile fastest
    size_t r = tile;
    const int tc = (int)(r % nt.tc);
    r /= nt.tc;
    const int tx = (int)(r % nt.tx);
    r /= nt.tx;
    const int ty = (int)(r % nt.ty);
    const int tz = (int)(r / nt.ty);
    const int i0 = tx * kQ1Tx, j0 = ty * kQ1Ty, c0 = tc * kQ1Tc;
    const int k0 = tz * kQ1Chunk, k1 = min(k0 + kQ1Chunk, gr.nz);
    const int i = i0 + lx, c = c0 + lc;
    const Q1Share share = q1_share(gr, p, i0, j0, c0);
    T v[kQ1StagePer];
    __syncthreads();  // the previous tile's readers are done with both buffers
    q1_fetch(v, X, gr, p, share, k0 - 1);
    q1_put(L[0], v);
    q1_fetch(v, X, gr, p, share, k0);
    q1_put(L[1], v);
    q1_fetch(v, X, gr, p, share, k0 + 1);
    __syncthreads();
    double Pm[kQ1Ty][3], Pc[kQ1Ty][3];
#pragma unroll
    for (int rr = 0; rr < kQ1Ty; ++rr) {
      q1_sums(L[0], rr, lx, lc, Pm[rr]);
      q1_sums(L[1], rr, lx, lc, Pc[rr]);
    }
    __syncthreads();  // buffer 0 is refilled below
    int b = 0;
    for (int k = k0; k < k1; ++k) {
      q1_put(L[b], v);  // plane k + 1
      if (k + 1 < k1) q1_fetch(v, X, gr, p, share, k + 2);
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < kQ1Ty; ++rr) {
        double Pn[3];
        q1_sums(L[b], rr, lx, lc, Pn);
        const int j = j0 + rr;
        if (i < gr.nx && j < gr.ny && c < p) {
          const double s0 = Pc[rr][0];
          const double s1 = Pc[rr][1] + Pm[rr][0] + Pn[0];
          const double s2 = Pc[rr][2] + Pm[rr][1] + Pn[1];
          const double s3 = Pm[rr][2] + Pn[2];
          const double ax = gr.mu * (cf.a0 * s0 + cf.a2 * s2 + cf.a3 * s3);
          const double bx = cf.b0 * s0 + cf.b1 * s1 + cf.b2 * s2 + cf.b3 * s3;
          const size_t g = (size_t)i + (size_t)gr.nx * ((size_t)j + (size_t)gr.ny * k);
          const size_t o = g * p + c;
          if (kG) Y[o] = (T)(scale * (0.5 * ax + h3 * veff[g] * s0));
          BX[o] = (T)bx;
          if (kEnergy) kin += s0 * ax;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          Pm[rr][q] = Pc[rr][q];
          Pc[rr][q] = Pn[q];
        }
      }
      b ^= 1;
    }
  }
  if (kEnergy) {
    kin = block_sum(kin, sh);
    write_partial(pt, SL_KIN, lb, kin);
  }
}

// Thomas tables of M = (h/6) tridiag(1, 4, 1) on N nodes: tab[k] = m_k = 1/(b - a c_{k-1}),
// tab[N + k] = c_k = a m_k (a = h/6, b = 4h/6; c_{-1} = 0).
__global__ void k_mass_setup(double* tab, int N, double h) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double a = h / 6.0, b = 4.0 * h / 6.0;
  double c = 0.0;
  for (int k = 0; k < N; ++k) {
    const double m = 1.0 / (b - a * c);
    c = a * m;
    tab[k] = m;
    tab[N + k] = c;
  }
}

// One axis of B^{-1}: every line along `axis` (length N <= kN) and orbital c solves
// M u = d.  Forward elimination d'_k = (d_k - a d'_{k-1}) m_k, back substitution
// u_k = d'_k - c_k u_{k+1}.  in and out may alias (each thread reads its line first).
template <typename T, int kN>
__global__ __launch_bounds__(256) void k_mass_axis(const T* in, T* out, int p, Grid gr,
                                                   int axis, const double* __restrict__ tab,
                                                   double a) {
  const int nx = gr.nx, ny = gr.ny, nz = gr.nz;
  const int N = axis == 0 ? nx : (axis == 1 ? ny : nz);
  const size_t lines = (size_t)gr.n / N;
  const size_t total = lines * p;
  const double* mk = tab;
  const double* ck = tab + N;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const size_t line = t / (unsigned)p;
    const int c = (int)(t - line * p);
    size_t base;
    size_t stride;
    if (axis == 0) {
      base = line * nx;
      stride = 1;
    } else if (axis == 1) {
      const size_t i = line % nx, k = line / nx;
      base = i + (size_t)nx * ny * k;
      stride = nx;
    } else {
      base = line;
      stride = (size_t)nx * ny;
    }
    const T* src = in + base * p + c;
    T* dst = out + base * p + c;
    const size_t step = stride * p;
    double d[kN];
#pragma unroll
    for (int k = 0; k < kN; ++k)
      if (k < N) d[k] = (double)src[k * step];
    double prev = 0.0;
#pragma unroll
    for (int k = 0; k < kN; ++k)
      if (k < N) {
        prev = (d[k] - a * prev) * mk[k];
        d[k] = prev;
      }
    double next = 0.0;
#pragma unroll
    for (int k = kN - 1; k >= 0; --k)
      if (k < N) {
        next = (k == N - 1) ? d[k] : d[k] - ck[k] * next;
        dst[k * step] = (T)next;
      }
  }
}

// D = Gt + X W, BD = G + BX W on the matrix cores; ||D||_B^2 = sum D.BD and the BB sums
// of the B metric: ss = S.BS, sy = S.BYd, yy = Yd.BYd with S = X - Xc, BS = BX - BXc,
// Yd = D - Dc, BYd = BD - BDc.  The p_p x p_p weights (zero-padded) sit in LDS, shared by
// the block's wavefronts.  A wavefront owns a 16-row tile and a group of up to 64 output
// columns (four 16 x 16 FP64 MFMA tiles per product); per 16-wide slice of the
// contraction each lane loads four consecutive entries of its row of X and of BX (lane
// l: row l % 16, entries 4 (l / 16) .. + 3, so 16 lanes read one full cache line), which
// feed four MFMA steps against the matching weight rows.  The next slice's entries are
// loaded before the current slice's products.
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kQ1Threads = 512;
constexpr int kQ1Waves = kQ1Threads / kWave;
constexpr int kQ1MaxBlocks = 1024;
constexpr size_t kQ1LdsCap = 150 * 1024;

// v[e] = A[row][k + e] for e < 4 as stored, from a clamped address (row 0 past n, entry 0
// of the row past p): no guard and no select, so a prefetch into v stays in flight
template <typename T>
__device__ inline void q1_load4_raw(const T* __restrict__ A, size_t row, int n, int p, int k,
                                    T v[4]) {
  const size_t r0 = (row < (size_t)n ? row : 0) * p;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = A[r0 + (k + e < p ? k + e : 0)];
}

template <typename T>
__global__ __launch_bounds__(kQ1Threads) void k_q1_grad(Q1GradArgs a) {
  extern __shared__ double Ws[];
  __shared__ double sh[4][kQ1Waves];
  const int p = a.p, pp = a.pp, n = a.n;
  const int ncg = (pp + 63) / 64;  // column groups of four 16-wide tiles
  const int wc = 64 * ncg;         // LDS row: every group full width, zero beyond p
  for (int e = threadIdx.x; e < pp * wc; e += blockDim.x) {
    const int k = e / wc, j = e % wc;
    Ws[e] = (k < p && j < p) ? a.W[(size_t)k * pp + j] : 0.0;
  }
  __syncthreads();
  const T* __restrict__ Gt = static_cast<const T*>(a.Gt);
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const T* __restrict__ G = static_cast<const T*>(a.G);
  const T* __restrict__ BX = static_cast<const T*>(a.BX);
  T* __restrict__ D = static_cast<T*>(a.D);
  T* __restrict__ BD = static_cast<T*>(a.BD);
  const T* __restrict__ Xc = static_cast<const T*>(a.Xc);
  const T* __restrict__ BXc = static_cast<const T*>(a.BXc);
  const T* __restrict__ Dc = static_cast<const T*>(a.Dc);
  const T* __restrict__ BDc = static_cast<const T*>(a.BDc);
  const bool ref = Xc != nullptr;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int lr = lane % 16, lq = lane / 16;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const size_t tiles = ((size_t)n + 15) / 16;
  size_t tb, te;
  // contiguous range of row tiles for this block
  {
    const size_t per = (tiles + gridDim.x - 1) / gridDim.x;
    const size_t b0 = (size_t)lb * per;
    tb = b0 < tiles ? b0 : tiles;
    te = b0 + per < tiles ? b0 + per : tiles;
  }
  const size_t items = (te - tb) * ncg;
  double dd = 0.0, ss = 0.0, sy = 0.0, yy = 0.0;
  for (size_t it = wave; it < items; it += kQ1Waves) {
    const size_t g0 = (tb + it / ncg) * 16;
    const int c0 = (int)(it % ncg) * 64;
    d4 ax[4], ab[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) ax[t] = ab[t] = d4{0.0, 0.0, 0.0, 0.0};
    const size_t row = g0 + lr;
    // Operand loads are unconditional and select nothing (a guarded or selected load makes
    // the compiler wait for it before the current slice's products): rows past n read row
    // 0 (their products land in rows that are never stored) and entries past p read the
    // row's first entry, which meets the zero rows of the staged weights.
    T xa[4], ba[4];
    q1_load4_raw<T>(X, row, n, p, 4 * lq, xa);
    q1_load4_raw<T>(BX, row, n, p, 4 * lq, ba);
    for (int k0 = 0; k0 < pp; k0 += 16) {
      const int kn = k0 + 16 < pp ? k0 + 16 : k0;  // the last slice reloads itself
      T xn[4], bn[4];
      q1_load4_raw<T>(X, row, n, p, kn + 4 * lq, xn);
      q1_load4_raw<T>(BX, row, n, p, kn + 4 * lq, bn);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double* wr = Ws + (size_t)(k0 + 4 * lq + e) * wc + c0 + lr;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double w = wr[16 * t];
          ax[t] = mfma16((double)xa[e], w, ax[t]);
          ab[t] = mfma16((double)ba[e], w, ab[t]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        xa[e] = xn[e];
        ba[e] = bn[e];
      }
    }
    // one column tile at a time keeps the epilogue's loads few in flight; the four rows of
    // a tile are loaded together (clamped addresses, no guard) before any of them is used
    const int ntv = min(4, (p - c0 + 15) / 16);  // tiles holding columns below p
#pragma unroll 1
    for (int t = 0; t < ntv; ++t) {
      const d4 vx = t == 0 ? ax[0] : t == 1 ? ax[1] : t == 2 ? ax[2] : ax[3];
      const d4 vb = t == 0 ? ab[0] : t == 1 ? ab[1] : t == 2 ? ab[2] : ab[3];
      const int j = c0 + 16 * t + lr;
      size_t o[4];
      bool ok[4];
      T gt[4], gg[4], x[4], xc[4], bx[4], bxc[4], dc[4], bdc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t g = g0 + lq + 4 * r;
        ok[r] = g < (size_t)n && j < p;
        o[r] = ok[r] ? g * p + j : 0;
        gt[r] = Gt[o[r]];
        gg[r] = G[o[r]];
        if (ref) {
          x[r] = X[o[r]];
          xc[r] = Xc[o[r]];
          bx[r] = BX[o[r]];
          bxc[r] = BXc[o[r]];
          dc[r] = Dc[o[r]];
          bdc[r] = BDc[o[r]];
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!ok[r]) continue;
        const T dT = (T)((double)gt[r] + vx[r]);
        const T bT = (T)((double)gg[r] + vb[r]);
        D[o[r]] = dT;
        BD[o[r]] = bT;
        const double d = (double)dT, bd = (double)bT;
        dd += d * bd;
        if (ref) {
          const double sdx = (double)x[r] - (double)xc[r];
          const double bs = (double)bx[r] - (double)bxc[r];
          const double y = d - (double)dc[r];
          const double by = bd - (double)bdc[r];
          ss += sdx * bs;
          sy += sdx * by;
          yy += y * by;
        }
      }
    }
  }
  // fixed-order block reduction of the four sums
  double v[4] = {dd, ss, sy, yy};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    for (int o = kWave / 2; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, kWave);
    if (lane == 0) sh[q][wave] = v[q];
  }
  __syncthreads();
  // slots SL_DD .. SL_YY are consecutive
  for (int q = 0; q < 4; ++q) {
    double acc = 0.0;
    for (int w = 0; w < kQ1Waves; ++w) acc += sh[q][w];
    write_partial(a.pt, SL_DD + q, lb, acc);
  }
}

template <typename T, int kN>
void mass_axes(const T* in, T* out, int p, Grid g, const double* const tab[3], hipStream_t st) {
  const double a = g.h / 6.0;
  const int dims[3] = {g.nx, g.ny, g.nz};
  for (int axis = 0; axis < 3; ++axis) {
    const size_t total = (size_t)g.n / dims[axis] * p;
    size_t nb = (total + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL((k_mass_axis<T, kN>), dim3((unsigned)nb), dim3(256), 0, st,
                       axis == 0 ? in : out, out, p, g, axis, tab[axis], a);
  }
}

}  // namespace

int q1_apply_blocks(Grid g, int p) {
  const size_t t = q1_tiles(g, p).total();
  return (int)(t < (size_t)kQ1ApplyMaxBlocks ? (t < 1 ? 1 : t) : (size_t)kQ1ApplyMaxBlocks);
}
int q1_grad_blocks(int n, int p) {
  // a few rounds of (row tile, column group) items per wavefront
  const size_t items = ((size_t)n + 15) / 16 * ((round_up(p, 16) + 63) / 64);
  size_t b = (items + 4 * kQ1Waves - 1) / (4 * kQ1Waves);
  if (b > (size_t)kQ1MaxBlocks) b = kQ1MaxBlocks;
  return b < 1 ? 1 : (int)b;
}

size_t q1_grad_lds(int p) {
  const size_t pp = round_up(p, 16), wc = (pp + 63) / 64 * 64;
  return pp * wc * sizeof(double);
}

template <typename T>
void launch_q1_apply(const T* X, T* G, T* BX, const double* veff, Grid g,
                     int p, double scale, Partials* pt, hipStream_t st) {
  const int nb = q1_apply_blocks(g, p);
  const Q1Coef cf = q1_coef(g.h);
  if (G && pt)
    hipLaunchKernelGGL((k_q1_apply<T, true, true>), dim3(nb), dim3(kBlock), 0, st, X, G, BX,
                       veff, g, p, scale, cf, *pt);
  else if (G)
    hipLaunchKernelGGL((k_q1_apply<T, true, false>), dim3(nb), dim3(kBlock), 0, st, X, G, BX,
                       veff, g, p, scale, cf, Partials{nullptr, 0});
  else
    hipLaunchKernelGGL((k_q1_apply<T, false, false>), dim3(nb), dim3(kBlock), 0, st, X, G, BX,
                       veff, g, p, scale, cf, Partials{nullptr, 0});
}

void launch_mass_setup(double* tab, int N, double h, hipStream_t st) {
  hipLaunchKernelGGL(k_mass_setup, dim3(1), dim3(64), 0, st, tab, N, h);
}

template <typename T>
void launch_mass_solve(const T* in, T* out, int p, Grid g, const double* const tab[3],
                       hipStream_t st) {
  const int N = std::max(g.nx, std::max(g.ny, g.nz));
  if (N <= 32) mass_axes<T, 32>(in, out, p, g, tab, st);
  else if (N <= 64) mass_axes<T, 64>(in, out, p, g, tab, st);
  else if (N <= 96) mass_axes<T, 96>(in, out, p, g, tab, st);
  else mass_axes<T, 128>(in, out, p, g, tab, st);
}

void launch_q1_grad(const Q1GradArgs& a, hipStream_t st) {
  const int nb = q1_grad_blocks(a.n, a.p);
  const size_t lds = q1_grad_lds(a.p);
  // the limit set does not depend on p, so concurrent callers agree on it
  const void* k = a.f32 ? reinterpret_cast<const void*>(k_q1_grad<float>)
                        : reinterpret_cast<const void*>(k_q1_grad<double>);
  if (lds > 65536) set_dyn_lds_once(k, (int)kQ1LdsCap);
  if (a.f32)
    hipLaunchKernelGGL(k_q1_grad<float>, dim3(nb), dim3(kQ1Threads), lds, st, a);
  else
    hipLaunchKernelGGL(k_q1_grad<double>, dim3(nb), dim3(kQ1Threads), lds, st, a);
}

template void launch_q1_apply<double>(const double*, double*, double*, const double*, Grid,
                                      int, double, Partials*, hipStream_t);
template void launch_q1_apply<float>(const float*, float*, float*, const double*, Grid, int,
                                     double, Partials*, hipStream_t);
template void launch_mass_solve<double>(const double*, double*, int, Grid, const double* const*,
                                        hipStream_t);
template void launch_mass_solve<float>(const float*, float*, int, Grid, const double* const*,
                                       hipStream_t);

}  // namespace ks
