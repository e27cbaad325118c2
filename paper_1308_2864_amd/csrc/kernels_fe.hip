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

constexpr int kMaxStreamBlocks = 4096;

inline int stream_blocks(size_t work) {
  size_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (int)(b < (size_t)kMaxStreamBlocks ? b : (size_t)kMaxStreamBlocks);
}

__device__ inline void block_range(size_t work, int lb, int nb, size_t* beg, size_t* end) {
  size_t per = (work + nb - 1) / nb;
  per = (per + kBlock - 1) / kBlock * kBlock;
  size_t b0 = (size_t)lb * per;
  *beg = b0 < work ? b0 : work;
  size_t e = b0 + per;
  *end = e < work ? e : work;
}

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

// Y = scale ((1/2) A X + h3 veff X) and BX = B X.  A thread owns one (i, j, orbital) column
// and marches along z over kQ1Chunk planes.  Per plane it loads the 3 x 3 in-plane
// neighbourhood once and reduces it to three partial sums (centre P0, in-plane faces P1,
// in-plane corners P2); the 3-D neighbour classes of plane k are then
//   centre P0(k), faces P1(k) + P0(k-1) + P0(k+1), edges P2(k) + P1(k-1) + P1(k+1),
//   corners P2(k-1) + P2(k+1),
// so each output costs 9 loads instead of 27.  Consecutive threads take consecutive
// orbitals of one node: every load of a wavefront is one contiguous segment.
constexpr int kQ1Chunk = 16;

template <typename T>
__device__ inline void q1_plane(const T* __restrict__ X, int i, int j, int k, int nx, int ny,
                                int nz, ptrdiff_t sx, ptrdiff_t sy, ptrdiff_t sz, double* P) {
  P[0] = P[1] = P[2] = 0.0;
  if (k < 0 || k >= nz) return;
  const T* xp = X + k * sz;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy) {
    if (j + dy < 0 || j + dy >= ny) continue;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      if (i + dx < 0 || i + dx >= nx) continue;
      P[(dx != 0) + (dy != 0)] += (double)xp[dy * sy + dx * sx];
    }
  }
}

template <typename T, bool kG, bool kEnergy>
__global__ __launch_bounds__(256) void k_q1_apply(const T* __restrict__ X, T* __restrict__ Y,
                                                  T* __restrict__ BX,
                                                  const double* __restrict__ veff,
                                                  const double* __restrict__ vext, Grid gr,
                                                  int p, double scale, Q1Coef cf,
                                                  Partials pt) {
  __shared__ double sh[kBlock / kWave];
  const int nx = gr.nx, ny = gr.ny, nz = gr.nz;
  const int nzc = (nz + kQ1Chunk - 1) / kQ1Chunk;
  const size_t work = (size_t)nx * ny * p * nzc;
  const ptrdiff_t sx = p, sy = (ptrdiff_t)nx * p, sz = (ptrdiff_t)nx * ny * p;
  const double h3 = gr.dV;
  double kin = 0.0, ext = 0.0;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  for (size_t t = (size_t)lb * blockDim.x + threadIdx.x; t < work;
       t += (size_t)gridDim.x * blockDim.x) {
    // t -> (z chunk, j, i, orbital), orbital fastest
    const int c = (int)(t % (unsigned)p);
    size_t r = t / (unsigned)p;
    const int i = (int)(r % nx);
    r /= nx;
    const int j = (int)(r % ny);
    const int kc = (int)(r / ny);
    const int k0 = kc * kQ1Chunk;
    const int k1 = min(k0 + kQ1Chunk, nz);
    const T* col = X + (ptrdiff_t)(i + (size_t)nx * j) * p + c;
    double Pm[3], Pc[3], Pn[3];
    q1_plane(col, i, j, k0 - 1, nx, ny, nz, sx, sy, sz, Pm);
    q1_plane(col, i, j, k0, nx, ny, nz, sx, sy, sz, Pc);
    for (int k = k0; k < k1; ++k) {
      q1_plane(col, i, j, k + 1, nx, ny, nz, sx, sy, sz, Pn);
      const double s0 = Pc[0];
      const double s1 = Pc[1] + Pm[0] + Pn[0];
      const double s2 = Pc[2] + Pm[1] + Pn[1];
      const double s3 = Pm[2] + Pn[2];
      const double ax = cf.a0 * s0 + cf.a2 * s2 + cf.a3 * s3;
      const double bx = cf.b0 * s0 + cf.b1 * s1 + cf.b2 * s2 + cf.b3 * s3;
      const size_t g = i + (size_t)nx * (j + (size_t)ny * k);
      const size_t o = g * p + c;
      if (kG) Y[o] = (T)(scale * (0.5 * ax + h3 * veff[g] * s0));
      BX[o] = (T)bx;
      if (kEnergy) {
        kin += s0 * ax;
        ext += h3 * vext[g] * s0 * s0;
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        Pm[q] = Pc[q];
        Pc[q] = Pn[q];
      }
    }
  }
  if (kEnergy) {
    kin = block_sum(kin, sh);
    ext = block_sum(ext, sh);
    write_partial(pt, SL_KIN, lb, kin);
    write_partial(pt, SL_EXT, lb, ext);
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

// D = Gt + X W, BD = G + BX W with the p x p weights staged in LDS; ||D||_B^2 = sum D.BD and
// the BB sums of the B metric: ss = S.BS, sy = S.BYd, yy = Yd.BYd with S = X - Xc,
// BS = BX - BXc, Yd = D - Dc, BYd = BD - BDc.  A block takes q1_rows(p) rows at a time: their
// X and BX rows are staged in LDS with coalesced loads (each entry read from memory
// once), then a thread computes kQ1Cols adjacent columns of one row from LDS.
constexpr int kQ1Cols = 4;
constexpr int kQ1Rows = 16;  // rows per tile up to p = 64; 8 above, so the weights fit LDS
constexpr size_t kQ1LdsCap = 150 * 1024;

__host__ __device__ inline int q1_rows(int p) { return p > 64 ? kQ1Rows / 2 : kQ1Rows; }

template <typename T>
__global__ __launch_bounds__(256) void k_q1_grad(Q1GradArgs a) {
  extern __shared__ double lds[];
  __shared__ double sh[kBlock / kWave];
  const int p = a.p, pp = a.pp;
  const int pc = (p + kQ1Cols - 1) / kQ1Cols * kQ1Cols;  // padded row of Ws
  const int nrow = q1_rows(p);
  double* Ws = lds;                                     // p x pc
  double* Xs = Ws + (size_t)p * pc;                     // nrow x p
  double* Bs = Xs + (size_t)nrow * p;                   // nrow x p
  for (int e = threadIdx.x; e < p * pc; e += blockDim.x) {
    const int k = e / pc, j = e % pc;
    Ws[e] = j < p ? a.W[k * pp + j] : 0.0;
  }
  const T* Gt = static_cast<const T*>(a.Gt);
  const T* X = static_cast<const T*>(a.X);
  const T* G = static_cast<const T*>(a.G);
  const T* BX = static_cast<const T*>(a.BX);
  T* D = static_cast<T*>(a.D);
  T* BD = static_cast<T*>(a.BD);
  const T* Xc = static_cast<const T*>(a.Xc);
  const T* BXc = static_cast<const T*>(a.BXc);
  const T* Dc = static_cast<const T*>(a.Dc);
  const T* BDc = static_cast<const T*>(a.BDc);
  const bool ref = Xc != nullptr;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int groups = pc / kQ1Cols;
  const int tiles = (a.n + nrow - 1) / nrow;
  size_t tb, te;
  // contiguous range of row tiles for this block
  {
    const int per = (tiles + gridDim.x - 1) / gridDim.x;
    const long b0 = (long)lb * per;
    tb = (size_t)(b0 < tiles ? b0 : tiles);
    const long e0 = b0 + per;
    te = (size_t)(e0 < tiles ? e0 : tiles);
  }
  double dd = 0.0, ss = 0.0, sy = 0.0, yy = 0.0;
  for (size_t tile = tb; tile < te; ++tile) {
    const size_t r0 = tile * nrow;
    const int rows = (int)((size_t)a.n - r0 < (size_t)nrow ? (size_t)a.n - r0 : nrow);
    __syncthreads();  // previous tile's readers are done (and Ws is complete)
    for (int e = threadIdx.x; e < rows * p; e += blockDim.x) {
      Xs[e] = (double)X[r0 * p + e];
      Bs[e] = (double)BX[r0 * p + e];
    }
    __syncthreads();
    for (int q0 = threadIdx.x; q0 < rows * groups; q0 += blockDim.x) {
      const int r = q0 / groups;
      const int j0 = (q0 - r * groups) * kQ1Cols;
      const double* xr = Xs + r * p;
      const double* br = Bs + r * p;
      double u[kQ1Cols] = {}, v[kQ1Cols] = {};
      for (int k = 0; k < p; ++k) {
        const double xk = xr[k], bk = br[k];
        const double* w = Ws + k * pc + j0;
#pragma unroll
        for (int q = 0; q < kQ1Cols; ++q) {
          u[q] += xk * w[q];
          v[q] += bk * w[q];
        }
      }
#pragma unroll
      for (int q = 0; q < kQ1Cols; ++q) {
        const int j = j0 + q;
        if (j >= p) break;
        const size_t o = (r0 + r) * p + j;
        const T dT = (T)((double)Gt[o] + u[q]);
        const T bT = (T)((double)G[o] + v[q]);
        D[o] = dT;
        BD[o] = bT;
        const double d = (double)dT, bd = (double)bT;
        dd += d * bd;
        if (ref) {
          const double sdx = xr[j] - (double)Xc[o];
          const double bs = br[j] - (double)BXc[o];
          const double y = d - (double)Dc[o];
          const double by = bd - (double)BDc[o];
          ss += sdx * bs;
          sy += sdx * by;
          yy += y * by;
        }
      }
    }
  }
  dd = block_sum(dd, sh);
  ss = block_sum(ss, sh);
  sy = block_sum(sy, sh);
  yy = block_sum(yy, sh);
  write_partial(a.pt, SL_DD, lb, dd);
  write_partial(a.pt, SL_SS, lb, ss);
  write_partial(a.pt, SL_SY, lb, sy);
  write_partial(a.pt, SL_YY, lb, yy);
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

int q1_apply_blocks(int n, int p) { return stream_blocks((size_t)n * p / kQ1Chunk + 1); }
int q1_grad_blocks(int n, int p) {
  // a few row tiles per block; at most the streaming cap
  const int tiles = (n + q1_rows(p) - 1) / q1_rows(p);
  int b = (tiles + 3) / 4;
  if (b > kMaxStreamBlocks) b = kMaxStreamBlocks;
  return b < 1 ? 1 : b;
}

size_t q1_grad_lds(int p) {
  return ((size_t)p * ((p + kQ1Cols - 1) / kQ1Cols * kQ1Cols) + 2 * (size_t)q1_rows(p) * p) *
         sizeof(double);
}

template <typename T>
void launch_q1_apply(const T* X, T* G, T* BX, const double* veff, const double* vext, Grid g,
                     int p, double scale, Partials* pt, hipStream_t st) {
  const int nb = q1_apply_blocks(g.n, p);
  const Q1Coef cf = q1_coef(g.h);
  if (G && pt)
    hipLaunchKernelGGL((k_q1_apply<T, true, true>), dim3(nb), dim3(kBlock), 0, st, X, G, BX,
                       veff, vext, g, p, scale, cf, *pt);
  else if (G)
    hipLaunchKernelGGL((k_q1_apply<T, true, false>), dim3(nb), dim3(kBlock), 0, st, X, G, BX,
                       veff, vext, g, p, scale, cf, Partials{nullptr, 0});
  else
    hipLaunchKernelGGL((k_q1_apply<T, false, false>), dim3(nb), dim3(kBlock), 0, st, X, G, BX,
                       veff, vext, g, p, scale, cf, Partials{nullptr, 0});
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
  if (lds > 65536)
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kQ1LdsCap);
  if (a.f32)
    hipLaunchKernelGGL(k_q1_grad<float>, dim3(nb), dim3(kBlock), lds, st, a);
  else
    hipLaunchKernelGGL(k_q1_grad<double>, dim3(nb), dim3(kBlock), lds, st, a);
}

template void launch_q1_apply<double>(const double*, double*, double*, const double*,
                                      const double*, Grid, int, double, Partials*, hipStream_t);
template void launch_q1_apply<float>(const float*, float*, float*, const double*, const double*,
                                     Grid, int, double, Partials*, hipStream_t);
template void launch_mass_solve<double>(const double*, double*, int, Grid, const double* const*,
                                        hipStream_t);
template void launch_mass_solve<float>(const float*, float*, int, Grid, const double* const*,
                                       hipStream_t);

}  // namespace ks
