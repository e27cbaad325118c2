// Trilinear (Q1) finite elements on the uniform hexahedral mesh (Section 2.3, the
// finite-element form with the mass matrix B and the constraint X^T B X = I).
//
// On a uniform mesh the element matrices are tensor products of the 1D linear-element
// matrices K = (1/h) tridiag(-1, 2, -1) and M = (h/6) tridiag(1, 4, 1):
//   B = M x M x M,   A = K x M x M + M x K x M + M x M x K.
// Both are 27-point stencils with one coefficient per neighbour class (centre, face,
// edge, corner): A = (8h/3, 0, -h/6, -h/12) (the face couplings cancel exactly) and
// B = (8h^3/27, 2h^3/27, h^3/54, h^3/216).  The kernels apply them as stencils over the
// grid-major orbital block instead of as CSR matrices: no index arrays to stream, and the
// 27 loads of a node hit the same cache lines as its neighbours' loads.
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

// Y = scale ((1/2) A X + h3 veff X) and BX = B X for every (node, orbital) pair.
template <typename T, bool kG, bool kEnergy>
__global__ __launch_bounds__(256) void k_q1_apply(const T* __restrict__ X, T* __restrict__ Y,
                                                  T* __restrict__ BX,
                                                  const double* __restrict__ veff,
                                                  const double* __restrict__ vext, Grid gr,
                                                  int p, double scale, Q1Coef cf,
                                                  Partials pt) {
  __shared__ double sh[kBlock / kWave];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const size_t work = (size_t)gr.n * p;
  size_t beg, end;
  block_range(work, lb, gridDim.x, &beg, &end);
  const int nx = gr.nx, ny = gr.ny, nz = gr.nz;
  const ptrdiff_t sx = p, sy = (ptrdiff_t)nx * p, sz = (ptrdiff_t)nx * ny * p;
  const double h3 = gr.dV;
  double kin = 0.0, ext = 0.0;
  for (size_t t = beg + threadIdx.x; t < end; t += blockDim.x) {
    const size_t g = t / (unsigned)p;
    const int i = (int)(g % nx);
    const size_t gy = g / nx;
    const int j = (int)(gy % ny), k = (int)(gy / ny);
    const T* xp = X + t;
    double s[4] = {0.0, 0.0, 0.0, 0.0};  // sums per neighbour class
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      if (k + dz < 0 || k + dz >= nz) continue;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        if (j + dy < 0 || j + dy >= ny) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (i + dx < 0 || i + dx >= nx) continue;
          const int cls = (dx != 0) + (dy != 0) + (dz != 0);
          s[cls] += (double)xp[dz * sz + dy * sy + dx * sx];
        }
      }
    }
    const double x0 = s[0];
    const double ax = cf.a0 * s[0] + cf.a2 * s[2] + cf.a3 * s[3];
    const double bx = cf.b0 * s[0] + cf.b1 * s[1] + cf.b2 * s[2] + cf.b3 * s[3];
    if (kG) Y[t] = (T)(scale * (0.5 * ax + h3 * veff[g] * x0));
    BX[t] = (T)bx;
    if (kEnergy) {
      kin += x0 * ax;
      ext += h3 * vext[g] * x0 * x0;
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
// BS = BX - BXc, Yd = D - Dc, BYd = BD - BDc.
template <typename T>
__global__ __launch_bounds__(256) void k_q1_grad(Q1GradArgs a) {
  extern __shared__ double Ws[];
  __shared__ double sh[kBlock / kWave];
  const int p = a.p, pp = a.pp;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int k = e / p, j = e % p;
    Ws[e] = a.W[k * pp + j];
  }
  __syncthreads();
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
  const size_t work = (size_t)a.n * p;
  size_t beg, end;
  block_range(work, lb, gridDim.x, &beg, &end);
  double dd = 0.0, ss = 0.0, sy = 0.0, yy = 0.0;
  for (size_t t = beg + threadIdx.x; t < end; t += blockDim.x) {
    const size_t g = t / (unsigned)p;
    const int j = (int)(t - g * p);
    const T* xr = X + g * p;
    const T* br = BX + g * p;
    double u = 0.0, v = 0.0;
    for (int k = 0; k < p; ++k) {
      const double w = Ws[k * p + j];
      u += (double)xr[k] * w;
      v += (double)br[k] * w;
    }
    const T dT = (T)((double)Gt[t] + u);
    const T bT = (T)((double)G[t] + v);
    D[t] = dT;
    BD[t] = bT;
    const double d = (double)dT, bd = (double)bT;
    dd += d * bd;
    if (ref) {
      const double s = (double)X[t] - (double)Xc[t];
      const double bs = (double)BX[t] - (double)BXc[t];
      const double y = d - (double)Dc[t];
      const double by = bd - (double)BDc[t];
      ss += s * bs;
      sy += s * by;
      yy += y * by;
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

int q1_apply_blocks(int n, int p) { return stream_blocks((size_t)n * p); }
int q1_grad_blocks(int n, int p) { return stream_blocks((size_t)n * p); }

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
  const size_t lds = (size_t)a.p * a.p * sizeof(double);
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
