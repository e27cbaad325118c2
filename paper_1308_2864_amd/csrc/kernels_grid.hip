// Grid kernels of the energy/gradient assembly (the paper's "T0" part, Section 4.1):
// nuclear potential, density, Hartree conjugate gradients, Slater exchange and the
// 7-point Hamiltonian applied to the orbital block, with fused FP64 energy partials.
//
// Layout: n-vectors are double[n] in linear grid order g = i + nx*(j + ny*k); orbital
// blocks are n x ld row-major ("grid-major"): consecutive threads walk consecutive
// orbitals of one grid point, then the next point, so every wavefront load is one
// contiguous segment.
#include "ks_common.h"

namespace ks {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kMaxStreamBlocks = 4096;  // blocks of the grid-stride streaming kernels

inline int stream_blocks(size_t work) {
  size_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (int)(b < (size_t)kMaxStreamBlocks ? b : (size_t)kMaxStreamBlocks);
}

// Contiguous range [beg, end) of work items for logical block lb of nb.
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

// ---- setup ---------------------------------------------------------------------------

__global__ void k_vext(double* __restrict__ v, const double* __restrict__ R,
                       const double* __restrict__ Z, int M, Grid g, double rc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.n) return;
  const int i = idx % g.nx, j = (idx / g.nx) % g.ny, k = idx / (g.nx * g.ny);
  const double x = g.lo[0] + (i + 1) * g.h, y = g.lo[1] + (j + 1) * g.h,
               z = g.lo[2] + (k + 1) * g.h;
  double acc = 0.0;
  for (int a = 0; a < M; ++a) {
    const double dx = x - R[3 * a], dy = y - R[3 * a + 1], dz = z - R[3 * a + 2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    double t;
    if (d < 1e-6) {
      // series of erf(d/rc)/d about d = 0
      t = (2.0 / (sqrt(kPi) * rc)) * (1.0 - d * d / (3.0 * rc * rc));
    } else {
      t = erf(d / rc) / d;
    }
    acc -= Z[a] * t;
  }
  v[idx] = acc;
}

__global__ void k_enuc(double* out, const double* R, const double* Z, int M) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double e = 0.0;
  for (int a = 0; a < M; ++a)
    for (int b = a + 1; b < M; ++b) {
      const double dx = R[3 * a] - R[3 * b], dy = R[3 * a + 1] - R[3 * b + 1],
                   dz = R[3 * a + 2] - R[3 * b + 2];
      e += Z[a] * Z[b] / sqrt(dx * dx + dy * dy + dz * dz);
    }
  *out = e;
}

__global__ void k_fill(double* x, double v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] = v;
}

__global__ void k_copy_vec(double* __restrict__ d, const double* __restrict__ s, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) d[i] = s[i];
}

template <typename T>
__global__ void k_copy_block(T* __restrict__ d, int ldd, const T* __restrict__ s, int lds,
                             int n, int p) {
  const size_t work = (size_t)n * p;
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; t < work; t += (size_t)gridDim.x * blockDim.x) {
    const size_t g = t / p, c = t - g * p;
    d[g * ldd + c] = s[g * lds + c];
  }
}

// ---- density rho_g = scale * sum_i X_gi^2 ----------------------------------------------

// Up to 64 columns a thread sums its row in column order (the density of a start block;
// wide retractions use the grouped form below).
template <typename T>
__global__ void k_density_row(const T* __restrict__ X, int ld, int n, int p, double scale,
                              double* __restrict__ rho) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const T* row = X + (size_t)g * ld;
  double s = 0.0;
  for (int c = 0; c < p; ++c) {
    const double x = (double)row[c];
    s += x * x;
  }
  rho[g] = scale * s;
}

// Wider blocks: kG = 64 lanes share a row, each summing the squares of columns lane,
// lane + 64, ... (a wave reads one row of contiguous memory), then the lanes fold in a
// fixed order.
template <typename T, int kG>
__global__ __launch_bounds__(256) void k_density(const T* __restrict__ X, int ld, int n, int p,
                                                 double scale, double* __restrict__ rho) {
  constexpr int kRows = kWave / kG;
  const int lane = threadIdx.x % kWave, sub = lane % kG;
  const size_t g = ((size_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kRows +
                   lane / kG;
  double s = 0.0;
  if (g < (size_t)n) {
    const T* row = X + g * ld;
    for (int c = sub; c < p; c += kG) {
      const double x = (double)row[c];
      s += x * x;
    }
  }
#pragma unroll
  for (int m = kG / 2; m >= 1; m /= 2) s += __shfl_xor(s, m, kG);
  if (g < (size_t)n && sub == 0) rho[g] = scale * s;
}

// ---- Slater exchange, effective potential, Hartree/exchange energy partials ------------

__device__ inline void k_xc_body(const XcArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ rho = ka.rho;
  const double* __restrict__ vh = ka.vh;
  const double* __restrict__ vext = ka.vext;
  double* __restrict__ veff = ka.veff;
  Grid gr = ka.gr;
  int use_h = ka.use_h;
  int use_x = ka.use_x;
  const CgState* __restrict__ cg = ka.cg;
  Partials pt = ka.pt;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kBlock / kWave];
  const int lb = xcd_remap(ks_bid, ks_nb);
  size_t beg, end;
  block_range((size_t)gr.n, lb, ks_nb, &beg, &end);
  // (3/4)(3/pi)^{1/3} and (3/pi)^{1/3}
  const double cv = cbrt(3.0 / kPi), cx = 0.75 * cv;
  const bool trivial = use_h && cg != nullptr && cg->bb == 0.0;  // rho == 0: V_H = 0
  double eh = 0.0, ex = 0.0;
  for (size_t g = beg + threadIdx.x; g < end; g += blockDim.x) {
    const double r = rho[g];
    const double h = (use_h && !trivial) ? vh[g] : 0.0;
    double vx = 0.0, e = 0.0;
    if (use_x) {
      const double c = cbrt(r);
      vx = -cv * c;
      e = -cx * c;
    }
    veff[g] = vext[g] + h + vx;
    eh += r * h;
    ex += r * e;
  }
  eh = block_sum(eh, sh);
  ex = block_sum(ex, sh);
  write_partial(pt, SL_EH, lb, eh);
  write_partial(pt, SL_EX, lb, ex);
}

__global__ void k_xc(XcArgs ka) {
  k_xc_body(ka, blockIdx.x, gridDim.x);
}

__global__ void k_xc_batch(BatchPtrs<XcArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_xc_body(*b.a[s], blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// ---- Hamiltonian on the orbital block -----------------------------------------------
// Y = scale * ((1/2) L X + Diag(veff) X), L = -Laplacian_h (7 points, zero Dirichlet).
// With pt: per-block partials of sum X.(LX) and sum vext X^2 (kinetic/external energy).

// A thread owns kW orbitals (a column pair when p, ld are even and the blocks are
// pair-aligned) of one grid column (i, j) over kHxChunk consecutive planes.  The centre
// values of those planes and of the two planes around them are loaded first, so the z
// neighbours come from registers and each output needs only its four in-plane
// neighbours; all loads are branch-free (clamped addresses, zero outside the grid).
// Consecutive threads take consecutive orbitals of one point.
constexpr int kHxChunk = 8;

template <typename T, int kW>
struct HxVec {
  typedef T type __attribute__((ext_vector_type(kW)));
};
template <typename T>
struct HxVec<T, 1> {
  typedef T type;
};

template <typename T, int kW>
__device__ inline void hx_load(const T* ptr, bool ok, double (&v)[kW]) {
  const typename HxVec<T, kW>::type w = *reinterpret_cast<const typename HxVec<T, kW>::type*>(ptr);
  if constexpr (kW == 1) {
    v[0] = ok ? (double)w : 0.0;
  } else {
#pragma unroll
    for (int e = 0; e < kW; ++e) v[e] = ok ? (double)w[e] : 0.0;
  }
}

template <typename T, bool kEnergy, int kW>
__device__ inline void hx_items(const HxArgs<T>& ka, int lb, int nblk, double& kin,
                                double& ext) {
  const T* __restrict__ X = ka.X;
  const int ldx = ka.ldx, ldy = ka.ldy;
  T* __restrict__ Y = ka.Y;
  const double* __restrict__ veff = ka.veff;
  const double* __restrict__ vext = ka.vext;
  const Grid gr = ka.gr;
  const int nx = gr.nx, ny = gr.ny, nz = gr.nz;
  const int pw = ka.p / kW;
  const int nzc = (nz + kHxChunk - 1) / kHxChunk;
  const size_t work = (size_t)nx * ny * pw * nzc;
  const ptrdiff_t sy = (ptrdiff_t)nx * ldx, sz = (ptrdiff_t)nx * ny * ldx;
  const double ih2 = gr.inv_h2, scale = ka.scale;
  for (size_t t = (size_t)lb * blockDim.x + threadIdx.x; t < work;
       t += (size_t)nblk * blockDim.x) {
    const int c = (int)(t % (unsigned)pw) * kW;
    size_t r = t / (unsigned)pw;
    const int i = (int)(r % nx);
    r /= nx;
    const int j = (int)(r % ny);
    const int k0 = (int)(r / ny) * kHxChunk;
    const int k1 = min(k0 + kHxChunk, nz);
    const T* col = X + (ptrdiff_t)(i + (size_t)nx * j) * ldx + c;
    double zc[kHxChunk + 2][kW];
#pragma unroll
    for (int u = 0; u < kHxChunk + 2; ++u) {
      const int k = k0 - 1 + u;
      const bool ok = k >= 0 && k < nz;
      hx_load<T, kW>(col + (ok ? k * sz : 0), ok, zc[u]);
    }
    const bool hxm = i > 0, hxp = i < nx - 1, hym = j > 0, hyp = j < ny - 1;
#pragma unroll
    for (int u = 0; u < kHxChunk; ++u) {
      const int k = k0 + u;
      if (k >= k1) break;
      const T* xp = col + k * sz;
      double a[kW], b[kW], cc[kW], d[kW];
      hx_load<T, kW>(xp - (hxm ? ldx : 0), hxm, a);
      hx_load<T, kW>(xp + (hxp ? ldx : 0), hxp, b);
      hx_load<T, kW>(xp - (hym ? sy : 0), hym, cc);
      hx_load<T, kW>(xp + (hyp ? sy : 0), hyp, d);
      const size_t g = i + (size_t)nx * (j + (size_t)ny * k);
      const double ve = veff[g];
      double o[kW];
#pragma unroll
      for (int e = 0; e < kW; ++e) {
        const double cur = zc[u + 1][e];
        const double nb = a[e] + b[e] + cc[e] + d[e] + zc[u][e] + zc[u + 2][e];
        const double lx = (6.0 * cur - nb) * ih2;
        o[e] = scale * (0.5 * lx + ve * cur);
        if (kEnergy) {
          kin += cur * lx;
          ext += vext[g] * cur * cur;
        }
      }
      T* yp = Y + g * ldy + c;
      if constexpr (kW == 1) {
        *yp = (T)o[0];
      } else {
        typename HxVec<T, kW>::type w;
#pragma unroll
        for (int e = 0; e < kW; ++e) w[e] = (T)o[e];
        *reinterpret_cast<typename HxVec<T, kW>::type*>(yp) = w;
      }
    }
  }
}

// The Hamiltonian with the Gram blocks X^T X and X^T G of the same pass (p = 32, column
// pairs, ld = 32).  A wavefront takes 4 grid columns x 16 column pairs, so on every plane
// its lanes hold a 4-point slice of X and of G exactly as FP64 MFMA fragments with the grid
// points as the contraction index: lane l holds point l / 16, columns 2 (l % 16) + e.  The
// even and odd columns form two 16-column tiles each, so X^T G and X^T X are 4 + 4 tiles per
// plane step (entry (m, n) of tile (a, b) is column pair (2 m + a, 2 n + b)).  The loop is
// uniform over the wavefront (MFMAs need every lane); lanes past the grid or the z chunk
// contribute zeros.
struct HxGramAcc {
  d4 xg[4], xx[4];  // tiles (a, b) at index 2 a + b
};

template <typename T>
__device__ inline void hx_gram_items(const HxArgs<T>& ka, int lb, int nblk, double& kin,
                                     double& ext, HxGramAcc& g) {
  constexpr int kW = 2, pw = 16;
  const T* __restrict__ X = ka.X;
  constexpr int ld = 2 * pw;
  T* __restrict__ Y = ka.Y;
  const double* __restrict__ veff = ka.veff;
  const double* __restrict__ vext = ka.vext;
  const Grid gr = ka.gr;
  const int nx = gr.nx, ny = gr.ny, nz = gr.nz;
  const int nzc = (nz + kHxChunk - 1) / kHxChunk;
  const size_t work = (size_t)nx * ny * pw * nzc;
  const ptrdiff_t sy = (ptrdiff_t)nx * ld, sz = (ptrdiff_t)nx * ny * ld;
  const double ih2 = gr.inv_h2, scale = ka.scale;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  for (size_t tw = ((size_t)lb * (kBlock / kWave) + w) * kWave; tw < work;
       tw += (size_t)nblk * kBlock) {
    const size_t t0 = tw + lane;
    const bool live = t0 < work;
    const size_t t = live ? t0 : tw;
    const int c = (int)(t % (unsigned)pw) * kW;
    size_t r = t / (unsigned)pw;
    const int i = (int)(r % nx);
    r /= nx;
    const int j = (int)(r % ny);
    const int k0 = (int)(r / ny) * kHxChunk;
    const int k1 = min(k0 + kHxChunk, nz);
    const T* col = X + (ptrdiff_t)(i + (size_t)nx * j) * ld + c;
    double zc[kHxChunk + 2][kW];
#pragma unroll
    for (int u = 0; u < kHxChunk + 2; ++u) {
      const int k = k0 - 1 + u;
      const bool ok = k >= 0 && k < nz;
      hx_load<T, kW>(col + (ok ? k * sz : 0), ok, zc[u]);
    }
    const bool hxm = i > 0, hxp = i < nx - 1, hym = j > 0, hyp = j < ny - 1;
#pragma unroll
    for (int u = 0; u < kHxChunk; ++u) {
      const int k = k0 + u;
      const bool ok = live && k < k1;
      const int kk = ok ? k : k0;
      const T* xp = col + kk * sz;
      double a[kW], b[kW], cc[kW], d[kW];
      hx_load<T, kW>(xp - (hxm ? ld : 0), hxm, a);
      hx_load<T, kW>(xp + (hxp ? ld : 0), hxp, b);
      hx_load<T, kW>(xp - (hym ? sy : 0), hym, cc);
      hx_load<T, kW>(xp + (hyp ? sy : 0), hyp, d);
      const size_t gp = i + (size_t)nx * (j + (size_t)ny * kk);
      const double ve = veff[gp];
      const double vx = vext[gp];
      double xo[kW], go[kW];
      typename HxVec<T, kW>::type wv;
#pragma unroll
      for (int e = 0; e < kW; ++e) {
        const double cur = zc[u + 1][e];
        const double nb = a[e] + b[e] + cc[e] + d[e] + zc[u][e] + zc[u + 2][e];
        const double lx = (6.0 * cur - nb) * ih2;
        const T o = (T)(scale * (0.5 * lx + ve * cur));
        wv[e] = o;
        if (ok) {
          kin += cur * lx;
          ext += vx * cur * cur;
        }
        xo[e] = ok ? cur : 0.0;
        go[e] = ok ? (double)o : 0.0;
      }
      if (ok) *reinterpret_cast<typename HxVec<T, kW>::type*>(Y + gp * ld + c) = wv;
#pragma unroll
      for (int ea = 0; ea < kW; ++ea)
#pragma unroll
        for (int eb = 0; eb < kW; ++eb) {
          g.xg[2 * ea + eb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xo[ea], go[eb],
                                                                    g.xg[2 * ea + eb], 0, 0, 0);
          g.xx[2 * ea + eb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xo[ea], xo[eb],
                                                                    g.xx[2 * ea + eb], 0, 0, 0);
        }
    }
  }
}

// Fixed-order sum of one 16 x 16 tile over the four wavefronts of a block (waves 1..3 park
// it in LDS, wave 0 adds them in order).
__device__ inline void hx_reduce_tile(d4& v, double* red, int w, int lane) {
  if (w > 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) red[((w - 1) * 4 + r) * kWave + lane] = v[r];
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int ww = 0; ww < 3; ++ww)
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] += red[(ww * 4 + r) * kWave + lane];
  }
  __syncthreads();
}

template <typename T, bool kEnergy, bool kGram>
__device__ inline void k_hx_body(const HxArgs<T>& ka, int ks_bid, int ks_nb) {
  __shared__ double sh[kBlock / kWave];
  const int lb = xcd_remap(ks_bid, ks_nb);
  double kin = 0.0, ext = 0.0;
  if constexpr (kGram) {
    __shared__ double red[3 * 4 * kWave];
    HxGramAcc g;
#pragma unroll
    for (int q = 0; q < 4; ++q) g.xg[q] = g.xx[q] = d4{0.0, 0.0, 0.0, 0.0};
    hx_gram_items<T>(ka, lb, ks_nb, kin, ext, g);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      hx_reduce_tile(g.xg[q], red, w, lane);
      hx_reduce_tile(g.xx[q], red, w, lane);
    }
    if (w == 0) {
      // tile (a, b), lane (lr, lc), register r: entry (2 (lr + 4 r) + a, 2 lc + b)
      constexpr int pp = 32;
      double* o0 = ka.gram_part + ((size_t)lb * 3 + 0) * pp * pp;  // X^T X
      double* o1 = ka.gram_part + ((size_t)lb * 3 + 1) * pp * pp;  // X^T G
      const int lr = lane / 16, lc = lane % 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ea = q / 2, eb = q % 2;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 2 * (lr + 4 * r) + ea, col = 2 * lc + eb;
          o0[row * pp + col] = g.xx[q][r];
          o1[row * pp + col] = g.xg[q][r];
        }
      }
    }
  } else {
    constexpr uintptr_t kAl = 2 * sizeof(T) - 1;
    const bool vec = ((ka.p | ka.ldx | ka.ldy) & 1) == 0 &&
                     ((reinterpret_cast<uintptr_t>(ka.X) | reinterpret_cast<uintptr_t>(ka.Y)) &
                      kAl) == 0;
    if (vec)
      hx_items<T, kEnergy, 2>(ka, lb, ks_nb, kin, ext);
    else
      hx_items<T, kEnergy, 1>(ka, lb, ks_nb, kin, ext);
  }
  if (kEnergy) {
    kin = block_sum(kin, sh);
    ext = block_sum(ext, sh);
    write_partial(ka.pt, SL_KIN, lb, kin);
    write_partial(ka.pt, SL_EXT, lb, ext);
  }
}

template <typename T, bool kEnergy, bool kGram = false>
__global__ __launch_bounds__(256) void k_hx(HxArgs<T> ka) {
  k_hx_body<T, kEnergy, kGram>(ka, blockIdx.x, gridDim.x);
}

template <typename T, bool kEnergy, bool kGram = false>
__global__ __launch_bounds__(256) void k_hx_batch(BatchPtrs<HxArgs<T>> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_hx_body<T, kEnergy, kGram>(*b.a[s], blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// ---- fixed-order reduction of per-block partials: one block per slot ---------------

}  // namespace

// ---- launch wrappers ------------------------------------------------------------------

void launch_vext(double* v, const double* R, const double* Z, int M, Grid g, double rc,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_vext, dim3((g.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, v, R, Z,
                     M, g, rc);
}

void launch_enuc(double* out, const double* R, const double* Z, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_enuc, dim3(1), dim3(64), 0, st, out, R, Z, M);
}

void launch_fill(double* x, double v, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(stream_blocks(n)), dim3(kBlock), 0, st, x, v, n);
}

void launch_copy_vec(double* dst, const double* src, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_vec, dim3(stream_blocks(n)), dim3(kBlock), 0, st, dst, src, n);
}

template <typename T>
void launch_copy_block(T* dst, int ldd, const T* src, int lds, int n, int p, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_block<T>, dim3(stream_blocks((size_t)n * p)), dim3(kBlock), 0, st,
                     dst, ldd, src, lds, n, p);
}
template void launch_copy_block<double>(double*, int, const double*, int, int, int,
                                        hipStream_t);
template void launch_copy_block<float>(float*, int, const float*, int, int, int, hipStream_t);

template <typename T, int kG>
void launch_density_g(const T* X, int ld, int n, int p, double scale, double* rho,
                      hipStream_t st) {
  const size_t rows_per_block = (size_t)(kBlock / kWave) * (kWave / kG);
  const size_t nb = ((size_t)n + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL((k_density<T, kG>), dim3((unsigned)(nb < 1 ? 1 : nb)), dim3(kBlock), 0, st,
                     X, ld, n, p, scale, rho);
}

template <typename T>
void launch_density(const T* X, int ld, int n, int p, double scale, double* rho,
                    hipStream_t st) {
  if (p > 64) {
    launch_density_g<T, 64>(X, ld, n, p, scale, rho, st);
    return;
  }
  hipLaunchKernelGGL(k_density_row<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, X,
                     ld, n, p, scale, rho);
}
template void launch_density<double>(const double*, int, int, int, double, double*,
                                     hipStream_t);
template void launch_density<float>(const float*, int, int, int, double, double*, hipStream_t);

int scalar_blocks(int n) { return stream_blocks((size_t)n); }

void launch_xc(const double* rho, const double* vh, const double* vext, double* veff, Grid g,
               int use_h, int use_x, const CgState* cg, Partials pt, hipStream_t st) {
  hipLaunchKernelGGL(k_xc, dim3(scalar_blocks(g.n)), dim3(kBlock), 0, st,
                     XcArgs{rho, vh, vext, veff, g, use_h, use_x, cg, pt});
}

template <typename T>
void launch_hx(const T* X, int ldx, T* Y, int ldy, const double* veff, const double* vext,
               Grid g, int p, double scale, Partials* pt, double* gram_part, hipStream_t st) {
  if (gram_part) {
    hipLaunchKernelGGL((k_hx<T, true, true>), dim3(hx_gram_blocks(g.n)), dim3(kBlock), 0, st,
                       HxArgs<T>{X, ldx, Y, ldy, veff, vext, g, p, scale, *pt, gram_part});
    return;
  }
  const int nb = hx_blocks(g.n, p);
  if (pt) {
    hipLaunchKernelGGL((k_hx<T, true>), dim3(nb), dim3(kBlock), 0, st,
                       HxArgs<T>{X, ldx, Y, ldy, veff, vext, g, p, scale, *pt, nullptr});
  } else {
    Partials none{nullptr, 0};
    hipLaunchKernelGGL((k_hx<T, false>), dim3(nb), dim3(kBlock), 0, st,
                       HxArgs<T>{X, ldx, Y, ldy, veff, vext, g, p, scale, none, nullptr});
  }
}
template void launch_hx<double>(const double*, int, double*, int, const double*,
                                const double*, Grid, int, double, Partials*, double*,
                                hipStream_t);
template void launch_hx<float>(const float*, int, float*, int, const double*, const double*,
                               Grid, int, double, Partials*, double*, hipStream_t);

int hx_blocks(int n, int p) { return stream_blocks((size_t)n * p / (2 * kHxChunk) + 1); }

// Blocks of the Hamiltonian that also forms the Gram blocks of [X, G]: as many as the Gram
// launch would use (each block writes one partial tile set).
int hx_gram_blocks(int n) {
  const int c = (n + 63) / 64;
  return c < 1 ? 1 : (c > 512 ? 512 : c);
}

bool hx_fuses_gram(int p) { return p == 32; }


void launch_xc_batch(const BatchPtrs<XcArgs>& b, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_xc_batch, dim3(blocks), dim3(kBlock), 0, st, b);
}

template <typename T>
void launch_hx_batch(const BatchPtrs<HxArgs<T>>& b, int blocks, bool gram, hipStream_t st) {
  if (gram)
    hipLaunchKernelGGL((k_hx_batch<T, true, true>), dim3(blocks), dim3(kBlock), 0, st, b);
  else
    hipLaunchKernelGGL((k_hx_batch<T, true>), dim3(blocks), dim3(kBlock), 0, st, b);
}
template void launch_hx_batch<double>(const BatchPtrs<HxArgs<double>>&, int, bool,
                                      hipStream_t);
template void launch_hx_batch<float>(const BatchPtrs<HxArgs<float>>&, int, bool, hipStream_t);

}  // namespace ks
