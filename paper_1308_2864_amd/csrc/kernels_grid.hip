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

template <typename T>
__global__ void k_density(const T* __restrict__ X, int ld, int n, int p, double scale,
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

// ---- Slater exchange, effective potential, Hartree/exchange energy partials ------------

__global__ void k_xc(const double* __restrict__ rho, const double* __restrict__ vh,
                     const double* __restrict__ vext, double* __restrict__ veff, Grid gr,
                     int use_h, int use_x, const CgState* __restrict__ cg, Partials pt) {
  __shared__ double sh[kBlock / kWave];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  size_t beg, end;
  block_range((size_t)gr.n, lb, gridDim.x, &beg, &end);
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

// ---- Hamiltonian on the orbital block -----------------------------------------------
// Y = scale * ((1/2) L X + Diag(veff) X), L = -Laplacian_h (7 points, zero Dirichlet).
// With pt: per-block partials of sum X.(LX) and sum vext X^2 (kinetic/external energy).

template <typename T, bool kEnergy>
__global__ void k_hx(const T* __restrict__ X, int ldx, T* __restrict__ Y, int ldy,
                     const double* __restrict__ veff, const double* __restrict__ vext, Grid gr,
                     int p, double scale, Partials pt) {
  __shared__ double sh[kBlock / kWave];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const size_t work = (size_t)gr.n * p;
  size_t beg, end;
  block_range(work, lb, gridDim.x, &beg, &end);
  const int nx = gr.nx, ny = gr.ny, nz = gr.nz;
  const size_t sy = (size_t)nx * ldx, sz = (size_t)nx * ny * ldx;
  const double ih2 = gr.inv_h2;
  double kin = 0.0, ext = 0.0;
  for (size_t t = beg + threadIdx.x; t < end; t += blockDim.x) {
    const size_t g = t / (unsigned)p;
    const int c = (int)(t - g * p);
    const int i = (int)(g % nx);
    const size_t gy = g / nx;
    const int j = (int)(gy % ny), k = (int)(gy / ny);
    const T* xp = X + g * ldx + c;
    const double x0 = (double)xp[0];
    double nb = 0.0;
    if (i > 0) nb += (double)xp[-ldx];
    if (i < nx - 1) nb += (double)xp[ldx];
    if (j > 0) nb += (double)xp[-(ptrdiff_t)sy];
    if (j < ny - 1) nb += (double)xp[sy];
    if (k > 0) nb += (double)xp[-(ptrdiff_t)sz];
    if (k < nz - 1) nb += (double)xp[sz];
    const double lx = (6.0 * x0 - nb) * ih2;
    Y[g * ldy + c] = (T)(scale * (0.5 * lx + veff[g] * x0));
    if (kEnergy) {
      kin += x0 * lx;
      ext += vext[g] * x0 * x0;
    }
  }
  if (kEnergy) {
    kin = block_sum(kin, sh);
    ext = block_sum(ext, sh);
    write_partial(pt, SL_KIN, lb, kin);
    write_partial(pt, SL_EXT, lb, ext);
  }
}

// ---- Hartree: conjugate gradients on L v = 4 pi rho ---------------------------------
// The scalars alpha, beta, r.r live in CgState.  Each reduction is finished by the last
// block to arrive (fixed summation order over the per-block partials), so one CG
// iteration is two launches.  Every kernel returns at once when the solve is done, so
// the host can queue iterations ahead of the convergence check.

__device__ inline double lap_at(const double* __restrict__ u, int g, int i, int j, int k,
                                const Grid& gr) {
  double nb = 0.0;
  if (i > 0) nb += u[g - 1];
  if (i < gr.nx - 1) nb += u[g + 1];
  if (j > 0) nb += u[g - gr.nx];
  if (j < gr.ny - 1) nb += u[g + gr.nx];
  const int sz = gr.nx * gr.ny;
  if (k > 0) nb += u[g - sz];
  if (k < gr.nz - 1) nb += u[g + sz];
  return (6.0 * u[g] - nb) * gr.inv_h2;
}

// Fixed-order sum of part[0..nb) by one block; result valid in thread 0.
__device__ inline double last_block_sum(const double* part, int nb, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
  return block_sum(v, sh);
}

// Returns true in every thread of the block that arrives last.
__device__ inline bool arrive_last(unsigned int* count) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int prev = atomicAdd(count, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}

__global__ void k_cg_init(const double* __restrict__ rho, const double* __restrict__ x0,
                          double* __restrict__ x, double* __restrict__ r,
                          double* __restrict__ p0, CgState* cs, double tol, int maxit, Grid gr,
                          double* __restrict__ part) {
  __shared__ double sh[kBlock / kWave];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  size_t beg, end;
  block_range((size_t)gr.n, lb, gridDim.x, &beg, &end);
  double rr = 0.0, bb = 0.0;
  for (size_t gg = beg + threadIdx.x; gg < end; gg += blockDim.x) {
    const int g = (int)gg;
    const int i = g % gr.nx, j = (g / gr.nx) % gr.ny, k = g / (gr.nx * gr.ny);
    const double b = 4.0 * kPi * rho[g];
    const double ri = x0 ? b - lap_at(x0, g, i, j, k, gr) : b;
    x[g] = x0 ? x0[g] : 0.0;
    r[g] = ri;
    p0[g] = 0.0;
    rr += ri * ri;
    bb += b * b;
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[lb] = rr;
    part[gridDim.x + lb] = bb;
  }
  if (arrive_last(&cs->count)) {
    const double trr = last_block_sum(part, gridDim.x, sh);
    const double tbb = last_block_sum(part + gridDim.x, gridDim.x, sh);
    if (threadIdx.x == 0) {
      cs->rr = trr;
      cs->bb = tbb;
      cs->tol2 = tol * tol;
      cs->beta = 0.0;
      cs->alpha = 0.0;
      cs->it = 0;
      cs->maxit = maxit;
      cs->done = (tbb == 0.0 || !isfinite(trr) || !isfinite(tbb) || trr <= tol * tol * tbb)
                     ? 1 : 0;
      cs->count = 0;
    }
  }
}

// pn = r + beta*po ; q = L pn ; partial pn.q ; last block: alpha = rr/pq
__global__ void k_cg_dir(const double* __restrict__ r, const double* __restrict__ po,
                         double* __restrict__ pn, double* __restrict__ q, CgState* cs, Grid gr,
                         double* __restrict__ part) {
  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double beta = cs->beta;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  size_t beg, end;
  block_range((size_t)gr.n, lb, gridDim.x, &beg, &end);
  const int sz = gr.nx * gr.ny;
  double pq = 0.0;
  for (size_t gg = beg + threadIdx.x; gg < end; gg += blockDim.x) {
    const int g = (int)gg;
    const int i = g % gr.nx, j = (g / gr.nx) % gr.ny, k = g / sz;
    const double pc = r[g] + beta * po[g];
    double nb = 0.0;
    if (i > 0) nb += r[g - 1] + beta * po[g - 1];
    if (i < gr.nx - 1) nb += r[g + 1] + beta * po[g + 1];
    if (j > 0) nb += r[g - gr.nx] + beta * po[g - gr.nx];
    if (j < gr.ny - 1) nb += r[g + gr.nx] + beta * po[g + gr.nx];
    if (k > 0) nb += r[g - sz] + beta * po[g - sz];
    if (k < gr.nz - 1) nb += r[g + sz] + beta * po[g + sz];
    const double qq = (6.0 * pc - nb) * gr.inv_h2;
    pn[g] = pc;
    q[g] = qq;
    pq += pc * qq;
  }
  pq = block_sum(pq, sh);
  if (threadIdx.x == 0) part[lb] = pq;
  if (arrive_last(&cs->count)) {
    const double t = last_block_sum(part, gridDim.x, sh);
    if (threadIdx.x == 0) {
      cs->pq = t;
      cs->alpha = cs->rr / t;
      cs->count = 0;
    }
  }
}

// x += alpha p ; r -= alpha q ; partial r.r ; last block: beta, convergence
__global__ void k_cg_upd(double* __restrict__ x, double* __restrict__ r,
                         const double* __restrict__ pn, const double* __restrict__ q,
                         CgState* cs, Grid gr, double* __restrict__ part) {
  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double alpha = cs->alpha;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  size_t beg, end;
  block_range((size_t)gr.n, lb, gridDim.x, &beg, &end);
  double rr = 0.0;
  for (size_t g = beg + threadIdx.x; g < end; g += blockDim.x) {
    x[g] += alpha * pn[g];
    const double rn = r[g] - alpha * q[g];
    r[g] = rn;
    rr += rn * rn;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) part[gridDim.x + lb] = rr;
  if (arrive_last(&cs->count)) {
    const double t = last_block_sum(part + gridDim.x, gridDim.x, sh);
    if (threadIdx.x == 0) {
      cs->beta = t / cs->rr;
      cs->rr = t;
      cs->it += 1;
      cs->done = (!isfinite(t) || t <= cs->tol2 * cs->bb || cs->it >= cs->maxit) ? 1 : 0;
      cs->count = 0;
    }
  }
}

// ---- fixed-order reduction of per-block partials: one block per slot ---------------

struct NBlk {
  int v[kMaxScalarSlots];
};

__global__ void k_reduce_scalars(const double* __restrict__ part, int stride, NBlk nb,
                                 double* __restrict__ out) {
  __shared__ double sh[kBlock / kWave];
  const int s = blockIdx.x;
  const int m = nb.v[s];
  double v = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) v += part[(size_t)s * stride + i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) out[s] = v;
}

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

template <typename T>
void launch_density(const T* X, int ld, int n, int p, double scale, double* rho,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_density<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, X, ld,
                     n, p, scale, rho);
}
template void launch_density<double>(const double*, int, int, int, double, double*,
                                     hipStream_t);
template void launch_density<float>(const float*, int, int, int, double, double*, hipStream_t);

int scalar_blocks(int n) { return stream_blocks((size_t)n); }

void launch_xc(const double* rho, const double* vh, const double* vext, double* veff, Grid g,
               int use_h, int use_x, const CgState* cg, Partials pt, hipStream_t st) {
  hipLaunchKernelGGL(k_xc, dim3(scalar_blocks(g.n)), dim3(kBlock), 0, st, rho, vh, vext, veff,
                     g, use_h, use_x, cg, pt);
}

template <typename T>
void launch_hx(const T* X, int ldx, T* Y, int ldy, const double* veff, const double* vext,
               Grid g, int p, double scale, Partials* pt, hipStream_t st) {
  const int nb = stream_blocks((size_t)g.n * p);
  if (pt) {
    hipLaunchKernelGGL((k_hx<T, true>), dim3(nb), dim3(kBlock), 0, st, X, ldx, Y, ldy, veff,
                       vext, g, p, scale, *pt);
  } else {
    Partials none{nullptr, 0};
    hipLaunchKernelGGL((k_hx<T, false>), dim3(nb), dim3(kBlock), 0, st, X, ldx, Y, ldy, veff,
                       vext, g, p, scale, none);
  }
}
template void launch_hx<double>(const double*, int, double*, int, const double*,
                                const double*, Grid, int, double, Partials*, hipStream_t);
template void launch_hx<float>(const float*, int, float*, int, const double*, const double*,
                               Grid, int, double, Partials*, hipStream_t);

int hx_blocks(size_t work) { return stream_blocks(work); }

int cg_blocks(int n) {
  int b = (n + kBlock - 1) / kBlock;
  return b < 1024 ? (b < 1 ? 1 : b) : 1024;
}

void launch_cg_init(const double* rho, const double* x0, double* x, double* r, double* p0,
                    CgState* cs, double tol, int maxit, Grid g, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init, dim3(cg_blocks(g.n)), dim3(kBlock), 0, st, rho, x0, x, r, p0,
                     cs, tol, maxit, g, part);
}

void launch_cg_iter(double* x, double* r, double* pa, double* pb, double* q, CgState* cs,
                    Grid g, double* part, hipStream_t st) {
  const int nb = cg_blocks(g.n);
  hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(kBlock), 0, st, r, pa, pb, q, cs, g, part);
  hipLaunchKernelGGL(k_cg_upd, dim3(nb), dim3(kBlock), 0, st, x, r, pb, q, cs, g, part);
}

void launch_reduce_scalars(const double* part, int stride, const int* nblk, int nslots,
                           double* out, hipStream_t st) {
  NBlk nb{};
  for (int i = 0; i < nslots && i < kMaxScalarSlots; ++i) nb.v[i] = nblk[i];
  hipLaunchKernelGGL(k_reduce_scalars, dim3(nslots), dim3(kBlock), 0, st, part, stride, nb,
                     out);
}

}  // namespace ks
