// Hartree potential: L v = 4 pi rho with L = -Laplacian_h (7 points, zero Dirichlet).
//
// Two solvers share the device state CgState:
//  * plain conjugate gradients, warm started from the previous potential (the Hartree
//    solve of the paper's energy evaluation, Section 2.3);
//  * the same iteration preconditioned by the exact inverse of L in its eigenbasis
//    ("fast diagonalisation"): the Dirichlet 7-point L on a box is
//    L = (T_x (+) T_y (+) T_z)/h^2 with T = tridiag(-1, 2, -1), and T = S diag(lambda) S
//    with S the orthogonal, symmetric type-I sine transform,
//    S_jm = sqrt(2/(N+1)) sin(pi (j+1)(m+1)/(N+1)), lambda_m = 2 - 2 cos(pi (m+1)/(N+1)).
//    Hence L^{-1} = (S_z x S_y x S_x) diag(h^2/(lx+ly+lz)) (S_z x S_y x S_x); each factor is
//    a dense N x N contraction along one axis.  With it the conjugate-gradient
//    iteration converges in one or two steps.
//
// Reductions are fixed order: each grid kernel writes one partial per block and a
// one-block kernel finishes the sum and updates the scalars, so there are no grid-wide
// fences and results are reproducible bit for bit.
#include <algorithm>

#include "ks_common.h"

namespace ks {

int fd_rz_blocks(Grid g);

namespace {

constexpr int kCgBlocksMax = 1024;

inline int cg_nblocks(int n) {
  int b = (n + kBlock - 1) / kBlock;
  return b < 1 ? 1 : (b > kCgBlocksMax ? kCgBlocksMax : b);
}

__device__ inline void range_of(int n, int lb, int nb, int* beg, int* end) {
  int per = (n + nb - 1) / nb;
  per = (per + kBlock - 1) / kBlock * kBlock;
  const long b0 = (long)lb * per;
  *beg = (int)(b0 < n ? b0 : n);
  const long e = b0 + per;
  *end = (int)(e < n ? e : n);
}

__device__ inline double lap7(const double* __restrict__ u, int g, int i, int j, int k,
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

// part layout: [4][kCgBlocksMax]
__device__ inline void put2(double* part, int lb, double a, double b, double* sh, int sa,
                            int sb) {
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) {
    part[sa * kCgBlocksMax + lb] = a;
    part[sb * kCgBlocksMax + lb] = b;
  }
}

__device__ inline double fin_sum(const double* part, int slot, int nb, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[slot * kCgBlocksMax + i];
  return block_sum(v, sh);
}

// r = 4 pi rho - L x0 ; x = x0 (or 0) ; p = 0 ; partials r.r (slot 0), b.b (slot 1)
__global__ void k_init(const double* __restrict__ rho, const double* __restrict__ x0,
                       double* __restrict__ x, double* __restrict__ r, double* __restrict__ p0,
                       Grid gr, double* __restrict__ part) {
  __shared__ double sh[kBlock / kWave];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  int beg, end;
  range_of(gr.n, lb, gridDim.x, &beg, &end);
  double rr = 0.0, bb = 0.0;
  for (int g = beg + threadIdx.x; g < end; g += blockDim.x) {
    const int i = g % gr.nx, j = (g / gr.nx) % gr.ny, k = g / (gr.nx * gr.ny);
    const double b = 4.0 * kPi * rho[g];
    const double ri = x0 ? b - lap7(x0, g, i, j, k, gr) : b;
    x[g] = x0 ? x0[g] : 0.0;
    r[g] = ri;
    p0[g] = 0.0;
    rr += ri * ri;
    bb += b * b;
  }
  put2(part, lb, rr, bb, sh, 0, 1);
}

__global__ void k_fin_init(const double* __restrict__ part, int nb, CgState* cs, double tol,
                           int maxit) {
  __shared__ double sh[kBlock / kWave];
  const double rr = fin_sum(part, 0, nb, sh);
  const double bb = fin_sum(part, 1, nb, sh);
  if (threadIdx.x == 0) {
    cs->rr = rr;
    cs->bb = bb;
    cs->tol2 = tol * tol;
    cs->alpha = cs->beta = cs->pq = 0.0;
    cs->rz = 0.0;
    cs->it = 0;
    cs->maxit = maxit;
    cs->done = (bb == 0.0 || !isfinite(rr) || !isfinite(bb) || rr <= tol * tol * bb) ? 1 : 0;
  }
}

// pn = z + beta po ; q = L pn ; partial pn.q (slot 2).  z = r for plain CG.
__global__ void k_dir(const double* __restrict__ z, const double* __restrict__ po,
                      double* __restrict__ pn, double* __restrict__ q, const CgState* cs, Grid gr,
                      double* __restrict__ part) {
  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double beta = cs->beta;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  int beg, end;
  range_of(gr.n, lb, gridDim.x, &beg, &end);
  const int sz = gr.nx * gr.ny;
  double pq = 0.0;
  for (int g = beg + threadIdx.x; g < end; g += blockDim.x) {
    const int i = g % gr.nx, j = (g / gr.nx) % gr.ny, k = g / sz;
    const double pc = z[g] + beta * po[g];
    double nb = 0.0;
    if (i > 0) nb += z[g - 1] + beta * po[g - 1];
    if (i < gr.nx - 1) nb += z[g + 1] + beta * po[g + 1];
    if (j > 0) nb += z[g - gr.nx] + beta * po[g - gr.nx];
    if (j < gr.ny - 1) nb += z[g + gr.nx] + beta * po[g + gr.nx];
    if (k > 0) nb += z[g - sz] + beta * po[g - sz];
    if (k < gr.nz - 1) nb += z[g + sz] + beta * po[g + sz];
    const double qq = (6.0 * pc - nb) * gr.inv_h2;
    pn[g] = pc;
    q[g] = qq;
    pq += pc * qq;
  }
  pq = block_sum(pq, sh);
  if (threadIdx.x == 0) part[2 * kCgBlocksMax + lb] = pq;
}

// alpha = (r.z)/(p.q)   (r.z = r.r for plain CG)
__global__ void k_fin_dir(const double* __restrict__ part, int nb, CgState* cs, int pcg) {
  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double pq = fin_sum(part, 2, nb, sh);
  if (threadIdx.x == 0) {
    cs->pq = pq;
    cs->alpha = (pcg ? cs->rz : cs->rr) / pq;
  }
}

// x += alpha p ; r -= alpha q ; partial r.r (slot 0)
__global__ void k_upd(double* __restrict__ x, double* __restrict__ r,
                      const double* __restrict__ pn, const double* __restrict__ q,
                      const CgState* cs, Grid gr, double* __restrict__ part) {
  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double alpha = cs->alpha;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  int beg, end;
  range_of(gr.n, lb, gridDim.x, &beg, &end);
  double rr = 0.0;
  for (int g = beg + threadIdx.x; g < end; g += blockDim.x) {
    x[g] += alpha * pn[g];
    const double rn = r[g] - alpha * q[g];
    r[g] = rn;
    rr += rn * rn;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) part[0 * kCgBlocksMax + lb] = rr;
}

// plain CG: beta = rr_new/rr ; convergence
__global__ void k_fin_upd(const double* __restrict__ part, int nb, CgState* cs, int pcg) {
  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double rr = fin_sum(part, 0, nb, sh);
  if (threadIdx.x == 0) {
    if (!pcg) cs->beta = rr / cs->rr;
    cs->rr = rr;
    cs->it += 1;
    cs->done = (!isfinite(rr) || rr <= cs->tol2 * cs->bb || cs->it >= cs->maxit) ? 1 : 0;
  }
}

// PCG: rz_new = r.z (slot 3, written by the last transform) ; beta = rz_new/rz
__global__ void k_fin_rz(const double* __restrict__ part, int nb, CgState* cs) {
  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double rz = fin_sum(part, 3, nb, sh);
  if (threadIdx.x == 0) {
    cs->beta = (cs->it == 0) ? 0.0 : rz / cs->rz;
    cs->rz = rz;
  }
}

// ---- fast-diagonalisation preconditioner --------------------------------------------

// S (N x N) and lambda (N) for one axis.
__global__ void k_fd_setup(double* __restrict__ S, double* __restrict__ lam, int N, double h) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N * N) {
    const int j = e / N, m = e % N;
    S[e] = sqrt(2.0 / (N + 1)) * sin(kPi * (double)((j + 1) * (m + 1)) / (double)(N + 1));
  }
  if (e < N) lam[e] = (2.0 - 2.0 * cos(kPi * (double)(e + 1) / (double)(N + 1))) / (h * h);
}

struct FdArgs {
  const double* in;
  double* out;
  const double* S;     // N x N
  int N;               // transform length
  int stride;          // element stride along the axis
  int inner;           // number of lines adjacent in memory (= stride for y, z)
  int nouter;          // outer line index count
  // optional eigenvalue scaling (forward z transform): out *= 1/(lx[i]+ly[j]+lz[k])
  const double* lx; const double* ly; const double* lz; int nx;
  // optional partial r.z with the final output (slot 3)
  const double* r; double* part;
  int skip_if_done;
  const CgState* cs;
};

// Transform along an axis whose lines are adjacent in memory (y: stride nx, z: stride
// nx*ny).  Block = 64 adjacent lines x all N points, staged in LDS; wave w produces the
// outputs w, w+4, ... of every line.
__global__ __launch_bounds__(256) void k_fd_strided(FdArgs a) {
  extern __shared__ double tile[];  // N x 64
  __shared__ double sh[kBlock / kWave];
  if (a.skip_if_done && a.cs->done) return;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int l0 = blockIdx.x * 64, outer = blockIdx.y;
  const int line = l0 + lane;
  const bool ok = line < a.inner;
  const size_t base = (size_t)outer * a.N * a.stride + line;
  for (int m = w; m < a.N; m += 4) tile[m * 64 + lane] = ok ? a.in[base + (size_t)m * a.stride] : 0.0;
  __syncthreads();
  double rz = 0.0;
  for (int j = w; j < a.N; j += 4) {
    const double* Sj = a.S + (size_t)j * a.N;
    double acc = 0.0;
    for (int m = 0; m < a.N; ++m) acc += Sj[m] * tile[m * 64 + lane];
    if (ok) {
      const size_t o = base + (size_t)j * a.stride;
      if (a.lx) {
        // forward z transform: (i, jy) from the line index, k = j
        const int i = line % a.nx, jy = line / a.nx;
        acc /= (a.lx[i] + a.ly[jy] + a.lz[j]);
      }
      a.out[o] = acc;
      if (a.part) rz += acc * a.r[o];
    }
  }
  if (a.part) {
    rz = block_sum(rz, sh);
    if (threadIdx.x == 0) a.part[3 * kCgBlocksMax + blockIdx.y * gridDim.x + blockIdx.x] = rz;
  }
}

// Transform along x (lines contiguous).  Block = 64 lines, loaded coalesced and
// transposed into LDS; every block reads all points of its own lines before writing
// them, so the transform may run in place.
__global__ __launch_bounds__(256) void k_fd_x(FdArgs a) {
  extern __shared__ double tile[];  // N x 65 (padded against bank conflicts)
  if (a.skip_if_done && a.cs->done) return;
  const int N = a.N;
  const int l0 = blockIdx.x * 64;
  const int nl = min(64, a.nouter - l0);
  const size_t gbase = (size_t)l0 * N;
  for (int e = threadIdx.x; e < 64 * N; e += blockDim.x) {
    const int l = e / N, m = e % N;
    tile[m * 65 + l] = (l < nl) ? a.in[gbase + e] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  for (int i = w; i < N; i += 4) {
    const double* Si = a.S + (size_t)i * N;
    double acc = 0.0;
    for (int m = 0; m < N; ++m) acc += Si[m] * tile[m * 65 + lane];
    if (lane < nl) a.out[gbase + (size_t)lane * N + i] = acc;
  }
}

}  // namespace

size_t hartree_part_doubles() { return (size_t)4 * kCgBlocksMax; }

size_t fd_lds_bytes_max(int N) { return (size_t)N * 65 * sizeof(double); }

void launch_fd_setup(double* S, double* lam, int N, double h, hipStream_t st) {
  hipLaunchKernelGGL(k_fd_setup, dim3((N * N + 255) / 256), dim3(256), 0, st, S, lam, N, h);
}

void launch_hartree_init(const double* rho, const double* x0, double* x, double* r, double* p0,
                         CgState* cs, double tol, int maxit, Grid g, double* part,
                         hipStream_t st) {
  const int nb = cg_nblocks(g.n);
  hipLaunchKernelGGL(k_init, dim3(nb), dim3(kBlock), 0, st, rho, x0, x, r, p0, g, part);
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kBlock), 0, st, part, nb, cs, tol, maxit);
}

namespace {
void set_lds(const void* k, size_t bytes) {
  if (bytes > 32768)
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
}  // namespace

// z = L^{-1} r by the fast diagonalisation, with the partial r.z of the result; the
// transforms after the first run in place on z.
void launch_fd_apply(const double* r, double* z, const FdOps& fd, Grid g, const CgState* cs,
                     double* part, hipStream_t st) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const size_t lx = (size_t)nx * 65 * sizeof(double);
  const size_t ly = (size_t)ny * 64 * sizeof(double);
  const size_t lz = (size_t)nz * 64 * sizeof(double);
  set_lds(reinterpret_cast<const void*>(k_fd_x), lx);
  set_lds(reinterpret_cast<const void*>(k_fd_strided), std::max(ly, lz));
  auto xform_x = [&](const double* in) {
    FdArgs a{};
    a.skip_if_done = 1; a.cs = cs; a.nx = nx;
    a.in = in; a.out = z; a.S = fd.Sx; a.N = nx; a.nouter = ny * nz;
    hipLaunchKernelGGL(k_fd_x, dim3((ny * nz + 63) / 64), dim3(256), lx, st, a);
  };
  auto xform_y = [&](bool rz) {
    FdArgs a{};
    a.skip_if_done = 1; a.cs = cs; a.nx = nx;
    a.in = z; a.out = z; a.S = fd.Sy; a.N = ny; a.stride = nx; a.inner = nx; a.nouter = nz;
    if (rz) { a.r = r; a.part = part; }
    hipLaunchKernelGGL(k_fd_strided, dim3((nx + 63) / 64, nz), dim3(256), ly, st, a);
  };
  auto xform_z = [&](bool scale) {
    FdArgs a{};
    a.skip_if_done = 1; a.cs = cs; a.nx = nx;
    a.in = z; a.out = z; a.S = fd.Sz; a.N = nz; a.stride = nx * ny; a.inner = nx * ny;
    a.nouter = 1;
    if (scale) { a.lx = fd.lx; a.ly = fd.ly; a.lz = fd.lz; }
    hipLaunchKernelGGL(k_fd_strided, dim3((nx * ny + 63) / 64, 1), dim3(256), lz, st, a);
  };
  xform_x(r);       // forward, r -> z
  xform_y(false);
  xform_z(true);    // with 1/(lx + ly + lz)
  xform_z(false);   // inverse (S is symmetric and orthogonal)
  xform_x(z);
  xform_y(true);    // with the partial r.z
  hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kBlock), 0, st, part, fd_rz_blocks(g),
                     const_cast<CgState*>(cs));
}

int fd_rz_blocks(Grid g) { return ((g.nx + 63) / 64) * g.nz; }

void launch_hartree_iter(double* x, double* r, const double* z, double* pa, double* pb,
                         double* q, CgState* cs, Grid g, double* part, int pcg,
                         hipStream_t st) {
  const int nb = cg_nblocks(g.n);
  hipLaunchKernelGGL(k_dir, dim3(nb), dim3(kBlock), 0, st, pcg ? z : r, pa, pb, q, cs, g, part);
  hipLaunchKernelGGL(k_fin_dir, dim3(1), dim3(kBlock), 0, st, part, nb, cs, pcg);
  hipLaunchKernelGGL(k_upd, dim3(nb), dim3(kBlock), 0, st, x, r, pb, q, cs, g, part);
  hipLaunchKernelGGL(k_fin_upd, dim3(1), dim3(kBlock), 0, st, part, nb, cs, pcg);
}

}  // namespace ks
