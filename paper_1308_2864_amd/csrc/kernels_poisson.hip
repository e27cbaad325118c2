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
// The finite-element form runs the same two solvers on A v = 4 pi h^3 rho with the Q1
// stiffness stencil: A = K x M x M + M x K x M + M x M x K, and K, M share the sine
// eigenvectors, so the preconditioner is exact there too with the divisor
// lx my mz + mx ly mz + mx my lz.
//
// Reductions are fixed order: each grid kernel writes one partial per block and a
// one-block kernel finishes the sum and updates the scalars, so there are no grid-wide
// fences and results are reproducible bit for bit.
#include <algorithm>

#include "ks_common.h"

namespace ks {

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
__device__ inline void k_init_body(const InitArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ rho = ka.rho;
  const double* __restrict__ x0 = ka.x0;
  double* x = ka.x;  // may be nullptr (x0 is the iterate)
  double* __restrict__ r = ka.r;
  double* __restrict__ p0 = ka.p0;
  Grid gr = ka.gr;
  double* __restrict__ part = ka.part;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kBlock / kWave];
  const int lb = xcd_remap(ks_bid, ks_nb);
  int beg, end;
  range_of(gr.n, lb, ks_nb, &beg, &end);
  double rr = 0.0, bb = 0.0;
  for (int g = beg + threadIdx.x; g < end; g += blockDim.x) {
    const int i = g % gr.nx, j = (g / gr.nx) % gr.ny, k = g / (gr.nx * gr.ny);
    const double b = poisson_rhs(rho, g, gr);
    const double ri = x0 ? b - op_apply(x0, nullptr, 0.0, g, i, j, k, gr) : b;
    if (x) x[g] = x0 ? x0[g] : 0.0;
    r[g] = ri;
    p0[g] = 0.0;
    rr += ri * ri;
    bb += b * b;
  }
  put2(part, lb, rr, bb, sh, 0, 1);
}

__global__ void k_init(InitArgs ka) {
  k_init_body(ka, blockIdx.x, gridDim.x);
}

__global__ void k_init_batch(BatchPtrs<InitArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_init_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}



__device__ inline void k_fin_init_body(const FinInitArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ part = ka.part;
  int nb = ka.nb;
  CgState* cs = ka.cs;
  double tol = ka.tol;
  int maxit = ka.maxit;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kBlock / kWave];
  const double rr = fin_sum(part, 0, nb, sh);
  const double bb = fin_sum(part, 1, nb, sh);
  if (threadIdx.x == 0) {
    cs->rr = rr;
    cs->bb = bb;
    cs->tol2 = tol * tol;
    cs->alpha = cs->beta = cs->pq = 0.0;
    cs->rz = 0.0;
    cs->rr_best = rr;
    cs->stall = 0;
    cs->it = bb == 0.0 ? 0 : ka.it0;  // rho == 0: nothing was solved
    cs->maxit = maxit;
    cs->done = (bb == 0.0 || !isfinite(rr) || !isfinite(bb) || rr <= tol * tol * bb) ? 1 : 0;
  }
}

__global__ void k_fin_init(FinInitArgs ka) {
  k_fin_init_body(ka, blockIdx.x, gridDim.x);
}



// pn = z + beta po ; q = L pn ; partial pn.q (slot 2).  z = r for plain CG.
__device__ inline void k_dir_body(const DirArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ z = ka.z;
  const double* __restrict__ po = ka.po;
  double* __restrict__ pn = ka.pn;
  double* __restrict__ q = ka.q;
  const CgState* cs = ka.cs;
  Grid gr = ka.gr;
  double* __restrict__ part = ka.part;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double beta = cs->beta;
  const int lb = xcd_remap(ks_bid, ks_nb);
  int beg, end;
  range_of(gr.n, lb, ks_nb, &beg, &end);
  const int sz = gr.nx * gr.ny;
  double pq = 0.0;
  for (int g = beg + threadIdx.x; g < end; g += blockDim.x) {
    const int i = g % gr.nx, j = (g / gr.nx) % gr.ny, k = g / sz;
    const double pc = z[g] + beta * po[g];
    const double qq = op_apply(z, po, beta, g, i, j, k, gr);
    pn[g] = pc;
    q[g] = qq;
    pq += pc * qq;
  }
  pq = block_sum(pq, sh);
  if (threadIdx.x == 0) part[2 * kCgBlocksMax + lb] = pq;
}

__global__ void k_dir(DirArgs ka) {
  k_dir_body(ka, blockIdx.x, gridDim.x);
}

__global__ void k_dir_batch(BatchPtrs<DirArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_dir_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// alpha = (r.z)/(p.q)   (r.z = r.r for plain CG)
__device__ inline void k_fin_dir_body(const FinDirArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ part = ka.part;
  int nb = ka.nb;
  CgState* cs = ka.cs;
  int pcg = ka.pcg;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double pq = fin_sum(part, 2, nb, sh);
  if (threadIdx.x == 0) {
    cs->pq = pq;
    cs->alpha = (pcg ? cs->rz : cs->rr) / pq;
  }
}

__global__ void k_fin_dir(FinDirArgs ka) {
  k_fin_dir_body(ka, blockIdx.x, gridDim.x);
}

__global__ void k_fin_dir_batch(BatchPtrs<FinDirArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_fin_dir_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// x += alpha p ; r -= alpha q ; partial r.r (slot 0)
__device__ inline void k_upd_body(const UpdArgs& ka, int ks_bid, int ks_nb) {
  double* __restrict__ x = ka.x;
  double* __restrict__ r = ka.r;
  const double* __restrict__ pn = ka.pn;
  const double* __restrict__ q = ka.q;
  const CgState* cs = ka.cs;
  Grid gr = ka.gr;
  double* __restrict__ part = ka.part;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double alpha = cs->alpha;
  const int lb = xcd_remap(ks_bid, ks_nb);
  int beg, end;
  range_of(gr.n, lb, ks_nb, &beg, &end);
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

__global__ void k_upd(UpdArgs ka) {
  k_upd_body(ka, blockIdx.x, gridDim.x);
}

__global__ void k_upd_batch(BatchPtrs<UpdArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_upd_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// plain CG: beta = rr_new/rr ; convergence
__device__ inline void k_fin_upd_body(const FinUpdArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ part = ka.part;
  int nb = ka.nb;
  CgState* cs = ka.cs;
  int pcg = ka.pcg;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double rr = fin_sum(part, 0, nb, sh);
  if (threadIdx.x == 0) {
    if (!pcg) cs->beta = rr / cs->rr;
    cs->rr = rr;
    cs->it += 1;
    bool floor = false;
    if (pcg) {
      if (rr < 0.25 * cs->rr_best) {
        cs->stall = 0;
      } else {
        cs->stall += 1;
      }
      cs->rr_best = fmin(cs->rr_best, rr);
      floor = cs->stall >= kCgStall && rr <= kCgFloor * kCgFloor * cs->tol2 * cs->bb;
    }
    cs->done = (!isfinite(rr) || rr <= cs->tol2 * cs->bb || floor || cs->it >= cs->maxit) ? 1 : 0;
  }
}

__global__ void k_fin_upd(FinUpdArgs ka) {
  k_fin_upd_body(ka, blockIdx.x, gridDim.x);
}

__global__ void k_fin_upd_batch(BatchPtrs<FinUpdArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_fin_upd_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// PCG: rz_new = r.z (slot 3, written by the last transform) ; beta = rz_new/rz
__device__ inline void k_fin_rz_body(const FinRzArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ part = ka.part;
  int nb = ka.nb;
  CgState* cs = ka.cs;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kBlock / kWave];
  if (cs->done) return;
  const double rz = fin_sum(part, 3, nb, sh);
  if (threadIdx.x == 0) {
    cs->beta = (cs->rz == 0.0) ? 0.0 : rz / cs->rz;  // rz is 0 right after a (re)start
    cs->rz = rz;
  }
}

__global__ void k_fin_rz(FinRzArgs ka) {
  k_fin_rz_body(ka, blockIdx.x, gridDim.x);
}

__global__ void k_fin_rz_batch(BatchPtrs<FinRzArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_fin_rz_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// ---- fast-diagonalisation preconditioner --------------------------------------------

// S (N x N), the operator eigenvalues lam (N) and the mass eigenvalues mu (N) of one
// axis.  Differences: lam = (2 - 2 cos t)/h^2, mu = 1.  Q1 elements: the 1D stiffness
// (1/h) tridiag(-1, 2, -1) and mass (h/6) tridiag(1, 4, 1) share the sine eigenvectors,
// lam = (2/h)(1 - cos t), mu = (h/3)(2 + cos t); then A = S3 diag(lx my mz + mx ly mz +
// mx my lz) S3.
__global__ void k_fd_setup(double* __restrict__ S, double* __restrict__ lam,
                           double* __restrict__ mu, int N, double h, int q1) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N * N) {
    const int j = e / N, m = e % N;
    S[e] = sqrt(2.0 / (N + 1)) * sin(kPi * (double)((j + 1) * (m + 1)) / (double)(N + 1));
  }
  if (e < N) {
    const double c = cos(kPi * (double)(e + 1) / (double)(N + 1));
    lam[e] = q1 ? (2.0 / h) * (1.0 - c) : (2.0 - 2.0 * c) / (h * h);
    mu[e] = q1 ? (h / 3.0) * (2.0 + c) : 1.0;
  }
}

// The sine-transform contractions run on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
//   A fragment: lane l holds A[l % 16][l / 16];  B fragment: lane l holds B[l / 16][l % 16];
//   result:     lane l, register r holds D[(l / 16) + 4 r][l % 16].
// Transform lengths are padded to multiples of 16 with zero rows/columns of S.  Because S
// is symmetric, S[j][m] = S[m][j], so every fragment of S is read along a row (coalesced).
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline double sget(const double* S, int N, int row, int col) {
  return (row < N && col < N) ? S[row * N + col] : 0.0;
}

constexpr int kFdWaves = 8;     // waves per block of the transform kernels
constexpr int kFdTiles = 8;     // result tiles a wave can hold (covers 128 x 128)
constexpr int kZCols = 32;      // (i, j) lines per block of the z transform

// 2-D transform of one z-plane, split by 16-column strips of the output: block
// (plane k, strip c) computes T[:, strip] = P S_x[:, strip] and then
// Y[:, strip] = S_y T[:, strip] (row = y), which needs only that strip of T, so the strips
// of a plane are independent blocks.  The plane lives in LDS (row stride nxp + 1 doubles:
// conflict-free column reads), then the T strip, the S_x strip and (kStageSy, when it
// fits) S_y, so the MFMA operands of both steps come from LDS.  With part the partial r.Y
// of the block goes to slot 3 at the block's index.
constexpr int kPlaneWaves = 4;

template <bool kStageSy, bool kStageSx>
__device__ inline void k_fd_plane_body(const FdPlaneArgs& ka, int ks_bid, int ks_nb) {
  double* __restrict__ out = ka.out;
  const double* __restrict__ Sx = ka.Sxg;
  const double* __restrict__ Sy = ka.Syg;
  const int nx = ka.nx, ny = ka.ny;
  const double* __restrict__ r = ka.r;
  double* __restrict__ part = ka.part;
  const CgState* cs = ka.cs;
  (void)ks_nb;
  extern __shared__ double P[];
  __shared__ double sh[kBlock / kWave];
  if (cs && cs->done) return;
  const int nxp = (nx + 15) & ~15, nyp = (ny + 15) & ~15, sp = nxp + 1;
  const int ncs = nxp / 16;
  const int k = ks_bid / ncs, i0 = (ks_bid % ncs) * 16;
  const size_t base = (size_t)k * nx * ny;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  lds_stage<16>(
      nyp * nxp,
      [&](int e) {
        const int j = e / nxp, m = e % nxp;
        const bool ok = j < ny && m < nx;
        const double v = ka.in[ok ? base + (size_t)j * nx + m : base];
        return ok ? v : 0.0;
      },
      [&](int e, double v) { P[(e / nxp) * sp + e % nxp] = v; });
  double* Tt = P + nyp * sp;     // nyp x 17
  double* Sxs = Tt + nyp * 17;   // nxp x 16: S_x[:, i0 .. i0 + 15] (when staged)
  if (kStageSx)
    lds_stage<8>(
        nxp * 16,
        [&](int e) {
          const int m = e / 16, c = e % 16;
          const bool ok = m < nx && i0 + c < nx;
          const double v = Sx[ok ? m * nx + i0 + c : 0];
          return ok ? v : 0.0;
        },
        [&](int e, double v) { Sxs[e] = v; });
  // the strip of S_x as a B fragment: from LDS, or from global memory (L2-resident) when
  // the plane leaves no room for it
  auto sx = [&](int m, int c) -> double {
    if (kStageSx) return Sxs[m * 16 + c];
    const bool ok = m < nx && i0 + c < nx;
    return ok ? Sx[m * nx + i0 + c] : 0.0;
  };
  const double* SyL = Sy;
  if (kStageSy) {
    double* sy = Sxs + nxp * 16;
    lds_stage<16>(ny * ny, [&](int e) { return Sy[e]; }, [&](int e, double v) { sy[e] = v; });
    SyL = sy;
  }
  __syncthreads();
  const int ntile = nyp / 16;
  // step 1: T[j][i0 + c] = sum_m P[j][m] S_x[m][i0 + c]
  for (int t = w; t < ntile; t += kPlaneWaves) {
    const int j0 = t * 16;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nxp; k0 += 4)
      acc = mma(P[(j0 + lc) * sp + k0 + lr], sx(k0 + lr, lc), acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) Tt[(j0 + lr + 4 * q) * 17 + lc] = acc[q];
  }
  __syncthreads();
  // step 2: Y[j][i0 + c] = sum_m S_y[j][m] T[m][i0 + c]
  double rz = 0.0;
  for (int t = w; t < ntile; t += kPlaneWaves) {
    const int j0 = t * 16;
    d4 y = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nyp; k0 += 4)
      y = mma(sget(SyL, ny, k0 + lr, j0 + lc), Tt[(k0 + lr) * 17 + lc], y);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + lr + 4 * q, i = i0 + lc;
      if (j < ny && i < nx) {
        const size_t o = base + (size_t)j * nx + i;
        if (ka.add) y[q] += ka.add[o];
        out[o] = y[q];
        if (part) rz += y[q] * r[o];
      }
    }
  }
  if (part) {
    rz = block_sum(rz, sh);
    if (threadIdx.x == 0) part[3 * kCgBlocksMax + ks_bid] = rz;
  }
}

template <bool kStageSy, bool kStageSx>
__global__ __launch_bounds__(256) void k_fd_plane(FdPlaneArgs ka) {
  k_fd_plane_body<kStageSy, kStageSx>(ka, blockIdx.x, gridDim.x);
}

template <bool kStageSy, bool kStageSx>
__global__ __launch_bounds__(256) void k_fd_plane_batch(BatchPtrs<FdPlaneArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_fd_plane_body<kStageSy, kStageSx>(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// The same 2-D transform with one whole z-plane per block of kFullWaves waves, used when
// the plane, T, S_x and S_y all fit in LDS (planes up to 64 x 64): every operand is staged
// once per plane instead of once per strip, and each wave computes one 16 x 16 tile of T
// and then one of Y.
constexpr int kFullWaves = 16;

__device__ inline void k_fd_plane_full_body(const FdPlaneArgs& ka, int ks_bid, int ks_nb) {
  double* __restrict__ out = ka.out;
  const double* __restrict__ Sx = ka.Sxg;
  const double* __restrict__ Sy = ka.Syg;
  const int nx = ka.nx, ny = ka.ny;
  const double* __restrict__ r = ka.r;
  double* __restrict__ part = ka.part;
  const CgState* cs = ka.cs;
  (void)ks_nb;
  extern __shared__ double P[];
  __shared__ double sh[kFullWaves];
  if (cs && cs->done) return;
  const int nxp = (nx + 15) & ~15, nyp = (ny + 15) & ~15, sp = nxp + 1;
  const size_t base = (size_t)ks_bid * nx * ny;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  double* T = P + nyp * sp;      // nyp x sp
  double* Sxs = T + nyp * sp;    // nxp x nxp (zero padded)
  double* Sys = Sxs + nxp * nxp; // nyp x nyp (zero padded)
  lds_stage<4>(
      nyp * nxp,
      [&](int e) {
        const int j = e / nxp, m = e % nxp;
        const bool ok = j < ny && m < nx;
        const double v = ka.in[ok ? base + (size_t)j * nx + m : base];
        return ok ? v : 0.0;
      },
      [&](int e, double v) { P[(e / nxp) * sp + e % nxp] = v; });
  lds_stage<4>(
      nxp * nxp,
      [&](int e) {
        const int m = e / nxp, c = e % nxp;
        const bool ok = m < nx && c < nx;
        const double v = Sx[ok ? m * nx + c : 0];
        return ok ? v : 0.0;
      },
      [&](int e, double v) { Sxs[e] = v; });
  lds_stage<4>(
      nyp * nyp,
      [&](int e) {
        const int m = e / nyp, c = e % nyp;
        const bool ok = m < ny && c < ny;
        const double v = Sy[ok ? m * ny + c : 0];
        return ok ? v : 0.0;
      },
      [&](int e, double v) { Sys[e] = v; });
  __syncthreads();
  const int nti = nxp / 16, ntile = (nyp / 16) * nti;
  // T[j][i] = sum_m P[j][m] S_x[m][i]
  for (int t = w; t < ntile; t += kFullWaves) {
    const int j0 = (t / nti) * 16, i0 = (t % nti) * 16;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nxp; k0 += 4)
      acc = mma(P[(j0 + lc) * sp + k0 + lr], Sxs[(k0 + lr) * nxp + i0 + lc], acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) T[(j0 + lr + 4 * q) * sp + i0 + lc] = acc[q];
  }
  __syncthreads();
  // Y[j][i] = sum_m S_y[j][m] T[m][i]  (S_y symmetric: its fragments are read along rows)
  double rz = 0.0;
  for (int t = w; t < ntile; t += kFullWaves) {
    const int j0 = (t / nti) * 16, i0 = (t % nti) * 16;
    d4 y = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nyp; k0 += 4)
      y = mma(Sys[(k0 + lr) * nyp + j0 + lc], T[(k0 + lr) * sp + i0 + lc], y);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + lr + 4 * q, i = i0 + lc;
      if (j < ny && i < nx) {
        const size_t o = base + (size_t)j * nx + i;
        if (ka.add) y[q] += ka.add[o];
        out[o] = y[q];
        if (part) rz += y[q] * r[o];
      }
    }
  }
  if (part) {
    // fixed-order sum over the block's waves
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) rz += __shfl_down(rz, o, kWave);
    if (lane == 0) sh[w] = rz;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < kFullWaves; ++i) t += sh[i];
      part[3 * kCgBlocksMax + ks_bid] = t;
    }
  }
}

__global__ __launch_bounds__(kFullWaves * kWave) void k_fd_plane_full(FdPlaneArgs ka) {
  k_fd_plane_full_body(ka, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kFullWaves * kWave) void k_fd_plane_full_batch(
    BatchPtrs<FdPlaneArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_fd_plane_full_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// z lines (block = 64 adjacent (i, j) columns x nz): forward transform, division by
// lx[i] + ly[j] + lz[k], inverse transform (S_z is its own inverse), in place.
template <bool kStageS>
__device__ inline void k_fd_z_body(const FdZArgs& ka, int ks_bid, int ks_nb) {
  double* __restrict__ u = ka.u;
  const double* __restrict__ Szg = ka.Szg;
  const double* __restrict__ lx = ka.lx;
  const double* __restrict__ ly = ka.ly;
  const double* __restrict__ lz = ka.lz;
  const double* __restrict__ mx = ka.mx;
  const double* __restrict__ my = ka.my;
  const double* __restrict__ mz = ka.mz;
  int nx = ka.nx;
  int ny = ka.ny;
  int nz = ka.nz;
  const CgState* cs = ka.cs;
  (void)ks_bid;
  (void)ks_nb;

  extern __shared__ double A[];  // nzp x kZCols (then S_z when it fits)
  if (cs && cs->done) return;
  const int npl = nx * ny;
  const int nzp = (nz + 15) & ~15;
  const int l0 = ks_bid * kZCols;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  lds_stage<8>(
      nzp * kZCols,
      [&](int e) {
        const int m = e / kZCols, l = e % kZCols;
        const bool ok = m < nz && l0 + l < npl;
        const double v = u[ok ? (size_t)m * npl + l0 + l : 0];
        return ok ? v : 0.0;
      },
      [&](int e, double v) { A[e] = v; });
  const double* Sz = Szg;
  if (kStageS) {
    double* sz = A + nzp * kZCols;
    lds_stage<8>(nz * nz, [&](int e) { return Szg[e]; }, [&](int e, double v) { sz[e] = v; });
    Sz = sz;
  }
  __syncthreads();
  constexpr int kCT = kZCols / 16;  // column tiles per block
  const int ntile = (nzp / 16) * kCT;
  d4 acc[kFdTiles];
#pragma unroll
  for (int s = 0; s < kFdTiles; ++s) {
    acc[s] = d4{0.0, 0.0, 0.0, 0.0};
    const int t = w + s * kFdWaves;
    if (t < ntile) {
      const int k0t = (t / kCT) * 16, c0 = (t % kCT) * 16;
      for (int k0 = 0; k0 < nzp; k0 += 4)
        acc[s] = mma(sget(Sz, nz, k0 + lr, k0t + lc), A[(k0 + lr) * kZCols + c0 + lc], acc[s]);
      // divide by the eigenvalue at (i, j, k): lx my mz + mx ly mz + mx my lz (with unit
      // mass eigenvalues this is exactly lx + ly + lz)
      const int line = l0 + c0 + lc;
      const int ii = line % nx, jj = line / nx;
      const bool live = line < npl;
      const double lxi = live ? lx[ii] : 1.0, mxi = live ? mx[ii] : 1.0;
      const double lyj = live ? ly[jj] : 1.0, myj = live ? my[jj] : 1.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = k0t + lr + 4 * q;
        if (kk < nz) {
          const double mzk = mz[kk];
          const double den = (lxi * myj * mzk + mxi * lyj * mzk) + mxi * myj * lz[kk];
          acc[s][q] = acc[s][q] / den;
        } else {
          acc[s][q] = 0.0;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kFdTiles; ++s) {
    const int t = w + s * kFdWaves;
    if (t < ntile) {
      const int k0t = (t / kCT) * 16, c0 = (t % kCT) * 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) A[(k0t + lr + 4 * q) * kZCols + c0 + lc] = acc[s][q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kFdTiles; ++s) {
    const int t = w + s * kFdWaves;
    if (t < ntile) {
      const int k0t = (t / kCT) * 16, c0 = (t % kCT) * 16;
      d4 y = d4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < nzp; k0 += 4)
        y = mma(sget(Sz, nz, k0 + lr, k0t + lc), A[(k0 + lr) * kZCols + c0 + lc], y);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = k0t + lr + 4 * q, line = l0 + c0 + lc;
        if (kk < nz && line < npl) u[(size_t)kk * npl + line] = y[q];
      }
    }
  }
}

template <bool kStageS>
__global__ __launch_bounds__(512) void k_fd_z(FdZArgs ka) {
  k_fd_z_body<kStageS>(ka, blockIdx.x, gridDim.x);
}

template <bool kStageS>
__global__ __launch_bounds__(512) void k_fd_z_batch(BatchPtrs<FdZArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_fd_z_body<kStageS>(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


}  // namespace

size_t hartree_part_doubles() { return (size_t)4 * kCgBlocksMax; }


void launch_fd_setup(double* S, double* lam, double* mu, int N, double h, int q1,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_fd_setup, dim3((N * N + 255) / 256), dim3(256), 0, st, S, lam, mu, N, h,
                     q1);
}

void launch_hartree_init(const double* rho, const double* x0, double* x, double* r, double* p0,
                         CgState* cs, double tol, int maxit, int it0, Grid g, double* part,
                         hipStream_t st) {
  const int nb = cg_nblocks(g.n);
  hipLaunchKernelGGL(k_init, dim3(nb), dim3(kBlock), 0, st, InitArgs{rho, x0, x, r, p0, g, part});
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kBlock), 0, st,
                     FinInitArgs{part, nb, cs, tol, maxit, it0});
}

namespace {
constexpr size_t kFdLdsCap = 150 * 1024;  // stay inside the 160 KiB of LDS of a CU

// Raises the dynamic-LDS limit of a kernel to the cap.  The value does not depend on the
// grid, so concurrent callers on several host threads all set the same value.
void set_lds(const void* k, size_t bytes) {
  if (bytes > 32768) set_dyn_lds_once(k, (int)kFdLdsCap);
}
}  // namespace

// LDS of one plane-transform block in each mode (strips with S_y read from L2, strips
// with S_y staged, whole plane).
size_t fd_plane_bytes(int nx, int ny, int mode) {
  const size_t nxp = (nx + 15) & ~15, nyp = (ny + 15) & ~15;
  if (mode == kPlaneFull) return (2 * nyp * (nxp + 1) + nxp * nxp + nyp * nyp) * sizeof(double);
  if (mode == kPlaneStripG) return (nyp * (nxp + 1) + nyp * 17) * sizeof(double);
  const size_t strip = (nyp * (nxp + 1) + nyp * 17 + nxp * 16) * sizeof(double);
  return mode == kPlaneStripSy ? strip + (size_t)ny * ny * sizeof(double) : strip;
}

bool fd_plane_mode_fits(int nx, int ny, int mode) {
  return (mode == kPlaneFull || mode == kPlaneStripSy || mode == kPlaneStrip ||
          mode == kPlaneStripG) &&
         fd_plane_bytes(nx, ny, mode) <= kFdLdsCap;
}

int fd_plane_mode_of(const Grid& g) {
  return g.fd_mode != kTuneAuto && fd_plane_mode_fits(g.nx, g.ny, g.fd_mode)
             ? g.fd_mode
             : fd_plane_mode(g.nx, g.ny);
}

int fd_plane_mode(int nx, int ny) {
  if (fd_plane_bytes(nx, ny, kPlaneFull) <= kFdLdsCap) return kPlaneFull;
  if (fd_plane_bytes(nx, ny, kPlaneStripSy) <= kFdLdsCap) return kPlaneStripSy;
  return fd_plane_bytes(nx, ny, kPlaneStrip) <= kFdLdsCap ? kPlaneStrip : kPlaneStripG;
}

bool fd_fits(int nx, int ny, int nz) {
  const size_t nzp = (nz + 15) & ~15;
  return fd_plane_bytes(nx, ny, kPlaneStripG) <= kFdLdsCap &&
         nzp * (size_t)kZCols * sizeof(double) <= kFdLdsCap;
}

int fd_plane_blocks(int nx, int nz, int mode) {
  return mode == kPlaneFull ? nz : nz * ((nx + 15) / 16);
}

// LDS the preconditioner needs for an nx x ny x nz grid (the plane strips at least).
size_t fd_lds_bytes(int nx, int ny, int nz) {
  const size_t nzp = (nz + 15) & ~15;
  return std::max(fd_plane_bytes(nx, ny, kPlaneStripG), nzp * (size_t)kZCols * sizeof(double));
}

// Largest plane the register tiles of k_fd_plane cover (kFdWaves * kFdTiles tiles).
int fd_max_plane() { return kFdWaves * kFdTiles * 256; }

namespace {
void launch_fd_plane(const FdPlaneArgs& pa, int nz, int mode, hipStream_t st) {
  const size_t lds = fd_plane_bytes(pa.nx, pa.ny, mode);
  const int nb = fd_plane_blocks(pa.nx, nz, mode);
  if (mode == kPlaneFull) {
    set_lds(reinterpret_cast<const void*>(k_fd_plane_full), lds);
    hipLaunchKernelGGL(k_fd_plane_full, dim3(nb), dim3(kFullWaves * kWave), lds, st, pa);
  } else if (mode == kPlaneStripSy) {
    set_lds(reinterpret_cast<const void*>(k_fd_plane<true, true>), lds);
    hipLaunchKernelGGL((k_fd_plane<true, true>), dim3(nb), dim3(kPlaneWaves * kWave), lds, st,
                       pa);
  } else if (mode == kPlaneStrip) {
    set_lds(reinterpret_cast<const void*>(k_fd_plane<false, true>), lds);
    hipLaunchKernelGGL((k_fd_plane<false, true>), dim3(nb), dim3(kPlaneWaves * kWave), lds, st,
                       pa);
  } else {
    set_lds(reinterpret_cast<const void*>(k_fd_plane<false, false>), lds);
    hipLaunchKernelGGL((k_fd_plane<false, false>), dim3(nb), dim3(kPlaneWaves * kWave), lds, st,
                       pa);
  }
}

// The three fast-diagonalisation passes: in -> tmp (plane transform), the z pass
// with the eigenvalue division in place on tmp, tmp -> out (inverse plane transform, plus
// add when given; with part also the partials of out . rr).  The strips of a plane are separate blocks, so a
// plane pass never works in place.
void fd_passes(const double* in, double* out, const double* add, double* tmp,
               const FdOps& fd, Grid g, const CgState* cs, const double* rr, double* part,
               hipStream_t st) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const size_t nzp = (nz + 15) & ~15;
  const size_t lzb = nzp * kZCols * sizeof(double);
  const size_t lzs = lzb + (size_t)nz * nz * sizeof(double);
  const size_t cap = kFdLdsCap;
  const int threads = kFdWaves * kWave;
  const int mode = fd_plane_mode_of(g);
  auto plane = [&](const double* src, double* dst, const double* ad, const double* r,
                   double* pt) {
    launch_fd_plane(FdPlaneArgs{src, dst, fd.Sx, fd.Sy, nx, ny, r, pt, cs, ad}, nz, mode, st);
  };
  const int zblocks = (nx * ny + kZCols - 1) / kZCols;
  const FdZArgs za{tmp, fd.Sz, fd.lx, fd.ly, fd.lz, fd.mx, fd.my, fd.mz, nx, ny, nz, cs};
  plane(in, tmp, nullptr, nullptr, nullptr);
  if (lzs <= cap) {
    set_lds(reinterpret_cast<const void*>(k_fd_z<true>), lzs);
    hipLaunchKernelGGL(k_fd_z<true>, dim3(zblocks), dim3(threads), lzs, st, za);
  } else {
    set_lds(reinterpret_cast<const void*>(k_fd_z<false>), lzb);
    hipLaunchKernelGGL(k_fd_z<false>, dim3(zblocks), dim3(threads), lzb, st, za);
  }
  plane(tmp, out, add, rr, part);
}
}  // namespace

// z = L^{-1} r by the fast diagonalisation, then beta from r.z.
void launch_fd_apply(const double* r, double* z, double* tmp, const FdOps& fd, Grid g,
                     const CgState* cs, double* part, hipStream_t st) {
  fd_passes(r, z, nullptr, tmp, fd, g, cs, r, part, st);
  const int nb = fd_plane_blocks(g.nx, g.nz, fd_plane_mode_of(g));
  hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kBlock), 0, st,
                     FinRzArgs{part, nb, const_cast<CgState*>(cs)});
}

// x = x0 + L^{-1} r: with r = b - L x0 this is the first iterate of the preconditioned CG
// from x0 with the step length the exact preconditioner gives (exactly 1).
void launch_fd_correct(const double* r, const double* x0, double* x, double* tmp,
                       const FdOps& fd, Grid g, hipStream_t st) {
  fd_passes(r, x, x0, tmp, fd, g, nullptr, nullptr, nullptr, st);
}

void launch_cg_residual(const double* rho, const double* x0, double* r, double* p0, Grid g,
                        double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(cg_nblocks(g.n)), dim3(kBlock), 0, st,
                     InitArgs{rho, x0, nullptr, r, p0, g, part});
}

void launch_hartree_iter(double* x, double* r, const double* z, double* pa, double* pb,
                         double* q, CgState* cs, Grid g, double* part, int pcg,
                         hipStream_t st) {
  const int nb = cg_nblocks(g.n);
  hipLaunchKernelGGL(k_dir, dim3(nb), dim3(kBlock), 0, st,
                     DirArgs{pcg ? z : r, pa, pb, q, cs, g, part});
  hipLaunchKernelGGL(k_fin_dir, dim3(1), dim3(kBlock), 0, st, FinDirArgs{part, nb, cs, pcg});
  hipLaunchKernelGGL(k_upd, dim3(nb), dim3(kBlock), 0, st, UpdArgs{x, r, pb, q, cs, g, part});
  hipLaunchKernelGGL(k_fin_upd, dim3(1), dim3(kBlock), 0, st, FinUpdArgs{part, nb, cs, pcg});
}

// ---- batched launches (one launch for the systems of a BatchPtrs table) ---------------

void launch_init_batch(const BatchPtrs<InitArgs>& b, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_init_batch, dim3(blocks), dim3(kBlock), 0, st, b);
}

int hartree_blocks(int n) { return cg_nblocks(n); }

FdLaunch fd_launch(const Grid& g) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const size_t nzp = (nz + 15) & ~15;
  FdLaunch l;
  l.plane_mode = fd_plane_mode_of(g);
  l.z_bytes = nzp * kZCols * sizeof(double);
  l.z_bytes_staged = l.z_bytes + (size_t)nz * nz * sizeof(double);
  l.cap = kFdLdsCap;
  l.z_blocks = (nx * ny + kZCols - 1) / kZCols;
  return l;
}

void launch_dir_batch(const BatchPtrs<DirArgs>& b, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_dir_batch, dim3(blocks), dim3(kBlock), 0, st, b);
}
void launch_fin_dir_batch(const BatchPtrs<FinDirArgs>& b, hipStream_t st) {
  hipLaunchKernelGGL(k_fin_dir_batch, dim3(b.S), dim3(kBlock), 0, st, b);
}
void launch_upd_batch(const BatchPtrs<UpdArgs>& b, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_upd_batch, dim3(blocks), dim3(kBlock), 0, st, b);
}
void launch_fin_upd_batch(const BatchPtrs<FinUpdArgs>& b, hipStream_t st) {
  hipLaunchKernelGGL(k_fin_upd_batch, dim3(b.S), dim3(kBlock), 0, st, b);
}
void launch_fin_rz_batch(const BatchPtrs<FinRzArgs>& b, hipStream_t st) {
  hipLaunchKernelGGL(k_fin_rz_batch, dim3(b.S), dim3(kBlock), 0, st, b);
}
void launch_fd_plane_batch(const BatchPtrs<FdPlaneArgs>& b, int blocks, int mode, size_t lds,
                           hipStream_t st) {
  if (mode == kPlaneFull) {
    set_lds(reinterpret_cast<const void*>(k_fd_plane_full_batch), lds);
    hipLaunchKernelGGL(k_fd_plane_full_batch, dim3(blocks), dim3(kFullWaves * kWave), lds, st,
                       b);
  } else if (mode == kPlaneStripSy) {
    set_lds(reinterpret_cast<const void*>(k_fd_plane_batch<true, true>), lds);
    hipLaunchKernelGGL((k_fd_plane_batch<true, true>), dim3(blocks), dim3(kPlaneWaves * kWave),
                       lds, st, b);
  } else if (mode == kPlaneStrip) {
    set_lds(reinterpret_cast<const void*>(k_fd_plane_batch<false, true>), lds);
    hipLaunchKernelGGL((k_fd_plane_batch<false, true>), dim3(blocks), dim3(kPlaneWaves * kWave),
                       lds, st, b);
  } else {
    set_lds(reinterpret_cast<const void*>(k_fd_plane_batch<false, false>), lds);
    hipLaunchKernelGGL((k_fd_plane_batch<false, false>), dim3(blocks),
                       dim3(kPlaneWaves * kWave), lds, st, b);
  }
}
void launch_fd_z_batch(const BatchPtrs<FdZArgs>& b, int blocks, bool staged, size_t lds,
                       hipStream_t st) {
  const int threads = kFdWaves * kWave;
  if (staged) {
    set_lds(reinterpret_cast<const void*>(k_fd_z_batch<true>), lds);
    hipLaunchKernelGGL(k_fd_z_batch<true>, dim3(blocks), dim3(threads), lds, st, b);
  } else {
    set_lds(reinterpret_cast<const void*>(k_fd_z_batch<false>), lds);
    hipLaunchKernelGGL(k_fd_z_batch<false>, dim3(blocks), dim3(threads), lds, st, b);
  }
}

}  // namespace ks
