// Internal declarations shared by the HIP kernels and the host orchestration.
// Not part of the public ABI (include/ks.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ks.h"

namespace ks {

constexpr int kBlock = 256;          // threads per block of the streaming kernels
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kXcds = 8;             // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kMaxScalarSlots = 16;  // scalar reduction slots per evaluation
constexpr double kPi = 3.14159265358979323846;

// Scalar reduction slots (sums over the grid of one evaluation).
enum Slot : int {
  SL_KIN = 0,   // sum_g,i X_gi (L X)_gi
  SL_EXT = 1,   // sum_g V_ext,g rho_g
  SL_EH = 2,    // sum_g rho_g V_H,g
  SL_EX = 3,    // sum_g rho_g eps_x(rho_g)
  SL_DD = 4,    // ||D||_F^2, D = G - X G^T X
  SL_SS = 5,    // tr(S^T S),  S = X_t - X_k
  SL_SY = 6,    // tr(S^T Yd), Yd = D_t - D_k
  SL_YY = 7,    // tr(Yd^T Yd)
  SL_DEFECT = 8,  // ||X^T G (bf16) - X^T G (exact)||_F^2 (KS_PREC_MIXED_BF16, p > 64)
  SL_TF = 9,      // sum_g rho_g eps_TF(rho_g) (Thomas-Fermi term, KS_TERM_TF)
  SL_CGRR = 10,   // r.r of the Hartree residual checked inside the exchange pass
  SL_CGBB = 11,   // b.b, b = 4 pi rho (same pass)
  SL_EBC = 12,    // sum_g rho_g V_bc,g (monopole Hartree boundary, KS_HBC_MONOPOLE)
  SL_COUNT = 13
};

// Conjugate-gradient state kept on the device (one solve at a time per system).
struct CgState {
  double rr;       // current r.r
  double bb;       // b.b, b = 4 pi rho
  double pq;       // p.Lp of the current iteration
  double alpha, beta;
  double tol2;     // squared relative tolerance
  double rz;       // r.z of the preconditioned iteration
  int it;          // iterations done
  int maxit;
  int done;        // 1 once converged or at maxit
  int stall;       // preconditioned iterations since r.r last fell below rr_best / 4
  unsigned int count;  // arrival counter of the last-block reduction
  unsigned int pad2;
  double rr_best;  // smallest r.r of the preconditioned solve so far
};

// A preconditioned solve whose residual has stopped falling (kCgStall iterations without
// a 4x decrease) has reached the rounding floor of its operator, about eps cond(L) of the
// right-hand side, which for grids of 128^3 nodes lies just above the default tolerance;
// it ends there if r.r <= kCgFloor^2 tol^2 b.b.
constexpr int kCgStall = 3;
constexpr double kCgFloor = 100.0;

// Results of one energy/gradient evaluation, assembled on the device.
struct EvalOut {
  double total, kinetic, external, hartree, xc, nuclear;
  double g2;        // ||grad E||_F^2
  double ss, sy, yy;
  double orth2;     // ||X^T X - I||_F^2
  double defect2;   // SL_DEFECT of this evaluation (0 unless measured)
  double cg_relres;
  int cg_iters;
  int nonfinite;
};

// Optimiser parameters and state of Alg. 3 on the device.
struct LsParams {
  double tau0, rho1, delta, eta, eps_g, tau_min, tau_max, reorth_tol, stagnation_tol;
  double energy_target;  // stop once an accepted energy is <= this (-inf: never)
  int max_iter, bb_rule, h_max, retraction;
};

struct ScalarCounts {
  int v[SL_COUNT];  // partial blocks per scalar slot
};

struct LsState {
  double E, g2;        // at the current iterate X_k
  double C, Q;         // nonmonotone reference value and weight
  double tau_bb, tau;  // BB value of this iteration and the current trial step
  double df[3];        // last relative energy changes
  int ndf;
  int k;               // accepted iterations
  int h;               // backtracks in this iteration
  int accepted;        // last trial accepted
  int stop;            // KS_STOP_*
  int backtracks, ls_fail, nfe, reorth_flag;
  int error;           // KS_E_* raised by a device step
  int hartree_pending; // the trial's Hartree solve had not converged: nothing was judged
  double tau_acc;      // step of the last accepted trial (0 before the first)
  int bf16_off;        // KS_PREC_MIXED_BF16: the bf16 X^T G error reached kBf16Defect of
                       // ||grad E||; the run forms X^T G exactly from here on
};

// The bf16 X^T G of KS_PREC_MIXED_BF16 stays in use while its measured error is below this
// fraction of ||grad E||_F (the error enters the direction and the BB sums as noise).
constexpr double kBf16Defect = 0.05;

// The device records are carved at 256-byte boundaries and mirrored at fixed offsets in a
// 1 KiB pinned host buffer.
static_assert(sizeof(CgState) <= 256 && sizeof(LsState) <= 256 && sizeof(EvalOut) <= 256,
              "scalar records must fit their 256-byte slots");

// Constants of the discretisation, passed by value to kernels.
constexpr int kTuneAuto = -99;

struct Grid {
  int nx, ny, nz;
  int n;
  double h, inv_h2, dV;
  double lo[3];
  int q1;            // 0: 7-point finite differences; 1: trilinear finite elements
  double rhs_scale;  // Poisson right-hand side 4 pi * rhs_scale * rho (FE: h^3)
  double mu;         // weight of the kinetic (von Weizsaecker) term: H = mu/2 L + V_eff
  // launch shapes chosen by ks_autotune (kTuneAuto: the built-in rule)
  int fd_mode = kTuneAuto;  // plane-transform mode of the fast diagonalisation (kPlane*)
  int hx_zrun = kTuneAuto;  // planes per work item of the Gram-fused Hamiltonian (8, 16)
};

__host__ __device__ inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// (Op u)_g for u = z + beta po (po may be null): the 7-point -Laplacian_h, or for finite
// elements the Q1 stiffness stencil (centre 8h/3, edges -h/6, corners -h/12, faces 0).
__device__ inline double op_apply(const double* __restrict__ z, const double* __restrict__ po,
                                  double beta, int g, int i, int j, int k, const Grid& gr) {
  const int sy = gr.nx, sz = gr.nx * gr.ny;
  auto u = [&](int o) { return po ? z[g + o] + beta * po[g + o] : z[g + o]; };
  if (!gr.q1) {
    double nb = 0.0;
    if (i > 0) nb += u(-1);
    if (i < gr.nx - 1) nb += u(1);
    if (j > 0) nb += u(-sy);
    if (j < gr.ny - 1) nb += u(sy);
    if (k > 0) nb += u(-sz);
    if (k < gr.nz - 1) nb += u(sz);
    return (6.0 * u(0) - nb) * gr.inv_h2;
  }
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    if (k + dz < 0 || k + dz >= gr.nz) continue;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      if (j + dy < 0 || j + dy >= gr.ny) continue;
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (i + dx < 0 || i + dx >= gr.nx) continue;
        const int cls = (dx != 0) + (dy != 0) + (dz != 0);
        if (cls == 1) continue;
        s[cls] += u(dz * sz + dy * sy + dx);
      }
    }
  }
  return (8.0 * gr.h / 3.0) * s[0] - (gr.h / 6.0) * s[2] - (gr.h / 12.0) * s[3];
}

// The Poisson right-hand side 4 pi rhs_scale rho_g and the residual b - (Op x0)_g, in the one
// form every kernel that measures a Hartree residual uses (so their values agree bitwise).
__device__ inline double poisson_rhs(const double* __restrict__ rho, int g, const Grid& gr) {
  return 4.0 * kPi * gr.rhs_scale * rho[g];
}

// Blocks are dispatched round-robin over the 8 XCDs; map them so that each XCD gets
// one contiguous range of logical blocks (neighbouring grid planes share an L2).
__device__ inline int xcd_remap(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, idx = b / kXcds;
  return x * q + (x < r ? x : r) + idx;
}

// Copies n values into LDS: value e (e < n) is load(e), stored by store(e, v).  Each
// thread issues kB global loads before it stores any of them, so a block keeps kB loads
// per thread in flight instead of waiting on each one.  load must be safe to call for
// every e < n (clamp its address and select zero for padding).
template <int kB, typename Load, typename Store>
__device__ inline void lds_stage(int n, Load load, Store store) {
  for (int e0 = threadIdx.x; e0 < n; e0 += kB * blockDim.x) {
    double v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int e = e0 + u * blockDim.x;
      v[u] = load(e < n ? e : e0);
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < n) store(e, v[u]);
    }
  }
}

// Deterministic sum over a block of kBlock threads (fixed shuffle/LDS tree order).
// sh must hold kBlock/kWave doubles.  Result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s += sh[i];
  }
  __syncthreads();
  return s;
}

// block_sum of N values at once (one barrier): each value is summed in the same order as
// block_sum sums it, so the results are bitwise those of N block_sum calls.  sh holds
// N * (blockDim.x / kWave) doubles; the sums are valid in thread 0, whose values v[] are
// replaced by them.
template <int N>
__device__ inline void block_sum_n(double (&v)[N], double* sh) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += __shfl_down(v[k], o, kWave);
  }
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) sh[k * nw + w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int i = 0; i < nw; ++i) s += sh[k * nw + i];
      v[k] = s;
    }
  }
}

// ------------------------------------------------------------------------------------
// Batched launches.  A batched kernel runs the body of a single-system kernel for up to
// kMaxBatch systems in one launch: system s owns blocks [off[s], off[s+1]) and its
// argument record lives in device memory at a[s].  The body receives the block index and
// block count of its own system, so each system keeps the block partition (and the
// fixed-order reductions) of its lone launch and the results are bitwise the same.
// ------------------------------------------------------------------------------------
constexpr int kMaxBatch = 16;

template <typename A>
struct BatchPtrs {
  int S;
  int off[kMaxBatch + 1];
  const A* a[kMaxBatch];
  // With par: a[s] is the slot-0 record of system s and its record for the current slot
  // par[s] (device memory, read at run time) lies par[s] * rstride bytes further, so that a
  // captured launch serves every slot pattern.
  const int* par;
  int rstride;
};

template <typename A>
__device__ inline const A& batch_arg(const BatchPtrs<A>& b, int s) {
  const char* p = reinterpret_cast<const char*>(b.a[s]);
  if (b.par) p += (size_t)b.par[s] * b.rstride;
  return *reinterpret_cast<const A*>(p);
}

__device__ inline int batch_system(const int* off, int S, int b) {
  int s = 0;
  while (s + 1 < S && b >= off[s + 1]) ++s;
  return s;
}

// Lockstep runner (ks_api.hip): members run Alg. 3 with one launch per trial kernel for
// all of them.  batch_add starts a run on the system's stream (which must be the engine's
// stream); batch_tick advances every active member by one trial; batch_take pops a
// finished run.
struct BatchEngine;
BatchEngine* batch_create(hipStream_t st);
void batch_destroy(BatchEngine* e);
int batch_size(const BatchEngine* e);
int batch_add(BatchEngine* e, ks_system* s, void* X, const ks_opt_params* o, void* tag);
int batch_tick(BatchEngine* e);
bool batch_take(BatchEngine* e, void** tag, ks_result* r, int* code);

// ------------------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files).  All take the stream last.
// ------------------------------------------------------------------------------------
struct Partials {
  double* buf;      // [slot][block]
  int stride;       // max blocks per slot
};

// Argument records of the grid kernels (see BatchPtrs).
struct XcArgs {
  const double* rho;
  const double* vh;
  const double* vext;
  double* veff;
  Grid gr;
  int use_h;
  int use_x;        // bit 0: Slater exchange; bit 1: LDA correlation; bit 2: Thomas-Fermi
  const CgState* cg;
  Partials pt;
  // with cg_check: the residual test of the Hartree solve in the same pass (r.r and b.b of
  // r = b - L V_H to the SL_CGRR, SL_CGBB partials; a solve that fails it is restarted
  // from the CG start by the host, which forms r again)
  int cg_check;
  const double* vbc;  // monopole boundary potential added to V_eff (nullptr: none)
};

template <typename T>
struct HxArgs {
  const T* X;
  int ldx;
  T* Y;
  int ldy;
  const double* veff;
  Grid gr;
  int p;
  double scale;
  Partials pt;
  double* gram_part;  // optional (p = 32, ld = 32): partial X^T X, X^T G tiles
  int zrun;           // planes per work item of the Gram-fused kernel (hx_zrun)
};


// grid kernels (kernels_grid.hip)
void launch_vext(double* v, const double* R, const double* Z, int M, Grid g, double rc,
                 hipStream_t st);
// The GNH pseudopotential (Section 4.2) of nuclei R, Z on the grid through a radial table
// (gnh_table_doubles() doubles of device scratch, filled here).
size_t gnh_table_doubles();
void launch_vext_gnh(double* v, const double* R, const double* Z, int M, Grid g, double* table,
                     hipStream_t st);
void launch_enuc(double* out, const double* R, const double* Z, int M, hipStream_t st);
void launch_fill(double* x, double v, size_t n, hipStream_t st);
void launch_copy_vec(double* dst, const double* src, size_t n, hipStream_t st);
template <typename T>
void launch_copy_block(T* dst, int ldd, const T* src, int lds, int n, int p, hipStream_t st);
// Trilinear interpolation of an n_c x p block (row stride ldc) from the (cnx, cny, cnz)
// interior nodes to the nested (2cnx+1, 2cny+1, 2cnz+1) mesh (row stride ldf), times scale.
template <typename T>
void launch_prolong(const T* xc, int ldc, int cnx, int cny, int cnz, T* xf, int ldf, int p,
                    double scale, hipStream_t st);
template <typename T>
void launch_density(const T* X, int ld, int n, int p, double scale, double* rho,
                    hipStream_t st);
void launch_xc(const double* rho, const double* vh, const double* vext, double* veff,
               Grid g, int use_h, int use_x, const CgState* cg, Partials pt, hipStream_t st,
               bool cg_check = false, const double* vbc = nullptr);
// Monopole boundary of the Hartree potential: the interior right-hand side of the boundary
// values Q/|r_b - c|, divided by 4 pi rhs_scale so that the Hartree solver's own right-hand
// side 4 pi rhs_scale x reproduces it (7-point: face neighbours / h^2; Q1: edge neighbours
// h/6, corners h/12); then out = -(1/2) Q V(c) by trilinear interpolation of V at c.
void launch_bc_rhs(double* out, Grid g, double Q, double cx, double cy, double cz,
                   hipStream_t st);
void launch_bc_point(const double* v, Grid g, double Q, double cx, double cy, double cz,
                     double* out, hipStream_t st);
// Y = scale ((1/2) L X + Diag(veff) X); with pt the per-block partials of sum X.(L X)
template <typename T>
void launch_hx(const T* X, int ldx, T* Y, int ldy, const double* veff, Grid g, int p,
               double scale, Partials* pt, double* gram_part, hipStream_t st);
int hx_blocks(int n, int p);  // blocks (and energy partials) of launch_hx
// With gram_part (p = 32, ld = 32, pt given) launch_hx also forms the partial Gram tiles
// X^T X and X^T G (products 0 and 1) with hx_gram_blocks(n) blocks.
int hx_gram_blocks(int n);
bool hx_fuses_gram(int p);
int hx_zrun(int nxy, int nz);  // planes per work item of the Gram-fused launch
int hx_zrun_of(const Grid& g);  // the grid's tuned value, else hx_zrun
void launch_xc_batch(const BatchPtrs<XcArgs>& b, int blocks, hipStream_t st);
template <typename T>
void launch_hx_batch(const BatchPtrs<HxArgs<T>>& b, int blocks, bool gram, hipStream_t st);
int scalar_blocks(int n);
// Hartree solver (kernels_poisson.hip)
struct FdOps {
  const double *Sx, *Sy, *Sz;   // sine-transform matrices per axis
  const double *lx, *ly, *lz;   // eigenvalues of the 1D operator per axis
  const double *mx, *my, *mz;   // eigenvalues of the 1D mass matrix (1 for differences)
};
// Argument records of the Hartree kernels (one per launch; see BatchPtrs).
struct InitArgs {
  const double* rho;
  const double* x0;
  double* x;        // nullptr: x0 is the iterate (no copy)
  double* r;
  double* p0;
  Grid gr;
  double* part;
};

struct FinInitArgs {
  const double* part;
  int nb;
  CgState* cs;
  double tol;
  int maxit;
  int it0;          // iterations the start already stands for (1 after a direct solve)
};

struct DirArgs {
  const double* z;
  const double* po;
  double* pn;
  double* q;
  const CgState* cs;
  Grid gr;
  double* part;
};

struct FinDirArgs {
  const double* part;
  int nb;
  CgState* cs;
  int pcg;
};

struct UpdArgs {
  double* x;
  double* r;
  const double* pn;
  const double* q;
  const CgState* cs;
  Grid gr;
  double* part;
};

struct FinUpdArgs {
  const double* part;
  int nb;
  CgState* cs;
  int pcg;
};

struct FinRzArgs {
  const double* part;
  int nb;
  CgState* cs;
};

struct FdPlaneArgs {
  const double* in;
  double* out;
  const double* Sxg;
  const double* Syg;
  int nx;
  int ny;
  const double* r;
  double* part;
  const CgState* cs;  // nullptr: no early exit
  const double* add;  // optional: out = add + transform
};

struct FdZArgs {
  double* u;
  const double* Szg;
  const double* lx;
  const double* ly;
  const double* lz;
  const double* mx;
  const double* my;
  const double* mz;
  int nx;
  int ny;
  int nz;
  const CgState* cs;
};

size_t hartree_part_doubles();
// Launch shapes of the Hartree kernels for one system (blocks and dynamic LDS).
int hartree_blocks(int n);
// Plane-transform modes: 16-column strips (S_y read from L2), strips with S_y staged in
// LDS, one whole plane per block.
// plane transform modes, slowest first: S_x strip read from global memory, S_x strip in
// LDS, S_x strip and S_y in LDS, whole plane per block
enum { kPlaneStripG = -1, kPlaneStrip = 0, kPlaneStripSy = 1, kPlaneFull = 2 };
size_t fd_plane_bytes(int nx, int ny, int mode);
int fd_plane_mode(int nx, int ny);  // the fastest mode whose LDS fits
int fd_plane_mode_of(const Grid& g);  // the grid's tuned mode, else fd_plane_mode
bool fd_plane_mode_fits(int nx, int ny, int mode);
int fd_plane_blocks(int nx, int nz, int mode);
bool fd_fits(int nx, int ny, int nz);  // the transforms' LDS fits for this grid
struct FdLaunch {
  int plane_mode;
  size_t z_bytes, z_bytes_staged, cap;
  int z_blocks;
};
FdLaunch fd_launch(const Grid& g);
void launch_dir_batch(const BatchPtrs<DirArgs>& b, int blocks, hipStream_t st);
void launch_fin_dir_batch(const BatchPtrs<FinDirArgs>& b, hipStream_t st);
void launch_upd_batch(const BatchPtrs<UpdArgs>& b, int blocks, hipStream_t st);
void launch_fin_upd_batch(const BatchPtrs<FinUpdArgs>& b, hipStream_t st);
void launch_fin_rz_batch(const BatchPtrs<FinRzArgs>& b, hipStream_t st);
void launch_init_batch(const BatchPtrs<InitArgs>& b, int blocks, hipStream_t st);
void launch_fd_plane_batch(const BatchPtrs<FdPlaneArgs>& b, int blocks, int mode, size_t lds,
                           hipStream_t st);
void launch_fd_z_batch(const BatchPtrs<FdZArgs>& b, int blocks, bool staged, size_t lds,
                       hipStream_t st);
size_t fd_lds_bytes(int nx, int ny, int nz);
int fd_max_plane();
void launch_fd_setup(double* S, double* lam, double* mu, int N, double h, int q1,
                     hipStream_t st);
void launch_hartree_init(const double* rho, const double* x0, double* x, double* r, double* p0,
                         CgState* cs, double tol, int maxit, int it0, Grid g, double* part,
                         hipStream_t st);
// r = 4 pi rhs_scale rho - L x0 (x0 may be nullptr: r = b) with the partials r.r, b.b
void launch_cg_residual(const double* rho, const double* x0, double* r, double* p0, Grid g,
                        double* part, hipStream_t st);
// x = x0 + L^{-1} r (or A^{-1} r; x0 may be nullptr) in three fast-diagonalisation passes
// (plane, z with the eigenvalue division, plane); tmp is an n-vector of scratch.
void launch_fd_correct(const double* r, const double* x0, double* x, double* tmp,
                       const FdOps& fd, Grid g, hipStream_t st);
// z = L^{-1} r (or A^{-1} r) by the fast diagonalisation; tmp is an n-vector of scratch.
void launch_fd_apply(const double* r, double* z, double* tmp, const FdOps& fd, Grid g,
                     const CgState* cs, double* part, hipStream_t st);
void launch_hartree_iter(double* x, double* r, const double* z, double* pa, double* pb,
                         double* q, CgState* cs, Grid g, double* part, int pcg,
                         hipStream_t st);

// trilinear finite elements (kernels_fe.hip)
// G = scale ((1/2) A X + h^3 Diag(veff) X) (with kG) and BX = B X; with pt the partials
// sum X.(AX).  Blocks are n x p.
template <typename T>
void launch_q1_apply(const T* X, T* G, T* BX, const double* veff, Grid g, int p, double scale,
                     Partials* pt, hipStream_t st);
// Tables of the constant-coefficient tridiagonal solve with the 1D mass matrix (2N doubles)
void launch_mass_setup(double* tab, int N, double h, hipStream_t st);
// out = B^{-1} in (in and out may be the same block)
template <typename T>
void launch_mass_solve(const T* in, T* out, int p, Grid g, const double* const tab[3],
                       hipStream_t st);
// D = Gt + X W and BD = G + BX W (W: pp x pp), partials ||D||_B^2 and the B-metric BB
// sums against (Xc, BXc, Dc, BDc) when those are given.
struct Q1GradArgs {
  const void *Gt, *X, *G, *BX;
  const double* W;
  void *D, *BD;
  const void *Xc, *BXc, *Dc, *BDc;
  Partials pt;
  int n, p, pp;
  bool f32;
};
void launch_q1_grad(const Q1GradArgs& a, hipStream_t st);
int q1_grad_blocks(int n, int p);
size_t q1_grad_lds(int p);  // dynamic LDS of the gradient kernel (its weights; p <= 128)
// Sets the message ks_last_error(NULL) returns on the calling thread.
void set_thread_error(const char* msg);
// True when [ptr, ptr + bytes) starts and ends inside memory the HIP runtime knows as
// device (or managed) memory; a query the runtime refuses leaves no pending error.
bool device_range(const void* ptr, size_t bytes);
int q1_apply_blocks(Grid g, int p);

// Raises kernel k's dynamic-LDS limit to bytes the first time it is asked for that kernel
// and does nothing afterwards (each call site always asks the same value), so launches
// made later, for instance while a stream is being captured into a graph, issue no
// runtime call besides the launch.  Thread-safe.
void set_dyn_lds_once(const void* k, int bytes);

// dense kernels (kernels_dense.hip)
// Argument records of the Gram kernels (see BatchPtrs).
template <typename T>
struct GramArgs {
  const T* A;
  const T* B;
  int ld;
  int n;
  int p;
  double* part;
  int pb;  // columns of B when they differ from p (0: p)
};

struct GramReduceArgs {
  const double* part;
  int nchunks;
  int pp;
  int mask;
  double* out;
  double* W;
  // optional (p <= 64): product 1 (X^T D of D = G + X W) formed as X^T G + (X^T X) W from
  // these reduced blocks instead of from partials
  const double* xd_xg;
  const double* xd_xx;
  const double* xd_W;
};


constexpr int kGramAA = 1, kGramAB = 2, kGramBB = 4;  // product bits of a Gram launch
int gram_chunks(int n, int pp);
size_t gram_part_doubles(int n, int pp);
// A, B: n x ld blocks of float (f32) or double; products accumulate in FP64
void launch_gram(const void* A, const void* B, bool f32, int ld, int n, int p, int mask,
                 double* partials, int nchunks, hipStream_t st);
// out: [3][pp][pp]; products outside mask are not written; W (nullable) = -(A^T B)^T
void launch_gram_reduce(const double* partials, int nchunks, int pp, int mask, double* out,
                        double* W, hipStream_t st, const double* xd_xg = nullptr,
                        const double* xd_xx = nullptr, const double* xd_W = nullptr);
struct CombineArgs {
  // orbital blocks are float when f32, else double; weights and sums are double
  const void* X; const double* A;       // X (n x ld) times A (pp x pp)
  const void* Y; const double* B;       // optional Y (n x ld) times B
  const void* C0;                       // optional additive n x ld term
  void* out;                            // n x ld
  double* rho; double rho_scale;        // optional density of out
  // optional BB/gradient epilogue: out is D_t; uses Xt (= X), Xk, Dk
  const void* Xk; const void* Dk;
  Partials pt;                          // slots SL_DD.. SL_YY (by value)
  double* gram_part;                    // optional (p_p <= 32): partial X^T D, D^T D tiles
  int ld, n, p;
  bool f32;
  bool upper;                           // A and B are upper triangular (QR retraction)
  int lda;                              // row stride of A and B (0: p_p of the launch)
  int pk;                               // columns of X and Y to contract over (0: p)
  bool mc;                              // float data, blocks wider than 64 columns: fp32
                                        // matrix cores with FP64 sums across chains
  // BB sums of a QR trial without a pass over X_k (FP64, p_p <= 32).  Retraction: also the
  // partials of ||s||^2 (SL_SS) and <s, D_k> (SL_SY), s = out - X (X = X_k, Y = D_k).
  // Gradient: X_k is not read; the partials are ||D||^2 (SL_DD) and <D_k, D> (SL_YY).
  bool bbr;
  // optional with rho (7-point grid): resid = 4 pi rhs_scale rho - L resid_x0, the first
  // residual of the next Hartree solve from its warm start (the arithmetic of the CG start)
  double* resid;
  const double* resid_x0;
  int gnx, gny, gnz;
  double inv_h2, rhs_scale;
};
void launch_combine(const CombineArgs& a, hipStream_t st);
// Events for the next single-kernel combine launch of this host thread: that launch records
// them from its own dispatch (its exact start and end), and clears them.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
// Blocks of scalar partials a combine launch writes per slot (the persistent blocks of the
// wide combine when p > 64).
int combine_partial_blocks(int n, int p);
// Reduced Gram products (mask over A^T A, A^T B, B^T B) of blocks wider than 64 columns,
// written into out (3 x p_p x p_p, products outside the mask untouched) and, with W,
// W = -(A^T B)^T; sub is 3 x 64 x 64 doubles of scratch.  sym_ab: A^T B is symmetric, so
// only its blocks I <= J are formed (and mirrored).  bf16_mask (float storage only): the
// products whose bit is set run on the bf16 matrix cores with fp32 accumulation.
void launch_gram_full(const void* A, const void* B, bool f32, int ld, int n, int p, int mask,
                      double* partials, double* sub, double* out, double* W, hipStream_t st,
                      bool sym_ab = false, int bf16_mask = 0);
// Batched Gram (products kMask of [A, B], p_p <= 32), its reduction, and the two combine
// forms of a trial: the retraction (X A + Y B with the density) and the gradient
// (C0 + X A with the BB sums).
template <typename T>
void launch_gram_batch(const BatchPtrs<GramArgs<T>>& b, int pp, int mask, int blocks,
                       hipStream_t st);
void launch_gram_reduce_batch(const BatchPtrs<GramReduceArgs>& b, int blocks, hipStream_t st);
int gram_reduce_blocks(int pp);
template <typename T>
void launch_combine_retract_batch(const BatchPtrs<CombineArgs>& b, int pp, int blocks,
                                  hipStream_t st);
// (the gradient form also accumulates the Gram tiles X^T D, D^T D into gram_part)
template <typename T>
void launch_combine_grad_batch(const BatchPtrs<CombineArgs>& b, int pp, int blocks,
                               hipStream_t st);
int combine_blocks(int n);

// small dense kernels (kernels_small.hip)
// Argument records of the per-system small kernels (see BatchPtrs).
struct QrFactor2dArgs {
  const double* xx;
  const double* gxd;
  int p;
  int pp;
  const double* tau_p;
  double* A;
  double* B;
  int* status;
  // With sel, the factor of the next trial launched before the host has read the line-search
  // record: it returns at once when that trial will not run (a stop, an error or a pending
  // Hartree solve), and takes xx_rej, gxd_rej (the current point's blocks) when the last
  // trial was rejected.
  const LsState* sel;
  const double* xx_rej;
  const double* gxd_rej;
  double* R;  // optional (p <= 64): the Cholesky factor R itself, p_p x p_p, zero below
};

struct FinishEvalArgs {
  const double* part;
  int stride;
  ScalarCounts nb;
  double* sums;
  const double* xx;
  int p;
  int pp;
  double f;
  double dV;
  const double* enuc;
  const CgState* cg;
  EvalOut* out;
  LsState* ls;
  LsParams prm;
  // with cgw: the CG start of a solve whose residual was measured in the exchange pass
  // (SL_CGRR, SL_CGBB) is written here before the judgement reads it
  CgState* cgw;
  double htol;
  int hmaxit;
  const double* ebc;  // the constant -(1/2) Q V_bc(c) of the monopole boundary (or nullptr)
  // BB sums of a QR trial without X_k in the gradient pass (with ls; see CombineArgs::bbr):
  // R (p_p x p_p, the trial's Cholesky factor) and X_t^T D_t (p_p x p_p)
  const double* bbr_R;
  const double* bbr_xtd;
  // optional: mirror_bytes (a multiple of 16) from mirror_src copied to mirror (host memory
  // mapped for the device) at the end, after the records are written
  void* mirror;
  const void* mirror_src;
  int mirror_bytes;
};


void launch_grad_weights(const double* gram, int pp, double* W, hipStream_t st);
void launch_qr_factor(const double* xx, const double* gxd, int p, int pp, const double* tau,
                      double* A, double* B, double* work, int* status, hipStream_t st,
                      double* R = nullptr);
// Per-tile partials (ceil(p/16)^2 of them, written to part) of ||xg - (xd - xx W)||_F^2:
// with xd = X^T D and xx = X^T X exact products of the stored blocks (X^T B D, X^T B X for
// finite elements) and D = G + X W, xd - xx W is the exact X^T G, so this is the error of
// the bf16 X^T G in xg.
void launch_bf16_defect(const double* xg, const double* xd, const double* xx, const double* W,
                        int p, int pp, double* part, hipStream_t st);
int bf16_defect_blocks(int p);
// C = A + B W (p x p blocks of stride pp, FP64; C may not alias B or W).
void launch_small_gemm_add(const double* A, const double* B, const double* W, double* C, int p,
                           int pp, hipStream_t st);
// The p <= 64 factor in its speculative form (see QrFactor2dArgs::sel).
void launch_qr_factor_next(const QrFactor2dArgs& a, hipStream_t st);
void launch_wy_factor(const double* gram_xg, int p, int pp, const double* tau,
                      double reorth_tol, double* A, double* B, double* work, int* status,
                      int* reorth_flag, hipStream_t st);
size_t small_work_doubles(int p);
void launch_ls_reset(LsState* ls, hipStream_t st);
void launch_compact_gram(const double* gram, int pp, int p, double* out, hipStream_t st);
// Sums the scalar partials (nblk[slot] blocks per slot, slot stride `stride`) into sums,
// writes the evaluation summary and, with ls, judges the trial (Alg. 3 line search).
void launch_finish_eval(const double* part, int stride, const int* nblk, double* sums,
                        const double* gram_xx, int p, int pp, double f, double dV,
                        const double* enuc, const CgState* cg, EvalOut* out, LsState* ls,
                        const LsParams* prm, hipStream_t st, CgState* cgw = nullptr,
                        double htol = 0.0, int hmaxit = 0, const double* ebc = nullptr,
                        const double* bbr_R = nullptr, const double* bbr_xtd = nullptr,
                        void* mirror = nullptr, const void* mirror_src = nullptr,
                        int mirror_bytes = 0);
void launch_set_scalar(double* dst, double v, hipStream_t st);
void launch_qr_factor_batch(const BatchPtrs<QrFactor2dArgs>& b, int p_max, hipStream_t st);
void launch_finish_eval_batch(const BatchPtrs<FinishEvalArgs>& b, hipStream_t st);
// Copies `bytes` from each src[s] to dst + s * bytes (one block per system).
struct GatherArgs {
  int S, bytes;
  const char* src[kMaxBatch];
  char* dst;
};
void launch_gather(const GatherArgs& g, hipStream_t st);
// Writes n (at most kMaxBatch) integers, passed by value, to dst[0..n) on the device.
struct IntList {
  int n;
  int v[kMaxBatch];
};
void launch_set_ints(int* dst, const IntList& l, hipStream_t st);
void launch_ls_init(const EvalOut* ev, LsState* ls, LsParams prm, hipStream_t st);
// After the current iterate was re-orthonormalised and evaluated again (ev): the
// nonmonotone reference restarts there (C = E, Q = 1); k, the step and the stagnation
// history are kept, and the gradient and energy-target tests are applied to the new point.
void launch_ls_restart(const EvalOut* ev, LsState* ls, LsParams prm, hipStream_t st);
}  // namespace ks
