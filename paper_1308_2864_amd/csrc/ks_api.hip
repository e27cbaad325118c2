// C ABI of the library (include/ks.h): system lifecycle, workspace layout and the host
// side of Alg. 3.  The host only orders kernel launches on the caller's stream and reads
// back small scalar records (CG state, line-search state); every number on the data path
// is computed by the kernels in kernels_grid.hip, kernels_dense.hip, kernels_small.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ks_common.h"
#include "../../include/ks.h"

using namespace ks;

namespace ks {

bool device_range(const void* ptr, size_t bytes) {
  if (!ptr || bytes == 0) return false;
  const char* ends[2] = {static_cast<const char*>(ptr), static_cast<const char*>(ptr) + bytes - 1};
  for (const char* q : ends) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, q) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged &&
        at.type != hipMemoryTypeUnified)
      return false;
  }
  return true;
}

}  // namespace ks

namespace {
thread_local std::string g_err;
}  // namespace

namespace ks {
void set_thread_error(const char* msg) { g_err = msg ? msg : ""; }
}  // namespace ks

namespace {
constexpr int kPartStride = 4096;  // >= blocks of every streaming kernel
// argument records of the batched trial kernels: one 320-byte slot per kernel and parity
enum Rec {
  R_QR, R_RETRACT, R_RESID, R_PLANE1, R_FDZ, R_PLANE2, R_XC, R_HX, R_GRAM1,
  R_RED1, R_GRAD, R_RED2, R_FINISH, R_QR_NEXT, R_COUNT
};
constexpr size_t kRecSlot = 320;
constexpr size_t kRecBytes = 2 * R_COUNT * kRecSlot;
constexpr int kGatherBytes = 512;  // CgState and LsState of one system (adjacent)
constexpr size_t kHostBytes = 1024 + (size_t)kMaxBatch * kGatherBytes;
}  // namespace

namespace ks {
// State of one Alg. 3 run between its trials.  ks_minimize, the per-iteration calls, state
// save and restore, and the lockstep runner all keep it in the system handle, so every
// route takes the same decisions from the same device records.
struct MinRun {
  ks_opt_params prm{};
  LsParams lp{};
  bool qr = true;
  int c = 0;
  void* X_inout = nullptr;
  std::chrono::steady_clock::time_point t0;
  bool active = false;   // begun and not yet ended
  bool queued = false;   // the QR factor of the next trial is already on the stream
  bool records = false;  // the lockstep argument records of this run are on the device
  int reorths = 0;       // re-orthonormalisations requested by reorth_every
};
}  // namespace ks

struct ks_system {
  ks_system_desc d{};
  ks::MinRun run;
  std::vector<double> R, Z;
  hipStream_t st = nullptr;
  Grid grid{};
  int n = 0, p = 0, ld = 0, pp = 0;
  double f = 2.0;
  int use_ext = 1, use_h = 1, use_x = 1;
  double htol = 1e-13;
  int hmaxit = 5000;
  // device buffers carved from the caller's workspace
  double *vext = nullptr, *rho = nullptr, *vh[2] = {}, *veff[2] = {};
  double *cg_r = nullptr, *cg_p[2] = {}, *cg_q = nullptr, *cg_z = nullptr;
  int cg_par = 0;
  double *fdS[3] = {}, *fdL[3] = {}, *fdM[3] = {};
  // trilinear finite elements: B^{-1} tables and, per slot, B^{-1} G, B X, B grad E and the
  // Gram block X^T B X (slot 1 of a [3][pp][pp] buffer)
  bool q1 = false;
  double* mtab[3] = {};
  // batched runs: argument records of the trial kernels for both slot parities, and a
  // staging area for the scalar records of a whole batch (used when this system leads)
  char* rec = nullptr;
  char* gstage = nullptr;
  int* slots = nullptr;  // record slots of the members of a replayed batch tick (lead only)
  void *Gt[2] = {}, *BX[2] = {}, *BD[2] = {};
  double* feg[2] = {};
  // the Cayley system of the B metric per slot: [X^T B X, X^T G, G^T B^{-1} G]
  double* wyg[2] = {};
  int solver = KS_HARTREE_CG;
  double *Rd = nullptr, *Zd = nullptr, *enuc = nullptr, *tau_user = nullptr;
  double* gnh_tab = nullptr;  // radial table of the GNH pseudopotential (KS_VEXT_GNH)
  double* vbc = nullptr;      // monopole boundary potential of the Hartree problem
  double* ebc = nullptr;      // its energy constant -(1/2) Q V_bc(c)
  void *X[2] = {}, *G[2] = {}, *D[2] = {};  // float (FP32 modes) or double
  bool f32 = false;
  bool bf16 = false;  // KS_PREC_MIXED_BF16: float storage, Gram sub-products in bf16
  bool mc = false;    // KS_PREC_FP32_MFMA: float storage, wide products on fp32 matrix cores
  bool bf16_on = true;  // a run switches it off once the bf16 X^T G error is too large
  int es = 8;  // bytes per orbital element
  double *gxg[2] = {}, *gxd[2] = {}, *W = nullptr, *A = nullptr, *B = nullptr;
  double *work = nullptr, *gram_part = nullptr, *spart = nullptr, *cgpart = nullptr;
  double* gsub = nullptr;
  double* Rq = nullptr;  // the Cholesky factor R of the last QR trial (BB sums without X_k)
  double* sums[2] = {};
  CgState* cg = nullptr;
  EvalOut* ev[2] = {};
  LsState* ls = nullptr;
  int* status = nullptr;
  int* reorth_count = nullptr;
  int cur = 0;
  int gram_nchunks = 1;
  // pinned host mirror of the scalar records
  void* host = nullptr;
  void* host_dev = nullptr;     // the device's address of host (kernels write the mirror)
  bool mirror_written = false;  // the last summary wrote the CG and line-search records there
  std::string err;
  int last_cg_iters = 0;
  int pcg_extra = 0;     // PCG iterations queued after the exact step of a trial's solve
  bool fuse_cg = false;  // the next exchange pass measures the Hartree residual (see hartree)
  bool cg_fused = false;  // the last evaluation measured it there (its r was not stored)
  bool pcg_probe = false;  // the first trial of a run queues one to see whether it is needed
  bool resid_ready = false;  // the retraction formed the next Hartree solve's first residual
  long long cg_total = 0;
  // optional phase timers
  struct Pending {
    hipEvent_t a, b;
    int ph;
  };
  bool timers = false;
  unsigned timer_mask = ~0u;  // phases timed while timers are on
  // optional graph replay of the trial step of ks_minimize (one graph per slot parity)
  bool graphs = false;
  hipStream_t cap_st = nullptr;
  hipGraphExec_t gx[2] = {};
  std::vector<hipEvent_t> ev_free;
  hipEvent_t ev_rb = nullptr;  // marks the end of a trial's record copy (the wait ahead)
  std::vector<Pending> ev_pend;
  Pending ev_open[KS_NPHASES] = {};
  double ph_ms[KS_NPHASES] = {};
  long long ph_n[KS_NPHASES] = {};
};

namespace {

// ---- workspace layout ------------------------------------------------------------------

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) / 256 * 256;
    T* ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return ptr;
  }
};

void layout(ks_system* s, char* base, size_t* total) {
  Carver c{base};
  const size_t n = (size_t)s->n, np = (size_t)s->n * s->p, pp2 = (size_t)s->pp * s->pp;
  const int M = (int)s->R.size() / 3;
  s->vext = c.take<double>(n);
  s->rho = c.take<double>(n);
  for (int i = 0; i < 2; ++i) {
    s->vh[i] = c.take<double>(n);
    s->veff[i] = c.take<double>(n);
  }
  s->cg_r = c.take<double>(n);
  s->cg_p[0] = c.take<double>(n);
  s->cg_p[1] = c.take<double>(n);
  s->cg_q = c.take<double>(n);
  s->cg_z = c.take<double>(n);
  const int dims[3] = {s->grid.nx, s->grid.ny, s->grid.nz};
  for (int a = 0; a < 3; ++a) {
    s->fdS[a] = c.take<double>((size_t)dims[a] * dims[a]);
    s->fdL[a] = c.take<double>((size_t)dims[a]);
    s->fdM[a] = c.take<double>((size_t)dims[a]);
    if (s->q1) s->mtab[a] = c.take<double>(2 * (size_t)dims[a]);
  }
  s->Rd = c.take<double>(3 * (size_t)(M > 0 ? M : 1));
  s->Zd = c.take<double>((size_t)(M > 0 ? M : 1));
  s->enuc = c.take<double>(1);
  s->tau_user = c.take<double>(1);
  if (s->d.vext_kind == KS_VEXT_GNH) s->gnh_tab = c.take<double>(gnh_table_doubles());
  if (s->d.hartree_bc == KS_HBC_MONOPOLE && (s->d.terms & KS_TERM_HARTREE)) {
    s->vbc = c.take<double>(n);
    s->ebc = c.take<double>(1);
  }
  for (int i = 0; i < 2; ++i) {
    s->X[i] = c.take<char>(np * s->es);
    s->G[i] = c.take<char>(np * s->es);
    s->D[i] = c.take<char>(np * s->es);
    s->gxg[i] = c.take<double>(3 * pp2);
    s->gxd[i] = c.take<double>(3 * pp2);
    s->sums[i] = c.take<double>(kMaxScalarSlots);
    s->ev[i] = c.take<EvalOut>(1);
    if (s->q1) {
      s->Gt[i] = c.take<char>(np * s->es);
      s->BX[i] = c.take<char>(np * s->es);
      s->BD[i] = c.take<char>(np * s->es);
      s->feg[i] = c.take<double>(3 * pp2);
      s->wyg[i] = c.take<double>(3 * pp2);
    }
  }
  s->W = c.take<double>(pp2);
  s->A = c.take<double>(pp2);
  s->B = c.take<double>(pp2);
  s->Rq = c.take<double>(pp2);
  s->work = c.take<double>(small_work_doubles(s->p));
  s->gram_nchunks = gram_chunks(s->n, s->pp);
  s->gram_part = c.take<double>(gram_part_doubles(s->n, s->pp));
  s->gsub = c.take<double>(3 * 64 * 64);  // one reduced 64-column bf16 sub-product (p > 64)
  s->spart = c.take<double>((size_t)SL_COUNT * kPartStride);
  s->cgpart = c.take<double>(hartree_part_doubles());
  s->cg = c.take<CgState>(1);
  s->ls = c.take<LsState>(1);  // 256 bytes after cg, mirrored on the host the same way
  s->status = c.take<int>(1);
  s->reorth_count = c.take<int>(1);
  s->rec = c.take<char>(kRecBytes);
  s->gstage = c.take<char>((size_t)kMaxBatch * kGatherBytes);
  s->slots = c.take<int>(kMaxBatch);
  *total = c.off + 256;
}

int validate(const ks_system_desc* d, std::string* why) {
  if (!d) { *why = "null descriptor"; return KS_E_INVAL; }
  if (d->disc != KS_DISC_FD7 && d->disc != KS_DISC_Q1) {
    *why = "unknown discretisation";
    return KS_E_UNSUPPORTED;
  }
  if (d->disc == KS_DISC_Q1 && (d->nx > 128 || d->ny > 128 || d->nz > 128)) {
    *why = "the finite-element mass solve supports at most 128 nodes per axis";
    return KS_E_UNSUPPORTED;
  }
  if (d->precision != KS_PREC_FP64 && d->precision != KS_PREC_FP32 &&
      d->precision != KS_PREC_MIXED_BF16 && d->precision != KS_PREC_FP32_MFMA) {
    *why = "precision must be KS_PREC_FP64, KS_PREC_FP32, KS_PREC_MIXED_BF16 or "
           "KS_PREC_FP32_MFMA";
    return KS_E_UNSUPPORTED;
  }
  if (d->hartree_solver != KS_HARTREE_CG && d->hartree_solver != KS_HARTREE_PCG_FD) {
    *why = "unknown Hartree solver";
    return KS_E_UNSUPPORTED;
  }
  if (d->hartree_solver == KS_HARTREE_PCG_FD &&
      (((d->nx + 15) / 16) * ((d->ny + 15) / 16) * 256 > fd_max_plane() || d->nz > 128 ||
       !fd_fits(d->nx, d->ny, d->nz))) {
    *why = "the fast-diagonalisation solver needs a plane in LDS (at most 128 x 128 planes) "
           "and nz <= 128";
    return KS_E_UNSUPPORTED;
  }
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) { *why = "grid sizes must be >= 1"; return KS_E_INVAL; }
  if (!(d->h > 0.0) || !std::isfinite(d->h)) { *why = "h must be > 0"; return KS_E_INVAL; }
  if (d->p < 1 || d->p > 512) { *why = "p must be in [1, 512]"; return KS_E_INVAL; }
  if (d->disc == KS_DISC_Q1 && d->p > 128) {
    *why = "the finite-element gradient kernel supports p <= 128 (its weights live in LDS)";
    return KS_E_UNSUPPORTED;
  }
  const int ld = d->ld ? d->ld : d->p;
  if (ld < d->p) { *why = "ld must be >= p"; return KS_E_INVAL; }
  const double cells = (double)d->nx * d->ny * d->nz;
  if (cells * ld >= 2147483647.0 || cells * d->p >= 2147483647.0) {
    *why = "n * ld must be < 2^31";
    return KS_E_INVAL;
  }
  if (!(d->occupation > 0.0)) { *why = "occupation must be > 0"; return KS_E_INVAL; }
  if (d->n_nuclei < 0) { *why = "n_nuclei must be >= 0"; return KS_E_INVAL; }
  if (d->hartree_bc != KS_HBC_ZERO && d->hartree_bc != KS_HBC_MONOPOLE) {
    *why = "unknown hartree_bc";
    return KS_E_INVAL;
  }
  if (d->vext_kind != KS_VEXT_ERF && d->vext_kind != KS_VEXT_GNH) {
    *why = "unknown vext_kind";
    return KS_E_INVAL;
  }
  if (!(d->kinetic_scale >= 0.0) || !std::isfinite(d->kinetic_scale)) {
    *why = "kinetic_scale must be >= 0";
    return KS_E_INVAL;
  }
  if (d->n_nuclei > 0 && (!d->R || !d->Z)) { *why = "R and Z are required"; return KS_E_INVAL; }
  if ((d->terms & KS_TERM_EXT) && d->n_nuclei > 0 && !d->v_ext_override &&
      d->vext_kind == KS_VEXT_ERF && !(d->rc > 0.0)) {
    *why = "rc must be > 0";
    return KS_E_INVAL;
  }
  return KS_OK;
}

void init_dims(ks_system* s, const ks_system_desc* d) {
  s->d = *d;
  s->n = d->nx * d->ny * d->nz;
  s->p = d->p;
  s->ld = d->ld ? d->ld : d->p;
  s->pp = round_up(d->p, 16);
  s->f = d->occupation;
  s->use_ext = (d->terms & KS_TERM_EXT) ? 1 : 0;
  s->use_h = (d->terms & KS_TERM_HARTREE) ? 1 : 0;
  s->use_x = ((d->terms & KS_TERM_XC) ? 1 : 0) | ((d->terms & KS_TERM_CORR) ? 2 : 0) |
             ((d->terms & KS_TERM_TF) ? 4 : 0);
  s->htol = d->hartree_tol > 0.0 ? d->hartree_tol : 1e-13;
  s->hmaxit = d->hartree_maxit > 0 ? d->hartree_maxit : 5000;
  s->solver = d->hartree_solver;
  s->bf16 = d->precision == KS_PREC_MIXED_BF16;
  s->mc = d->precision == KS_PREC_FP32_MFMA;
  s->f32 = d->precision == KS_PREC_FP32 || s->bf16 || s->mc;
  s->es = s->f32 ? 4 : 8;
  s->R.assign(d->R ? d->R : nullptr, d->R ? d->R + 3 * d->n_nuclei : nullptr);
  s->Z.assign(d->Z ? d->Z : nullptr, d->Z ? d->Z + d->n_nuclei : nullptr);
  s->grid.nx = d->nx;
  s->grid.ny = d->ny;
  s->grid.nz = d->nz;
  s->grid.n = s->n;
  s->grid.h = d->h;
  s->grid.inv_h2 = 1.0 / (d->h * d->h);
  s->grid.dV = d->h * d->h * d->h;
  for (int i = 0; i < 3; ++i) s->grid.lo[i] = d->box_lo[i];
  s->q1 = d->disc == KS_DISC_Q1;
  s->grid.q1 = s->q1 ? 1 : 0;
  // the finite-element Poisson problem is A V_H = 4 pi h^3 rho (nodal quadrature)
  s->grid.rhs_scale = s->q1 ? s->grid.dV : 1.0;
  s->grid.mu = d->kinetic_scale > 0.0 ? d->kinetic_scale : 1.0;
}

// Density scale: rho_g = (f/h^3) sum X^2 on the grid (X^T X = I); rho_k = f sum X^2 at the
// finite-element nodes (X^T B X = I).
double rho_scale(const ks_system* s) { return s->q1 ? s->f : s->f / s->grid.dV; }

int fail(ks_system* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  g_err = msg;
  return code;
}

int hip_check(ks_system* s, hipError_t e, const char* what) {
  if (e == hipSuccess) return KS_OK;
  return fail(s, KS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int launch_check(ks_system* s, const char* what) {
  return hip_check(s, hipGetLastError(), what);
}

// ---- orbital-block launches in the system's storage precision -----------------------

void copy_block(ks_system* s, void* dst, int ldd, const void* src, int lds) {
  if (s->f32)
    launch_copy_block<float>(static_cast<float*>(dst), ldd, static_cast<const float*>(src), lds,
                             s->n, s->p, s->st);
  else
    launch_copy_block<double>(static_cast<double*>(dst), ldd, static_cast<const double*>(src),
                              lds, s->n, s->p, s->st);
}

void density(ks_system* s, const void* X, int ld, double* rho) {
  const double scale = rho_scale(s);
  if (s->f32)
    launch_density<float>(static_cast<const float*>(X), ld, s->n, s->p, scale, rho, s->st);
  else
    launch_density<double>(static_cast<const double*>(X), ld, s->n, s->p, scale, rho, s->st);
}

void hamiltonian(ks_system* s, const void* X, int ldx, void* Y, int ldy, const double* veff,
                 double scale, Partials* pt, double* gram_part = nullptr) {
  if (s->f32)
    launch_hx<float>(static_cast<const float*>(X), ldx, static_cast<float*>(Y), ldy, veff,
                     s->grid, s->p, scale, pt, gram_part, s->st);
  else
    launch_hx<double>(static_cast<const double*>(X), ldx, static_cast<double*>(Y), ldy, veff,
                      s->grid, s->p, scale, pt, gram_part, s->st);
}

void q1_apply(ks_system* s, const void* X, void* G, void* BX, const double* veff, double scale,
              Partials* pt) {
  if (s->f32)
    launch_q1_apply<float>(static_cast<const float*>(X), static_cast<float*>(G),
                           static_cast<float*>(BX), veff, s->grid, s->p, scale, pt,
                           s->st);
  else
    launch_q1_apply<double>(static_cast<const double*>(X), static_cast<double*>(G),
                            static_cast<double*>(BX), veff, s->grid, s->p, scale, pt,
                            s->st);
}

void mass_solve(ks_system* s, const void* in, void* out) {
  const double* const tab[3] = {s->mtab[0], s->mtab[1], s->mtab[2]};
  if (s->f32)
    launch_mass_solve<float>(static_cast<const float*>(in), static_cast<float*>(out), s->p,
                             s->grid, tab, s->st);
  else
    launch_mass_solve<double>(static_cast<const double*>(in), static_cast<double*>(out), s->p,
                              s->grid, tab, s->st);
}

void gram(ks_system* s, const void* A, const void* B, int mask) {
  launch_gram(A, B, s->f32, s->p, s->n, s->p, mask, s->gram_part, s->gram_nchunks, s->st);
}

// Gram products of [A, B] (mask) reduced into out (and W = -(A^T B)^T with W); blocks wider
// than 64 columns run on 128 x 128 output tiles (bf16 products: 64-column sub-products).
// sym_ab: A^T B is symmetric (X^T B X, D^T B D); beyond 64 columns only its tiles I <= J
// are formed and mirrored
// KS_PREC_MIXED_BF16 takes A^T B (the calls marked bf16_ok: X^T G) on the bf16 matrix
// cores; every other product stays exact.  X^T G sets only the weights W = -(X^T G)^T of
// the direction D = G + X W.  The Cholesky factor of the retraction needs Y^T Y of the Y
// actually formed, so with float storage X^T D (X^T B D) is a product of the stored D,
// never X^T G + (X^T X) W: that sum misses the rounding of the stored D (about 1e-7 of
// each entry, enough to put X off the manifold by 1e-4 at p = 130) and, with bf16 error d
// in X^T G, the d + d^T that the true X^T D + D^T X carries.  Formed from D, the factor is
// exact; d then only rotates X within its span to first order, which leaves the energy
// unchanged.
void gram_reduced(ks_system* s, const void* A, const void* B, int mask, double* out,
                  double* W, bool sym_ab = false, bool bf16_ok = false) {
  if (s->pp > 64) {
    const int bf16_mask = s->bf16 && s->bf16_on && bf16_ok ? kGramAB : 0;
    launch_gram_full(A, B, s->f32, s->p, s->n, s->p, mask, s->gram_part, s->gsub, out, W,
                     s->st, sym_ab, bf16_mask);
    return;
  }
  gram(s, A, B, mask);
  launch_gram_reduce(s->gram_part, s->gram_nchunks, s->pp, mask, out, W, s->st);
}

// Pinned host mirror: CgState at 0 and LsState at 256 (the same offsets as on the device,
// so one copy brings both back), EvalOut at 512, ints at 768.
CgState* host_cg(ks_system* s) { return reinterpret_cast<CgState*>(s->host); }
LsState* host_ls(ks_system* s) {
  return reinterpret_cast<LsState*>(static_cast<char*>(s->host) + 256);
}
EvalOut* host_ev(ks_system* s) {
  return reinterpret_cast<EvalOut*>(static_cast<char*>(s->host) + 512);
}
int* host_int(ks_system* s) { return reinterpret_cast<int*>(static_cast<char*>(s->host) + 768); }

void harvest(ks_system* s);

// The CG and line-search records with one copy and one synchronisation (they are
// adjacent on the device, see layout()).
// QR trials of FP64 runs on the 7-point grid with p_p <= 32 take their BB sums without a
// pass over X_k (CombineArgs::bbr): the retraction sums ||s||^2 and <s, D_k>, the gradient
// pass <D_k, D_t>, and the summary combines them with R and X_t^T D_t.
bool bbr_ok(const ks_system* s) { return !s->q1 && !s->f32 && s->pp <= 32; }

int readback_cg_ls(ks_system* s) {
  const size_t bytes = reinterpret_cast<char*>(s->ls + 1) - reinterpret_cast<char*>(s->cg);
  hipError_t e = hipMemcpyAsync(s->host, s->cg, bytes, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e == hipSuccess && s->timers) harvest(s);
  return hip_check(s, e, "read-back");
}

void tbeg(ks_system* s, int ph);
void tend(ks_system* s, int ph);

// As readback_cg_ls for a trial from slot c, with the QR factor of the next trial queued
// behind the record copy before the host waits (for the copy only): the factor picks slot
// 1 - c or c on the device from the same record (QrFactor2dArgs::sel), so the GPU works
// while the host wakes up and decides.  (Queuing the retraction as well measured slower:
// it then starts with a dependent load of the record.)
int readback_cg_ls_ahead(ks_system* s, int c) {
  const int t = 1 - c;
  const int pp2 = s->pp * s->pp;
  const size_t bytes = reinterpret_cast<char*>(s->ls + 1) - reinterpret_cast<char*>(s->cg);
  // the summary kernel of the trial wrote the records into the host mirror itself
  hipError_t e = s->mirror_written
                     ? hipSuccess
                     : hipMemcpyAsync(s->host, s->cg, bytes, hipMemcpyDeviceToHost, s->st);
  s->mirror_written = false;
  if (e == hipSuccess && !s->ev_rb) e = hipEventCreateWithFlags(&s->ev_rb, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(s->ev_rb, s->st);
  if (e == hipSuccess) {
    QrFactor2dArgs a{};
    a.xx = s->q1 ? s->feg[t] + pp2 : s->gxg[t];
    a.gxd = s->gxd[t];
    a.p = s->p;
    a.pp = s->pp;
    a.tau_p = &s->ls->tau;
    a.A = s->A;
    a.B = s->B;
    a.status = &s->ls->error;
    a.sel = s->ls;
    a.xx_rej = s->q1 ? s->feg[c] + pp2 : s->gxg[c];
    a.gxd_rej = s->gxd[c];
    a.R = bbr_ok(s) ? s->Rq : nullptr;
    tbeg(s, KS_PH_SMALL);
    launch_qr_factor_next(a, s->st);
    tend(s, KS_PH_SMALL);
    e = hipEventSynchronize(s->ev_rb);
  }
  if (e == hipSuccess && s->timers) harvest(s);
  return hip_check(s, e, "read-back");
}

template <typename T>
int readback(ks_system* s, T* host, const T* dev) {
  hipError_t e = hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e == hipSuccess && s->timers) harvest(s);
  return hip_check(s, e, "read-back");
}

// ---- phase timers -----------------------------------------------------------------------

hipEvent_t take_event(ks_system* s) {
  if (s->ev_free.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = s->ev_free.back();
  s->ev_free.pop_back();
  return e;
}

void tbeg(ks_system* s, int ph) {
  if (!s->timers || !((s->timer_mask >> ph) & 1u)) return;
  ks_system::Pending p{take_event(s), take_event(s), ph};
  if (p.a) (void)hipEventRecord(p.a, s->st);
  s->ev_open[ph] = p;
}

// (Re)records the end event of an open phase.
void tmark(ks_system* s, int ph) {
  if (!s->timers || !s->ev_open[ph].b) return;
  (void)hipEventRecord(s->ev_open[ph].b, s->st);
}

// Closes an open phase whose end event has been recorded.
void tcommit(ks_system* s, int ph) {
  if (!s->timers) return;
  ks_system::Pending p = s->ev_open[ph];
  if (!p.a || !p.b) return;
  s->ev_pend.push_back(p);
  s->ev_open[ph] = ks_system::Pending{};
}

void tend(ks_system* s, int ph) {
  tmark(s, ph);
  tcommit(s, ph);
}

// Times a phase that is one combine launch by the launch's own dispatch (no event packets
// around it); false when the phase is not timed.  Close it with tcommit.
bool tbeg_launch(ks_system* s, int ph) {
  if (!s->timers || !((s->timer_mask >> ph) & 1u)) return false;
  ks_system::Pending p{take_event(s), take_event(s), ph};
  if (!p.a || !p.b) {
    if (p.a) s->ev_free.push_back(p.a);
    if (p.b) s->ev_free.push_back(p.b);
    return false;
  }
  set_launch_events(p.a, p.b);
  s->ev_open[ph] = p;
  return true;
}

// Accumulates every finished pair (called after stream synchronisations).
void harvest(ks_system* s) {
  std::vector<ks_system::Pending> keep;
  for (auto& p : s->ev_pend) {
    if (hipEventQuery(p.b) != hipSuccess) {
      keep.push_back(p);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      s->ph_ms[p.ph] += ms;
      s->ph_n[p.ph] += 1;
    }
    s->ev_free.push_back(p.a);
    s->ev_free.push_back(p.b);
  }
  s->ev_pend.swap(keep);
}

// ---- Hartree solve ---------------------------------------------------------------------
// CG iterations are queued in chunks; each kernel exits at once after convergence, and
// the host checks the device flag between chunks.
// Queues Hartree iterations on the current CG state until the device flag says done
// (checked between chunks).  With wait == false a PCG solve only queues its usual two
// iterations; whoever reads the CG state later must check the flag.
FdOps fd_ops(const ks_system* s) {
  return FdOps{s->fdS[0], s->fdS[1], s->fdS[2], s->fdL[0], s->fdL[1], s->fdL[2],
               s->fdM[0], s->fdM[1], s->fdM[2]};
}

int hartree_iterate(ks_system* s, double* x, int first_chunk, bool wait, int* iters,
                    double* relres) {
  const bool pcg = s->solver == KS_HARTREE_PCG_FD;
  const FdOps fd = fd_ops(s);
  int launched = 0;
  int chunk = first_chunk;
  CgState* hc = host_cg(s);
  for (;;) {
    const int c = std::min(chunk, s->hmaxit - launched);
    for (int i = 0; i < c; ++i) {
      if (pcg) launch_fd_apply(s->cg_r, s->cg_z, s->cg_q, fd, s->grid, s->cg, s->cgpart, s->st);
      launch_hartree_iter(x, s->cg_r, s->cg_z, s->cg_p[s->cg_par], s->cg_p[1 - s->cg_par],
                          s->cg_q, s->cg, s->grid, s->cgpart, pcg ? 1 : 0, s->st);
      s->cg_par = 1 - s->cg_par;
    }
    launched += c;
    tmark(s, KS_PH_HARTREE);
    int rc = launch_check(s, "hartree");
    if (rc) return rc;
    if (!wait) {
      tcommit(s, KS_PH_HARTREE);
      return KS_OK;
    }
    rc = readback(s, hc, s->cg);
    if (rc) return rc;
    if (hc->done || launched >= s->hmaxit) {
      tcommit(s, KS_PH_HARTREE);
      break;
    }
    chunk = pcg ? 2 : 16;
  }
  s->last_cg_iters = hc->it;
  s->cg_total += hc->it;
  if (iters) *iters = hc->it;
  if (relres) *relres = hc->bb > 0.0 ? std::sqrt(hc->rr / hc->bb) : 0.0;
  return KS_OK;
}

int hartree(ks_system* s, const double* rho, const double* x0, double* x, bool wait,
            int* iters, double* relres, bool fuse = false) {
  tbeg(s, KS_PH_HARTREE);
  s->cg_par = 0;
  if (s->solver == KS_HARTREE_PCG_FD) {
    // One preconditioned CG iteration from x0 with the exact step length of the exact
    // preconditioner: x = x0 + L^{-1}(b - L x0).  The CG start then measures the residual
    // of x and counts the iteration; only a solve that misses the tolerance continues with
    // PCG iterations (for a queued trial the caller does that: hartree_pending).
    // (a trial's retraction forms r = b - L x0 with its density: CombineArgs::resid)
    if (!s->resid_ready) launch_cg_residual(rho, x0, s->cg_r, s->cg_p[0], s->grid, s->cgpart, s->st);
    s->resid_ready = false;
    launch_fd_correct(s->cg_r, x0, x, s->cg_q, fd_ops(s), s->grid, s->st);
    if (fuse && s->pcg_extra == 0) {
      // a trial that queues no continuation: its exchange pass measures the residual and
      // the evaluation summary writes the CG start (one pass and one launch fewer)
      s->fuse_cg = true;
      tmark(s, KS_PH_HARTREE);
      tcommit(s, KS_PH_HARTREE);
      return launch_check(s, "hartree");
    }
    launch_hartree_init(rho, x, nullptr, s->cg_r, s->cg_p[0], s->cg, s->htol, s->hmaxit, 1,
                        s->grid, s->cgpart, s->st);
    // pcg_extra: a run whose exact steps miss the tolerance (large grids: eps cond(L) above
    // it) queues one more PCG iteration with each solve, so that its trials do not come back
    // pending (the iteration exits at once when the solve has converged)
    return hartree_iterate(s, x, s->pcg_extra, wait, iters, relres);
  }
  launch_hartree_init(rho, x0, x, s->cg_r, s->cg_p[0], s->cg, s->htol, s->hmaxit, 0, s->grid,
                      s->cgpart, s->st);
  // first chunk sized by the previous solve (warm starts need similar counts)
  const int chunk = s->last_cg_iters > 0 ? s->last_cg_iters + 2 : 32;
  return hartree_iterate(s, x, chunk, wait, iters, relres);
}

// ---- one energy/gradient evaluation on internal slot `idx` -------------------------
// rho of X[idx] is either ready (fused into the retraction) or computed here.  With
// bb_ref >= 0 the gradient epilogue also forms the BB sums against slot bb_ref.
// warm: slot whose V_H starts the CG.  Writes G, D, gram blocks, sums, ev of the slot.
int evaluate_tail(ks_system* s, int idx, int bb_ref, bool want_gxd, bool want_gg,
                  const LsParams* judge = nullptr);
int evaluate_tail_q1(ks_system* s, int idx, int bb_ref, bool want_gxd, bool want_gg,
                     const LsParams* judge);

// With judge, the summary kernel also runs the line-search judgement of the trial.
int evaluate(ks_system* s, int idx, bool rho_ready, int bb_ref, int warm, bool want_gxd,
             bool want_gg, bool wait_hartree = true, const LsParams* judge = nullptr) {
  const double scale = s->f / s->grid.dV;
  (void)scale;
  const void* Xs = s->X[idx];
  if (!rho_ready) {
    tbeg(s, KS_PH_DENSITY);
    density(s, Xs, s->p, s->rho);
    tend(s, KS_PH_DENSITY);
  }
  int rc = launch_check(s, "density");
  if (rc) return rc;
  if (s->use_h) {
    rc = hartree(s, s->rho, s->vh[warm], s->vh[idx], wait_hartree, nullptr, nullptr,
                 judge != nullptr);
    if (rc) return rc;
  }
  return evaluate_tail(s, idx, bb_ref, want_gxd, want_gg, judge);
}

// Everything after the Hartree solve: exchange, Hamiltonian, Gram blocks, gradient,
// reductions and the evaluation summary of slot idx.
int evaluate_tail(ks_system* s, int idx, int bb_ref, bool want_gxd, bool want_gg,
                  const LsParams* judge) {
  if (s->q1) return evaluate_tail_q1(s, idx, bb_ref, want_gxd, want_gg, judge);
  const void* Xs = s->X[idx];
  Partials pt{s->spart, kPartStride};
  const bool fuse_cg = s->fuse_cg;
  s->fuse_cg = false;
  s->cg_fused = fuse_cg;
  tbeg(s, KS_PH_XC);
  launch_xc(s->rho, s->vh[idx], s->vext, s->veff[idx], s->grid, s->use_h, s->use_x,
            s->use_h && !fuse_cg ? s->cg : nullptr, pt, s->st, fuse_cg, s->vbc);
  tend(s, KS_PH_XC);
  // Gram blocks of [X, G]: X^T X and X^T G (and G^T G for the Cayley system); at p = 32
  // without G^T G the Hamiltonian pass forms them itself
  const bool hxg = !want_gg && hx_fuses_gram(s->p);
  tbeg(s, KS_PH_HAMILTONIAN);
  hamiltonian(s, Xs, s->p, s->G[idx], s->p, s->veff[idx], 2.0 * s->f, &pt,
              hxg ? s->gram_part : nullptr);
  tend(s, KS_PH_HAMILTONIAN);
  const int mask1 = kGramAA | kGramAB | (want_gg ? kGramBB : 0);
  if (hxg) {
    tbeg(s, KS_PH_SMALL);
    launch_gram_reduce(s->gram_part, hx_gram_blocks(s->n), s->pp, mask1, s->gxg[idx], s->W,
                       s->st);
    tend(s, KS_PH_SMALL);
  } else {
    tbeg(s, KS_PH_GRAM);
    // bf16 only for the QR retraction: the Cayley system takes X^T G as it is
    gram_reduced(s, Xs, s->G[idx], mask1, s->gxg[idx], s->W, false, !want_gg);
    tend(s, KS_PH_GRAM);
  }
  // D = G - X (G^T X) with ||D||^2, the BB sums and (QR) the Gram blocks X^T D, D^T D:
  // up to 32 columns they come out of the same kernel, wider blocks take a Gram launch
  const bool fused = want_gxd && s->pp <= 32;
  // a QR trial (want_gxd) judged here: BB sums without X_k
  const bool bbr = bb_ref >= 0 && want_gxd && judge != nullptr && bbr_ok(s);
  CombineArgs ca{};
  ca.bbr = bbr;
  ca.X = Xs;
  ca.A = s->W;
  ca.C0 = s->G[idx];
  ca.out = s->D[idx];
  ca.Xk = bb_ref >= 0 ? s->X[bb_ref] : Xs;
  ca.Dk = bb_ref >= 0 ? s->D[bb_ref] : s->D[idx];
  ca.pt = pt;
  ca.gram_part = fused ? s->gram_part : nullptr;
  ca.f32 = s->f32;
  ca.mc = s->mc;
  ca.ld = s->p;
  ca.n = s->n;
  ca.p = s->p;
  // one launch up to 64 columns: timed by its own dispatch
  const bool exact = s->pp <= 64 && tbeg_launch(s, KS_PH_GRADIENT);
  if (!exact) tbeg(s, KS_PH_GRADIENT);
  launch_combine(ca, s->st);
  if (exact) {
    set_launch_events(nullptr, nullptr);
    tcommit(s, KS_PH_GRADIENT);
  } else {
    tend(s, KS_PH_GRADIENT);
  }
  const int mask2 = kGramAB | kGramBB;
  if (want_gxd && !fused) {
    tbeg(s, KS_PH_GRAM);
    if (s->pp > 64 && !s->f32) {
      // X^T D = X^T G + (X^T X) W from the blocks already reduced; only D^T D is a pass
      const int pp2 = s->pp * s->pp;
      gram_reduced(s, Xs, s->D[idx], kGramBB, s->gxd[idx], nullptr);
      launch_small_gemm_add(s->gxg[idx] + pp2, s->gxg[idx], s->W, s->gxd[idx] + pp2, s->p,
                            s->pp, s->st);
    } else {
      gram_reduced(s, Xs, s->D[idx], mask2, s->gxd[idx], nullptr);
    }
    tend(s, KS_PH_GRAM);
  }
  // the error of the bf16 X^T G, from the exact X^T D just formed
  const bool defect = want_gxd && !fused && s->bf16 && s->bf16_on && s->pp > 64;
  if (defect) {
    const int pp2 = s->pp * s->pp;
    launch_bf16_defect(s->gxg[idx] + pp2, s->gxd[idx] + pp2, s->gxg[idx], s->W, s->p, s->pp,
                       s->spart + (size_t)SL_DEFECT * kPartStride, s->st);
  }
  tbeg(s, KS_PH_SMALL);
  if (fused) {
    // after the gradient pass of a QR trial (bbr), X^T D = X^T G + (X^T X) W comes from the
    // reduced blocks; that pass formed only D^T D
    const int pp2 = s->pp * s->pp;
    launch_gram_reduce(s->gram_part, combine_blocks(s->n), s->pp, mask2, s->gxd[idx], nullptr,
                       s->st, bbr ? s->gxg[idx] + pp2 : nullptr, bbr ? s->gxg[idx] : nullptr,
                       bbr ? s->W : nullptr);
  }
  int nblk[kMaxScalarSlots] = {};
  nblk[SL_KIN] = hxg ? hx_gram_blocks(s->n) : hx_blocks(s->n, s->p);
  nblk[SL_EH] = nblk[SL_EX] = nblk[SL_EXT] = nblk[SL_TF] = scalar_blocks(s->n);
  nblk[SL_DD] = nblk[SL_SS] = nblk[SL_SY] = nblk[SL_YY] = combine_partial_blocks(s->n, s->p);
  nblk[SL_DEFECT] = defect ? bf16_defect_blocks(s->p) : 0;
  nblk[SL_CGRR] = nblk[SL_CGBB] = fuse_cg ? scalar_blocks(s->n) : 0;
  nblk[SL_EBC] = s->vbc ? scalar_blocks(s->n) : 0;
  // a judged trial also writes its CG and line-search records into the host mirror
  const bool mirror = judge != nullptr && s->host_dev != nullptr;
  launch_finish_eval(s->spart, kPartStride, nblk, s->sums[idx], s->gxg[idx], s->p, s->pp, s->f,
                     s->grid.dV, s->enuc, s->use_h ? s->cg : nullptr, s->ev[idx],
                     judge ? s->ls : nullptr, judge, s->st, fuse_cg ? s->cg : nullptr, s->htol,
                     s->hmaxit, s->ebc, bbr ? s->Rq : nullptr,
                     bbr ? s->gxd[idx] + s->pp * s->pp : nullptr,
                     mirror ? s->host_dev : nullptr, s->cg,
                     (int)(reinterpret_cast<char*>(s->ls + 1) - reinterpret_cast<char*>(s->cg)));
  s->mirror_written = mirror;
  tend(s, KS_PH_SMALL);
  return launch_check(s, "evaluate");
}

// The Cayley system in the B metric (Section 3 with Y = B^{1/2} X): with U = [B^{-1} G, X],
// V = [X, -B^{-1} G] and the B inner product, V^T B U needs [X^T B X, X^T G, G^T B^{-1} G]
// where the Euclidean form has [X^T X, X^T G, G^T G]; the same factor kernel then gives
// X+ = X A + (B^{-1} G) B.  Called after B^{-1} G, X^T G and X^T B X of slot idx exist.
void wy_blocks_q1(ks_system* s, int idx) {
  const int pp2 = s->pp * s->pp;
  launch_copy_vec(s->wyg[idx], s->feg[idx] + pp2, (size_t)pp2, s->st);
  launch_copy_vec(s->wyg[idx] + pp2, s->gxg[idx] + pp2, (size_t)pp2, s->st);
  // G^T (B^{-1} G) lands in product slot 1 of wyg + pp2, i.e. slot 2 of wyg
  gram_reduced(s, s->G[idx], s->Gt[idx], kGramAB, s->wyg[idx] + pp2, nullptr, true);
}

// The finite-element evaluation in the B metric: G = E_X, BX = B X, Gt = B^{-1} G,
// M = G^T X, D = grad E = Gt - X M and BD = B D = G - BX M (same weights), the Gram blocks
// X^T B X (orthonormality and the Cholesky of the retraction), X^T BD and D^T BD (with
// want_gxd), ||D||_B^2 and the BB sums of the B metric against slot bb_ref.
int evaluate_tail_q1(ks_system* s, int idx, int bb_ref, bool want_gxd, bool want_gg,
                     const LsParams* judge) {
  const void* Xs = s->X[idx];
  const int pp2 = s->pp * s->pp;
  Partials pt{s->spart, kPartStride};
  const bool fuse_cg = s->fuse_cg;
  s->fuse_cg = false;
  s->cg_fused = fuse_cg;
  tbeg(s, KS_PH_XC);
  launch_xc(s->rho, s->vh[idx], s->vext, s->veff[idx], s->grid, s->use_h, s->use_x,
            s->use_h && !fuse_cg ? s->cg : nullptr, pt, s->st, fuse_cg, s->vbc);
  tend(s, KS_PH_XC);
  tbeg(s, KS_PH_HAMILTONIAN);
  q1_apply(s, Xs, s->G[idx], s->BX[idx], s->veff[idx], 2.0 * s->f, &pt);
  tend(s, KS_PH_HAMILTONIAN);
  // B^{-1} G is part of the B-metric gradient
  tbeg(s, KS_PH_GRADIENT);
  mass_solve(s, s->G[idx], s->Gt[idx]);
  tend(s, KS_PH_GRADIENT);
  tbeg(s, KS_PH_GRAM);
  gram_reduced(s, Xs, s->G[idx], kGramAB, s->gxg[idx], s->W, false, !want_gg);
  gram_reduced(s, Xs, s->BX[idx], kGramAB, s->feg[idx], nullptr, true);
  if (want_gg) wy_blocks_q1(s, idx);
  tend(s, KS_PH_GRAM);
  Q1GradArgs ga{};
  ga.Gt = s->Gt[idx];
  ga.X = Xs;
  ga.G = s->G[idx];
  ga.BX = s->BX[idx];
  ga.W = s->W;
  ga.D = s->D[idx];
  ga.BD = s->BD[idx];
  if (bb_ref >= 0) {
    ga.Xc = s->X[bb_ref];
    ga.BXc = s->BX[bb_ref];
    ga.Dc = s->D[bb_ref];
    ga.BDc = s->BD[bb_ref];
  }
  ga.pt = pt;
  ga.n = s->n;
  ga.p = s->p;
  ga.pp = s->pp;
  ga.f32 = s->f32;
  tbeg(s, KS_PH_GRADIENT);
  launch_q1_grad(ga, s->st);
  tend(s, KS_PH_GRADIENT);
  if (want_gxd) {
    tbeg(s, KS_PH_GRAM);
    if (s->pp > 64 && !s->f32) {
      // X^T BD = X^T G + (X^T B X) W from the blocks already reduced
      launch_small_gemm_add(s->gxg[idx] + pp2, s->feg[idx] + pp2, s->W, s->gxd[idx] + pp2,
                            s->p, s->pp, s->st);
    } else {
      gram_reduced(s, Xs, s->BD[idx], kGramAB, s->gxd[idx], nullptr);
    }
    // D^T BD lands in product slot 2 of gxd
    gram_reduced(s, s->D[idx], s->BD[idx], kGramAB, s->gxd[idx] + pp2, nullptr, true);
    tend(s, KS_PH_GRAM);
  }
  // the error of the bf16 X^T G, from the exact X^T B D and X^T B X
  const bool defect = want_gxd && s->bf16 && s->bf16_on && s->pp > 64;
  if (defect)
    launch_bf16_defect(s->gxg[idx] + pp2, s->gxd[idx] + pp2, s->feg[idx] + pp2, s->W, s->p,
                       s->pp, s->spart + (size_t)SL_DEFECT * kPartStride, s->st);
  tbeg(s, KS_PH_SMALL);
  int nblk[kMaxScalarSlots] = {};
  nblk[SL_KIN] = q1_apply_blocks(s->grid, s->p);
  nblk[SL_EH] = nblk[SL_EX] = nblk[SL_EXT] = nblk[SL_TF] = scalar_blocks(s->n);
  nblk[SL_DD] = nblk[SL_SS] = nblk[SL_SY] = nblk[SL_YY] = q1_grad_blocks(s->n, s->p);
  nblk[SL_DEFECT] = defect ? bf16_defect_blocks(s->p) : 0;
  nblk[SL_CGRR] = nblk[SL_CGBB] = fuse_cg ? scalar_blocks(s->n) : 0;
  nblk[SL_EBC] = s->vbc ? scalar_blocks(s->n) : 0;
  launch_finish_eval(s->spart, kPartStride, nblk, s->sums[idx], s->feg[idx] + pp2, s->p, s->pp,
                     s->f, s->grid.dV, s->enuc, s->use_h ? s->cg : nullptr, s->ev[idx],
                     judge ? s->ls : nullptr, judge, s->st, fuse_cg ? s->cg : nullptr, s->htol,
                     s->hmaxit, s->ebc);
  tend(s, KS_PH_SMALL);
  return launch_check(s, "evaluate");
}

// Monopole boundary values of the Hartree problem (KS_HBC_MONOPOLE): V_bc is the solution
// of the interior system whose right-hand side carries the boundary values Q/|r_b - c|
// (Q = f p electrons, c the nuclear-charge centre, or the box centre without nuclei),
// formed with the system's own Hartree solver; then the energy constant -(1/2) Q V_bc(c).
int setup_monopole(ks_system* s) {
  double c[3] = {0.0, 0.0, 0.0}, zs = 0.0;
  for (size_t a = 0; a < s->Z.size(); ++a) {
    zs += s->Z[a];
    for (int d = 0; d < 3; ++d) c[d] += s->Z[a] * s->R[3 * a + d];
  }
  const int dims[3] = {s->grid.nx, s->grid.ny, s->grid.nz};
  for (int d = 0; d < 3; ++d)
    c[d] = zs != 0.0 ? c[d] / zs : s->grid.lo[d] + 0.5 * (dims[d] + 1) * s->grid.h;
  const double Q = s->f * s->p;
  launch_bc_rhs(s->rho, s->grid, Q, c[0], c[1], c[2], s->st);
  int it = 0;
  double rr = 0.0;
  int rc = hartree(s, s->rho, nullptr, s->vbc, true, &it, &rr);
  if (rc) return rc;
  const CgState* hc = host_cg(s);
  if (rr > s->htol && !(hc->stall >= kCgStall && rr <= kCgFloor * s->htol))
    return fail(s, KS_E_NOT_CONVERGED, "monopole boundary potential: Hartree solve did not converge");
  launch_bc_point(s->vbc, s->grid, Q, c[0], c[1], c[2], s->ebc, s->st);
  return launch_check(s, "monopole boundary");
}

// Cholesky QR of slot idx in place (Alg. 2): X <- X R^{-1} with X^T X = R^T R (finite
// differences) or X^T B X = R^T R (finite elements), the Gram block formed in FP64 from the
// stored X.  Uses slot 1 - idx as scratch.
int orthonormalize_slot(ks_system* s, int idx) {
  const int o = 1 - idx;
  const int pp2 = s->pp * s->pp;
  const double* xx = nullptr;
  if (s->q1) {
    q1_apply(s, s->X[idx], nullptr, s->BX[idx], nullptr, 1.0, nullptr);
    gram_reduced(s, s->X[idx], s->BX[idx], kGramAB, s->feg[idx], nullptr, true);
    xx = s->feg[idx] + pp2;
  } else {
    gram_reduced(s, s->X[idx], s->X[idx], kGramAA, s->gxg[idx], nullptr);
    xx = s->gxg[idx];
  }
  // tau = 0: the factor reduces to the Cholesky of the Gram block; X^T D and D^T D are not
  // used
  launch_fill(s->gxd[idx], 0.0, 3 * (size_t)pp2, s->st);
  launch_set_scalar(s->tau_user, 0.0, s->st);
  int* hstat = host_int(s);
  hstat[0] = 0;
  int rc = hip_check(s, hipMemcpyAsync(s->status, hstat, sizeof(int), hipMemcpyHostToDevice,
                                       s->st), "status upload");
  if (rc) return rc;
  launch_qr_factor(xx, s->gxd[idx], s->p, s->pp, s->tau_user, s->A, s->B, s->work, s->status,
                   s->st);
  CombineArgs ca{};
  ca.X = s->X[idx];
  ca.A = s->A;
  ca.ld = s->p;
  ca.n = s->n;
  ca.p = s->p;
  ca.f32 = s->f32;
  ca.mc = s->mc;
  ca.out = s->X[o];
  launch_combine(ca, s->st);
  copy_block(s, s->X[idx], s->p, s->X[o], s->p);
  rc = launch_check(s, "B-orthonormalisation");
  if (rc) return rc;
  rc = readback(s, hstat, s->status);
  if (rc) return rc;
  if (hstat[0] != 0)
    return fail(s, KS_E_NOT_SPD, s->q1 ? "block is rank deficient in the B metric"
                                       : "block is rank deficient");
  return KS_OK;
}

void to_energy(const EvalOut& e, ks_energy* out) {
  out->total = e.total;
  out->kinetic = e.kinetic;
  out->external = e.external;
  out->hartree = e.hartree;
  out->xc = e.xc;
  out->nuclear = e.nuclear;
  out->grad_norm = std::sqrt(std::max(e.g2, 0.0));
  out->orth_error = std::sqrt(std::max(e.orth2, 0.0));
  out->hartree_iters = e.cg_iters;
  out->hartree_relres = e.cg_relres;
}

LsParams to_params(const ks_opt_params& o) {
  LsParams p{};
  p.tau0 = o.tau0;
  p.rho1 = o.rho1;
  p.delta = o.delta;
  p.eta = o.eta;
  p.eps_g = o.eps_g;
  p.tau_min = o.tau_min;
  p.tau_max = o.tau_max;
  p.reorth_tol = o.reorth_tol;
  p.stagnation_tol = o.stagnation_tol;
  p.energy_target = o.energy_target;
  p.max_iter = o.max_iter;
  p.bb_rule = o.bb_rule;
  p.h_max = o.h_max;
  p.retraction = o.retraction;
  return p;
}

}  // namespace

namespace {

// One trial step of Alg. 3 from slot c into slot t = 1 - c: the retraction factor and
// combine (with the density of the trial point), the evaluation and the line-search
// judgement, all on the device.  Nothing in it waits for the host, so it can be captured
// into a graph; with the plain CG Hartree solver the evaluation waits for convergence.
// queued: the QR factor of this trial was already queued by readback_cg_ls_ahead.
// Fields of a retraction combine that also forms r = 4 pi rhs_scale rho - L x0.
void set_resid(CombineArgs& ca, const ks_system* s, const double* x0) {
  ca.resid = s->cg_r;
  ca.resid_x0 = x0;
  ca.gnx = s->grid.nx;
  ca.gny = s->grid.ny;
  ca.gnz = s->grid.nz;
  ca.inv_h2 = s->grid.inv_h2;
  ca.rhs_scale = s->grid.rhs_scale;
}

int enqueue_trial(ks_system* s, int c, bool qr, const LsParams& lp, const ks_opt_params& prm,
                  bool queued = false) {
  const int t = 1 - c;
  CombineArgs ca{};
  ca.X = s->X[c];
  ca.A = s->A;
  ca.B = s->B;
  ca.out = s->X[t];
  ca.rho = s->rho;
  ca.rho_scale = rho_scale(s);
  ca.f32 = s->f32;
  ca.mc = s->mc;
  ca.ld = s->p;
  ca.n = s->n;
  ca.p = s->p;
  if (qr) {
    if (!queued) {
      tbeg(s, KS_PH_SMALL);
      launch_qr_factor(s->q1 ? s->feg[c] + s->pp * s->pp : s->gxg[c], s->gxd[c], s->p, s->pp,
                       &s->ls->tau, s->A, s->B, s->work, &s->ls->error, s->st,
                       bbr_ok(s) ? s->Rq : nullptr);
      tend(s, KS_PH_SMALL);
    }
    ca.Y = s->D[c];
    ca.upper = true;
    ca.bbr = bbr_ok(s);
    ca.pt = Partials{s->spart, kPartStride};
  } else {
    tbeg(s, KS_PH_SMALL);
    launch_wy_factor(s->q1 ? s->wyg[c] : s->gxg[c], s->p, s->pp, &s->ls->tau, prm.reorth_tol,
                     s->A, s->B, s->work, &s->ls->error, s->reorth_count, s->st);
    tend(s, KS_PH_SMALL);
    ca.Y = s->q1 ? s->Gt[c] : s->G[c];
  }
  const bool pcg = s->solver == KS_HARTREE_PCG_FD;
  if (pcg && s->use_h && !s->q1) {
    // the first residual of the trial's Hartree solve, from its warm start V_H(c)
    set_resid(ca, s, s->vh[c]);
    s->resid_ready = true;
  }
  tbeg(s, KS_PH_RETRACT);
  launch_combine(ca, s->st);
  tend(s, KS_PH_RETRACT);
  int rc = evaluate(s, t, true, c, c, qr, !qr, !pcg, &lp);
  s->resid_ready = false;  // consumed by that solve (or dropped with an error)
  if (rc) return rc;
  return launch_check(s, "line search");
}

void drop_graphs(ks_system* s) {
  for (auto& g : s->gx) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

// Records enqueue_trial(c) on the capture stream into s->gx[c].  A failed capture leaves
// gx[c] empty and the trial runs eagerly.
int capture_trial(ks_system* s, int c, bool qr, const LsParams& lp, const ks_opt_params& prm) {
  hipStream_t orig = s->st;
  s->st = s->cap_st;
  hipError_t e = hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal);
  int rc = KS_OK;
  if (e == hipSuccess) rc = enqueue_trial(s, c, qr, lp, prm);
  hipGraph_t g = nullptr;
  hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(s->st, &g) : e;
  s->st = orig;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e2 == hipSuccess && g) {
    if (hipGraphInstantiate(&s->gx[c], g, nullptr, nullptr, 0) != hipSuccess) s->gx[c] = nullptr;
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();  // a refused capture is not an error of the run
  return KS_OK;
}

}  // namespace

namespace {

// Validation, start block, first evaluation and line-search initialisation.
int run_begin(ks_system* s, void* X_inout, const ks_opt_params* o, MinRun* m) {
  if (!s || !X_inout) return fail(s, KS_E_INVAL, "null argument");
  m->t0 = std::chrono::steady_clock::now();
  if (o) m->prm = *o;
  else ks_default_params(&m->prm);
  const ks_opt_params& prm = m->prm;
  if (prm.retraction != KS_QR && prm.retraction != KS_WY)
    return fail(s, KS_E_INVAL, "unknown retraction");
  if (!(prm.delta > 0.0 && prm.delta < 1.0) || !(prm.tau0 > 0.0) || prm.h_max < 0)
    return fail(s, KS_E_INVAL, "bad line-search parameters");
  if (prm.reorth_every < 0 || std::isnan(prm.energy_target))
    return fail(s, KS_E_INVAL, "reorth_every must be >= 0 and energy_target not NaN");
  m->lp = to_params(prm);
  m->qr = prm.retraction == KS_QR;
  m->X_inout = X_inout;
  m->active = true;
  m->queued = false;
  m->records = false;
  m->reorths = 0;
  s->bf16_on = true;
  s->cg_total = 0;
  // each run starts from the same solver settings: its first trial queues one PCG
  // iteration after the exact step, and whether that iteration ran decides the rest
  s->pcg_extra = 1;
  s->pcg_probe = true;
  drop_graphs(s);  // graphs hold the parameters of the run that captured them
  int c = s->cur;
  m->c = c;
  copy_block(s, s->X[c], s->p, X_inout, s->ld);
  if (s->q1) {
    // the start block needs full column rank only: make it B-orthonormal first
    int rb = orthonormalize_slot(s, c);
    if (rb) return rb;
  }
  launch_ls_reset(s->ls, s->st);
  int* hint = host_int(s);
  hint[1] = 0;
  int rc = hip_check(s, hipMemcpyAsync(s->reorth_count, &hint[1], sizeof(int),
                                       hipMemcpyHostToDevice, s->st), "counter upload");
  if (rc) return rc;
  // the first Hartree solve starts from V_H = 0, so a run depends only on X_inout
  launch_fill(s->vh[c], 0.0, s->n, s->st);
  rc = evaluate(s, c, false, -1, c, m->qr, !m->qr);
  if (rc) return rc;
  launch_ls_init(s->ev[c], s->ls, m->lp, s->st);
  return readback(s, host_ls(s), s->ls);
}

// After a trial's CG and line-search records are in the host mirror: finish a Hartree
// solve that had not converged (rare), then accept or keep the slot.
int run_after_trial(ks_system* s, MinRun* m, bool cg_read) {
  LsState* hl = host_ls(s);
  const int c = m->c, t = 1 - c;
  if (cg_read && !hl->hartree_pending) s->cg_total += host_cg(s)->it;
  if (hl->hartree_pending) {
    // the queued PCG iteration did not reach the tolerance; finish the solve and evaluate
    // the trial again, and queue one more iteration with the solves of later trials
    s->pcg_probe = false;
    if (!s->pcg_extra) {
      s->pcg_extra = 1;
      drop_graphs(s);
    }
    // a residual measured in the exchange pass left only its norm: the CG start is formed
    // again from the trial's V_H; then PCG iterations until the solve converges
    if (s->cg_fused) {
      s->cg_par = 0;
      launch_hartree_init(s->rho, s->vh[t], nullptr, s->cg_r, s->cg_p[0], s->cg, s->htol,
                          s->hmaxit, 1, s->grid, s->cgpart, s->st);
    }
    int rc = hartree_iterate(s, s->vh[t], 2, true, nullptr, nullptr);
    if (rc) return rc;
    rc = evaluate_tail(s, t, c, m->qr, !m->qr, &m->lp);
    if (rc) return rc;
    rc = readback(s, hl, s->ls);
    if (rc) return rc;
    if (hl->hartree_pending) return fail(s, KS_E_NOT_CONVERGED, "Hartree solve did not converge");
  } else if (cg_read && s->pcg_probe) {
    // the first trial of the run: keep the queued iteration only if it had to run (the
    // exact step counts as iteration 1; a converged solve skips the rest)
    s->pcg_probe = false;
    const int need = host_cg(s)->it > 1 ? 1 : 0;
    if (need != s->pcg_extra) {
      s->pcg_extra = need;
      drop_graphs(s);
    }
  }
  if (hl->bf16_off) s->bf16_on = false;  // exact X^T G for the rest of the run
  if (hl->error) return KS_OK;
  if (hl->accepted) {
    m->c = t;
    s->cur = t;
  }
  return KS_OK;
}

// reorth_every: the accepted iterate is re-orthonormalised in FP64 (Cholesky QR of its
// stored values), evaluated again, and the nonmonotone reference restarts there.
int run_reorth(ks_system* s, MinRun* m) {
  const int c = m->c;
  int rc = orthonormalize_slot(s, c);
  if (rc) return rc;
  rc = evaluate(s, c, false, -1, c, m->qr, !m->qr);
  if (rc) return rc;
  launch_ls_restart(s->ev[c], s->ls, m->lp, s->st);
  m->reorths += 1;
  m->queued = false;
  return readback(s, host_ls(s), s->ls);
}

// One trial step of Alg. 3 from the current slot, judged on the device, then accepted or
// rejected on the host side of the run (and, every reorth_every accepted iterations, the
// re-orthonormalisation of the new iterate).
int run_trial(ks_system* s, MinRun* m) {
  LsState* hl = host_ls(s);
  const int c = m->c;
  const bool pcg = s->solver == KS_HARTREE_PCG_FD;
  // graph replay from the second trial on (the first runs eagerly and initialises the
  // launch attributes); the CG solver's host-side convergence checks cannot be captured
  const bool replay = s->graphs && s->cap_st && (pcg || !s->use_h) && !s->timers &&
                      hl->nfe > 1;
  int rc = KS_OK;
  if (replay && !s->gx[c]) {
    rc = capture_trial(s, c, m->qr, m->lp, m->prm);
    if (rc) return rc;
  }
  if (replay && s->gx[c]) {
    rc = hip_check(s, hipGraphLaunch(s->gx[c], s->st), "graph launch");
  } else {
    rc = enqueue_trial(s, c, m->qr, m->lp, m->prm, m->queued);
  }
  m->queued = false;
  if (rc) return rc;
  const bool cg_read = pcg && s->use_h;
  // eager QR runs queue the next trial's factor behind the record copy
  const bool ahead = cg_read && m->qr && s->p <= 64 && !s->graphs;
  if (ahead) rc = readback_cg_ls_ahead(s, c);
  else rc = cg_read ? readback_cg_ls(s) : readback(s, hl, s->ls);
  if (rc) return rc;
  // a pending Hartree solve re-evaluates the trial first; the queued factor then returned
  // without writing, and the next trial queues its own
  m->queued = ahead && !hl->hartree_pending;
  rc = run_after_trial(s, m, cg_read);
  if (rc) return rc;
  if (m->prm.reorth_every > 0 && hl->accepted && hl->stop == KS_STOP_NONE && !hl->error &&
      hl->k % m->prm.reorth_every == 0)
    return run_reorth(s, m);
  return KS_OK;
}

// Copies the result out (into X_out when given, else the run's X_inout) and fills the
// statistics.
int run_end(ks_system* s, MinRun* m, ks_result* r, void* X_out = nullptr) {
  LsState* hl = host_ls(s);
  int* hint = host_int(s);
  drop_graphs(s);
  m->active = false;
  m->queued = false;
  s->bf16_on = true;
  if (!X_out) X_out = m->X_inout;
  if (X_out) copy_block(s, X_out, s->ld, s->X[m->c], s->p);
  int rc = launch_check(s, "minimize");
  if (rc) return rc;
  EvalOut* he = host_ev(s);
  rc = readback(s, he, s->ev[m->c]);
  if (rc) return rc;
  rc = readback(s, &hint[1], s->reorth_count);
  if (rc) return rc;
  if (r) {
    std::memset(r, 0, sizeof(*r));
    r->iters = hl->k;
    r->nfe = hl->nfe;
    r->backtracks = hl->backtracks;
    r->ls_fail = hl->ls_fail;
    r->reorths = hint[1] + m->reorths;
    r->stop_reason = hl->stop;
    r->energy = he->total;
    r->grad_norm = std::sqrt(std::max(he->g2, 0.0));
    to_energy(*he, &r->terms);
    r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - m->t0).count();
    r->hartree_iters_total = s->cg_total;
  }
  if (hl->error) return fail(s, hl->error, ks_status_string(hl->error));
  if (hl->stop == KS_STOP_MAXIT) return fail(s, KS_E_NOT_CONVERGED, "max_iter reached");
  return KS_OK;
}

}  // namespace

namespace {

// ---- batched runs ----------------------------------------------------------------------
// Systems that share the trial's launch shapes (finite differences, PCG with the exact
// preconditioner, QR retraction, p_p <= 32, one storage precision) run their trials in
// lockstep: each kernel of a trial is one launch for all of them, every system reading
// its own argument record.  The records hold exactly the arguments the lone trial passes,
// and each system keeps its lone block counts, so every result equals its lone run.

static_assert(sizeof(QrFactor2dArgs) <= kRecSlot && sizeof(CombineArgs) <= kRecSlot &&
                  sizeof(InitArgs) <= kRecSlot && sizeof(FinInitArgs) <= kRecSlot &&
                  sizeof(FdPlaneArgs) <= kRecSlot && sizeof(FdZArgs) <= kRecSlot &&
                  sizeof(FinRzArgs) <= kRecSlot && sizeof(DirArgs) <= kRecSlot &&
                  sizeof(FinDirArgs) <= kRecSlot && sizeof(UpdArgs) <= kRecSlot &&
                  sizeof(FinUpdArgs) <= kRecSlot && sizeof(XcArgs) <= kRecSlot &&
                  sizeof(HxArgs<double>) <= kRecSlot && sizeof(GramArgs<double>) <= kRecSlot &&
                  sizeof(GramReduceArgs) <= kRecSlot && sizeof(FinishEvalArgs) <= kRecSlot,
              "argument records must fit their slots");

bool batchable(const ks_system* s, const MinRun& m) {
  return !s->q1 && s->solver == KS_HARTREE_PCG_FD && s->use_h && m.qr && s->pp <= 32 &&
         !s->timers && m.prm.reorth_every == 0;
}

template <typename A>
const A* rec_at(const ks_system* s, int c, int r) {
  return reinterpret_cast<const A*>(s->rec + ((size_t)c * R_COUNT + r) * kRecSlot);
}

template <typename A>
void put_rec(std::vector<char>& buf, int c, int r, const A& a) {
  std::memcpy(buf.data() + ((size_t)c * R_COUNT + r) * kRecSlot, &a, sizeof(A));
}

template <typename T>
void fill_typed(ks_system* s, std::vector<char>& buf, int c) {
  const int t = 1 - c;
  Partials pt{s->spart, kPartStride};
  // retraction: X_t = X_c A + D_c B with the density (QR weights)
  double* rq = bbr_ok(s) ? s->Rq : nullptr;
  put_rec(buf, c, R_QR, QrFactor2dArgs{s->gxg[c], s->gxd[c], s->p, s->pp, &s->ls->tau, s->A,
                                        s->B, &s->ls->error, nullptr, nullptr, nullptr, rq});
  // the factor of the trial after a trial from slot c, queued before the host reads the
  // record: slot t when that trial is accepted, slot c otherwise (QrFactor2dArgs::sel)
  put_rec(buf, c, R_QR_NEXT, QrFactor2dArgs{s->gxg[t], s->gxd[t], s->p, s->pp, &s->ls->tau,
                                             s->A, s->B, &s->ls->error, s->ls, s->gxg[c],
                                             s->gxd[c], rq});
  CombineArgs rt{};
  rt.X = s->X[c];
  rt.A = s->A;
  rt.Y = s->D[c];
  rt.upper = true;
  rt.B = s->B;
  rt.out = s->X[t];
  rt.rho = s->rho;
  rt.rho_scale = rho_scale(s);
  rt.ld = s->p;
  rt.n = s->n;
  rt.p = s->p;
  rt.f32 = s->f32;
  rt.bbr = bbr_ok(s);
  rt.pt = pt;
  set_resid(rt, s, s->vh[c]);  // the first residual of the Hartree solve (no k_init launch)
  put_rec(buf, c, R_RETRACT, rt);
  // Hartree: V_H of slot t = V_H(c) + L^{-1}(b - L V_H(c)) by the fast diagonalisation,
  // then the CG start that measures its residual (a solve that misses the tolerance is
  // finished by the host)
  const FdOps fd = fd_ops(s);
  put_rec(buf, c, R_RESID, InitArgs{s->rho, s->vh[c], nullptr, s->cg_r, s->cg_p[0], s->grid,
                                    s->cgpart});
  put_rec(buf, c, R_PLANE1, FdPlaneArgs{s->cg_r, s->cg_q, fd.Sx, fd.Sy, s->grid.nx, s->grid.ny,
                                        nullptr, nullptr, nullptr, nullptr});
  put_rec(buf, c, R_FDZ, FdZArgs{s->cg_q, fd.Sz, fd.lx, fd.ly, fd.lz, fd.mx, fd.my, fd.mz,
                                 s->grid.nx, s->grid.ny, s->grid.nz, nullptr});
  put_rec(buf, c, R_PLANE2, FdPlaneArgs{s->cg_q, s->vh[t], fd.Sx, fd.Sy, s->grid.nx, s->grid.ny,
                                        nullptr, nullptr, nullptr, s->vh[c]});
  // evaluation of slot t; the exchange pass measures the Hartree residual (the summary
  // writes the CG start), as a lone trial that queues no continuation does
  put_rec(buf, c, R_XC, XcArgs{s->rho, s->vh[t], s->vext, s->veff[t], s->grid, s->use_h,
                               s->use_x, nullptr, pt, 1, s->vbc});
  const bool hxg = hx_fuses_gram(s->p);
  put_rec(buf, c, R_HX, HxArgs<T>{static_cast<const T*>(s->X[t]), s->p,
                                  static_cast<T*>(s->G[t]), s->p, s->veff[t], s->grid,
                                  s->p, 2.0 * s->f, pt, hxg ? s->gram_part : nullptr,
                                  hx_zrun_of(s->grid)});
  put_rec(buf, c, R_GRAM1, GramArgs<T>{static_cast<const T*>(s->X[t]),
                                       static_cast<const T*>(s->G[t]), s->p, s->n, s->p,
                                       s->gram_part});
  put_rec(buf, c, R_RED1, GramReduceArgs{s->gram_part,
                                         hxg ? hx_gram_blocks(s->n) : s->gram_nchunks, s->pp,
                                         kGramAA | kGramAB, s->gxg[t], s->W});
  CombineArgs gd{};
  gd.X = s->X[t];
  gd.A = s->W;
  gd.C0 = s->G[t];
  gd.out = s->D[t];
  gd.Xk = s->X[c];
  gd.Dk = s->D[c];
  gd.pt = pt;
  gd.gram_part = s->gram_part;  // X^T D, D^T D from the same kernel
  gd.ld = s->p;
  gd.n = s->n;
  gd.p = s->p;
  gd.f32 = s->f32;
  gd.bbr = bbr_ok(s);  // the FP64 batch kernel always takes this form
  put_rec(buf, c, R_GRAD, gd);
  const bool bbr = bbr_ok(s);  // the FP64 gradient kernel forms only D^T D
  put_rec(buf, c, R_RED2, GramReduceArgs{s->gram_part, combine_blocks(s->n), s->pp,
                                         kGramAB | kGramBB, s->gxd[t], nullptr,
                                         bbr ? s->gxg[t] + s->pp * s->pp : nullptr,
                                         bbr ? s->gxg[t] : nullptr, bbr ? s->W : nullptr});
}

int upload_records(ks_system* s, const MinRun& m) {
  std::vector<char> buf(kRecBytes, 0);
  for (int c = 0; c < 2; ++c) {
    if (s->f32) fill_typed<float>(s, buf, c);
    else fill_typed<double>(s, buf, c);
    const int t = 1 - c;
    int nblk[kMaxScalarSlots] = {};
    nblk[SL_KIN] = hx_fuses_gram(s->p) ? hx_gram_blocks(s->n) : hx_blocks(s->n, s->p);
    nblk[SL_EH] = nblk[SL_EX] = nblk[SL_EXT] = nblk[SL_TF] = scalar_blocks(s->n);
    nblk[SL_DD] = nblk[SL_SS] = nblk[SL_SY] = nblk[SL_YY] = combine_blocks(s->n);
    nblk[SL_CGRR] = nblk[SL_CGBB] = scalar_blocks(s->n);
    nblk[SL_EBC] = s->vbc ? scalar_blocks(s->n) : 0;
    ScalarCounts sc{};
    for (int i = 0; i < SL_COUNT; ++i) sc.v[i] = nblk[i];
    const bool bbr = bbr_ok(s);
    put_rec(buf, c, R_FINISH, FinishEvalArgs{s->spart, kPartStride, sc, s->sums[t], s->gxg[t],
                                             s->p, s->pp, s->f, s->grid.dV, s->enuc, s->cg,
                                             s->ev[t], s->ls, m.lp, s->cg, s->htol,
                                             s->hmaxit, s->ebc, bbr ? s->Rq : nullptr,
                                             bbr ? s->gxd[t] + s->pp * s->pp : nullptr});
  }
  int rc = hip_check(s, hipMemcpyAsync(s->rec, buf.data(), kRecBytes, hipMemcpyHostToDevice,
                                       s->st), "record upload");
  if (rc) return rc;
  rc = hip_check(s, hipStreamSynchronize(s->st), "record upload sync");
  if (rc == KS_OK) s->run.records = true;
  return rc;
}

}  // namespace

namespace ks {

struct BatchMember {
  ks_system* s = nullptr;  // its run state is s->run
  bool queued = false;  // the QR factor of its next trial is already on the engine stream
  void* tag = nullptr;
  int code = KS_OK;
  ks_result r{};
};

struct BatchEngine {
  hipStream_t st = nullptr;
  bool finish = true;       // stopped runs are ended (result copied out) by the engine
  hipEvent_t ev = nullptr;  // end of the record copy of a tick
  std::vector<BatchMember*> act;
  std::vector<BatchMember*> fin;
  // Graph replay of a tick's trial launches (every member has graphs enabled and its
  // factor queued): captured for one ordered membership and replayed while it lasts; the
  // launches find each member's records through its current slot, kept in the lead
  // member's workspace (slots) and captured on the lead's capture stream.
  hipGraphExec_t gexec = nullptr;
  std::vector<const ks_system*> gkey;
};

namespace {

// The launch table of record kind r for group g.  par (device, one int per member of g):
// the records are addressed by the slot in par at run time (graph replay); otherwise by
// each member's current slot now.
template <typename A, typename F>
BatchPtrs<A> table(const std::vector<BatchMember*>& g, int r, F blocks, int* total,
                   const int* par = nullptr) {
  BatchPtrs<A> b{};
  b.S = (int)g.size();
  b.par = par;
  b.rstride = (int)(R_COUNT * kRecSlot);
  int off = 0;
  for (int i = 0; i < b.S; ++i) {
    b.off[i] = off;
    b.a[i] = rec_at<A>(g[i]->s, par ? 0 : g[i]->s->run.c, r);
    off += blocks(g[i]->s);
  }
  b.off[b.S] = off;
  *total = off;
  return b;
}

int one(const ks_system*) { return 1; }

// One trial of every member of g (same precision and p_p), then their records back.
// par: see table (graph capture; every member's factor is then already queued).
template <typename T>
void launch_trial_batch(const std::vector<BatchMember*>& g, hipStream_t st,
                        const int* par = nullptr) {
  int tot = 0;
  const int pp = g[0]->s->pp;
  int pmax = 0;
  for (auto* m : g) pmax = std::max(pmax, m->s->p);
  // the factor of members whose factor was queued at the end of the last tick is in place
  std::vector<BatchMember*> fresh;
  for (auto* m : g)
    if (!m->queued) fresh.push_back(m);
  for (auto* m : g) m->queued = false;
  if (!fresh.empty()) {
    int pf = 0;
    for (auto* m : fresh) pf = std::max(pf, m->s->p);
    auto qr = table<QrFactor2dArgs>(fresh, R_QR, one, &tot);
    launch_qr_factor_batch(qr, pf <= 16 ? 16 : 32, st);
  }
  auto cb = [](const ks_system* s) { return combine_blocks(s->n); };
  auto rt = table<CombineArgs>(g, R_RETRACT, cb, &tot, par);
  launch_combine_retract_batch<T>(rt, pp, tot, st);
  // one plane mode for the group (the slowest any member needs), LDS for the largest
  int mode = kPlaneFull;
  bool stage_z = true;
  for (auto* m : g) {
    const FdLaunch l = fd_launch(m->s->grid);
    mode = std::min(mode, l.plane_mode);
    stage_z = stage_z && l.z_bytes_staged <= l.cap;
  }
  size_t lds_p = 0, lds_z = 0;
  for (auto* m : g) {
    const FdLaunch l = fd_launch(m->s->grid);
    lds_p = std::max(lds_p, fd_plane_bytes(m->s->grid.nx, m->s->grid.ny, mode));
    lds_z = std::max(lds_z, stage_z ? l.z_bytes_staged : l.z_bytes);
  }
  auto pb = [mode](const ks_system* s) { return fd_plane_blocks(s->grid.nx, s->grid.nz, mode); };
  auto zb = [](const ks_system* s) {
    return fd_launch(s->grid).z_blocks;
  };
  auto hb = [](const ks_system* s) { return hartree_blocks(s->n); };
  (void)hb;  // the retraction formed each member's first Hartree residual
  auto p1 = table<FdPlaneArgs>(g, R_PLANE1, pb, &tot, par);
  launch_fd_plane_batch(p1, tot, mode, lds_p, st);
  auto fz = table<FdZArgs>(g, R_FDZ, zb, &tot, par);
  launch_fd_z_batch(fz, tot, stage_z, lds_z, st);
  auto p2 = table<FdPlaneArgs>(g, R_PLANE2, pb, &tot, par);
  launch_fd_plane_batch(p2, tot, mode, lds_p, st);
  auto sb = [](const ks_system* s) { return scalar_blocks(s->n); };
  auto xc = table<XcArgs>(g, R_XC, sb, &tot, par);
  launch_xc_batch(xc, tot, st);
  // the members of a group agree on whether the Hamiltonian forms the [X, G] Gram blocks
  const bool hxg = hx_fuses_gram(g[0]->s->p);
  auto hxb = [hxg](const ks_system* s) {
    return hxg ? hx_gram_blocks(s->n) : hx_blocks(s->n, s->p);
  };
  auto hx = table<HxArgs<T>>(g, R_HX, hxb, &tot, par);
  launch_hx_batch<T>(hx, tot, hxg, st);
  auto gb = [](const ks_system* s) { return s->gram_nchunks; };
  auto rb = [](const ks_system* s) { return gram_reduce_blocks(s->pp); };
  if (!hxg) {
    auto g1 = table<GramArgs<T>>(g, R_GRAM1, gb, &tot, par);
    launch_gram_batch<T>(g1, pp, kGramAA | kGramAB, tot, st);
  }
  auto r1 = table<GramReduceArgs>(g, R_RED1, rb, &tot, par);
  launch_gram_reduce_batch(r1, tot, st);
  auto gd = table<CombineArgs>(g, R_GRAD, cb, &tot, par);
  launch_combine_grad_batch<T>(gd, pp, tot, st);
  auto r2 = table<GramReduceArgs>(g, R_RED2, rb, &tot, par);
  launch_gram_reduce_batch(r2, tot, st);
  launch_finish_eval_batch(table<FinishEvalArgs>(g, R_FINISH, one, &tot, par), st);
}

}  // namespace

BatchEngine* batch_create(hipStream_t st) {
  BatchEngine* e = new BatchEngine();
  e->st = st;
  return e;
}

void batch_destroy(BatchEngine* e) {
  if (!e) return;
  if (e->ev) (void)hipEventDestroy(e->ev);
  if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
  for (auto* m : e->act) delete m;
  for (auto* m : e->fin) delete m;
  delete e;
}

int batch_size(const BatchEngine* e) { return (int)e->act.size(); }

// Starts a run (first evaluation on the system's own stream).  A run that cannot start,
// or that stops at once, goes straight to the finished list.
int batch_add(BatchEngine* e, ks_system* s, void* X, const ks_opt_params* o, void* tag) {
  if ((int)e->act.size() >= kMaxBatch) return KS_E_INVAL;
  // a captured tick names its members' buffers: a new member (possibly a new system at the
  // address of a destroyed one) always means a new capture
  if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
  e->gexec = nullptr;
  e->gkey.clear();
  BatchMember* m = new BatchMember();
  m->s = s;
  m->tag = tag;
  int rc = run_begin(s, X, o, &s->run);
  if (rc == KS_OK && !batchable(s, s->run)) rc = fail(s, KS_E_UNSUPPORTED, "not batchable");
  if (rc == KS_OK) rc = upload_records(s, s->run);
  if (rc != KS_OK) {
    s->run.active = false;
    m->code = rc;
    e->fin.push_back(m);
    return rc;
  }
  const LsState* hl = host_ls(s);
  if (hl->stop != KS_STOP_NONE || hl->error) {
    m->code = run_end(s, &s->run, &m->r);
    e->fin.push_back(m);
    return KS_OK;
  }
  e->act.push_back(m);
  return KS_OK;
}

// The trial launches and the record gather of a tick as a graph: captured when the ordered
// membership differs from the captured one, then replayed after the members' current slots
// are written to the lead member's slot array.  The membership key holds the lead, so a
// replayed graph always reads the slot array it was captured with.
int batch_replay(BatchEngine* e, const std::vector<std::vector<BatchMember*>>& groups,
                 const GatherArgs& ga) {
  ks_system* lead = e->act[0]->s;
  std::vector<const ks_system*> key;
  for (auto* m : e->act) key.push_back(m->s);
  IntList sl{};
  for (auto& g : groups)
    for (auto* m : g) sl.v[sl.n++] = m->s->run.c;
  launch_set_ints(lead->slots, sl, e->st);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess && (!e->gexec || key != e->gkey)) {
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    e->gexec = nullptr;
    e->gkey.clear();
    hipGraph_t graph = nullptr;
    hipStream_t cs = lead->cap_st;
    he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
      int base = 0;
      for (auto& g : groups) {
        if (g[0]->s->f32) launch_trial_batch<float>(g, cs, lead->slots + base);
        else launch_trial_batch<double>(g, cs, lead->slots + base);
        base += (int)g.size();
      }
      launch_gather(ga, cs);
      he = hipStreamEndCapture(cs, &graph);
    }
    if (he == hipSuccess) he = hipGraphInstantiate(&e->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (he == hipSuccess) e->gkey = key;
  }
  if (he == hipSuccess) he = hipGraphLaunch(e->gexec, e->st);
  return hip_check(lead, he, "batch graph replay");
}

// One trial for every active member; members that stop move to the finished list.
int batch_tick(BatchEngine* e) {
  if (e->act.empty()) return KS_OK;
  // groups of equal storage precision, p_p and Hamiltonian form (with or without the Gram)
  std::vector<std::vector<BatchMember*>> groups;
  for (auto* m : e->act) {
    bool placed = false;
    for (auto& g : groups)
      if (g[0]->s->f32 == m->s->f32 && g[0]->s->pp == m->s->pp &&
          hx_fuses_gram(g[0]->s->p) == hx_fuses_gram(m->s->p)) {
        g.push_back(m);
        placed = true;
        break;
      }
    if (!placed) groups.push_back({m});
  }
  // the CG and line-search records of all members come back in one copy
  ks_system* lead = e->act[0]->s;
  GatherArgs ga{};
  ga.S = (int)e->act.size();
  ga.bytes = kGatherBytes;
  for (int i = 0; i < ga.S; ++i) ga.src[i] = reinterpret_cast<const char*>(e->act[i]->s->cg);
  ga.dst = lead->gstage;
  bool replay = true;
  for (auto* m : e->act) replay = replay && m->s->graphs && m->s->cap_st && m->queued;
  if (replay) {
    const int rc0 = batch_replay(e, groups, ga);
    if (rc0) return rc0;
  } else {
    for (auto& g : groups) {
      if (g[0]->s->f32) launch_trial_batch<float>(g, e->st);
      else launch_trial_batch<double>(g, e->st);
    }
    launch_gather(ga, e->st);
  }
  char* hstage = static_cast<char*>(lead->host) + 1024;
  hipError_t he = hipMemcpyAsync(hstage, lead->gstage, (size_t)ga.S * kGatherBytes,
                                 hipMemcpyDeviceToHost, e->st);
  // the QR factors of every member's next trial go behind the copy; each picks its slot
  // from its own line-search record on the device, and the host waits for the copy only
  if (he == hipSuccess && !e->ev) he = hipEventCreateWithFlags(&e->ev, hipEventDisableTiming);
  if (he == hipSuccess) he = hipEventRecord(e->ev, e->st);
  if (he == hipSuccess) {
    int tot = 0, pm = 0;
    for (auto* m : e->act) pm = std::max(pm, m->s->p);
    launch_qr_factor_batch(table<QrFactor2dArgs>(e->act, R_QR_NEXT, one, &tot),
                           pm <= 16 ? 16 : 32, e->st);
    he = hipEventSynchronize(e->ev);
  }
  int rc = hip_check(lead, he, "batch read-back");
  if (rc) return rc;
  bool pending = false;
  for (int i = 0; i < ga.S; ++i) {
    std::memcpy(e->act[i]->s->host, hstage + (size_t)i * kGatherBytes, kGatherBytes);
    pending = pending || host_ls(e->act[i]->s)->hartree_pending;
  }
  // a pending member is re-evaluated on its own stream: the queued factors (which return at
  // once for it) finish first
  if (pending) {
    rc = hip_check(lead, hipStreamSynchronize(e->st), "batch factor wait");
    if (rc) return rc;
  }
  std::vector<BatchMember*> keep;
  for (int i = 0; i < ga.S; ++i) {
    BatchMember* m = e->act[i];
    m->queued = !host_ls(m->s)->hartree_pending;
    m->s->run.queued = false;  // the lone path's speculative factor is not in place
    m->s->cg_par = 0;  // the host state a lone trial leaves (no PCG iteration queued)
    m->s->cg_fused = true;  // the batched exchange pass measured the Hartree residual
    int code = run_after_trial(m->s, &m->s->run, true);
    const LsState* hl = host_ls(m->s);
    if (code != KS_OK) {
      m->code = code;
      m->s->run.active = false;
      e->fin.push_back(m);
    } else if (hl->stop != KS_STOP_NONE || hl->error) {
      m->code = e->finish ? run_end(m->s, &m->s->run, &m->r) : KS_OK;
      e->fin.push_back(m);
    } else {
      keep.push_back(m);
    }
  }
  e->act.swap(keep);
  return KS_OK;
}

// Pops one finished run: its tag, result and return code.
bool batch_take(BatchEngine* e, void** tag, ks_result* r, int* code) {
  if (e->fin.empty()) return false;
  BatchMember* m = e->fin.front();
  e->fin.erase(e->fin.begin());
  if (tag) *tag = m->tag;
  if (r) *r = m->r;
  if (code) *code = m->code;
  delete m;
  return true;
}

}  // namespace ks

extern "C" {

void ks_default_params(ks_opt_params* o) {
  if (!o) return;
  o->tau0 = 1e-3;
  o->rho1 = 1e-4;
  o->delta = 0.1;
  o->eta = 0.85;
  o->eps_g = 1e-6;
  o->max_iter = 10000;
  o->bb_rule = KS_BB_ALT;
  o->retraction = KS_QR;
  o->tau_min = 1e-20;
  o->tau_max = 1e20;
  o->h_max = 20;
  o->reorth_tol = 1e-12;
  o->stagnation_tol = 1e-13;
  o->reorth_every = 0;
  o->energy_target = -HUGE_VAL;
}

const char* ks_status_string(int code) {
  switch (code) {
    case KS_OK: return "ok";
    case KS_E_INVAL: return "invalid argument";
    case KS_E_NOMEM: return "workspace too small";
    case KS_E_HIP: return "HIP runtime error";
    case KS_E_NOT_SPD: return "Cholesky breakdown (matrix not positive definite)";
    case KS_E_SINGULAR: return "singular Sherman-Morrison-Woodbury system";
    case KS_E_NONFINITE: return "non-finite value";
    case KS_E_NOT_CONVERGED: return "not converged";
    case KS_E_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* ks_last_error(const ks_system* s) {
  return s ? s->err.c_str() : g_err.c_str();
}

size_t ks_workspace_bytes(const ks_system_desc* d) {
  std::string why;
  if (validate(d, &why) != KS_OK) {
    g_err = why;
    return 0;
  }
  ks_system tmp;
  init_dims(&tmp, d);
  size_t total = 0;
  layout(&tmp, nullptr, &total);
  return total;
}

int ks_create_system(const ks_system_desc* d, void* dev_workspace, size_t ws_bytes,
                     void* hip_stream, ks_system** out) {
  if (!out) return fail(nullptr, KS_E_INVAL, "out is null");
  *out = nullptr;
  std::string why;
  int rc = validate(d, &why);
  if (rc) return fail(nullptr, rc, why);
  if (!dev_workspace) return fail(nullptr, KS_E_INVAL, "workspace is null");
  if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0)
    return fail(nullptr, KS_E_INVAL, "workspace must be 256-byte aligned");
  ks_system* s = new ks_system();
  init_dims(s, d);
  size_t need = 0;
  layout(s, nullptr, &need);
  if (ws_bytes < need) {
    delete s;
    return fail(nullptr, KS_E_NOMEM, "workspace smaller than ks_workspace_bytes()");
  }
  // every later step writes into the workspace from kernels: an address the runtime does
  // not know as device memory is refused here, before any launch
  if (!device_range(dev_workspace, need)) {
    delete s;
    return fail(nullptr, KS_E_INVAL, "workspace is not device memory of ws_bytes bytes");
  }
  layout(s, static_cast<char*>(dev_workspace), &need);
  s->st = static_cast<hipStream_t>(hip_stream);
  if (hipHostMalloc(&s->host, kHostBytes, hipHostMallocDefault) != hipSuccess) {
    delete s;
    return fail(nullptr, KS_E_HIP, "pinned host buffer");
  }
  std::memset(s->host, 0, kHostBytes);
  if (hipHostGetDevicePointer(&s->host_dev, s->host, 0) != hipSuccess) {
    (void)hipGetLastError();
    s->host_dev = nullptr;  // the records are then copied
  }
  const int M = d->n_nuclei;
  hipError_t e = hipSuccess;
  if (M > 0) {
    e = hipMemcpyAsync(s->Rd, s->R.data(), 3 * M * sizeof(double), hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->Zd, s->Z.data(), M * sizeof(double), hipMemcpyHostToDevice, s->st);
  }
  if (e == hipSuccess && d->v_ext_override)
    e = hipMemcpyAsync(s->vext, d->v_ext_override, (size_t)s->n * sizeof(double),
                       hipMemcpyHostToDevice, s->st);
  if (e != hipSuccess) {
    rc = hip_check(s, e, "upload");
    ks_destroy_system(s);
    return rc;
  }
  if (!d->v_ext_override) {
    if (s->use_ext && M > 0 && d->vext_kind == KS_VEXT_GNH)
      launch_vext_gnh(s->vext, s->Rd, s->Zd, M, s->grid, s->gnh_tab, s->st);
    else if (s->use_ext && M > 0) launch_vext(s->vext, s->Rd, s->Zd, M, s->grid, d->rc, s->st);
    else launch_fill(s->vext, 0.0, s->n, s->st);
  }
  if (!d->v_ext_override && s->use_ext && M > 1) launch_enuc(s->enuc, s->Rd, s->Zd, M, s->st);
  else launch_set_scalar(s->enuc, 0.0, s->st);
  for (int i = 0; i < 2; ++i) {
    launch_fill(s->vh[i], 0.0, s->n, s->st);
    launch_copy_vec(s->veff[i], s->vext, s->n, s->st);
  }
  const int dims[3] = {s->grid.nx, s->grid.ny, s->grid.nz};
  for (int a = 0; a < 3; ++a) {
    launch_fd_setup(s->fdS[a], s->fdL[a], s->fdM[a], dims[a], s->grid.h, s->q1 ? 1 : 0, s->st);
    if (s->q1) launch_mass_setup(s->mtab[a], dims[a], s->grid.h, s->st);
  }
  launch_ls_reset(s->ls, s->st);
  // the CG arrival counter must start at zero
  launch_fill(reinterpret_cast<double*>(s->cg), 0.0, sizeof(CgState) / sizeof(double), s->st);
  rc = launch_check(s, "setup");
  if (rc == KS_OK && s->vbc) rc = setup_monopole(s);
  if (rc == KS_OK) rc = hip_check(s, hipStreamSynchronize(s->st), "setup sync");
  if (rc) {
    std::string m = s->err;
    ks_destroy_system(s);
    return fail(nullptr, rc, m);
  }
  *out = s;
  return KS_OK;
}

void ks_destroy_system(ks_system* s) {
  if (!s) return;
  if (s->host) {
    (void)hipStreamSynchronize(s->st);
    (void)hipHostFree(s->host);
  }
  for (auto& p : s->ev_pend) {
    s->ev_free.push_back(p.a);
    s->ev_free.push_back(p.b);
  }
  for (auto& p : s->ev_open) {
    if (p.a) s->ev_free.push_back(p.a);
    if (p.b) s->ev_free.push_back(p.b);
  }
  for (hipEvent_t e : s->ev_free) (void)hipEventDestroy(e);
  if (s->ev_rb) (void)hipEventDestroy(s->ev_rb);
  drop_graphs(s);
  if (s->cap_st) (void)hipStreamDestroy(s->cap_st);
  delete s;
}

int ks_timer_phases(ks_system* s, unsigned mask) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  s->timer_mask = mask;
  return KS_OK;
}

int ks_enable_graphs(ks_system* s, int on) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  if (on && !s->cap_st) {
    int rc = hip_check(s, hipStreamCreateWithFlags(&s->cap_st, hipStreamNonBlocking),
                       "capture stream");
    if (rc) return rc;
  }
  s->graphs = on != 0;
  drop_graphs(s);
  return KS_OK;
}

int ks_enable_timers(ks_system* s, int on) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  s->timers = on != 0;
  s->timer_mask = ~0u;
  return KS_OK;
}

int ks_read_timers(ks_system* s, ks_phase_times* out, int reset) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  int rc = hip_check(s, hipStreamSynchronize(s->st), "timer sync");
  if (rc) return rc;
  harvest(s);
  if (out) {
    for (int i = 0; i < KS_NPHASES; ++i) {
      out->ms[i] = s->ph_ms[i];
      out->count[i] = s->ph_n[i];
    }
  }
  if (reset) {
    for (int i = 0; i < KS_NPHASES; ++i) {
      s->ph_ms[i] = 0.0;
      s->ph_n[i] = 0;
    }
  }
  return KS_OK;
}

int ks_density(ks_system* s, const void* X, double* rho) {
  if (!s || !X || !rho) return fail(s, KS_E_INVAL, "null argument");
  density(s, X, s->ld, rho);
  int rc = launch_check(s, "density");
  return rc ? rc : hip_check(s, hipStreamSynchronize(s->st), "density sync");
}

int ks_hartree_solve(ks_system* s, const double* rho, double* v_h, int warm, int* iters,
                     double* relres) {
  if (!s || !rho || !v_h) return fail(s, KS_E_INVAL, "null argument");
  int it = 0;
  double rr = 0.0;
  int rc = hartree(s, rho, warm ? v_h : nullptr, v_h, true, &it, &rr);
  if (rc) return rc;
  if (host_cg(s)->bb == 0.0) launch_fill(v_h, 0.0, s->n, s->st);
  rc = hip_check(s, hipStreamSynchronize(s->st), "hartree sync");
  if (iters) *iters = it;
  if (relres) *relres = rr;
  if (rc) return rc;
  const CgState* hc = host_cg(s);
  const bool at_floor = hc->stall >= kCgStall && rr <= kCgFloor * s->htol;
  if (rr > s->htol && !at_floor)
    return fail(s, KS_E_NOT_CONVERGED, "Hartree CG reached its iteration cap");
  return KS_OK;
}

int ks_apply_hamiltonian(ks_system* s, const void* X, void* Y, const double* v_eff) {
  if (!s || !X || !Y) return fail(s, KS_E_INVAL, "null argument");
  if (X == Y) return fail(s, KS_E_INVAL, "X and Y must differ");
  if (s->q1) {
    // Y = (1/2) A X + h^3 Diag(v_eff) X on dense internal copies
    const int t = 1 - s->cur;
    copy_block(s, s->X[t], s->p, X, s->ld);
    q1_apply(s, s->X[t], s->G[t], s->BX[t], v_eff ? v_eff : s->veff[s->cur], 1.0, nullptr);
    copy_block(s, Y, s->ld, s->G[t], s->p);
  } else {
    tbeg(s, KS_PH_HAMILTONIAN);
    hamiltonian(s, X, s->ld, Y, s->ld, v_eff ? v_eff : s->veff[s->cur], 1.0, nullptr);
    tend(s, KS_PH_HAMILTONIAN);
  }
  int rc = launch_check(s, "hamiltonian");
  if (rc == KS_OK) rc = hip_check(s, hipStreamSynchronize(s->st), "hamiltonian sync");
  if (rc == KS_OK && s->timers) harvest(s);
  return rc;
}

int ks_get_potentials(ks_system* s, double* v_ext, double* v_h, double* v_eff) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  if (v_ext) launch_copy_vec(v_ext, s->vext, s->n, s->st);
  if (v_h) launch_copy_vec(v_h, s->vh[s->cur], s->n, s->st);
  if (v_eff) launch_copy_vec(v_eff, s->veff[s->cur], s->n, s->st);
  int rc = launch_check(s, "potentials");
  return rc ? rc : hip_check(s, hipStreamSynchronize(s->st), "potentials sync");
}

int ks_gram(ks_system* s, const void* Ain, const void* Bin, double* out) {
  if (!s || !Ain || !Bin || !out) return fail(s, KS_E_INVAL, "null argument");
  const int t = 1 - s->cur;
  copy_block(s, s->X[t], s->p, Ain, s->ld);
  copy_block(s, s->G[t], s->p, Bin, s->ld);
  const int all = kGramAA | kGramAB | kGramBB;
  gram_reduced(s, s->X[t], s->G[t], all, s->gxg[t], nullptr, false, true);
  launch_compact_gram(s->gxg[t], s->pp, s->p, out, s->st);
  int rc = launch_check(s, "gram");
  return rc ? rc : hip_check(s, hipStreamSynchronize(s->st), "gram sync");
}

int ks_energy_grad(ks_system* s, const void* X, void* G, void* gradE, ks_energy* out) {
  if (!s || !X) return fail(s, KS_E_INVAL, "null argument");
  const int c = s->cur;
  copy_block(s, s->X[c], s->p, X, s->ld);
  int rc = evaluate(s, c, false, -1, c, false, false);
  if (rc) return rc;
  if (G)
    copy_block(s, G, s->ld, s->G[c], s->p);
  if (gradE)
    copy_block(s, gradE, s->ld, s->D[c], s->p);
  rc = launch_check(s, "energy_grad");
  if (rc) return rc;
  EvalOut* he = host_ev(s);
  rc = readback(s, he, s->ev[c]);
  if (rc) return rc;
  if (out) to_energy(*he, out);
  if (he->nonfinite) return fail(s, KS_E_NONFINITE, "non-finite energy or gradient");
  return KS_OK;
}

int ks_retract(ks_system* s, const void* X, const void* G, double tau, int kind, void* X_out) {
  if (!s || !X || !G || !X_out) return fail(s, KS_E_INVAL, "null argument");
  if (kind != KS_QR && kind != KS_WY) return fail(s, KS_E_INVAL, "unknown retraction");
  if (X_out == X || X_out == G) return fail(s, KS_E_INVAL, "X_out must not alias X or G");
  if (!std::isfinite(tau)) return fail(s, KS_E_INVAL, "tau must be finite");
  const int t = 1 - s->cur, c = s->cur;
  copy_block(s, s->X[t], s->p, X, s->ld);
  copy_block(s, s->G[t], s->p, G, s->ld);
  const int all = kGramAA | kGramAB | kGramBB;
  if (s->q1) {
    // grad E = B^{-1} G - X (G^T X) and the B-metric Gram blocks, as in an evaluation
    const int pp2 = s->pp * s->pp;
    q1_apply(s, s->X[t], nullptr, s->BX[t], nullptr, 1.0, nullptr);
    mass_solve(s, s->G[t], s->Gt[t]);
    gram_reduced(s, s->X[t], s->G[t], kGramAB, s->gxg[t], s->W, false, kind == KS_QR);
    gram_reduced(s, s->X[t], s->BX[t], kGramAB, s->feg[t], nullptr, true);
    Q1GradArgs ga{};
    ga.Gt = s->Gt[t];
    ga.X = s->X[t];
    ga.G = s->G[t];
    ga.BX = s->BX[t];
    ga.W = s->W;
    ga.D = s->D[t];
    ga.BD = s->BD[t];
    ga.pt = Partials{s->spart, kPartStride};
    ga.n = s->n;
    ga.p = s->p;
    ga.pp = s->pp;
    ga.f32 = s->f32;
    launch_q1_grad(ga, s->st);
    gram_reduced(s, s->X[t], s->BD[t], kGramAB, s->gxd[t], nullptr);
    gram_reduced(s, s->D[t], s->BD[t], kGramAB, s->gxd[t] + pp2, nullptr, true);
    if (kind == KS_WY) wy_blocks_q1(s, t);
  } else {
    gram_reduced(s, s->X[t], s->G[t], all, s->gxg[t], s->W, false, kind == KS_QR);
  }
  launch_set_scalar(s->tau_user, tau, s->st);
  int* hstat = host_int(s);
  hstat[0] = 0;
  int rc0 = hip_check(s, hipMemcpyAsync(s->status, hstat, sizeof(int), hipMemcpyHostToDevice,
                                        s->st), "status upload");
  if (rc0) return rc0;
  CombineArgs ca{};
  ca.ld = s->p;
  ca.n = s->n;
  ca.p = s->p;
  ca.f32 = s->f32;
  ca.mc = s->mc;
  if (kind == KS_QR && s->q1) {
    launch_qr_factor(s->feg[t] + s->pp * s->pp, s->gxd[t], s->p, s->pp, s->tau_user, s->A, s->B,
                     s->work, s->status, s->st);
    ca.Y = s->D[t];
    ca.upper = true;
  } else if (kind == KS_QR) {
    CombineArgs cd{};
    cd.f32 = s->f32;
    cd.mc = s->mc;
    cd.X = s->X[t];
    cd.A = s->W;
    cd.C0 = s->G[t];
    cd.out = s->D[t];
    cd.ld = s->p;
    cd.n = s->n;
    cd.p = s->p;
    launch_combine(cd, s->st);
    const int m2 = kGramAB | kGramBB;
    gram_reduced(s, s->X[t], s->D[t], m2, s->gxd[t], nullptr);
    launch_qr_factor(s->gxg[t], s->gxd[t], s->p, s->pp, s->tau_user, s->A, s->B, s->work,
                     s->status, s->st);
    ca.Y = s->D[t];
    ca.upper = true;
  } else {
    launch_wy_factor(s->q1 ? s->wyg[t] : s->gxg[t], s->p, s->pp, s->tau_user, INFINITY, s->A,
                     s->B, s->work, s->status, nullptr, s->st);
    ca.Y = s->q1 ? s->Gt[t] : s->G[t];
  }
  ca.X = s->X[t];
  ca.A = s->A;
  ca.B = s->B;
  ca.out = s->D[c];
  launch_combine(ca, s->st);
  copy_block(s, X_out, s->ld, s->D[c], s->p);
  int rc = launch_check(s, "retract");
  if (rc) return rc;
  rc = readback(s, hstat, s->status);
  if (rc) return rc;
  if (hstat[0] == KS_E_NOT_SPD) return fail(s, KS_E_NOT_SPD, "Cholesky breakdown of Y^T Y");
  if (hstat[0] == KS_E_SINGULAR) return fail(s, KS_E_SINGULAR, "singular SMW system");
  if (hstat[0] != 0) return fail(s, hstat[0], "retraction failed");
  return KS_OK;
}

int ks_minimize(ks_system* s, void* X_inout, const ks_opt_params* o, ks_result* r) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  MinRun* m = &s->run;
  int rc = run_begin(s, X_inout, o, m);
  if (rc) {
    m->active = false;
    return rc;
  }
  LsState* hl = host_ls(s);
  while (hl->stop == KS_STOP_NONE && !hl->error) {
    rc = run_trial(s, m);
    if (rc) {
      m->active = false;
      return rc;
    }
  }
  return run_end(s, m, r);
}

extern "C++" {
namespace {
using TuneKey = std::tuple<int, int, int, int, int, int, int>;
std::mutex g_tune_mu;
// a candidate must beat the built-in shape by 10%: tuning-time timings of the Hartree passes
// vary by several percent from run to run and have ranked shapes against the times the
// same kernels take inside a solve
constexpr double kTuneMargin = 0.10;
constexpr int kTuneRounds = 3;
std::map<TuneKey, std::pair<int, int>> g_tune;  // (fd_mode, hx_zrun)

// Mean device time of fn() over reps launches on the system's stream, after two warm-ups.
template <typename F>
int time_us(ks_system* s, int reps, F fn, double* us) {
  fn();
  fn();
  hipEvent_t a, b;
  int rc = hip_check(s, hipEventCreate(&a), "tune event");
  if (rc) return rc;
  rc = hip_check(s, hipEventCreate(&b), "tune event");
  if (rc) {
    (void)hipEventDestroy(a);
    return rc;
  }
  (void)hipEventRecord(a, s->st);
  for (int i = 0; i < reps; ++i) fn();
  (void)hipEventRecord(b, s->st);
  rc = hip_check(s, hipEventSynchronize(b), "tune timing");
  float ms = 0.0f;
  if (!rc) rc = hip_check(s, hipEventElapsedTime(&ms, a, b), "tune timing");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (!rc) rc = launch_check(s, "tune launches");
  *us = 1e3 * (double)ms / reps;
  return rc;
}
}  // namespace
}  // extern "C++"

int ks_autotune(ks_system* s, int force, ks_tune_info* out) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  if (s->run.active) return fail(s, KS_E_INVAL, "a run is in progress");
  ks_tune_info info{};
  info.fd_plane_mode = info.hx_zrun = KS_TUNE_AUTO;
  const bool tune_fd = s->use_h && s->solver == KS_HARTREE_PCG_FD;
  const bool tune_hx = !s->q1 && hx_fuses_gram(s->p);
  const TuneKey key{s->grid.nx, s->grid.ny, s->grid.nz, s->p, s->f32 ? 1 : 0, s->q1 ? 1 : 0,
                    s->solver};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end() && !force) {
      s->grid.fd_mode = it->second.first;
      s->grid.hx_zrun = it->second.second;
      info.fd_plane_mode = tune_fd ? fd_plane_mode_of(s->grid) : KS_TUNE_AUTO;
      info.hx_zrun = tune_hx ? hx_zrun_of(s->grid) : KS_TUNE_AUTO;
      info.cached = 1;
      if (out) *out = info;
      return KS_OK;
    }
  }
  const size_t nb = (size_t)s->n * sizeof(double);
  const int reps = 10;
  int rc = KS_OK;
  if (tune_fd) {
    for (double* v : {s->cg_r, s->cg_q, s->vh[0], s->vh[1]})
      if (!rc) rc = hip_check(s, hipMemsetAsync(v, 0, nb, s->st), "tune clear");
    double best = 0.0;
    int best_mode = KS_TUNE_AUTO;
    const int dflt = fd_plane_mode(s->grid.nx, s->grid.ny);
    double dflt_us = 0.0;
    // interleaved rounds, the fastest round of each candidate: a single timing per
    // candidate mixes clock ramp-up and noise of a few percent into the comparison
    const int modes[4] = {kPlaneFull, kPlaneStripSy, kPlaneStrip, kPlaneStripG};
    double tmin[4] = {0.0, 0.0, 0.0, 0.0};
    for (int round = 0; round < kTuneRounds && !rc; ++round)
      for (int m = 0; m < 4 && !rc; ++m) {
        if (!fd_plane_mode_fits(s->grid.nx, s->grid.ny, modes[m])) continue;
        s->grid.fd_mode = modes[m];
        double us = 0.0;
        rc = time_us(s, reps, [&] {
          launch_fd_correct(s->cg_r, s->vh[0], s->vh[1], s->cg_q, fd_ops(s), s->grid, s->st);
        }, &us);
        if (round == 0 || us < tmin[m]) tmin[m] = us;
      }
    for (int m = 0; m < 4 && !rc; ++m) {
      const int mode = modes[m];
      if (!fd_plane_mode_fits(s->grid.nx, s->grid.ny, mode)) continue;
      const double us = tmin[m];
      info.fd_modes[info.n_fd] = mode;
      info.fd_us[info.n_fd++] = us;
      if (mode == dflt) dflt_us = us;
      if (best_mode == KS_TUNE_AUTO || us < best) {
        best = us;
        best_mode = mode;
      }
    }
    // a shape replaces the built-in rule only when it is clearly faster (timing noise must
    // not flip the choice, which changes the last bits of the results)
    if (!rc && dflt_us > 0.0 && best > (1.0 - kTuneMargin) * dflt_us) best_mode = dflt;
    s->grid.fd_mode = best_mode;
    info.fd_plane_mode = best_mode;
  }
  if (tune_hx && !rc) {
    const size_t xb = (size_t)s->n * s->p * s->es;
    rc = hip_check(s, hipMemsetAsync(s->X[0], 0, xb, s->st), "tune clear");
    if (!rc) rc = hip_check(s, hipMemsetAsync(s->veff[0], 0, nb, s->st), "tune clear");
    Partials pt{s->spart, kPartStride};
    double best = 0.0;
    int best_z = KS_TUNE_AUTO;
    const int dflt = hx_zrun(s->grid.nx * s->grid.ny, s->grid.nz);
    double dflt_us = 0.0;
    const int zs[2] = {16, 8};
    double tmin[2] = {0.0, 0.0};
    for (int round = 0; round < kTuneRounds && !rc; ++round)
      for (int m = 0; m < 2 && !rc; ++m) {
        s->grid.hx_zrun = zs[m];
        double us = 0.0;
        rc = time_us(s, reps, [&] {
          hamiltonian(s, s->X[0], s->p, s->G[0], s->p, s->veff[0], 1.0, &pt, s->gram_part);
        }, &us);
        if (round == 0 || us < tmin[m]) tmin[m] = us;
      }
    for (int m = 0; m < 2 && !rc; ++m) {
      const int z = zs[m];
      const double us = tmin[m];
      info.hx_zruns[info.n_hx] = z;
      info.hx_us[info.n_hx++] = us;
      if (z == dflt) dflt_us = us;
      if (best_z == KS_TUNE_AUTO || us < best) {
        best = us;
        best_z = z;
      }
    }
    if (!rc && dflt_us > 0.0 && best > (1.0 - kTuneMargin) * dflt_us) best_z = dflt;
    s->grid.hx_zrun = best_z;
    info.hx_zrun = best_z;
  }
  if (rc) return rc;
  drop_graphs(s);  // captured launches carry the old shapes
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {s->grid.fd_mode, s->grid.hx_zrun};
  }
  if (out) *out = info;
  return KS_OK;
}

int ks_prolong(ks_system* coarse, const void* Xc, ks_system* fine, void* Xf) {
  if (!coarse || !fine || !Xc || !Xf) return fail(fine ? fine : coarse, KS_E_INVAL,
                                                  "null argument");
  if (coarse == fine) return fail(fine, KS_E_INVAL, "coarse and fine are the same system");
  const Grid& c = coarse->grid;
  const Grid& f = fine->grid;
  const bool nested = f.nx == 2 * c.nx + 1 && f.ny == 2 * c.ny + 1 && f.nz == 2 * c.nz + 1 &&
                      std::fabs(2.0 * f.h - c.h) <= 1e-12 * c.h &&
                      std::fabs(f.lo[0] - c.lo[0]) <= 1e-12 * std::max(1.0, std::fabs(c.lo[0])) &&
                      std::fabs(f.lo[1] - c.lo[1]) <= 1e-12 * std::max(1.0, std::fabs(c.lo[1])) &&
                      std::fabs(f.lo[2] - c.lo[2]) <= 1e-12 * std::max(1.0, std::fabs(c.lo[2]));
  if (!nested)
    return fail(fine, KS_E_INVAL, "fine is not the uniform refinement of coarse (2N + 1 "
                                  "nodes per axis, half the spacing, the same box)");
  if (coarse->q1 != fine->q1 || coarse->f32 != fine->f32 || coarse->bf16 != fine->bf16 ||
      coarse->p != fine->p)
    return fail(fine, KS_E_INVAL, "coarse and fine differ in discretisation, precision or p");
  if (fine->run.active) return fail(fine, KS_E_INVAL, "a run of the fine system is in progress");
  int rc = hip_check(coarse, hipStreamSynchronize(coarse->st), "coarse stream");
  if (rc) return rc;
  // phi = X h^{-3/2} on the grid: halving h scales the nodal values by 2^{-3/2}; a Q1
  // block is the same finite-element function on the finer mesh
  const double scale = fine->q1 ? 1.0 : 1.0 / (2.0 * std::sqrt(2.0));
  const int slot = fine->cur;
  if (fine->f32)
    launch_prolong<float>(static_cast<const float*>(Xc), coarse->ld, c.nx, c.ny, c.nz,
                          static_cast<float*>(fine->X[slot]), fine->p, fine->p, scale, fine->st);
  else
    launch_prolong<double>(static_cast<const double*>(Xc), coarse->ld, c.nx, c.ny, c.nz,
                           static_cast<double*>(fine->X[slot]), fine->p, fine->p, scale,
                           fine->st);
  rc = launch_check(fine, "prolong");
  if (rc) return rc;
  rc = orthonormalize_slot(fine, slot);
  if (rc) return rc;
  copy_block(fine, Xf, fine->ld, fine->X[slot], fine->p);
  rc = launch_check(fine, "prolong copy");
  if (rc) return rc;
  return hip_check(fine, hipStreamSynchronize(fine->st), "prolong");
}

int ks_minimize_levels(ks_system* const* levels, int nlev, void* const* X,
                       const ks_opt_params* o, ks_result* r) {
  if (!levels || !X || !r || nlev < 1 || nlev > 16)
    return fail(levels && nlev > 0 ? levels[0] : nullptr, KS_E_INVAL,
                "levels, X and r are required, 1 <= nlev <= 16");
  for (int i = 0; i < nlev; ++i)
    if (!levels[i] || !X[i]) return fail(nullptr, KS_E_INVAL, "null level or block");
  int rc = KS_OK;
  for (int i = 0; i < nlev; ++i) {
    if (i > 0) {
      rc = ks_prolong(levels[i - 1], X[i - 1], levels[i], X[i]);
      if (rc) {
        levels[i]->err = "level " + std::to_string(i) + ": " + levels[i]->err;
        g_err = levels[i]->err;
        return rc;
      }
    }
    rc = ks_minimize(levels[i], X[i], o, &r[i]);
    if (rc != KS_OK && rc != KS_E_NOT_CONVERGED) {
      levels[i]->err = "level " + std::to_string(i) + ": " + levels[i]->err;
      g_err = levels[i]->err;
      return rc;
    }
  }
  return rc;
}

namespace {

void fill_info(ks_system* s, ks_iter_info* info) {
  if (!info) return;
  const LsState* hl = host_ls(s);
  info->k = hl->k;
  info->nfe = hl->nfe;
  info->backtracks = hl->backtracks;
  info->stop_reason = hl->stop;
  info->energy = hl->E;
  info->grad_norm = std::sqrt(std::max(hl->g2, 0.0));
  info->tau = hl->tau_acc;
  info->C = hl->C;
}

// The saved state of a run: this header, then the device records of the current slot.
struct StateHeader {
  uint64_t magic;
  int version, disc, precision, n, p, es;
  size_t bytes;
  ks_opt_params prm;
  int reorths, pcg_extra, pcg_probe, last_cg_iters;
  long long cg_total;
};
constexpr uint64_t kStateMagic = 0x3145544154534b53ull;  // "KSSTATE1"
constexpr size_t kStateHead = 512;
static_assert(sizeof(StateHeader) <= kStateHead, "state header must fit its slot");

struct Part {
  void* ptr;
  size_t bytes;
};

// Device records a trial from slot c reads (see enqueue_trial): the orbital blocks and
// their Gram blocks, the warm-start Hartree potential, the evaluation summary and the
// line-search state.
std::vector<Part> state_parts(ks_system* s, int c) {
  const size_t blk = (size_t)s->n * s->p * s->es, pp2 = (size_t)s->pp * s->pp;
  std::vector<Part> v = {{s->X[c], blk}, {s->G[c], blk}, {s->D[c], blk},
                         {s->vh[c], (size_t)s->n * sizeof(double)},
                         {s->gxg[c], 3 * pp2 * sizeof(double)},
                         {s->gxd[c], 3 * pp2 * sizeof(double)},
                         {s->ev[c], sizeof(EvalOut)}, {s->ls, sizeof(LsState)},
                         {s->reorth_count, sizeof(int)}};
  if (s->q1) {
    v.push_back({s->Gt[c], blk});
    v.push_back({s->BX[c], blk});
    v.push_back({s->BD[c], blk});
    v.push_back({s->feg[c], 3 * pp2 * sizeof(double)});
    v.push_back({s->wyg[c], 3 * pp2 * sizeof(double)});
  }
  return v;
}

size_t state_size(ks_system* s) {
  size_t off = kStateHead;
  for (const Part& q : state_parts(s, 0)) off += (q.bytes + 255) / 256 * 256;
  return off;
}

}  // namespace

int ks_minimize_begin(ks_system* s, const void* X0, const ks_opt_params* o, ks_iter_info* info) {
  if (!s || !X0) return fail(s, KS_E_INVAL, "null argument");
  MinRun* m = &s->run;
  int rc = run_begin(s, const_cast<void*>(X0), o, m);
  m->X_inout = nullptr;  // results leave through ks_minimize_end
  if (rc) {
    m->active = false;
    return rc;
  }
  fill_info(s, info);
  const LsState* hl = host_ls(s);
  if (hl->error) return fail(s, hl->error, ks_status_string(hl->error));
  return KS_OK;
}

int ks_minimize_step(ks_system* s, ks_iter_info* info) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  MinRun* m = &s->run;
  if (!m->active) return fail(s, KS_E_INVAL, "no run in progress (ks_minimize_begin)");
  LsState* hl = host_ls(s);
  while (hl->stop == KS_STOP_NONE && !hl->error) {
    int rc = run_trial(s, m);
    if (rc) {
      m->active = false;
      return rc;
    }
    if (hl->accepted) break;
  }
  fill_info(s, info);
  if (hl->error) return fail(s, hl->error, ks_status_string(hl->error));
  return KS_OK;
}

int ks_minimize_end(ks_system* s, void* X_out, ks_result* r) {
  if (!s) return fail(s, KS_E_INVAL, "null system");
  if (!s->run.active) return fail(s, KS_E_INVAL, "no run in progress (ks_minimize_begin)");
  return run_end(s, &s->run, r, X_out);
}

size_t ks_state_bytes(ks_system* s) { return s ? state_size(s) : 0; }

int ks_get_state(ks_system* s, void* buf) {
  if (!s || !buf) return fail(s, KS_E_INVAL, "null argument");
  MinRun* m = &s->run;
  if (!m->active) return fail(s, KS_E_INVAL, "no run in progress (ks_minimize_begin)");
  StateHeader h{};
  h.magic = kStateMagic;
  h.version = 1;
  h.disc = s->d.disc;
  h.precision = s->d.precision;
  h.n = s->n;
  h.p = s->p;
  h.es = s->es;
  h.bytes = state_size(s);
  h.prm = m->prm;
  h.reorths = m->reorths;
  h.pcg_extra = s->pcg_extra;
  h.pcg_probe = s->pcg_probe ? 1 : 0;
  h.last_cg_iters = s->last_cg_iters;
  h.cg_total = s->cg_total;
  char* dst = static_cast<char*>(buf);
  hipError_t e = hipMemcpyAsync(dst, &h, sizeof(h), hipMemcpyDefault, s->st);
  size_t off = kStateHead;
  for (const Part& q : state_parts(s, m->c)) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst + off, q.ptr, q.bytes, hipMemcpyDefault, s->st);
    off += (q.bytes + 255) / 256 * 256;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  return hip_check(s, e, "state copy");
}

int ks_set_state(ks_system* s, const void* buf) {
  if (!s || !buf) return fail(s, KS_E_INVAL, "null argument");
  StateHeader h{};
  hipError_t e = hipMemcpyAsync(&h, buf, sizeof(h), hipMemcpyDefault, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  int rc = hip_check(s, e, "state header copy");
  if (rc) return rc;
  if (h.magic != kStateMagic || h.version != 1)
    return fail(s, KS_E_INVAL, "not a saved run state");
  if (h.disc != s->d.disc || h.precision != s->d.precision || h.n != s->n || h.p != s->p ||
      h.es != s->es || h.bytes != state_size(s))
    return fail(s, KS_E_INVAL, "saved state belongs to a system of another shape");
  MinRun* m = &s->run;
  const int c = s->cur;
  const char* src = static_cast<const char*>(buf);
  size_t off = kStateHead;
  for (const Part& q : state_parts(s, c)) {
    if (e == hipSuccess) e = hipMemcpyAsync(q.ptr, src + off, q.bytes, hipMemcpyDefault, s->st);
    off += (q.bytes + 255) / 256 * 256;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->host, s->cg,
                       reinterpret_cast<char*>(s->ls + 1) - reinterpret_cast<char*>(s->cg),
                       hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  rc = hip_check(s, e, "state copy");
  if (rc) return rc;
  drop_graphs(s);
  m->prm = h.prm;
  m->lp = to_params(h.prm);
  m->qr = h.prm.retraction == KS_QR;
  m->c = c;
  m->X_inout = nullptr;
  m->t0 = std::chrono::steady_clock::now();
  m->active = true;
  m->queued = false;
  m->records = false;
  m->reorths = h.reorths;
  s->bf16_on = !host_ls(s)->bf16_off;
  s->pcg_extra = h.pcg_extra;
  s->pcg_probe = h.pcg_probe != 0;
  s->last_cg_iters = h.last_cg_iters;
  s->cg_total = h.cg_total;
  return KS_OK;
}

int ks_batch_step(ks_system* const* sys, int count, ks_iter_info* info) {
  if (!sys || count < 1 || count > kMaxBatch) return fail(nullptr, KS_E_INVAL, "bad batch");
  for (int i = 0; i < count; ++i) {
    if (!sys[i]) return fail(nullptr, KS_E_INVAL, "null system");
    for (int j = 0; j < i; ++j)
      if (sys[j] == sys[i]) return fail(nullptr, KS_E_INVAL, "a system is listed twice");
    if (!sys[i]->run.active)
      return fail(sys[i], KS_E_INVAL, "no run in progress (ks_minimize_begin)");
    if (!batchable(sys[i], sys[i]->run))
      return fail(sys[i], KS_E_UNSUPPORTED, "run outside the lockstep runner's limits");
  }
  BatchEngine e;
  e.st = sys[0]->st;
  e.finish = false;
  int rc = KS_OK;
  for (int i = 0; i < count && rc == KS_OK; ++i) {
    ks_system* s = sys[i];
    rc = hip_check(s, hipStreamSynchronize(s->st), "batch start");
    if (rc == KS_OK && !s->run.records) rc = upload_records(s, s->run);
    const LsState* hl = host_ls(s);
    if (rc == KS_OK && hl->stop == KS_STOP_NONE && !hl->error) {
      BatchMember* bm = new BatchMember();
      bm->s = s;
      e.act.push_back(bm);
    }
  }
  if (rc == KS_OK && !e.act.empty()) rc = batch_tick(&e);
  if (rc == KS_OK) rc = hip_check(sys[0], hipStreamSynchronize(e.st), "batch step sync");
  for (auto* bm : e.act) delete bm;
  for (auto* bm : e.fin) {
    if (rc == KS_OK && bm->code != KS_OK) rc = bm->code;
    delete bm;
  }
  e.act.clear();
  e.fin.clear();
  if (e.ev) (void)hipEventDestroy(e.ev);
  e.ev = nullptr;
  for (int i = 0; i < count; ++i) fill_info(sys[i], info ? info + i : nullptr);
  return rc;
}

int ks_minimize_batch(ks_system* const* sys, int count, void* const* X_inout,
                      const ks_opt_params* o, ks_result* r, int* codes) {
  if (!sys || !X_inout || count < 1 || count > kMaxBatch)
    return fail(nullptr, KS_E_INVAL, "bad batch");
  for (int i = 0; i < count; ++i)
    if (!sys[i] || !X_inout[i]) return fail(nullptr, KS_E_INVAL, "null system or block");
  BatchEngine* e = batch_create(sys[0]->st);
  for (int i = 0; i < count; ++i) {
    hipError_t he = hipStreamSynchronize(sys[i]->st);
    if (he != hipSuccess) {
      batch_destroy(e);
      return hip_check(sys[i], he, "batch start");
    }
    (void)batch_add(e, sys[i], X_inout[i], o, reinterpret_cast<void*>((intptr_t)i));
  }
  int rc = KS_OK;
  while (batch_size(e) > 0 && rc == KS_OK) rc = batch_tick(e);
  void* tag = nullptr;
  ks_result res{};
  int code = KS_OK;
  int worst = rc;
  while (batch_take(e, &tag, &res, &code)) {
    const int i = (int)(intptr_t)tag;
    if (r) r[i] = res;
    if (codes) codes[i] = code;
    if (worst == KS_OK && code != KS_OK && code != KS_E_NOT_CONVERGED) worst = code;
  }
  batch_destroy(e);
  return worst;
}

}  // extern "C"
